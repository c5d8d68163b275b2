"""Parity of the HIP path (through the C ABI) with the CPU oracle and with
closed forms.  Tolerances: the exact discrete adjoint (serial method) must
match the oracle to rounding (1e-11); the Paraexp path replaces the RK4
propagation of the homogeneous pieces by exact exponentials, so it differs
from the oracle by the RK4 time-discretisation gap plus the Krylov
tolerance: rel L2 <= 1e-8 (FP64 gate).
"""
import math
import sys

import numpy as np
import pytest

import fourier
from conftest import rel
from paper_2004_00546_amd import _lib, api, workloads

pytestmark = pytest.mark.gpu

FP64_GATE = 1e-8


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    _lib.load()
    return _t


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run(inst, method="paraexp", **kw):
    r = api.GradientRunner([inst], method=method, **kw)
    r.run()
    out = r.results()[0]
    code, est = r.status()
    out["status"] = code
    out["est"] = est
    return out


def small_advdiff(n=64, T=0.5, nt=500, P=4, m=30, K=3, seed=0, nu=0.05):
    rng = np.random.default_rng(seed)
    L = 2 * math.pi
    G = workloads.gaussian_pulses_1d(n, L, L * rng.uniform(0, 1, K), 0.3)
    return dict(op="advdiff1d", control="forcing", nx=n, ny=1, L=L, vx=1.0,
                vy=0.0, nu=nu, T=T, omega=1.0, beta=1e-3, n_steps=nt, P=P, m=m,
                basis=G, a=rng.standard_normal(K), u_tgt=rng.standard_normal(n),
                q0=np.zeros(n))


# ---- serial method: exact discrete adjoint -------------------------------

@pytest.mark.parametrize("n", [64, 128, 2048])
def test_serial_matches_oracle_to_rounding(torch, orc, n):
    inst = small_advdiff(n=n, T=0.25, nt=250 if n <= 512 else 2500, P=5,
                         nu=0.01 if n > 512 else 0.05)
    say("serial parity n=%d" % n)
    got = run(inst, "serial")
    want = orc.gradient(inst)
    assert rel(got["qT"], want["qT"]) < 1e-12
    assert abs(got["J"] - want["J"]) < 1e-12 * abs(want["J"])
    assert rel(got["lam"], want["Lambda"]) < 1e-11
    assert rel(got["grad"], want["grad"]) < 1e-11


def test_serial_workload_n128(torch, orc):
    inst = workloads.make("advdiff1d_n128")[0]
    got = run(inst, "serial")
    want = orc.gradient(inst)
    say("n128 serial", rel(got["grad"], want["grad"]))
    assert rel(got["grad"], want["grad"]) < 1e-11
    assert rel(got["qT"], want["qT"]) < 1e-12


# ---- Krylov exponential pieces against closed forms ----------------------

@pytest.mark.parametrize("krylov", ["poly", "shift_invert"])
@pytest.mark.parametrize("wl", ["advdiff1d_n128", "advdiff1d_n4096"])
def test_adjoint_piece_vs_fourier(torch, wl, krylov):
    """paraexp_adjoint propagates lamT by exp(tau A^T) and forms
    Lambda = int_0^T sin(w(T - s)) exp(s A^T) lamT ds: both against the
    Fourier closed form (no RK4 involved)."""
    inst = workloads.make(wl)[0]
    say("adjoint piece", wl, krylov)
    n = inst["nx"]
    rng = np.random.default_rng(1)
    lamT = np.asarray(inst["u_tgt"]) + 0.1 * np.sin(np.arange(n) * 2 * np.pi / n * 3)
    p = api.make_problem(inst, krylov=krylov, tol=1e-12)
    # lam0 needs IC control semantics: ask for both outputs directly.
    dev = torch.device("cuda:0")
    f64 = dict(dtype=torch.float64, device=dev)
    ws = torch.empty(_lib.pxp_workspace_size([p]), dtype=torch.uint8, device=dev)
    _lib.pxp_workspace_init(ws)
    lt = torch.tensor(lamT, **f64)
    lam0 = torch.zeros(n, **f64)
    Lam = torch.zeros(n, **f64)
    _lib.paraexp_adjoint([p], lt, lam0, Lam, ws)
    code, est = _lib.pxp_device_status(ws)
    torch.cuda.synchronize()
    lam_eig = fourier.eigenvalues(inst)
    want0 = fourier.exp_action_T(inst, inst["T"], lamT, lam_eig)
    mu = np.conj(lam_eig)
    T, w = inst["T"], inst["omega"]
    tr = (w * np.exp(mu * T) - mu * np.sin(w * T) - w * np.cos(w * T)) / (mu ** 2 + w ** 2)
    wantL = np.fft.ifft(tr * np.fft.fft(lamT)).real
    e0 = rel(lam0.cpu().numpy(), want0)
    eL = rel(Lam.cpu().numpy(), wantL)
    say("  lam0 %.2e Lambda %.2e est %.2e status %d" % (e0, eL, est, code))
    assert code == 0
    assert e0 < 1e-9 and eL < 1e-9


@pytest.mark.parametrize("n,kblock", [(64, 0), (256, 0), (512, 64), (1024, 0), (1024, 256),
                                      (2048, 64), (2048, 128), (4096, 256)])
def test_shift_invert_chunk_shapes_vs_fourier(torch, n, kblock):
    """The uniform shift-and-invert solve eliminates each thread's chunk of
    N/B points and reduces the B chunk interfaces cyclically: every chunk
    length 1..32 and workgroup size 64..512 must give the same exponential
    and integral as the Fourier closed form."""
    h = 2 * np.pi / n
    nt = max(500, int(0.5 * (4 * 0.02 / h ** 2 + 1.0 / h) / 2.0) + 1)  # RK4-stable grid
    inst = small_advdiff(n=n, T=0.5, nt=nt, P=1, m=48, nu=0.02)
    p = api.make_problem(inst, krylov="shift_invert", tol=1e-11, kblock=kblock)
    dev = torch.device("cuda:0")
    f64 = dict(dtype=torch.float64, device=dev)
    ws = torch.empty(_lib.pxp_workspace_size([p]), dtype=torch.uint8, device=dev)
    _lib.pxp_workspace_init(ws)
    x = np.arange(n) * 2 * np.pi / n
    # smooth data (a pulse and two modes): the space converges well within
    # m on every grid, so the comparison tests the solve, not convergence
    lamT = np.exp(-(x - np.pi) ** 2 / (2 * 0.3 ** 2)) + np.sin(3 * x) + 0.5 * np.cos(7 * x)
    lam0 = torch.zeros(n, **f64)
    Lam = torch.zeros(n, **f64)
    _lib.paraexp_adjoint([p], torch.tensor(lamT, **f64), lam0, Lam, ws)
    code, est = _lib.pxp_device_status(ws)
    lam_eig = fourier.eigenvalues(inst)
    want0 = fourier.exp_action_T(inst, inst["T"], lamT, lam_eig)
    mu = np.conj(lam_eig)
    T, w = inst["T"], inst["omega"]
    tr = (w * np.exp(mu * T) - mu * np.sin(w * T) - w * np.cos(w * T)) / (mu ** 2 + w ** 2)
    wantL = np.fft.ifft(tr * np.fft.fft(lamT)).real
    e0, eL = rel(lam0.cpu().numpy(), want0), rel(Lam.cpu().numpy(), wantL)
    say("si chunks n=%d kblock=%d: lam0 %.2e Lambda %.2e est %.1e status %d"
        % (n, kblock, e0, eL, est, code))
    assert code == 0
    assert e0 < 1e-9 and eL < 1e-9


def test_krylov_full_dimension_is_exact(torch):
    """m = N on a tiny grid: the Krylov space exhausts the space (happy
    breakdown at dimension N), so exp(T A^T) v must match to rounding."""
    inst = small_advdiff(n=16, T=0.3, nt=300, P=1, m=16, nu=0.05)
    p = api.make_problem(inst, krylov="poly", tol=1e-12, m=16)
    dev = torch.device("cuda:0")
    f64 = dict(dtype=torch.float64, device=dev)
    ws = torch.empty(_lib.pxp_workspace_size([p]), dtype=torch.uint8, device=dev)
    _lib.pxp_workspace_init(ws)
    v = np.random.default_rng(2).standard_normal(16)
    lam0 = torch.zeros(16, **f64)
    _lib.paraexp_adjoint([p], torch.tensor(v, **f64), lam0, None, ws)
    code, _ = _lib.pxp_device_status(ws)
    want = fourier.exp_action_T(inst, inst["T"], v)
    say("full-dim", rel(lam0.cpu().numpy(), want))
    assert rel(lam0.cpu().numpy(), want) < 1e-12


# ---- Paraexp end to end ---------------------------------------------------

@pytest.mark.parametrize("krylov,sched", [("poly", "classic"), ("poly", "chain"),
                                          ("shift_invert", "classic"),
                                          ("shift_invert", "chain")])
def test_paraexp_workload_n128(torch, orc, krylov, sched):
    inst = workloads.make("advdiff1d_n128")[0]
    # per-piece estimate tolerance; m = 30 shift-and-invert spaces on this
    # mildly stiff grid reach about 1e-9 on the longest piece
    got = run(inst, krylov=krylov, sched=sched,
              tol=1e-8 if krylov == "shift_invert" else 1e-10)
    want = orc.gradient(inst)
    eq, eg = rel(got["qT"], want["qT"]), rel(got["grad"], want["grad"])
    say("n128 paraexp %s/%s: qT %.2e grad %.2e est %.1e st %d"
        % (krylov, sched, eq, eg, got["est"], got["status"]))
    assert got["status"] == 0
    assert eq < FP64_GATE and eg < FP64_GATE
    assert abs(got["J"] - want["J"]) < FP64_GATE * abs(want["J"])


def test_paraexp_single_slice_equals_serial(torch):
    """P = 1: the direct solve has no homogeneous piece; q(T) must equal the
    serial march bit for bit."""
    inst = small_advdiff(n=128, P=1)
    a = run(inst, "paraexp")
    b = run(inst, "serial")
    assert np.array_equal(a["qT"], b["qT"])


@pytest.mark.parametrize("P", [2, 5, 25])
def test_paraexp_slice_counts(torch, orc, P):
    inst = small_advdiff(n=128, T=0.5, nt=500, P=P)
    got = run(inst, krylov="poly", sched="classic")
    want = orc.gradient(inst)
    say("P=%d qT %.2e grad %.2e" % (P, rel(got["qT"], want["qT"]), rel(got["grad"], want["grad"])))
    assert rel(got["qT"], want["qT"]) < FP64_GATE
    assert rel(got["grad"], want["grad"]) < FP64_GATE


@pytest.mark.parametrize("P,krylov,sched", [(500, "poly", "classic"),
                                            (500, "poly", "chain"),
                                            (250, "auto", "chain"),
                                            (100, "taylor", "classic")])
def test_paraexp_many_short_slices(torch, orc, P, krylov, sched):
    """Degenerate partitions: one or two RK4 steps per slice, so nearly all of
    the horizon is carried by the exponentials of the homogeneous pieces
    (hundreds of them in one launch, or one chain of that length).  At two
    steps per slice tau*rho is about 0.2 on this grid, so AUTO takes Taylor;
    shift-and-invert is not meant for such short pieces (its inverse is
    nearly the identity) and its estimate says so."""
    inst = small_advdiff(n=128, T=0.5, nt=500, P=P)
    got = run(inst, krylov=krylov, sched=sched, tol=1e-10)
    want = orc.gradient(inst)
    eq, eg = rel(got["qT"], want["qT"]), rel(got["grad"], want["grad"])
    say("P=%d %s/%s qT %.2e grad %.2e st %d" % (P, krylov, sched, eq, eg, got["status"]))
    assert got["status"] == 0
    assert eq < FP64_GATE and eg < FP64_GATE


def test_ragged_batch_equals_one_by_one(torch):
    insts = [small_advdiff(n=64, seed=3), small_advdiff(n=256, seed=4, P=5),
             small_advdiff(n=128, seed=5, P=2)]
    r = api.GradientRunner(insts, krylov="poly")
    r.run()
    batch = r.results()
    for inst, b in zip(insts, batch):
        one = run(inst, krylov="poly")
        assert np.array_equal(one["grad"], b["grad"])
        assert np.array_equal(one["qT"], b["qT"])


def test_deterministic(torch):
    inst = workloads.make("advdiff1d_n128")[0]
    a = run(inst, krylov="shift_invert")
    b = run(inst, krylov="shift_invert")
    assert np.array_equal(a["grad"], b["grad"]) and np.array_equal(a["qT"], b["qT"])


def test_nonconvergence_is_flagged(torch):
    """A Krylov dimension of 2 with a 1e-14 tolerance cannot meet the
    estimate in one shift-and-invert space: the device status says so."""
    inst = workloads.make("advdiff1d_n128")[0]
    got = run(inst, krylov="shift_invert", m=2, tol=1e-14)
    assert got["status"] == _lib.PXP_EKRYLOV_NOCONV


def test_paraexp_workload_n4096(torch, orc):
    inst = workloads.make("advdiff1d_n4096")[0]
    say("n4096: oracle (about 12 s)")
    want = orc.gradient(inst)
    # per-piece tolerances: the 40-dimensional shift-and-invert spaces of
    # the longest pieces estimate about 1e-10
    for krylov, sched, tol in [("shift_invert", "classic", 1e-9), ("poly", "chain", 1e-10)]:
        got = run(inst, krylov=krylov, sched=sched, tol=tol)
        eq, eg = rel(got["qT"], want["qT"]), rel(got["grad"], want["grad"])
        say("n4096 %s/%s qT %.2e grad %.2e est %.1e st %d"
            % (krylov, sched, eq, eg, got["est"], got["status"]))
        assert got["status"] == 0
        assert eq < FP64_GATE and eg < FP64_GATE
    got = run(inst, "serial")
    assert rel(got["grad"], want["grad"]) < 1e-11


# ---- Burgers: serial direct with checkpoints, time-varying adjoint --------

def small_burgers(n=256, T=0.5, nt=1024, P=16, nu=0.02, K=8, seed=7, ckpt=64):
    rng = np.random.default_rng(seed)
    phases = rng.uniform(0, 2 * math.pi, K)
    return dict(op="burgers1d", control="ic", nx=n, ny=1, L=2 * math.pi, vx=0.0,
                vy=0.0, nu=nu, T=T, omega=1.0, beta=1e-3, n_steps=nt, P=P, m=30,
                ckpt_every=ckpt,
                basis=workloads.burgers_ic_modes(n, 2 * math.pi, phases),
                a=0.3 * rng.standard_normal(K) / np.arange(1, K + 1),
                u_tgt=rng.standard_normal(n), q0=np.zeros(n))


@pytest.mark.parametrize("ckpt", [16, 64])
def test_burgers_serial_matches_oracle_to_rounding(torch, orc, ckpt):
    inst = small_burgers(ckpt=ckpt)
    got = run(inst, "serial")
    want = orc.gradient(inst)
    say("burgers serial ckpt=%d: qT %.2e lam0 %.2e grad %.2e" % (
        ckpt, rel(got["qT"], want["qT"]), rel(got["lam"], want["lam0"]),
        rel(got["grad"], want["grad"])))
    assert rel(got["qT"], want["qT"]) < 1e-12
    assert rel(got["lam"], want["lam0"]) < 1e-11
    assert rel(got["grad"], want["grad"]) < 1e-11


# The Magnus macro step is one slice; its fourth-order error needs slices of
# at most 64 RK4 steps here (P = 4, i.e. 256 steps, measures 9e-7).  The
# a posteriori Magnus check estimates up to 1.3e-8 at P = 16 (the adjoint's
# actual error 3.8e-9): the piece tolerance 1e-7 lets every P pass it.
@pytest.mark.parametrize("P", [16, 32, 64])
def test_burgers_paraexp_small(torch, orc, P):
    inst = small_burgers(P=P)
    got = run(inst, "paraexp", krylov="poly", tol=1e-7)
    want = orc.gradient(inst)
    el, eg = rel(got["lam"], want["lam0"]), rel(got["grad"], want["grad"])
    say("burgers paraexp P=%d: lam0 %.2e grad %.2e st %d est %.1e" % (P, el, eg, got["status"], got["est"]))
    assert got["status"] == 0
    assert rel(got["qT"], want["qT"]) < 1e-12  # direct is the same serial march
    assert el < FP64_GATE and eg < FP64_GATE


def test_magnus_check_flags_long_slices(torch, orc):
    """The a posteriori Magnus check: one macro step against two half steps
    of lambda_T on the first and the last slice, the fourth-order Richardson
    estimate of the step's relative error.  At a 1e-9 piece tolerance,
    slices of 256 and 64 RK4 steps are flagged as not converged and the
    estimate follows the adjoint's actual error (within a factor 10); slices
    of 16 steps pass."""
    inst = small_burgers()
    want = orc.gradient(inst)
    for P, flagged in [(4, True), (16, True), (64, False)]:
        got = run(dict(inst, P=P), "paraexp", krylov="poly", tol=1e-9)
        e = rel(got["lam"], want["lam0"])
        say("magnus check P=%d: adjoint error %.2e estimate %.2e status %d"
            % (P, e, got["est"], got["status"]))
        assert (got["status"] == _lib.PXP_EKRYLOV_NOCONV) == flagged
        if flagged:
            assert 0.1 * e <= got["est"] <= 10.0 * e


def test_magnus_check_batched_per_instance(torch, orc):
    """The same check on the batched Burgers path: each instance's report
    carries its own estimate, within a factor 20 of its adjoint's actual
    error where the Magnus error dominates, and the batch status is
    flagged at a 1e-9 tolerance."""
    insts = ragged_burgers(seed=40)
    r = api.GradientRunner(insts, method="paraexp", krylov="poly", tol=1e-9)
    _lib.pxp_last_report(r.problems, r.ws)
    r.run()
    res = r.results()
    rep = _lib.pxp_last_report(r.problems, r.ws)
    code, _ = r.status()
    assert code == _lib.PXP_EKRYLOV_NOCONV
    for inst, b, x in zip(insts, res, rep):
        e = rel(b["lam"], orc.gradient(inst)["lam0"])
        say("batched magnus check n=%d P=%d: adjoint error %.2e estimate %.2e"
            % (inst["nx"], inst["P"], e, x["max_est"]))
        if e > 1e-9:
            assert e / 20.0 <= x["max_est"] <= 20.0 * e


def test_burgers_workload_n2048(torch, orc):
    inst = workloads.make("burgers1d_n2048")[0]
    want = orc.gradient(inst)
    # the Magnus check estimates 1e-10 here (adjoint error 2e-10)
    got = run(inst, "paraexp", krylov="poly", tol=1e-9)
    el, eg = rel(got["lam"], want["lam0"]), rel(got["grad"], want["grad"])
    say("burgers n2048 paraexp: lam0 %.2e grad %.2e st %d est %.1e" % (el, eg, got["status"], got["est"]))
    assert got["status"] == 0
    assert el < FP64_GATE and eg < FP64_GATE
    ser = run(inst, "serial")
    assert rel(ser["grad"], want["grad"]) < 1e-11


# ---- FP32 bulk: stencil/RK in FP32 (compensated), Krylov algebra in FP64 ----

FP32_GATE = 1e-5


@pytest.mark.parametrize("wl,krylov", [("advdiff1d_n128", "poly"),
                                       ("advdiff1d_n4096", "shift_invert"),
                                       ("burgers1d_n2048", "poly")])
def test_fp32_bulk_within_gate(torch, orc, wl, krylov):
    inst = workloads.make(wl)[0]
    want = orc.gradient(inst)
    lam_key = "Lambda" if inst["control"] == "forcing" else "lam0"
    for method in ("paraexp", "serial"):
        # the Krylov estimate cannot go below the FP32 noise of the slice
        # states: tolerance 1e-6 in this mode
        got = run(inst, method, krylov=krylov, prec="fp32_bulk", tol=1e-6)
        e = dict(qT=rel(got["qT"], want["qT"]), adj=rel(got["lam"], want[lam_key]),
                 grad=rel(got["grad"], want["grad"]))
        say("fp32 bulk %s %s: %s st %d" % (wl, method, e, got["status"]))
        assert got["status"] == 0
        assert max(e.values()) < FP32_GATE


def test_fp32_bulk_compensation_matters(torch, orc):
    """The compensated FP32 state update keeps the serial march near FP64
    accuracy over 40 000 steps (plain FP32 accumulation drifts far more)."""
    inst = workloads.make("advdiff1d_n4096")[0]
    got = run(inst, "serial", prec="fp32_bulk")
    want = orc.gradient(inst)
    say("fp32 serial n4096 qT %.2e" % rel(got["qT"], want["qT"]))
    assert rel(got["qT"], want["qT"]) < 1e-6


# ---- ragged Burgers batches (one launch per phase) -------------------------

def ragged_burgers(seed=21):
    out = []
    for i, (n, nu, T) in enumerate([(256, 0.02, 0.4), (512, 0.01, 0.3),
                                    (1024, 0.02, 0.2), (512, 0.015, 0.5),
                                    (256, 0.03, 0.25)]):
        dt = 0.8 * workloads.burgers_dt_bound(n, nu)
        nt = 64 * int(math.ceil(T / (64 * dt)))
        # Magnus macro steps of at most T/16 (as in the ragged workload)
        inst = small_burgers(n=n, T=T, nt=nt, P=nt // 4, nu=nu, seed=seed + i,
                             ckpt=16)
        out.append(inst)
    return out


@pytest.mark.parametrize("method", ["paraexp", "serial"])
def test_ragged_burgers_batch_equals_one_by_one(torch, method):
    insts = ragged_burgers()
    # slices of four RK4 steps: Magnus estimates up to about 1e-8
    r = api.GradientRunner(insts, method=method, krylov="poly", tol=1e-7)
    r.run()
    code, _ = r.status()
    assert code == 0
    batch = r.results()
    for inst, b in zip(insts, batch):
        one = run(inst, method, krylov="poly", tol=1e-7)
        assert np.array_equal(one["qT"], b["qT"])
        assert np.array_equal(one["grad"], b["grad"]), (inst["nx"], method)


def test_ragged_burgers_serial_sweep_512(torch, orc):
    """Every instance a multiple of 512 points (2, 4 and 8 per thread at 512
    threads): the batched reverse sweep runs at 512 threads.  It must agree
    with the one-by-one calls and, at the small size, with the oracle."""
    insts = []
    for i, (n, nu) in enumerate([(1024, 0.02), (2048, 0.02), (4096, 0.03), (1024, 0.01)]):
        dt = 0.8 * workloads.burgers_dt_bound(n, nu)
        nt = 64 * int(math.ceil(0.02 / (64 * dt)))
        insts.append(small_burgers(n=n, T=0.02, nt=nt, P=nt // 16, nu=nu, seed=60 + i,
                                   ckpt=16))
    r = api.GradientRunner(insts, method="serial")
    r.run()
    code, _ = r.status()
    assert code == 0
    batch = r.results()
    for inst, b in zip(insts, batch):
        one = run(inst, "serial")
        e = rel(b["grad"], one["grad"])
        say("serial sweep 512 n=%d nt=%d: batch vs one %.2e" % (inst["nx"], inst["n_steps"], e))
        assert np.array_equal(one["qT"], b["qT"])
        assert e < 1e-13
    want = orc.gradient(insts[0])
    assert rel(batch[0]["grad"], want["grad"]) < 1e-11


def test_ragged_burgers_batch_vs_oracle(torch, orc):
    insts = ragged_burgers(seed=40)
    r = api.GradientRunner(insts, method="paraexp", krylov="poly")
    r.run()
    for inst, b in zip(insts, r.results()):
        want = orc.gradient(inst)
        e = rel(b["grad"], want["grad"])
        say("ragged n=%d nt=%d P=%d grad %.2e" % (inst["nx"], inst["n_steps"], inst["P"], e))
        assert e < FP64_GATE


def test_ragged_workload_sample_vs_oracle(torch, orc):
    """Four instances of the 64-instance ragged workload (N = 1024 .. 8192)
    with the horizon cut to a quarter: same grids, viscosities, time steps
    and Magnus macro-step lengths, FP32 bulk."""
    full = workloads.make("burgers1d_ragged")
    picks = [full[i] for i in (0, 1, 4, 5)]
    insts = []
    for inst in picks:
        nt = inst["n_steps"] // 4
        insts.append(dict(inst, n_steps=nt, T=inst["T"] / 4, P=inst["P"] // 4))
    r = api.GradientRunner(insts, method="paraexp", krylov="poly", prec="fp32_bulk", tol=1e-6)
    r.run()
    code, _ = r.status()
    assert code == 0
    for inst, b in zip(insts, r.results()):
        want = orc.gradient(inst)
        e = rel(b["grad"], want["grad"])
        say("ragged workload n=%d nt=%d fp32 grad %.2e" % (inst["nx"], inst["n_steps"], e))
        assert e < FP32_GATE


# ---- shift-and-invert Magnus factors for the Burgers adjoint ---------------
# (I - gamma J(W)^T) is periodic tridiagonal with variable coefficients; the
# kernel solves it by chunk elimination plus cyclic reduction of the chunk
# interfaces.  n = 256 and 512 give one point per thread (the interface
# system is the whole system), larger n give 2 and 4 points per chunk.

@pytest.mark.parametrize("n", [256, 512, 1024, 2048])
def test_burgers_shift_invert_matches_oracle(torch, orc, n):
    nu = 0.02 if n <= 512 else 0.01
    dt = 0.8 * workloads.burgers_dt_bound(n, nu)
    nt = 64 * int(math.ceil(0.4 / (64 * dt)))
    inst = small_burgers(n=n, T=0.4, nt=nt, P=nt // 4 if nt // 4 <= 64 else 64,
                         nu=nu, seed=50 + n, ckpt=16)
    if nt % inst["P"]:
        inst["P"] = 16
    got = run(inst, "paraexp", krylov="shift_invert")
    want = orc.gradient(inst)
    e = rel(got["grad"], want["grad"])
    say("burgers SI n=%d nt=%d P=%d: grad %.2e lam0 %.2e" % (
        n, nt, inst["P"], e, rel(got["lam"], want["lam0"])))
    assert e < FP64_GATE


def test_burgers_shift_invert_workload(torch, orc):
    inst = workloads.make("burgers1d_n2048")[0]
    got = run(inst, "paraexp", krylov="shift_invert")
    want = orc.gradient(inst)
    e = rel(got["grad"], want["grad"])
    say("burgers SI C3: grad %.2e" % e)
    assert e < FP64_GATE


def test_ragged_burgers_shift_invert_batch(torch, orc):
    """Batched shift-and-invert equals one-by-one runs bitwise and the
    polynomial-Krylov result at the same macro steps (both flavours compute
    the same Magnus factors); against the oracle with macro steps of two RK4
    steps, so that the Magnus error stays far below the gate."""
    insts = ragged_burgers(seed=60)
    r = api.GradientRunner(insts, method="paraexp", krylov="shift_invert", tol=1e-7)
    r.run()
    code, _ = r.status()
    assert code == 0
    for inst, b in zip(insts, r.results()):
        one = run(inst, "paraexp", krylov="shift_invert", tol=1e-7)
        assert np.array_equal(one["grad"], b["grad"]), inst["nx"]
        poly = run(inst, "paraexp", krylov="poly", tol=1e-7)
        d = rel(b["grad"], poly["grad"])
        fine = dict(inst, P=inst["n_steps"] // 2)
        sif = run(fine, "paraexp", krylov="shift_invert")
        want = orc.gradient(inst)["grad"]
        say("ragged SI n=%d P=%d: SI vs poly %.2e; vs oracle SI %.2e poly %.2e; P=%d SI %.2e"
            % (inst["nx"], inst["P"], d, rel(b["grad"], want), rel(poly["grad"], want),
               fine["P"], rel(sif["grad"], want)))
        assert d < 1e-9
        assert rel(sif["grad"], want) < FP64_GATE


def test_auto_flavour_ragged_equals_explicit_choice(torch):
    """AUTO picks the Chebyshev flavour per instance where its chain kernel
    covers the grid; elsewhere shift-and-invert where half a slice times the
    diffusion spectral radius exceeds 64, else Taylor; each batched result
    equals the run with that flavour named explicitly."""
    def chain_shape(n):
        return (n <= 256 and n % 64 == 0) or any(
            n % b == 0 and (n // b) & (n // b - 1) == 0 and n // b <= cap
            for b, cap in ((256, 8), (512, 16)))
    insts = ragged_burgers(seed=70)
    insts[2] = dict(insts[2], P=insts[2]["n_steps"] // 64)  # long macro steps
    # (long macro steps: a loose piece tolerance keeps the Magnus check
    # quiet; the test is about the flavour choice)
    r = api.GradientRunner(insts, method="paraexp", krylov="auto", tol=1e-5)
    r.run()
    assert r.status()[0] == 0
    rep = _lib.pxp_last_report(r.problems, r.ws)
    for inst, b, rp in zip(insts, r.results(), rep):
        h = inst["L"] / inst["nx"]
        si = 0.5 * inst["T"] / inst["P"] * 4 * inst["nu"] / h**2 > 64
        kr = "chebyshev" if chain_shape(inst["nx"]) else ("shift_invert" if si else "taylor")
        assert rp["krylov_adjoint"] == kr, (inst["nx"], rp)
        one = run(inst, "paraexp", krylov=kr, tol=1e-5)
        assert np.array_equal(one["grad"], b["grad"]), (inst["nx"], si)


# ---- absorbed adjoint: the batch of adjoint inhomogeneous slices ----------

@pytest.mark.parametrize("wl,krylov,sched", [("advdiff1d_n128", "poly", "classic"),
                                             ("advdiff1d_n128", "poly", "chain"),
                                             ("advdiff1d_n4096", "shift_invert", "classic")])
def test_absorbed_adjoint_matches_oracle(torch, orc, wl, krylov, sched):
    """The absorbed form (adjoint slices from zero with source A^T lamT as one
    batch, their end states propagated by classic pieces) against the oracle
    and against the unabsorbed form (one homogeneous piece from lamT)."""
    inst = workloads.make(wl)[0]
    tol = 1e-9 if krylov == "shift_invert" else 1e-10
    a = run(inst, "paraexp", krylov=krylov, sched=sched, tol=tol, absorbed=True)
    b = run(inst, "paraexp", krylov=krylov, sched=sched, tol=tol)
    want = orc.gradient(inst)
    ea = rel(a["grad"], want["grad"])
    say("absorbed %s %s %s: grad %.2e (unabsorbed %.2e), Lambda %.2e vs unabsorbed %.2e, status %d"
        % (wl, krylov, sched, ea, rel(b["grad"], want["grad"]),
           rel(a["lam"], want["Lambda"]), rel(a["lam"], b["lam"]), a["status"]))
    assert a["status"] == 0
    assert ea < FP64_GATE
    assert rel(a["lam"], b["lam"]) < 1e-8


def test_absorbed_adjoint_ic_control(torch, orc):
    inst = small_advdiff(n=64, T=0.5, nt=500, P=5)
    inst = dict(inst, control="ic")
    a = run(inst, "paraexp", krylov="poly", absorbed=True)
    want = orc.gradient(inst)
    say("absorbed IC: lam0 %.2e grad %.2e" % (rel(a["lam"], want["lam0"]),
                                              rel(a["grad"], want["grad"])))
    assert rel(a["grad"], want["grad"]) < FP64_GATE
    assert rel(a["lam"], want["lam0"]) < FP64_GATE


@pytest.mark.parametrize("case", ["advdiff1d_n128", "burgers_small"])
def test_taylor_flavour_matches_oracle(torch, orc, case):
    """The Taylor flavour (no Arnoldi process) on the register-resident 1D
    pieces and on the Burgers Magnus factors (the Jacobian bounds its own
    norm in the kernel)."""
    if case == "burgers_small":
        inst = small_burgers(n=512, T=0.3, nt=128, P=32, nu=0.01, seed=9, ckpt=16)
    else:
        inst = workloads.make(case)[0]
    # Burgers: the Magnus check estimates a little above 1e-10 for these
    # slices (gradient error 9e-11), so the piece tolerance is 1e-9 there
    got = run(inst, "paraexp", krylov="taylor",
              tol=1e-9 if case == "burgers_small" else 1e-10)
    want = orc.gradient(inst)
    e = rel(got["grad"], want["grad"])
    say("taylor %s: grad %.2e status %d est %.1e" % (case, e, got["status"], got["est"]))
    assert got["status"] == 0
    assert e < FP64_GATE


@pytest.mark.parametrize("n,nu,P", [(256, 0.02, 16), (512, 0.01, 32), (2048, 0.005, 128)])
def test_chebyshev_flavour_matches_oracle_and_taylor(torch, orc, n, nu, P):
    """The Chebyshev flavour of the Burgers Magnus factors (series on the
    Gershgorin interval, coefficients from the Bessel recurrence in the
    kernel): against the oracle, against the Taylor flavour (both are
    within the piece tolerance of the same factors), and with fewer stencil
    applications where the interval is wide.  The N = 2048 case has
    half-widths of about 8 per factor (no substeps); the coarse cases cover
    small intervals, where both flavours need about as many terms."""
    if n == 2048:
        inst = workloads.make("burgers1d_n2048")[0]
    else:
        inst = small_burgers(n=n, T=0.3, nt=256, P=P, nu=nu, seed=9, ckpt=16)
    want = orc.gradient(inst)
    res = {}
    for kr in ("chebyshev", "taylor"):
        r = api.GradientRunner([inst], method="paraexp", krylov=kr, tol=1e-10)
        _lib.pxp_last_report(r.problems, r.ws)
        r.run()
        out = r.results()[0]
        code, est = r.status()
        rep = _lib.pxp_last_report(r.problems, r.ws)[0]
        res[kr] = (out, code, est, rep)
        say("%s n=%d: grad %.2e lam0 %.2e status %d est %.1e terms %d" % (
            kr, n, rel(out["grad"], want["grad"]), rel(out["lam"], want["lam0"]), code, est,
            rep["iterations"]))
    ch, ta = res["chebyshev"], res["taylor"]
    assert ch[3]["krylov_adjoint"] == "chebyshev"
    assert rel(ch[0]["grad"], want["grad"]) < FP64_GATE
    assert rel(ch[0]["lam"], want["lam0"]) < FP64_GATE
    assert rel(ch[0]["lam"], ta[0]["lam"]) < 1e-9
    assert ch[1] == ta[1]
    if n == 2048:
        assert ch[3]["iterations"] < ta[3]["iterations"]


# ---- non-finite inputs reach the device status ------------------------------

@pytest.mark.parametrize("case", ["advdiff_paraexp", "advdiff_serial", "burgers_paraexp",
                                  "burgers_serial"])
def test_nan_input_sets_nonfinite_status(torch, case):
    """A NaN in the initial state must come back as PXP_ENONFINITE (not a
    silent NaN gradient with PXP_OK) on every path."""
    if case.startswith("advdiff"):
        inst = small_advdiff(n=128, T=0.25, nt=250, P=5)
        q0 = np.zeros(inst["nx"])
        q0[17] = np.nan
        inst = dict(inst, q0=q0)
    else:
        inst = small_burgers()
        inst = dict(inst, q0=np.zeros(inst["nx"]))
        inst["q0"][5] = np.nan
    method = "serial" if case.endswith("serial") else "paraexp"
    say("nan input: %s" % case)
    r = api.GradientRunner([inst], method=method, krylov="auto", tol=1e-10)
    r.run()
    code, _ = r.status()
    assert code == _lib.PXP_ENONFINITE, (case, code)
    # the status is cleared by the read: a clean run reports OK again
    r2 = api.GradientRunner([dict(inst, q0=np.zeros(inst["nx"]))], method=method,
                            krylov="auto", tol=1e-7)
    r2.run()
    assert r2.status()[0] == _lib.PXP_OK


# ---- the one-call boundary entry point ----------------------------------------

@pytest.mark.parametrize("wl", ["advdiff1d_n128", "advdiff1d_n4096"])
def test_gradient_entry_point_matches_oracle(torch, orc, wl):
    """gradient() (include/paraexp.h) called through ctypes on the workload as
    stated, compared with the oracle at the FP64 gate."""
    inst = workloads.make(wl)[0]
    r = api.GradientRunner([inst], method="paraexp", krylov="auto", tol=1e-9)
    say("gradient() on %s" % wl)
    _lib.gradient(r.problems, r.ctrl, r.basis, r.q0, r.u_tgt, r.J, r.grad, r.qT, r.ws)
    got = r.results()[0]
    code, est = r.status()
    want = orc.gradient(inst)
    eg, eq = rel(got["grad"], want["grad"]), rel(got["qT"], want["qT"])
    say("  grad %.2e  qT %.2e  J %.2e  status %d" % (eg, eq, abs(got["J"] - want["J"]) /
                                                     abs(want["J"]), code))
    assert code == 0
    assert eg <= FP64_GATE and eq <= FP64_GATE
    assert abs(got["J"] - want["J"]) <= FP64_GATE * abs(want["J"])
    # no single component far off either (max-abs relative to the largest)
    assert np.max(np.abs(got["grad"] - want["grad"])) <= FP64_GATE * np.max(np.abs(want["grad"]))


# ---- per-instance report and per-class counters ---------------------------------

def test_last_report_per_instance(torch):
    """A mixed batch (1D linear, Burgers, 2D) reports each instance's resolved
    flavours, its own substeps and iterations, and an estimate within the
    tolerance; reading clears the statistics."""
    import test_gpu_2d_uniform as u2
    insts = [small_advdiff(n=128, T=0.25, nt=250, P=5), small_burgers(P=128),
             u2.small2d(P=16)]
    probs = [api.make_problem(x, krylov="auto", sched=sc, tol=1e-10)
             for x, sc in zip(insts, ("classic", "classic", "tree"))]
    r = api.GradientRunner(insts, method="paraexp", problems=probs)
    r.run()
    assert r.status()[0] == 0
    rep = _lib.pxp_last_report(r.problems, r.ws)
    say("report", rep)
    a, b, c = rep
    assert a["P"] == 5 and a["sched"] == "classic" and a["krylov_direct"] == "taylor"
    assert a["substeps"] >= 5 and a["iterations"] > 0 and 0.0 <= a["max_est"] <= 1e-10
    assert b["krylov_direct"] is None and b["sched"] is None
    assert b["krylov_adjoint"] in ("chebyshev", "shift_invert") and b["substeps"] > 0
    assert c["krylov_direct"] == "uniform" and c["krylov_adjoint"] == "uniform"
    assert c["sched"] == "tree" and c["substeps"] >= 16 and c["iterations"] > 0
    assert 0.0 < c["max_est"] <= 1e-12
    again = _lib.pxp_last_report(r.problems, r.ws)
    assert all(x["substeps"] == 0 and x["iterations"] == 0 for x in again)


def test_counters_by_class(torch):
    """Direct pieces and the adjoint piece count separately: P-1 classic
    pieces of at least one substep each, one adjoint exponential."""
    inst = small_advdiff(n=128, T=0.25, nt=250, P=5)
    r = api.GradientRunner([inst], method="paraexp", krylov="poly", sched="classic", tol=1e-10)
    _lib.pxp_device_counters(r.ws)
    r.run()
    d = _lib.pxp_device_counters_class(r.ws, 0)
    j = _lib.pxp_device_counters_class(r.ws, 1)
    tot = _lib.pxp_device_counters(r.ws)
    say("counters direct %s adjoint %s total %s" % (d, j, tot))
    assert d[0] >= 4 and j[0] >= 1
    assert tot == tuple(x + y for x, y in zip(d, j))


def test_ragged_workload_full_autotuned_graph_vs_oracle(torch, orc):
    """The 64-instance ragged Burgers workload as stated: full horizons, FP32
    bulk, slice counts autotuned within 32..256, the whole gradient captured
    in a hipGraph and replayed (bit-equal to the eager call); the oracle
    checks the cheapest instance of every grid size, N = 1024, 2048, 4096
    and 8192, at the FP32-bulk gate."""
    import time
    from concurrent.futures import ThreadPoolExecutor
    full = workloads.make("burgers1d_ragged")
    t0 = time.perf_counter()
    probs, rep = api.autotune(full, p_min=32, p_max=256, rtol=5e-6, krylov="auto",
                              prec="fp32_bulk", tol=1e-6)
    say("ragged autotune %.1f s: P %s" % (time.perf_counter() - t0,
                                           sorted({int(p.P) for p in probs})))
    assert all(32 <= int(p.P) <= 256 and x["n_steps"] % int(p.P) == 0
               for p, x in zip(probs, full))
    r = api.GradientRunner(full, method="paraexp", problems=probs)
    r.run()
    assert r.status()[0] == 0
    eager = [dict(grad=b["grad"].copy(), qT=b["qT"].copy()) for b in r.results()]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        r.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        r.run()
    for rep_i in range(2):
        r.grad.zero_()
        r.qT.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(eager, r.results()):
            assert np.array_equal(a["grad"], b["grad"]), rep_i
            assert np.array_equal(a["qT"], b["qT"]), rep_i
    assert r.status()[0] == 0
    res = r.results()
    cost = [x["nx"] * x["n_steps"] for x in full]
    picks = {}
    for i, x in enumerate(full):
        if x["nx"] not in picks or cost[i] < cost[picks[x["nx"]]]:
            picks[x["nx"]] = i
    assert sorted(picks) == [1024, 2048, 4096, 8192]
    say("oracle on instances %s" % sorted(picks.values()))
    with ThreadPoolExecutor(max_workers=4) as ex:
        refs = dict(zip(picks.values(), ex.map(lambda i: orc.gradient(full[i]), picks.values())))
    for i, want in refs.items():
        eg, eq = rel(res[i]["grad"], want["grad"]), rel(res[i]["qT"], want["qT"])
        say("  N=%d steps=%d P=%d: qT %.2e grad %.2e" % (full[i]["nx"], full[i]["n_steps"],
                                                       int(probs[i].P), eq, eg))
        assert eg < FP32_GATE and eq < FP32_GATE
