"""2D upwind advection-diffusion through the C ABI: the band RK4 marches
(slices, serial march and its exact discrete adjoint), the streamed 2D
Krylov pieces, and the whole Paraexp gradient, against the CPU oracle and
the Fourier closed forms.  Tolerances as for 1D: serial to rounding, Paraexp
within the FP64 gate 1e-8."""
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


def small2d(nx=64, ny=32, T=0.5, nt=64, P=16, m=30, K=3, seed=3, nu=0.02,
            control="forcing"):
    rng = np.random.default_rng(seed)
    L = 2 * math.pi
    G = workloads.gaussian_blobs_2d(nx, ny, L, L * rng.uniform(0, 1, (K, 2)), 0.05 * L)
    return dict(op="advdiff2d_upwind", control=control, nx=nx, ny=ny, L=L, vx=1.0,
                vy=0.5, nu=nu, T=T, omega=1.0, beta=1e-3, n_steps=nt, P=P, m=m,
                basis=G, a=rng.standard_normal(K), u_tgt=rng.standard_normal(nx * ny),
                q0=np.zeros(nx * ny))


def run(inst, method="paraexp", **kw):
    r = api.GradientRunner([inst], method=method, krylov="poly", **kw)
    r.run()
    out = r.results()[0]
    out["status"], out["est"] = r.status()
    return out


@pytest.mark.parametrize("nx,ny,nt", [(64, 32, 64), (128, 64, 37), (256, 16, 9)])
def test_serial_2d_matches_oracle_to_rounding(torch, orc, nx, ny, nt):
    """Serial band march and exact discrete adjoint; n_t not a multiple of the
    four steps per launch exercises the partial last launch."""
    inst = small2d(nx=nx, ny=ny, nt=nt, P=1, T=0.3 * nt / 64)
    got = run(inst, "serial")
    want = orc.gradient(inst)
    say("2d serial %dx%d nt=%d: qT %.2e Lam %.2e grad %.2e" % (
        nx, ny, nt, rel(got["qT"], want["qT"]), rel(got["lam"], want["Lambda"]),
        rel(got["grad"], want["grad"])))
    assert rel(got["qT"], want["qT"]) < 1e-12
    assert rel(got["lam"], want["Lambda"]) < 1e-11
    assert rel(got["grad"], want["grad"]) < 1e-11


def test_serial_2d_ic_control(torch, orc):
    inst = small2d(control="ic", P=1)
    inst["basis"] = inst["basis"] * 0.5
    got = run(inst, "serial")
    want = orc.gradient(inst)
    assert rel(got["lam"], want["lam0"]) < 1e-11
    assert rel(got["grad"], want["grad"]) < 1e-11


def test_slices_2d_p1_equals_serial(torch):
    """With one slice of at most four steps, the slice march from zero is
    the serial march."""
    inst = small2d(nt=4, P=1, T=0.03)
    a = run(inst, "paraexp")
    b = run(inst, "serial")
    assert rel(a["qT"], b["qT"]) < 1e-14


def test_adjoint_piece_2d_vs_fourier(torch):
    inst = small2d(nx=64, ny=64, T=0.7, nt=64, P=16, m=40)
    n = inst["nx"] * inst["ny"]
    lamT = np.asarray(inst["u_tgt"])
    p = api.make_problem(inst, krylov="poly", tol=1e-12)
    dev = torch.device("cuda:0")
    f64 = dict(dtype=torch.float64, device=dev)
    ws = torch.empty(_lib.pxp_workspace_size([p]), dtype=torch.uint8, device=dev)
    _lib.pxp_workspace_init(ws)
    lam0 = torch.zeros(n, **f64)
    Lam = torch.zeros(n, **f64)
    _lib.paraexp_adjoint([p], torch.tensor(lamT, **f64), lam0, Lam, ws)
    code, est = _lib.pxp_device_status(ws)
    lam_eig = fourier.eigenvalues(inst)
    want0 = fourier.exp_action_T(inst, inst["T"], lamT, lam_eig)
    mu = np.conj(lam_eig)
    T, w = inst["T"], inst["omega"]
    tr = (w * np.exp(mu * T) - mu * np.sin(w * T) - w * np.cos(w * T)) / (mu ** 2 + w ** 2)
    wantL = fourier._ifft(inst, tr * fourier._fft(inst, lamT))
    e0, eL = rel(lam0.cpu().numpy(), want0), rel(Lam.cpu().numpy(), wantL)
    say("2d adjoint piece: lam0 %.2e Lambda %.2e est %.1e" % (e0, eL, est))
    assert code == 0
    assert e0 < 1e-10 and eL < 1e-10


@pytest.mark.parametrize("sched", ["chain", "classic"])
@pytest.mark.parametrize("P", [16, 32])
def test_paraexp_2d_matches_oracle(torch, orc, sched, P):
    inst = small2d(P=P)
    got = run(inst, "paraexp", sched=sched, tol=1e-11)
    want = orc.gradient(inst)
    e = rel(got["grad"], want["grad"])
    say("2d paraexp %s P=%d: qT %.2e Lam %.2e grad %.2e status %d" % (
        sched, P, rel(got["qT"], want["qT"]), rel(got["lam"], want["Lambda"]), e,
        got["status"]))
    assert got["status"] == 0
    assert rel(got["qT"], want["qT"]) < FP64_GATE
    assert e < FP64_GATE


def test_batch_2d_equals_one_by_one(torch):
    insts = [small2d(seed=10), small2d(nx=128, ny=32, seed=11, T=0.4),
             small2d(nx=64, ny=64, seed=12, nt=32, P=8, T=0.25)]
    for method in ("paraexp", "serial"):
        r = api.GradientRunner(insts, method=method, krylov="poly", sched="chain")
        r.run()
        for inst, b in zip(insts, r.results()):
            one = run(inst, method, sched="chain")
            assert np.array_equal(one["grad"], b["grad"]), (method, inst["nx"])
            assert np.array_equal(one["qT"], b["qT"]), (method, inst["nx"])


def test_workload_2d_sample_vs_oracle(torch, orc):
    """Two instances of the 16-instance 256 x 256 workload (shortest
    horizons), batched, chain schedule, against the oracle."""
    full = workloads.make("advdiff2d_256")
    picks = sorted(range(len(full)), key=lambda i: full[i]["n_steps"])[:2]
    insts = [full[i] for i in picks]
    r = api.GradientRunner(insts, method="paraexp", krylov="poly", sched="chain")
    r.run()
    code, est = r.status()
    for inst, b in zip(insts, r.results()):
        want = orc.gradient(inst)
        e = rel(b["grad"], want["grad"])
        say("2d workload T=%.3f nt=%d: qT %.2e grad %.2e" % (
            inst["T"], inst["n_steps"], rel(b["qT"], want["qT"]), e))
        assert e < FP64_GATE
    assert code == 0


# ---- Taylor flavour: exp(tau A) v by the scaled truncated Taylor series ----

def test_adjoint_piece_2d_taylor_vs_fourier(torch):
    inst = small2d(nx=64, ny=64, T=0.7, nt=64, P=16, m=40)
    n = inst["nx"] * inst["ny"]
    lamT = np.asarray(inst["u_tgt"])
    p = api.make_problem(inst, krylov="taylor", tol=1e-12)
    dev = torch.device("cuda:0")
    f64 = dict(dtype=torch.float64, device=dev)
    ws = torch.empty(_lib.pxp_workspace_size([p]), dtype=torch.uint8, device=dev)
    _lib.pxp_workspace_init(ws)
    lam0 = torch.zeros(n, **f64)
    Lam = torch.zeros(n, **f64)
    _lib.paraexp_adjoint([p], torch.tensor(lamT, **f64), lam0, Lam, ws)
    code, est = _lib.pxp_device_status(ws)
    lam_eig = fourier.eigenvalues(inst)
    want0 = fourier.exp_action_T(inst, inst["T"], lamT, lam_eig)
    mu = np.conj(lam_eig)
    T, w = inst["T"], inst["omega"]
    tr = (w * np.exp(mu * T) - mu * np.sin(w * T) - w * np.cos(w * T)) / (mu ** 2 + w ** 2)
    wantL = fourier._ifft(inst, tr * fourier._fft(inst, lamT))
    e0, eL = rel(lam0.cpu().numpy(), want0), rel(Lam.cpu().numpy(), wantL)
    say("2d taylor adjoint piece: lam0 %.2e Lambda %.2e est %.1e" % (e0, eL, est))
    assert code == 0
    assert e0 < 1e-10 and eL < 1e-10


@pytest.mark.parametrize("sched", ["chain", "classic"])
def test_paraexp_2d_taylor_matches_oracle(torch, orc, sched):
    inst = small2d(P=16)
    got = run_flavour(inst, "taylor", sched=sched, tol=1e-11)
    want = orc.gradient(inst)
    e = rel(got["grad"], want["grad"])
    say("2d taylor %s: grad %.2e status %d" % (sched, e, got["status"]))
    assert got["status"] == 0 and e < FP64_GATE


def test_workload_2d_taylor_sample(torch, orc):
    full = workloads.make("advdiff2d_256")
    inst = min(full, key=lambda x: x["n_steps"])
    got = run_flavour(inst, "taylor", sched="chain")
    want = orc.gradient(inst)
    e = rel(got["grad"], want["grad"])
    say("2d workload taylor chain: grad %.2e" % e)
    assert got["status"] == 0 and e < FP64_GATE


def run_flavour(inst, krylov, **kw):
    r = api.GradientRunner([inst], method="paraexp", krylov=krylov, **kw)
    r.run()
    out = r.results()[0]
    out["report"] = _lib.pxp_last_report(r.problems, r.ws)[0]
    out["status"], out["est"] = r.status()
    return out


# ---- shift-and-invert flavour: Krylov on (I - gamma A)^{-1}, Fourier solve ----

@pytest.mark.parametrize("nx,ny,nt,tol,gate", [(64, 64, 64, 1e-11, 1e-9),
                                              (128, 32, 128, 1e-10, 1e-9),
                                              (256, 16, 128, 1e-9, 1e-8)])
def test_adjoint_piece_2d_si_vs_fourier(torch, nx, ny, nt, tol, gate):
    """lambda(0) = exp(T A^T) lambda_T and its time integral Lambda from one
    shift-and-invert space of the transposed operator (the 2D periodic
    solve by Fourier diagonalisation in every Arnoldi step), against the
    Fourier closed forms, on square and flat grids (a 16-point column
    transform on the 256 x 16 grid).  A random lambda_T excites every mode;
    the flat grids' wider spectra converge more slowly, hence their looser
    tolerances."""
    inst = small2d(nx=nx, ny=ny, T=0.7, nt=nt, P=16, m=50)
    n = inst["nx"] * inst["ny"]
    lamT = np.asarray(inst["u_tgt"])
    p = api.make_problem(inst, krylov="shift_invert", tol=tol)
    dev = torch.device("cuda:0")
    f64 = dict(dtype=torch.float64, device=dev)
    ws = torch.empty(_lib.pxp_workspace_size([p]), dtype=torch.uint8, device=dev)
    _lib.pxp_workspace_init(ws)
    lam0 = torch.zeros(n, **f64)
    Lam = torch.zeros(n, **f64)
    say("2d si adjoint piece: %d x %d, m=50" % (nx, ny))
    _lib.paraexp_adjoint([p], torch.tensor(lamT, **f64), lam0, Lam, ws)
    code, est = _lib.pxp_device_status(ws)
    lam_eig = fourier.eigenvalues(inst)
    want0 = fourier.exp_action_T(inst, inst["T"], lamT, lam_eig)
    mu = np.conj(lam_eig)
    T, w = inst["T"], inst["omega"]
    tr = (w * np.exp(mu * T) - mu * np.sin(w * T) - w * np.cos(w * T)) / (mu ** 2 + w ** 2)
    wantL = fourier._ifft(inst, tr * fourier._fft(inst, lamT))
    e0, eL = rel(lam0.cpu().numpy(), want0), rel(Lam.cpu().numpy(), wantL)
    say("2d si adjoint piece: lam0 %.2e Lambda %.2e est %.1e code %d" % (e0, eL, est, code))
    assert code == 0
    assert e0 < gate and eL < gate


@pytest.mark.parametrize("sched", ["chain", "classic"])
def test_paraexp_2d_si_matches_oracle(torch, orc, sched):
    inst = small2d(P=16)
    say("2d si paraexp %s: 64 x 32, P=16" % sched)
    got = run_flavour(inst, "shift_invert", sched=sched, tol=1e-11)
    want = orc.gradient(inst)
    e = rel(got["grad"], want["grad"])
    say("2d si %s: qT %.2e grad %.2e status %d" % (
        sched, rel(got["qT"], want["qT"]), e, got["status"]))
    assert got["status"] == 0
    assert rel(got["qT"], want["qT"]) < FP64_GATE and e < FP64_GATE
    rep = got["report"]
    assert rep["krylov_direct"] == "shift_invert" and rep["krylov_adjoint"] == "shift_invert"
    assert rep["sched"] == sched and rep["iterations"] > 0


def test_mixed_flavour_2d_batch_equals_one_by_one(torch):
    """A batch with polynomial and shift-and-invert instances (two launches
    of the 2D Krylov kernel, one per flavour) gives each instance the
    bits of its own call."""
    insts = [small2d(seed=20), small2d(nx=128, ny=32, seed=21, T=0.4),
             small2d(nx=64, ny=64, seed=22, nt=32, P=8, T=0.25)]
    kinds = ["shift_invert", "poly", "shift_invert"]
    say("2d mixed flavour batch")
    probs = [api.make_problem(i, krylov=k, sched="classic", tol=1e-11)
             for i, k in zip(insts, kinds)]
    r = api.GradientRunner(insts, method="paraexp", problems=probs)
    r.run()
    code, _ = r.status()
    assert code == 0
    for inst, k, b in zip(insts, kinds, r.results()):
        one = run_flavour(inst, k, sched="classic", tol=1e-11)
        assert np.array_equal(one["grad"], b["grad"]), k
        assert np.array_equal(one["qT"], b["qT"]), k


def test_workload_2d_si_sample(torch, orc):
    """The shortest instance of the 256 x 256 workload (P = 256, Krylov
    dimension 50) with shift-and-invert pieces, classic schedule (255
    independent pieces, each its own space), against the oracle."""
    import time
    full = workloads.make("advdiff2d_256")
    inst = min(full, key=lambda x: x["n_steps"])
    say("2d workload si classic: T=%.3f nt=%d" % (inst["T"], inst["n_steps"]))
    t0 = time.perf_counter()
    got = run_flavour(inst, "shift_invert", sched="classic")
    dt = time.perf_counter() - t0
    want = orc.gradient(inst)
    e = rel(got["grad"], want["grad"])
    say("2d workload si classic: grad %.2e qT %.2e status %d (%.2f s with setup)" % (
        e, rel(got["qT"], want["qT"]), got["status"], dt))
    assert got["status"] == 0 and e < FP64_GATE


@pytest.mark.parametrize("krylov,sched", [("shift_invert", "classic"), ("poly", "chain"),
                                          ("auto", "tree")])
def test_nan_input_2d_sets_nonfinite_status(torch, krylov, sched):
    """A NaN in the 2D initial state comes back as PXP_ENONFINITE on the
    Krylov flavours and on uniformisation, and a clean run after it reports
    OK again."""
    inst = small2d(P=16)
    q0 = np.zeros(inst["nx"] * inst["ny"])
    q0[100] = np.nan
    say("2d nan input: %s %s" % (krylov, sched))
    r = api.GradientRunner([dict(inst, q0=q0)], method="paraexp", krylov=krylov,
                           sched=sched, tol=1e-10)
    r.run()
    code, _ = r.status()
    assert code == _lib.PXP_ENONFINITE, (krylov, code)
    r2 = api.GradientRunner([inst], method="paraexp", krylov=krylov, sched=sched, tol=1e-10)
    r2.run()
    code2, _ = r2.status()
    assert code2 == 0, (krylov, code2)


def test_graph_replay_mixed_flavour_2d(torch):
    """A 2D batch of shift-and-invert and polynomial instances (two table
    uploads and two launches of the 2D Krylov kernel per phase) captured in
    a graph: every replay, with eager runs in between, gives the eager
    bits."""
    insts = [small2d(seed=30), small2d(nx=128, ny=32, seed=31, T=0.4)]
    probs = [api.make_problem(i, krylov=k, sched="classic", tol=1e-11)
             for i, k in zip(insts, ["shift_invert", "poly"])]
    say("2d mixed flavour graph replay")
    r = api.GradientRunner(insts, method="paraexp", problems=probs)
    r.run()
    eager = r.results()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        r.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        r.run()
    for rep in range(3):
        r.grad.zero_()
        r.qT.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(r.results(), eager):
            assert np.array_equal(a["grad"], b["grad"]), rep
            assert np.array_equal(a["qT"], b["qT"]), rep
        r.run()
        torch.cuda.synchronize()
    assert r.status()[0] == 0
