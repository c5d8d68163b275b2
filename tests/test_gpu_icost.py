"""Integral cost of section 4.2 (eq. cost) through the C ABI.

J = 1/T int_0^T |q - u_tgt|^2 dt + beta |a|^2 by the trapezoidal rule over the
RK4 step states; every step state is an argument of J and the adjoint is
driven by the step sources (eq. adjEquation).  Checked against the oracle's
exact discrete adjoint of that cost:
  - the Paraexp path (slices; the tree kept level by level and walked back
    down for the corrected slice-start states; every slice marched again from
    its corrected start, writing the sources and the cost; the adjoint slices
    with the sources as one batch; the tree of their pieces with their exact
    shares of Lambda) for several slice counts, both control kinds and every
    row length;
  - the serial march and its discrete adjoint with sources;
  - the step-source argument of paraexp_adjoint;
  - the four-diffusivity workload of section 4.2 at full size;
  - hipGraph replays.

Tolerances: the serial path does the oracle's arithmetic (RK4 steps, the
same sources), so it meets it to 1e-11; the Paraexp path replaces the RK4
propagation of the homogeneous pieces by exact exponentials (uniformised,
a priori tail krylov_tol / 100), so it differs from the oracle by the RK4
time error, well inside the FP64 gate 1e-8."""
import math
import sys

import numpy as np
import pytest

from conftest import rel, rel_max
from paper_2004_00546_amd import _lib, api, workloads

pytestmark = pytest.mark.gpu

FP64_GATE = 1e-8
SERIAL_GATE = 1e-11


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


def small_icost(nx=64, ny=32, T=0.5, nt=64, P=16, K=3, seed=5, nu=0.02, control="forcing",
                rough=False, width=0.05):
    """A small integral-cost instance.  The target is a few low Fourier modes
    (rough: white noise, which excites the grid's highest modes, where the
    RK4 step and the exact exponential differ most)."""
    rng = np.random.default_rng(seed)
    L = 2 * math.pi
    G = workloads.gaussian_blobs_2d(nx, ny, L, L * rng.uniform(0, 1, (K, 2)), width * L)
    a = rng.standard_normal(K)
    if rough:
        tgt = 0.1 * rng.standard_normal(nx * ny)
    else:
        x = np.arange(nx) * (L / nx)
        y = np.arange(ny) * (L / ny)
        tgt = np.zeros((ny, nx))
        for j in range(3):
            p, q = rng.integers(1, 4, 2)
            tgt += 0.1 * rng.standard_normal() * np.sin(p * x[None, :] + q * y[:, None]
                                                        + rng.uniform(0, L))
        tgt = tgt.ravel()
    return dict(op="advdiff2d_upwind", control=control, cost="integral", nx=nx, ny=ny,
                L=L, vx=1.0, vy=0.5, nu=nu, T=T, omega=1.0, beta=1e-3, n_steps=nt, P=P,
                m=30, basis=G, a=a, u_tgt=tgt, q0=np.zeros(nx * ny))


def check(got, want, gate, tag):
    eJ = abs(got["J"] - want["J"]) / abs(want["J"])
    eq = rel(got["qT"], want["qT"])
    eg = rel(got["grad"], want["grad"])
    say("%s: J %.2e qT %.2e lam %.2e grad %.2e (max %.2e)" % (
        tag, eJ, eq, got.get("elam", float("nan")), eg, rel_max(got["grad"], want["grad"])))
    assert eJ < gate and eq < gate and eg < gate
    assert rel_max(got["grad"], want["grad"]) < gate


def run(insts, method="paraexp", tol=1e-11):
    r = api.GradientRunner(insts, method=method, krylov="uniform", sched="tree", tol=tol)
    r.run()
    res = r.results()
    code, est = r.status()
    return res, code


@pytest.mark.parametrize("P,nt,T", [(16, 64, 0.5), (13, 52, 0.40625), (6, 24, 0.1875),
                                    (64, 64, 0.5), (1, 4, 0.03125)])
def test_icost_paraexp_matches_oracle(torch, orc, P, nt, T):
    inst = small_icost(P=P, nt=nt, T=T)
    res, code = run([inst])
    got = res[0]
    want = orc.gradient(inst)
    got["elam"] = rel(got["lam"], want["Lambda"])
    assert code == 0
    check(got, want, FP64_GATE, "icost paraexp P=%d nt=%d" % (P, nt))
    assert got["elam"] < FP64_GATE


def test_icost_rough_target_lambda_is_rk4_time_error(torch, orc):
    """With a white-noise target the adjoint sources reach the grid's highest
    modes, and the Lambda field differs from the oracle's (RK4 everywhere) by
    the RK4 time error of the homogeneous propagation, which the Paraexp path
    does exactly: halving the step shrinks it about 16-fold, fourth order,
    while the gradient stays inside the gate."""
    errs = []
    for nt in (64, 128):
        inst = small_icost(P=nt // 4, nt=nt, rough=True)
        res, code = run([inst])
        want = orc.gradient(inst)
        assert code == 0
        e = rel(res[0]["lam"], want["Lambda"])
        eg = rel(res[0]["grad"], want["grad"])
        say("rough target nt=%d: Lambda %.2e grad %.2e" % (nt, e, eg))
        assert eg < FP64_GATE
        errs.append(e)
    assert errs[0] / errs[1] > 10.0


def test_icost_ic_control_matches_oracle(torch, orc):
    # a smooth initial state: the comparison is then not dominated by the
    # RK4 time error of the grid's highest modes
    inst = small_icost(control="ic", P=16, width=0.15)
    res, code = run([inst])
    got = res[0]
    want = orc.gradient(inst)
    got["elam"] = rel(got["lam"], want["lam0"])
    assert code == 0
    check(got, want, FP64_GATE, "icost paraexp ic")
    assert got["elam"] < FP64_GATE


@pytest.mark.parametrize("control", ["forcing", "ic"])
def test_icost_serial_matches_oracle(torch, orc, control):
    # 66 steps: the last serial launch takes the two-step tail
    inst = small_icost(control=control, P=6, nt=66, T=0.515625)
    res, code = run([inst], method="serial")
    got = res[0]
    want = orc.gradient(inst)
    got["elam"] = rel(got["lam"], want["Lambda" if control == "forcing" else "lam0"])
    assert code == 0
    check(got, want, SERIAL_GATE, "icost serial %s" % control)
    assert got["elam"] < SERIAL_GATE


@pytest.mark.parametrize("nx,ny", [(128, 32), (256, 16)])
def test_icost_row_lengths(torch, orc, nx, ny):
    inst = small_icost(nx=nx, ny=ny, T=0.25, nt=64, P=16)
    res, code = run([inst])
    got = res[0]
    want = orc.gradient(inst)
    got["elam"] = rel(got["lam"], want["Lambda"])
    assert code == 0
    check(got, want, FP64_GATE, "icost %dx%d" % (nx, ny))
    assert got["elam"] < FP64_GATE


def test_icost_mixed_batch(torch, orc):
    """Integral-cost and terminal-cost instances of different row lengths and
    slice counts in one call."""
    a = small_icost(P=16)
    b = dict(small_icost(nx=128, ny=32, T=0.25, nt=48, P=12, seed=9), cost="terminal")
    c = small_icost(nx=128, ny=32, T=0.375, nt=96, P=24, seed=11)
    res, code = run([a, b, c])
    assert code == 0
    for inst, got, tag in zip([a, b, c], res, "abc"):
        want = orc.gradient(inst)
        got["elam"] = rel(got["lam"], want["Lambda"])
        check(got, want, FP64_GATE, "mixed %s" % tag)
        assert got["elam"] < FP64_GATE


def test_icost_adjoint_source_argument(torch, orc):
    """paraexp_adjoint with step sources built on the host from the oracle's
    trajectory (dJ/dq_n of the trapezoidal cost), without and with a final
    condition: equals the oracle's integral-cost adjoint (plus, by linearity,
    its terminal adjoint of that final condition)."""
    inst = small_icost(P=16)
    n = inst["nx"] * inst["ny"]
    nt, T = inst["n_steps"], inst["T"]
    F = inst["a"] @ inst["basis"]
    _, tr = orc.direct(inst, np.zeros(n), F, traj=True)
    w = np.full(nt + 1, T / nt / T)
    w[0] = w[-1] = 0.5 / nt
    g = 2.0 * w[:, None] * (tr - inst["u_tgt"][None, :])
    want = orc.gradient(inst)
    dev = torch.device("cuda:0")
    f64 = dict(dtype=torch.float64, device=dev)
    p = api.make_problem(inst, krylov="uniform", sched="tree", tol=1e-11)
    ws = torch.empty(_lib.pxp_workspace_size([p]), dtype=torch.uint8, device=dev)
    _lib.pxp_workspace_init(ws)
    src = torch.tensor(g.ravel(), **f64)
    lam0 = torch.zeros(n, **f64)
    Lam = torch.zeros(n, **f64)
    _lib.paraexp_adjoint([p], None, lam0, Lam, ws, jI_src=src)
    e0, eL = rel(lam0.cpu().numpy(), want["lam0"]), rel(Lam.cpu().numpy(), want["Lambda"])
    say("source argument: lam0 %.2e Lambda %.2e" % (e0, eL))
    assert _lib.pxp_device_status(ws)[0] == 0
    assert e0 < FP64_GATE and eL < FP64_GATE
    # with a final condition as well
    lamT = 10.0 * inst["u_tgt"]  # smooth (a few low modes)
    t0, tL = orc.adjoint(dict(inst, cost="terminal"), tr, F, lamT)
    _lib.paraexp_adjoint([p], torch.tensor(lamT, **f64), lam0, Lam, ws, jI_src=src)
    e0 = rel(lam0.cpu().numpy(), want["lam0"] + t0)
    eL = rel(Lam.cpu().numpy(), want["Lambda"] + tL)
    say("source argument + final condition: lam0 %.2e Lambda %.2e" % (e0, eL))
    assert e0 < FP64_GATE and eL < FP64_GATE


def test_icost_workload_full_size_vs_oracle(torch, orc):
    """The section 4.2 stand-in as stated: four diffusivities on 128^2,
    T = 10, 2048 steps in 512 slices, one call; the oracle checks the least
    and the most diffusive instance (the largest adjoint piece has Poisson
    parameter about 1000 there)."""
    full = workloads.make("advdiff2d_icost")
    res, code = run(full, tol=1e-9)
    assert code == 0
    for i in (0, 3):
        say("oracle for D=%g (%d steps)" % (full[i]["nu"], full[i]["n_steps"]))
        want = orc.gradient(full[i])
        got = res[i]
        got["elam"] = rel(got["lam"], want["Lambda"])
        check(got, want, FP64_GATE, "icost workload D=%g" % full[i]["nu"])
        assert got["elam"] < FP64_GATE
    for b in res:
        assert np.all(np.isfinite(b["grad"])) and b["J"] > 0.0


def test_icost_graph_replay(torch):
    """The integral-cost gradient captured in a hipGraph and replayed three
    times with eager work in between: every replay equals the eager result
    bit for bit."""
    insts = [small_icost(P=16), small_icost(nx=128, ny=32, T=0.375, nt=48, P=24, seed=11)]
    r = api.GradientRunner(insts, method="paraexp", krylov="uniform", sched="tree",
                           tol=1e-11)
    r.run()
    ref = [dict(grad=b["grad"].copy(), J=b["J"], lam=b["lam"].copy()) for b in r.results()]
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
        r.J.zero_()
        r.lam.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(ref, r.results()):
            assert np.array_equal(a["grad"], b["grad"]), rep
            assert a["J"] == b["J"], rep
            assert np.array_equal(a["lam"], b["lam"]), rep
    assert r.status()[0] == 0


# ---- Burgers: the hybrid serial-direct-parallel-adjoint scheme (section 3.3) --

def small_burgers_icost(n=256, T=0.5, nt=1024, P=64, nu=0.02, K=8, seed=7, ckpt=16, **hyb):
    rng = np.random.default_rng(seed)
    phases = rng.uniform(0, 2 * math.pi, K)
    x = np.arange(n) * (2 * math.pi / n)
    inst = dict(op="burgers1d", control="ic", cost="integral", nx=n, ny=1, L=2 * math.pi,
                vx=0.0, vy=0.0, nu=nu, T=T, omega=1.0, beta=1e-3, n_steps=nt, P=P, m=30,
                ckpt_every=ckpt,
                basis=workloads.burgers_ic_modes(n, 2 * math.pi, phases),
                a=0.3 * rng.standard_normal(K) / np.arange(1, K + 1),
                u_tgt=0.1 * np.sin(2 * x + 0.3), q0=np.zeros(n))
    inst.update(hyb)
    return inst


def run_b(insts, method="paraexp", tol=1e-9, krylov="poly"):
    r = api.GradientRunner(insts, method=method, krylov=krylov, tol=tol)
    r.run()
    res = r.results()
    code, est = r.status()
    return res, code, r


def test_burgers_icost_serial_matches_oracle(torch, orc):
    """The serial march writes the step sources; the discrete adjoint adds
    them after every reverse step, from dJ/dq(T): the oracle's arithmetic."""
    inst = small_burgers_icost()
    res, code, _ = run_b([inst], method="serial")
    got, want = res[0], orc.gradient(inst)
    eJ = abs(got["J"] - want["J"]) / abs(want["J"])
    say("burgers icost serial: J %.2e lam0 %.2e grad %.2e" % (
        eJ, rel(got["lam"], want["lam0"]), rel(got["grad"], want["grad"])))
    assert code == 0
    assert eJ < SERIAL_GATE
    assert rel(got["qT"], want["qT"]) < SERIAL_GATE
    assert rel(got["lam"], want["lam0"]) < SERIAL_GATE
    assert rel(got["grad"], want["grad"]) < SERIAL_GATE


@pytest.mark.parametrize("hyb", [dict(), dict(hyb_group=1), dict(hyb_slices=16, hyb_k=2.0),
                                 dict(hyb_slices=7, hyb_k=1.0, hyb_group=3)])
def test_burgers_icost_hybrid_matches_oracle(torch, orc, hyb):
    """The hybrid scheme: march launches per adjoint slice, the adjoint
    slices with their sources on the side stream as the march passes them,
    then the Magnus chain from dJ/dq(T) adding each slice's end state.
    Equal slices (one per macro step), one slice per adjoint launch, and the
    partition of eq. nonEquiP with k = 2 and k = 1 (slices shrinking toward
    T, rounded to the macro-step grid)."""
    inst = small_burgers_icost(**hyb)
    res, code, _ = run_b([inst])
    got, want = res[0], orc.gradient(inst)
    eJ = abs(got["J"] - want["J"]) / abs(want["J"])
    el, eg = rel(got["lam"], want["lam0"]), rel(got["grad"], want["grad"])
    say("burgers icost hybrid %s: J %.2e qT %.2e lam0 %.2e grad %.2e" % (
        hyb, eJ, rel(got["qT"], want["qT"]), el, eg))
    assert code == 0
    # the direct is the serial march, split into launches: rounding only
    assert rel(got["qT"], want["qT"]) < 1e-12 and eJ < 1e-12
    assert el < FP64_GATE and eg < FP64_GATE


def test_burgers_icost_hybrid_graph_replay(torch):
    """The hybrid scheme's fork and join of the side stream captured in a
    hipGraph: three replays, with eager work in between, equal the eager
    result bit for bit."""
    insts = [small_burgers_icost(hyb_slices=16, hyb_k=2.0)]
    r = api.GradientRunner(insts, method="paraexp", krylov="poly", tol=1e-9)
    r.run()
    ref = r.results()[0]
    ref = dict(grad=ref["grad"].copy(), J=ref["J"], lam=ref["lam"].copy())
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
        r.J.zero_()
        r.lam.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        b = r.results()[0]
        assert np.array_equal(ref["grad"], b["grad"]), rep
        assert ref["J"] == b["J"], rep
        assert np.array_equal(ref["lam"], b["lam"]), rep
        r.run()
        torch.cuda.synchronize()
    assert r.status()[0] == 0


def test_burgers_icost_workload_vs_oracle(torch, orc):
    """The N = 2048 Burgers workload (T = 2, 8192 steps, 128 Magnus steps,
    checkpoints every 64) with the integral cost: hybrid scheme with 128
    equal adjoint slices and with 32 slices of eq. nonEquiP (k = 2.5); the
    serial method beside it."""
    base = workloads.make("burgers1d_n2048")[0]
    inst = dict(base, cost="integral")
    say("burgers icost n2048: oracle (about 20 s)")
    want = orc.gradient(inst)
    for hyb in (dict(), dict(hyb_slices=32, hyb_k=2.5)):
        res, code, _ = run_b([dict(inst, **hyb)])
        got = res[0]
        el, eg = rel(got["lam"], want["lam0"]), rel(got["grad"], want["grad"])
        say("  hybrid %s: lam0 %.2e grad %.2e status %d" % (hyb, el, eg, code))
        assert code == 0
        assert el < FP64_GATE and eg < FP64_GATE
    res, code, _ = run_b([inst], method="serial")
    assert rel(res[0]["grad"], want["grad"]) < SERIAL_GATE
