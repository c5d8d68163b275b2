"""2D exponentials by uniformisation (krylov "uniform") through the C ABI:
the adjoint piece and its time integral against the Fourier closed forms of
the circulant operator, the tree and chain schedules of the direct pieces
against the CPU oracle, the full 16-instance 256 x 256 workload against the
oracle on its longest and shortest horizons, and hipGraph replays.

Tolerances: the uniformised exponential is exact up to the a priori Poisson
tail (krylov_tol / 100) and rounding, so the pieces meet the closed forms to
1e-10; the Paraexp gradient differs from the oracle's RK4 by the RK4 time
error, well inside the FP64 gate 1e-8."""
import math
import sys

import numpy as np
import pytest

import fourier
from conftest import rel, rel_max
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


def small2d(nx=64, ny=32, T=0.5, nt=64, P=16, K=3, seed=3, nu=0.02, control="forcing"):
    rng = np.random.default_rng(seed)
    L = 2 * math.pi
    G = workloads.gaussian_blobs_2d(nx, ny, L, L * rng.uniform(0, 1, (K, 2)), 0.05 * L)
    return dict(op="advdiff2d_upwind", control=control, nx=nx, ny=ny, L=L, vx=1.0,
                vy=0.5, nu=nu, T=T, omega=1.0, beta=1e-3, n_steps=nt, P=P, m=30,
                basis=G, a=rng.standard_normal(K), u_tgt=rng.standard_normal(nx * ny),
                q0=np.zeros(nx * ny))


def adjoint_piece(torch, inst, want0=True, wantL=True, tol=1e-12):
    n = inst["nx"] * inst["ny"]
    p = api.make_problem(inst, krylov="uniform", sched="tree", tol=tol)
    dev = torch.device("cuda:0")
    f64 = dict(dtype=torch.float64, device=dev)
    ws = torch.empty(_lib.pxp_workspace_size([p]), dtype=torch.uint8, device=dev)
    _lib.pxp_workspace_init(ws)
    lam0 = torch.zeros(n, **f64) if want0 else None
    Lam = torch.zeros(n, **f64) if wantL else None
    lamT = np.asarray(inst["u_tgt"])
    _lib.paraexp_adjoint([p], torch.tensor(lamT, **f64), lam0, Lam, ws)
    code, est = _lib.pxp_device_status(ws)
    return (lam0.cpu().numpy() if want0 else None,
            Lam.cpu().numpy() if wantL else None, code, est)


def fourier_adjoint(inst):
    lamT = np.asarray(inst["u_tgt"])
    lam_eig = fourier.eigenvalues(inst)
    want0 = fourier.exp_action_T(inst, inst["T"], lamT, lam_eig)
    mu = np.conj(lam_eig)
    T, w = inst["T"], inst["omega"]
    tr = (w * np.exp(mu * T) - mu * np.sin(w * T) - w * np.cos(w * T)) / (mu ** 2 + w ** 2)
    wantL = fourier._ifft(inst, tr * fourier._fft(inst, lamT))
    return want0, wantL


@pytest.mark.parametrize("outs", [(True, True), (True, False), (False, True)])
def test_uniform_adjoint_piece_vs_fourier(torch, outs):
    inst = small2d(nx=64, ny=64, T=0.7, nt=64, P=16)
    l0, L, code, est = adjoint_piece(torch, inst, *outs)
    want0, wantL = fourier_adjoint(inst)
    e0 = rel(l0, want0) if outs[0] else 0.0
    eL = rel(L, wantL) if outs[1] else 0.0
    say("uniform adjoint piece %s: lam0 %.2e Lambda %.2e est %.1e" % (outs, e0, eL, est))
    assert code == 0
    assert e0 < 1e-10 and eL < 1e-10
    assert 0.0 < est <= 1e-14


@pytest.mark.parametrize("nx,ny", [(128, 32), (256, 16)])
def test_uniform_adjoint_row_lengths(torch, nx, ny):
    inst = small2d(nx=nx, ny=ny, T=0.4, nt=64, P=16)
    l0, L, code, est = adjoint_piece(torch, inst)
    want0, wantL = fourier_adjoint(inst)
    e0, eL = rel(l0, want0), rel(L, wantL)
    say("uniform adjoint %dx%d: lam0 %.2e Lambda %.2e" % (nx, ny, e0, eL))
    assert code == 0 and e0 < 1e-10 and eL < 1e-10


def test_uniform_adjoint_substeps_vs_fourier(torch):
    """mu T above the largest Poisson parameter of one series: the piece is
    split into substeps, Lambda summed over them with shifted phases."""
    inst = small2d(nx=64, ny=64, T=30.0, nt=1024, P=256, nu=0.02)
    l0, L, code, est = adjoint_piece(torch, inst)
    want0, wantL = fourier_adjoint(inst)
    e0, eL = rel(l0, want0), rel(L, wantL)
    say("uniform adjoint substeps T=30: lam0 %.2e Lambda %.2e" % (e0, eL))
    assert code == 0 and e0 < 1e-10 and eL < 1e-10


@pytest.mark.parametrize("sched", ["tree", "chain"])
@pytest.mark.parametrize("P,nt,T", [(16, 64, 0.5), (6, 24, 0.1875), (13, 52, 0.40625),
                                    (64, 64, 0.5)])
def test_uniform_paraexp_2d_matches_oracle(torch, orc, sched, P, nt, T):
    inst = small2d(P=P, nt=nt, T=T)
    r = api.GradientRunner([inst], method="paraexp", krylov="uniform", sched=sched,
                           tol=1e-11)
    r.run()
    got = r.results()[0]
    code, est = r.status()
    want = orc.gradient(inst)
    eq, eg = rel(got["qT"], want["qT"]), rel(got["grad"], want["grad"])
    say("uniform %s P=%d nt=%d: qT %.2e Lam %.2e grad %.2e" % (
        sched, P, nt, eq, rel(got["lam"], want["Lambda"]), eg))
    assert code == 0
    assert eq < FP64_GATE and eg < FP64_GATE
    assert rel_max(got["qT"], want["qT"]) < FP64_GATE


def test_uniform_ic_control_matches_oracle(torch, orc):
    inst = small2d(control="ic", P=16)
    inst["basis"] = inst["basis"] * 0.5
    r = api.GradientRunner([inst], method="paraexp", krylov="auto", sched="tree", tol=1e-11)
    r.run()
    got = r.results()[0]
    want = orc.gradient(inst)
    say("uniform ic: lam0 %.2e grad %.2e" % (rel(got["lam"], want["lam0"]),
                                             rel(got["grad"], want["grad"])))
    assert r.status()[0] == 0
    assert rel(got["grad"], want["grad"]) < FP64_GATE


def test_workload_2d_full_batch_tree_vs_oracle(torch, orc):
    """All 16 instances of the 256 x 256 workload (horizons 0.5..2, 256 slices)
    in one call, tree schedule; the oracle checks the two longest horizons
    (1024 RK4 steps) and the shortest."""
    full = workloads.make("advdiff2d_256")
    r = api.GradientRunner(full, method="paraexp", krylov="auto", sched="tree", tol=1e-9)
    r.run()
    code, est = r.status()
    res = r.results()
    order = sorted(range(len(full)), key=lambda i: full[i]["n_steps"])
    for i in [order[-1], order[-2], order[0]]:
        say("oracle for instance %d (T=%.3f, %d steps)" % (i, full[i]["T"], full[i]["n_steps"]))
        want = orc.gradient(full[i])
        eq, eg = rel(res[i]["qT"], want["qT"]), rel(res[i]["grad"], want["grad"])
        eL = rel(res[i]["lam"], want["Lambda"])
        say("  qT %.2e Lambda %.2e grad %.2e  max-abs grad %.2e" % (
            eq, eL, eg, rel_max(res[i]["grad"], want["grad"])))
        assert eq < FP64_GATE and eg < FP64_GATE
        assert rel_max(res[i]["grad"], want["grad"]) < FP64_GATE
    assert code == 0
    for b in res:
        assert np.all(np.isfinite(b["grad"]))


def test_workload_2d_tree_graph_replay(torch):
    """The whole tree-schedule gradient of four 256 x 256 instances captured in
    a hipGraph and replayed three times, with eager work in between; every
    replay equals the eager result bit for bit."""
    full = workloads.make("advdiff2d_256")[:4]
    r = api.GradientRunner(full, method="paraexp", krylov="auto", sched="tree", tol=1e-9)
    r.run()
    ref = [dict(grad=b["grad"].copy(), qT=b["qT"].copy()) for b in r.results()]
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
        for a, b in zip(ref, r.results()):
            assert np.array_equal(a["grad"], b["grad"]), rep
            assert np.array_equal(a["qT"], b["qT"]), rep
    assert r.status()[0] == 0
