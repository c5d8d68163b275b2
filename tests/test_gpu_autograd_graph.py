"""torch.autograd.Function over the C ABI, and hipGraph capture of the
whole gradient call."""
import numpy as np
import pytest

from conftest import rel
from paper_2004_00546_amd import _lib, api, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    _lib.load()
    return _t


@pytest.mark.parametrize("wl,krylov", [("advdiff1d_n128", "poly"),
                                       ("advdiff1d_n128", "shift_invert"),
                                       ("burgers1d_n2048", "poly"),
                                       ("burgers1d_n2048", "auto"),
                                       ("burgers1d_nl", "auto"),
                                       ("advdiff2d_256", "auto"),
                                       ("advdiff2d_256", "shift_invert")])
def test_autograd_matches_oracle(torch, orc, wl, krylov):
    from paper_2004_00546_amd.autograd import Problem, paraexp_loss
    insts = workloads.make(wl)
    # 2D: the shortest of the 256 x 256 instances; AUTO on the tree
    # (uniformisation), shift-and-invert on independent pieces
    inst = min(insts, key=lambda x: x["n_steps"]) if wl.startswith("advdiff2d") else insts[0]
    sched = "tree" if wl.startswith("advdiff2d") and krylov == "auto" else "classic"
    # the 30-dimensional shift-and-invert space reaches about 1e-9 on the
    # longest N=128 pieces (mild stiffness converges slowest)
    # (Burgers: the Magnus check estimates 1e-10 for the workload's slices)
    tol = (1e-8 if krylov == "shift_invert" and wl == "advdiff1d_n128" else
           (1e-9 if wl.startswith("burgers") else 1e-10))
    prob = Problem(inst, krylov=krylov, sched=sched, tol=tol)
    a = torch.tensor(inst["a"], dtype=torch.float64, device="cuda:0", requires_grad=True)
    J = paraexp_loss(a, prob)
    (3.0 * J).backward()
    want = orc.gradient(inst)
    print("autograd %s/%s: J %.2e grad %.2e" % (wl, krylov, abs(J.item() - want["J"]) / want["J"],
                                                rel(a.grad.cpu().numpy() / 3.0, want["grad"])),
          flush=True)
    assert abs(J.item() - want["J"]) < 1e-8 * abs(want["J"])
    assert rel(a.grad.cpu().numpy() / 3.0, want["grad"]) < 1e-8


def test_autograd_gradient_vs_central_differences(torch):
    """J is quadratic in a for the linear problem: central differences of
    the GPU forward are exact up to rounding and the Krylov tolerance."""
    from paper_2004_00546_amd.autograd import Problem, paraexp_loss
    inst = workloads.make("advdiff1d_n128")[0]
    prob = Problem(inst, krylov="poly")
    a0 = torch.tensor(inst["a"], dtype=torch.float64, device="cuda:0", requires_grad=True)
    paraexp_loss(a0, prob).backward()
    g = a0.grad.cpu().numpy()
    for d in inst["fd_dirs"][:4]:
        dd = torch.tensor(d, dtype=torch.float64, device="cuda:0")
        eps = 1e-2
        jp = paraexp_loss(a0.detach() + eps * dd, prob).item()
        jm = paraexp_loss(a0.detach() - eps * dd, prob).item()
        fd = (jp - jm) / (2 * eps)
        assert abs(fd - g @ d) < 1e-7 * (abs(fd) + np.linalg.norm(g))


@pytest.mark.parametrize("wl,krylov", [("advdiff1d_n128", "shift_invert"),
                                       ("burgers1d_n2048", "poly")])
def test_graph_replay_equals_eager(torch, wl, krylov):
    inst = workloads.make(wl)[0]
    r = api.GradientRunner([inst], krylov=krylov, tol=1e-9)
    r.run()
    eager = r.results()[0]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        r.run()  # warm up on the side stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        r.run()
    for rep in range(3):
        r.J.zero_()
        r.grad.zero_()
        r.qT.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = r.results()[0]
        assert np.array_equal(got["grad"], eager["grad"]), rep
        assert np.array_equal(got["qT"], eager["qT"]), rep
        assert got["J"] == eager["J"]
        # eager work between replays
        r.run()
        torch.cuda.synchronize()


def test_graph_replay_two_launch_groups(torch):
    """A ragged Burgers batch whose Magnus chains need two workgroup sizes
    (N=8192 at 256 threads, N<=2048 at 512): the second launch group runs on
    the library's side stream, forked and joined by events.  A captured
    graph must replay the whole gradient exactly, with eager work between
    the replays."""
    full = workloads.make("burgers1d_ragged")
    big = min((x for x in full if x["nx"] == 8192), key=lambda x: x["n_steps"])
    small = min((x for x in full if x["nx"] <= 2048), key=lambda x: x["n_steps"])
    r = api.GradientRunner([small, big], krylov="auto", tol=1e-9)
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
        r.J.zero_()
        r.grad.zero_()
        r.qT.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for got, want in zip(r.results(), eager):
            assert np.array_equal(got["grad"], want["grad"]), rep
            assert np.array_equal(got["qT"], want["qT"]), rep
        r.run()
        torch.cuda.synchronize()


def test_autograd_two_forwards_then_backward(torch, orc):
    """Two Burgers forwards at different controls, then one backward through
    both: each backward must read its own forward's checkpoints."""
    from paper_2004_00546_amd.autograd import Problem, paraexp_loss
    base = workloads.make("burgers1d_n2048")[0]
    inst = workloads.scaled(base, n_steps=1024, T=0.25, P=64)
    prob = Problem(inst, krylov="auto", tol=1e-10)
    a1 = torch.tensor(inst["a"], dtype=torch.float64, device="cuda:0", requires_grad=True)
    a2v = np.asarray(inst["a"]) * -1.5 + 0.01
    a2 = torch.tensor(a2v, dtype=torch.float64, device="cuda:0", requires_grad=True)
    J1 = paraexp_loss(a1, prob)
    J2 = paraexp_loss(a2, prob)
    (J1 + 2.0 * J2).backward()
    w1 = orc.gradient(inst)
    w2 = orc.gradient(dict(inst, a=a2v))
    e1 = rel(a1.grad.cpu().numpy(), w1["grad"])
    e2 = rel(a2.grad.cpu().numpy() / 2.0, w2["grad"])
    print("two forwards: grad errors %.2e %.2e" % (e1, e2), flush=True)
    assert e1 < 1e-8 and e2 < 1e-8
