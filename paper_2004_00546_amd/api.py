"""Convenience layer over the C ABI: problem descriptions from workload dicts
and device buffers held as torch tensors.  Marshalling only; the arithmetic
runs in libparaexp.so."""
from __future__ import annotations

import numpy as np

from . import _lib


def make_problem(inst: dict, krylov: str = "shift_invert", sched: str = "classic",
                 tol: float = 1e-10, block: int = 0, kblock: int = 0,
                 si_gamma: float = 0.0, absorbed: bool = False,
                 P: int | None = None, m: int | None = None,
                 prec: str = "fp64") -> _lib.pxp_problem:
    p = _lib.pxp_problem()
    p.op = _lib.OP[inst["op"]]
    p.prec = _lib.PREC[prec]
    p.ctrl = _lib.CTRL[inst["control"]]
    p.krylov = _lib.KRYLOV[krylov]
    p.sched = _lib.SCHED[sched]
    p.nx = int(inst["nx"])
    p.ny = int(inst.get("ny", 1))
    p.P = int(inst["P"] if P is None else P)
    p.m = int(inst["m"] if m is None else m)
    p.K = int(np.asarray(inst["basis"]).shape[0])
    p.ckpt_every = int(inst.get("ckpt_every", 64))
    p.block = int(block)
    p.kblock = int(kblock)
    p.flags = _lib.FLAG_ABSORBED_ADJOINT if absorbed else 0
    # the integral cost of section 4.2 (eq. cost) instead of the terminal one
    if inst.get("cost", "terminal") == "integral":
        p.flags |= _lib.FLAG_INTEGRAL_COST
    p.n_steps = int(inst["n_steps"])
    p.L = float(inst["L"])
    p.vx = float(inst.get("vx", 0.0))
    p.vy = float(inst.get("vy", 0.0))
    p.nu = float(inst["nu"])
    p.T = float(inst["T"])
    p.omega = float(inst.get("omega", 1.0))
    p.beta = float(inst.get("beta", 0.0))
    p.krylov_tol = float(tol)
    p.si_gamma = float(si_gamma)  # 0: the library's default for the operator
    # hybrid scheme of the Burgers integral cost: adjoint slices and their
    # partition (eq. nonEquiP)
    p.hyb_slices = int(inst.get("hyb_slices", 0))
    p.hyb_group = int(inst.get("hyb_group", 0))
    p.hyb_k = float(inst.get("hyb_k", 0.0))
    # the iterative nonlinear Paraexp of section 3.2 for the Burgers direct
    if inst.get("nl_paraexp", False):
        p.flags |= _lib.FLAG_NL_PARAEXP
    p.nl_iters = int(inst.get("nl_iters", 0))
    p.nl_slices = int(inst.get("nl_slices", 0))
    p.nl_tol = float(inst.get("nl_tol", 0.0))
    return p


class GradientRunner:
    """Device buffers for a batch of instances and one gradient call.
    ``problems`` (optional) replaces the problem descriptions built from the
    instances, e.g. by tuned ones."""

    def __init__(self, instances, method: str = "paraexp", device: str = "cuda:0",
                 a=None, problems=None, **prob_kw):
        import torch
        self.torch = torch
        self.instances = list(instances)
        self.method = method
        self.device = torch.device(device)
        self.problems = (list(problems) if problems is not None else
                         [make_problem(inst, **prob_kw) for inst in self.instances])
        f64 = dict(dtype=torch.float64, device=self.device)
        ctrl = [np.asarray(inst["a"] if a is None else a[i], dtype=np.float64)
                for i, inst in enumerate(self.instances)]
        self.ctrl = torch.tensor(np.concatenate(ctrl), **f64)
        self.basis = torch.tensor(np.concatenate(
            [np.asarray(inst["basis"], dtype=np.float64).ravel() for inst in self.instances]), **f64)
        q0 = np.concatenate(
            [np.asarray(inst.get("q0", np.zeros(inst["nx"] * inst.get("ny", 1))),
                        dtype=np.float64) for inst in self.instances])
        # an all-zero base state is passed as null (the C ABI's zero), which
        # lets the library drop the initial-state source term
        self.q0 = torch.tensor(q0, **f64) if np.any(q0 != 0.0) else None
        self.u_tgt = torch.tensor(np.concatenate(
            [np.asarray(inst["u_tgt"], dtype=np.float64) for inst in self.instances]), **f64)
        ntot = self.u_tgt.numel()
        self.J = torch.zeros(len(self.instances), **f64)
        self.grad = torch.zeros(self.ctrl.numel(), **f64)
        self.qT = torch.zeros(ntot, **f64)
        self.lam = torch.zeros(ntot, **f64)
        nbytes = _lib.pxp_workspace_size(self.problems)
        self.ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        _lib.pxp_workspace_init(self.ws)
        self.sizes = [int(inst["nx"]) * int(inst.get("ny", 1)) for inst in self.instances]
        self.ks = [int(np.asarray(inst["basis"]).shape[0]) for inst in self.instances]

    def run(self, stream=None):
        _lib.pxp_gradient(self.problems, self.method, self.ctrl, self.basis, self.q0,
                          self.u_tgt, self.J, self.grad, self.qT, self.lam, self.ws,
                          stream)

    def status(self):
        return _lib.pxp_device_status(self.ws)

    def counters(self):
        return _lib.pxp_device_counters(self.ws)

    def results(self):
        self.torch.cuda.synchronize(self.device)
        J = self.J.cpu().numpy()
        g = self.grad.cpu().numpy()
        qT = self.qT.cpu().numpy()
        lam = self.lam.cpu().numpy()
        out = []
        o = ko = 0
        for i, (n, K) in enumerate(zip(self.sizes, self.ks)):
            out.append(dict(J=float(J[i]), grad=g[ko:ko + K], qT=qT[o:o + n],
                            lam=lam[o:o + n]))
            o += n
            ko += K
        return out


def autotune(instances, p_min: int = 0, p_max: int = 0, rtol: float = 1e-9,
             reps: int = 2, device: str = "cuda:0", **prob_kw):
    """Run the library's autotuner on the instances (their own controls as
    the sample point); returns (tuned problems, per-instance reports)."""
    r = GradientRunner(instances, method="paraexp", device=device, **prob_kw)
    torch = r.torch
    nbytes = _lib.pxp_tune_workspace_size(r.problems, p_min, p_max)
    ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=r.device)
    rep = _lib.pxp_autotune(r.problems, r.ctrl, r.basis, r.q0, r.u_tgt, ws, p_min, p_max,
                            rtol, reps)
    return r.problems, rep
