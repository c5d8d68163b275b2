"""Oracle: plain serial FP64 CPU reference of the direct-adjoint loop.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The HIP
library never imports, links or calls it, and it imports nothing from the
HIP package.

The arithmetic lives in ``oracle.c`` (serial RK4 direct march and its exact
discrete adjoint, paper section 2 and sections 4.2-4.3 for the operators);
this module is argument marshalling with ctypes plus the build step.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "liboracle.so")

OPS = {"advdiff1d": 0, "advdiff2d_upwind": 1, "burgers1d": 2}
CONTROLS = {"forcing": 0, "ic": 1}


class _Problem(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("L", ctypes.c_double), ("vx", ctypes.c_double),
                ("vy", ctypes.c_double), ("nu", ctypes.c_double),
                ("T", ctypes.c_double), ("omega", ctypes.c_double),
                ("beta", ctypes.c_double), ("n_steps", ctypes.c_long)]


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (no FMA contraction) into _build/."""
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        os.makedirs(_BUILD, exist_ok=True)
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC",
                               "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_Problem)
        lib.orc_rhs.argtypes = [pp, dp, dp]
        lib.orc_rhs_adjoint.argtypes = [pp, dp, dp, dp]
        lib.orc_direct.argtypes = [pp, dp, dp, dp, dp]
        lib.orc_direct.restype = ctypes.c_int
        lib.orc_adjoint.argtypes = [pp, dp, dp, dp, dp, dp]
        lib.orc_adjoint.restype = ctypes.c_int
        lib.orc_gradient.argtypes = [pp, ctypes.c_int, ctypes.c_int, dp, dp, dp,
                                     dp, dp, dp, dp, dp, dp]
        lib.orc_gradient.restype = ctypes.c_int
        lib.orc_gradient_icost.argtypes = lib.orc_gradient.argtypes
        lib.orc_gradient_icost.restype = ctypes.c_int
        _lib = lib
    return _lib


def _prob(inst: dict) -> _Problem:
    return _Problem(OPS[inst["op"]], int(inst["nx"]), int(inst.get("ny", 1)),
                    float(inst["L"]), float(inst.get("vx", 0.0)),
                    float(inst.get("vy", 0.0)), float(inst["nu"]),
                    float(inst["T"]), float(inst.get("omega", 1.0)),
                    float(inst.get("beta", 0.0)), int(inst["n_steps"]))


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def size(inst: dict) -> int:
    return int(inst["nx"]) * int(inst.get("ny", 1))


def rhs(inst: dict, u) -> np.ndarray:
    """A u for the linear operators, N(u) for Burgers."""
    u = _f64(u)
    out = np.empty(size(inst))
    p = _prob(inst)
    _load().orc_rhs(ctypes.byref(p), _ptr(u), _ptr(out))
    return out


def rhs_adjoint(inst: dict, U, lam) -> np.ndarray:
    """J(U)^T lam (U ignored by the linear operators)."""
    U = _f64(U if U is not None else np.zeros(size(inst)))
    lam = _f64(lam)
    out = np.empty(size(inst))
    p = _prob(inst)
    _load().orc_rhs_adjoint(ctypes.byref(p), _ptr(U), _ptr(lam), _ptr(out))
    return out


def direct(inst: dict, q0, F=None, traj: bool = False):
    """RK4 march; returns q(T) (and all step states if traj)."""
    q0 = _f64(q0)
    F = _f64(F)
    n = size(inst)
    qT = np.empty(n)
    tr = np.empty((int(inst["n_steps"]) + 1, n)) if traj else None
    p = _prob(inst)
    rc = _load().orc_direct(ctypes.byref(p), _ptr(q0), _ptr(F), _ptr(qT),
                            _ptr(tr))
    if rc:
        raise MemoryError("oracle direct march failed")
    return (qT, tr) if traj else qT


def adjoint(inst: dict, traj, F, lamT):
    """Exact discrete adjoint sweep; returns (lambda_0, Lambda)."""
    n = size(inst)
    lam0 = np.empty(n)
    Lam = np.empty(n)
    p = _prob(inst)
    rc = _load().orc_adjoint(ctypes.byref(p), _ptr(_f64(traj)), _ptr(_f64(F)),
                             _ptr(_f64(lamT)), _ptr(lam0), _ptr(Lam))
    if rc:
        raise MemoryError("oracle adjoint sweep failed")
    return lam0, Lam


def gradient(inst: dict, a=None) -> dict:
    """One direct-adjoint loop: q(T), J, dJ/da, lambda_0 and Lambda.  An
    instance with cost "integral" takes the integral cost of section 4.2
    (trapezoidal rule over the step states), else the terminal cost."""
    basis = _f64(inst["basis"])
    a = _f64(inst["a"] if a is None else a)
    K = basis.shape[0]
    n = size(inst)
    q0 = _f64(inst.get("q0", np.zeros(n)))
    tgt = _f64(inst["u_tgt"])
    qT = np.empty(n)
    J = np.empty(1)
    g = np.empty(K)
    lam0 = np.empty(n)
    Lam = np.empty(n)
    p = _prob(inst)
    fn = (_load().orc_gradient_icost if inst.get("cost", "terminal") == "integral"
          else _load().orc_gradient)
    rc = fn(ctypes.byref(p), CONTROLS[inst["control"]], K,
                              _ptr(basis), _ptr(a), _ptr(q0), _ptr(tgt),
                              _ptr(qT), _ptr(J), _ptr(g), _ptr(lam0), _ptr(Lam))
    if rc:
        raise MemoryError("oracle gradient failed")
    return dict(qT=qT, J=float(J[0]), grad=g, lam0=lam0, Lambda=Lam)


def cost(inst: dict, a) -> float:
    """J(a) from the direct march alone (for finite differences); the
    integral cost sums the trapezoidal weights over the stored states."""
    basis = _f64(inst["basis"])
    a = _f64(a)
    n = size(inst)
    q0 = _f64(inst.get("q0", np.zeros(n))).copy()
    if inst["control"] == "forcing":
        F = a @ basis
    else:
        F = None
        q0 = q0 + a @ basis
    if inst.get("cost", "terminal") == "integral":
        _, tr = direct(inst, q0, F, traj=True)
        nt = int(inst["n_steps"])
        d = tr - np.asarray(inst["u_tgt"])[None, :]
        s = np.einsum("ij,ij->i", d, d)
        w = np.full(nt + 1, 1.0 / nt)
        w[0] = w[-1] = 0.5 / nt
        return float(w @ s) + float(inst["beta"]) * float(a @ a)
    qT = direct(inst, q0, F)
    d = qT - inst["u_tgt"]
    return 0.5 * float(d @ d) + float(inst["beta"]) * float(a @ a)
