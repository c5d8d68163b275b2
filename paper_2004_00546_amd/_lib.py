"""ctypes binding of libparaexp.so (the C ABI declared in include/paraexp.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device buffers are torch tensors on a ROCm device; their
``data_ptr()`` is passed through.  The library must have been built
(``python -m paper_2004_00546_amd.build``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libparaexp.so")

# enums (include/paraexp.h)
PXP_OK, PXP_EINVAL, PXP_EUNSUPPORTED, PXP_EWORKSPACE = 0, 1, 2, 3
PXP_EUNSTABLE_DT, PXP_EKRYLOV_NOCONV, PXP_ENONFINITE, PXP_EHIP = 4, 5, 6, 7
OP = {"advdiff1d": 0, "advdiff2d_upwind": 1, "burgers1d": 2}
PREC = {"fp64": 0, "fp32_bulk": 1}
CTRL = {"forcing": 0, "ic": 1}
KRYLOV = {"poly": 0, "shift_invert": 1, "auto": 2, "taylor": 3, "uniform": 4,
          "chebyshev": 5}
FLAG_ABSORBED_ADJOINT = 1
FLAG_INTEGRAL_COST = 2
FLAG_NL_PARAEXP = 4
SCHED = {"classic": 0, "chain": 1, "tree": 2}
METHOD = {"paraexp": 0, "serial": 1}

STATUS_NAMES = {0: "PXP_OK", 1: "PXP_EINVAL", 2: "PXP_EUNSUPPORTED",
                3: "PXP_EWORKSPACE", 4: "PXP_EUNSTABLE_DT",
                5: "PXP_EKRYLOV_NOCONV", 6: "PXP_ENONFINITE", 7: "PXP_EHIP"}

EXPORTED = ("pxp_workspace_size", "pxp_workspace_init", "paraexp_direct",
            "paraexp_adjoint", "pxp_gradient", "gradient", "pxp_device_status",
            "pxp_device_counters", "pxp_status_str", "pxp_version",
            "pxp_profile_enable", "pxp_profile_read", "pxp_assemble",
            "pxp_cost", "pxp_reduce_gradient", "pxp_tune_workspace_size",
            "pxp_autotune", "pxp_gradient_noalloc", "pxp_device_counters_class",
            "pxp_last_report")
KCLASS = {"slices": 0, "krylov_direct": 1, "krylov_adjoint": 2,
          "serial_direct": 3, "serial_reverse": 4, "ltv_adjoint": 5,
          "ltv_nodes": 6, "sources": 7, "adj_slices": 8,
          "ltv_check": 9, "nl_iter": 10}


class pxp_problem(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("ctrl", ctypes.c_int32), ("krylov", ctypes.c_int32),
                ("sched", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("P", ctypes.c_int32),
                ("m", ctypes.c_int32), ("K", ctypes.c_int32),
                ("ckpt_every", ctypes.c_int32), ("block", ctypes.c_int32),
                ("kblock", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("n_steps", ctypes.c_int64),
                ("L", ctypes.c_double), ("vx", ctypes.c_double),
                ("vy", ctypes.c_double), ("nu", ctypes.c_double),
                ("T", ctypes.c_double), ("omega", ctypes.c_double),
                ("beta", ctypes.c_double), ("krylov_tol", ctypes.c_double),
                ("si_gamma", ctypes.c_double),
                ("hyb_slices", ctypes.c_int32), ("hyb_group", ctypes.c_int32),
                ("hyb_k", ctypes.c_double),
                ("nl_iters", ctypes.c_int32), ("nl_slices", ctypes.c_int32),
                ("nl_tol", ctypes.c_double)]


class pxp_tune_report(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int32), ("krylov", ctypes.c_int32),
                ("sched", ctypes.c_int32), ("kblock", ctypes.c_int32),
                ("candidates", ctypes.c_int32), ("group", ctypes.c_int32),
                ("ms", ctypes.c_double), ("serial_ms", ctypes.c_double),
                ("rel_err", ctypes.c_double)]


class pxp_report(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int32), ("sched", ctypes.c_int32),
                ("krylov_direct", ctypes.c_int32), ("krylov_adjoint", ctypes.c_int32),
                ("substeps", ctypes.c_uint64), ("iterations", ctypes.c_uint64),
                ("max_est", ctypes.c_double), ("nl_iterations", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class PxpError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__("%s failed: %s (%s)" % (where, STATUS_NAMES.get(code, code),
                                                 status_str(code)))


_lib = None


def load() -> ctypes.CDLL:
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libparaexp.so is not built (run python -m "
                           "paper_2004_00546_amd.build); there is no fallback")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(pxp_problem)
    vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32
    st = ctypes.c_int
    sig = {
        "pxp_workspace_size": (st, [P, i32, ctypes.POINTER(sz)]),
        "pxp_workspace_init": (st, [vp, sz, vp]),
        "paraexp_direct": (st, [P, i32, vp, vp, vp, vp, sz, vp]),
        "paraexp_adjoint": (st, [P, i32, vp, vp, vp, vp, vp, sz, vp]),
        "pxp_gradient": (st, [P, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                              sz, vp]),
        "gradient": (st, [P, i32, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]),
        "pxp_device_status": (st, [vp, sz, vp, ctypes.POINTER(ctypes.c_double)]),
        "pxp_device_counters": (st, [vp, sz, vp, ctypes.POINTER(ctypes.c_uint64),
                                     ctypes.POINTER(ctypes.c_uint64),
                                     ctypes.POINTER(ctypes.c_uint64)]),
        "pxp_status_str": (ctypes.c_char_p, [st]),
        "pxp_assemble": (st, [P, i32, vp, vp, vp, vp, vp]),
        "pxp_cost": (st, [P, i32, vp, vp, vp, vp, vp, vp]),
        "pxp_reduce_gradient": (st, [P, i32, vp, vp, vp, vp, vp]),
        "pxp_profile_enable": (st, [i32]),
        "pxp_profile_read": (st, [i32, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_int32)]),
        "pxp_version": (ctypes.c_char_p, []),
        "pxp_tune_workspace_size": (st, [P, i32, i32, i32, ctypes.POINTER(sz)]),
        "pxp_autotune": (st, [P, i32, vp, vp, vp, vp, i32, i32, ctypes.c_double, i32,
                              vp, sz, ctypes.POINTER(pxp_tune_report), vp]),
        "pxp_gradient_noalloc": (st, [P, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                      vp]),
        "pxp_last_report": (st, [P, i32, vp, sz, vp, ctypes.POINTER(pxp_report)]),
        "pxp_device_counters_class": (st, [vp, sz, vp, i32, ctypes.POINTER(ctypes.c_uint64),
                                           ctypes.POINTER(ctypes.c_uint64),
                                           ctypes.POINTER(ctypes.c_uint64)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def status_str(code: int) -> str:
    try:
        return load().pxp_status_str(code).decode()
    except Exception:  # library absent: still describe the code
        return STATUS_NAMES.get(code, str(code))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(int(stream))


def problems_array(problems):
    arr = (pxp_problem * len(problems))(*problems)
    return arr, len(problems)


def _check(code, where):
    if code != PXP_OK:
        raise PxpError(code, where)


def pxp_workspace_size(problems) -> int:
    arr, n = problems_array(problems)
    out = ctypes.c_size_t(0)
    _check(load().pxp_workspace_size(arr, n, ctypes.byref(out)), "pxp_workspace_size")
    return out.value


def pxp_workspace_init(ws, stream=None):
    _check(load().pxp_workspace_init(_ptr(ws), ws.numel(), _stream(stream)),
           "pxp_workspace_init")


def paraexp_direct(problems, q0, F, qT, ws, stream=None):
    arr, n = problems_array(problems)
    _check(load().paraexp_direct(arr, n, _ptr(q0), _ptr(F), _ptr(qT), _ptr(ws),
                                 ws.numel(), _stream(stream)), "paraexp_direct")


def paraexp_adjoint(problems, lamT, lam0, Lambda, ws, stream=None, jI_src=None):
    arr, n = problems_array(problems)
    _check(load().paraexp_adjoint(arr, n, _ptr(lamT), _ptr(jI_src), _ptr(lam0),
                                  _ptr(Lambda), _ptr(ws), ws.numel(), _stream(stream)),
           "paraexp_adjoint")


def pxp_gradient(problems, method, ctrl, basis, q0, u_tgt, J, grad, qT, lam_out,
                 ws, stream=None):
    arr, n = problems_array(problems)
    _check(load().pxp_gradient(arr, n, METHOD[method] if isinstance(method, str)
                               else method, _ptr(ctrl), _ptr(basis), _ptr(q0),
                               _ptr(u_tgt), _ptr(J), _ptr(grad), _ptr(qT),
                               _ptr(lam_out), _ptr(ws), ws.numel(),
                               _stream(stream)), "pxp_gradient")


NOALLOC_SCRATCH_BYTES = 64 << 20  # PXP_NOALLOC_SCRATCH_BYTES


def pxp_gradient_noalloc(problems, method, ctrl, basis, q0, u_tgt, J, grad, qT, lam_out,
                         status_out=None, stream=None):
    """pxp_gradient with the library's fixed device workspace (no caller
    workspace, no allocation)."""
    arr, n = problems_array(problems)
    _check(load().pxp_gradient_noalloc(arr, n, METHOD[method] if isinstance(method, str)
                                       else method, _ptr(ctrl), _ptr(basis), _ptr(q0),
                                       _ptr(u_tgt), _ptr(J), _ptr(grad), _ptr(qT),
                                       _ptr(lam_out), _ptr(status_out), _stream(stream)),
           "pxp_gradient_noalloc")


def gradient(problems, ctrl, basis, q0, u_tgt, J, grad, qT, ws, stream=None):
    arr, n = problems_array(problems)
    _check(load().gradient(arr, n, _ptr(ctrl), _ptr(basis), _ptr(q0),
                           _ptr(u_tgt), _ptr(J), _ptr(grad), _ptr(qT), _ptr(ws),
                           ws.numel(), _stream(stream)), "gradient")


def pxp_device_status(ws, stream=None):
    est = ctypes.c_double(0.0)
    code = load().pxp_device_status(_ptr(ws), ws.numel(), _stream(stream),
                                    ctypes.byref(est))
    return code, est.value


def pxp_device_counters(ws, stream=None):
    """(substeps, Arnoldi iterations, second Gram-Schmidt passes)"""
    a, b, c = ctypes.c_uint64(0), ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(load().pxp_device_counters(_ptr(ws), ws.numel(), _stream(stream),
                                      ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
           "pxp_device_counters")
    return a.value, b.value, c.value


def pxp_device_counters_class(ws, cls, stream=None):
    """(substeps, iterations or Taylor terms, second Gram-Schmidt passes) of
    the direct (cls 0) or adjoint (cls 1) exponentials"""
    a, b, c = ctypes.c_uint64(0), ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(load().pxp_device_counters_class(_ptr(ws), ws.numel(), _stream(stream), cls,
                                            ctypes.byref(a), ctypes.byref(b),
                                            ctypes.byref(c)),
           "pxp_device_counters_class")
    return a.value, b.value, c.value


def pxp_last_report(problems, ws, stream=None):
    """Per-instance statistics since the last report (dicts); clears them."""
    arr, n = problems_array(problems)
    rep = (pxp_report * n)()
    _check(load().pxp_last_report(arr, n, _ptr(ws), ws.numel(), _stream(stream), rep),
           "pxp_last_report")
    names = {v: k for k, v in KRYLOV.items()}
    out = []
    for r in rep:
        d = dict((f, getattr(r, f)) for f, _ in pxp_report._fields_ if f != "pad")
        d["krylov_direct"] = names.get(d["krylov_direct"], None)
        d["krylov_adjoint"] = names.get(d["krylov_adjoint"], None)
        d["sched"] = {0: "classic", 1: "chain", 2: "tree"}.get(d["sched"], None)
        out.append(d)
    return out


def pxp_profile_enable(on: bool):
    _check(load().pxp_profile_enable(1 if on else 0), "pxp_profile_enable")


def pxp_profile_read(kernel_class) -> tuple[float, int]:
    """Summed milliseconds and launch count of one kernel class."""
    k = KCLASS[kernel_class] if isinstance(kernel_class, str) else kernel_class
    ms, cnt = ctypes.c_double(0.0), ctypes.c_int32(0)
    _check(load().pxp_profile_read(k, ctypes.byref(ms), ctypes.byref(cnt)),
           "pxp_profile_read")
    return ms.value, cnt.value


def pxp_assemble(problems, ctrl, basis, base, out, stream=None):
    arr, n = problems_array(problems)
    _check(load().pxp_assemble(arr, n, _ptr(ctrl), _ptr(basis), _ptr(base),
                               _ptr(out), _stream(stream)), "pxp_assemble")


def pxp_cost(problems, qT, u_tgt, ctrl, J, lamT, stream=None):
    arr, n = problems_array(problems)
    _check(load().pxp_cost(arr, n, _ptr(qT), _ptr(u_tgt), _ptr(ctrl), _ptr(J),
                           _ptr(lamT), _stream(stream)), "pxp_cost")


def pxp_reduce_gradient(problems, basis, v, ctrl, grad, stream=None):
    arr, n = problems_array(problems)
    _check(load().pxp_reduce_gradient(arr, n, _ptr(basis), _ptr(v), _ptr(ctrl),
                                      _ptr(grad), _stream(stream)),
           "pxp_reduce_gradient")


def pxp_tune_workspace_size(problems, p_min=0, p_max=0) -> int:
    arr, n = problems_array(problems)
    out = ctypes.c_size_t(0)
    _check(load().pxp_tune_workspace_size(arr, n, p_min, p_max, ctypes.byref(out)),
           "pxp_tune_workspace_size")
    return out.value


def pxp_autotune(problems, ctrl, basis, q0, u_tgt, ws, p_min=0, p_max=0, rtol=1e-9,
                 reps=2, stream=None):
    """Tunes the problems in place (the ctypes structures are updated) and
    returns the per-instance reports."""
    arr, n = problems_array(problems)
    rep = (pxp_tune_report * n)()
    _check(load().pxp_autotune(arr, n, _ptr(ctrl), _ptr(basis), _ptr(q0), _ptr(u_tgt),
                               p_min, p_max, rtol, reps, _ptr(ws), ws.numel(), rep,
                               _stream(stream)), "pxp_autotune")
    for i in range(n):
        ctypes.memmove(ctypes.byref(problems[i]), ctypes.byref(arr[i]),
                       ctypes.sizeof(pxp_problem))
    return [dict((f, getattr(r, f)) for f, _ in pxp_tune_report._fields_) for r in rep]
