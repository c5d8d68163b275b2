"""The C-ABI library loads and exports every entry point the header declares,
and rejects malformed problems on the host before anything is enqueued
(no GPU needed: these paths make no HIP call)."""
import ctypes
import os
import re

import pytest

from paper_2004_00546_amd import _lib, api, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "paraexp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*"
                       r"([A-Za-z_][A-Za-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libparaexp.so not built: run python -m paper_2004_00546_amd.build")
    return _lib.load()


def test_header_declares_the_north_star_calls():
    names = declared_functions()
    for n in ("paraexp_direct", "paraexp_adjoint", "gradient"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(_lib.EXPORTED) == set(names)


def test_version_and_status_strings(lib):
    assert lib.pxp_version().decode().startswith("paraexp")
    for code in range(8):
        assert len(_lib.status_str(code)) > 0


def test_struct_layout_matches_header():
    # 12 int32, 1 int64, 9 doubles
    assert ctypes.sizeof(_lib.pxp_problem) == 14 * 4 + 8 + 9 * 8


def _size_status(probs):
    arr, n = _lib.problems_array(probs)
    out = ctypes.c_size_t(0)
    return _lib.load().pxp_workspace_size(arr, n, ctypes.byref(out)), out.value


def test_workspace_size_valid_and_monotone(lib):
    inst = workloads.make("advdiff1d_n128")[0]
    st, b1 = _size_status([api.make_problem(inst)])
    assert st == 0 and b1 > 0
    st, b2 = _size_status([api.make_problem(inst)] * 3)
    assert st == 0 and b2 > 2 * b1
    st, b0 = _size_status([])
    assert st == 0


@pytest.mark.parametrize("field,value,code", [
    ("n_steps", 1001, _lib.PXP_EINVAL),        # not a multiple of P
    ("P", 0, _lib.PXP_EINVAL),
    ("nx", 1, _lib.PXP_EINVAL),
    ("m", 0, _lib.PXP_EUNSUPPORTED),
    ("m", 200, _lib.PXP_EUNSUPPORTED),
    ("T", -1.0, _lib.PXP_EINVAL),
    ("krylov_tol", 0.0, _lib.PXP_EINVAL),
    ("n_steps", 8, _lib.PXP_EUNSTABLE_DT),     # dt = 0.125 on N=128
])
def test_host_validation(lib, field, value, code):
    inst = workloads.make("advdiff1d_n128")[0]
    p = api.make_problem(inst)
    setattr(p, field, value)
    st, _ = _size_status([p])
    assert st == code


def test_stiff_dt_rejected_on_unit_box(lib):
    """The N=4096 workload on [0,1) instead of [0,2 pi) makes dt=1e-4 leave
    the RK4 stability region; the host check must catch it."""
    inst = dict(workloads.make("advdiff1d_n4096")[0], L=1.0)
    st, _ = _size_status([api.make_problem(inst)])
    assert st == _lib.PXP_EUNSTABLE_DT


def test_shift_invert_needs_power_of_two(lib):
    inst = dict(workloads.make("advdiff1d_n128")[0], nx=96)
    st, _ = _size_status([api.make_problem(inst, krylov="shift_invert")])
    assert st == _lib.PXP_EUNSUPPORTED
    st, _ = _size_status([api.make_problem(inst, krylov="poly")])
    assert st == 0


def test_calls_fail_before_enqueue(lib):
    """Argument errors return without touching the device."""
    inst = workloads.make("advdiff1d_n128")[0]
    p = api.make_problem(inst)
    arr, n = _lib.problems_array([p])
    # missing workspace
    st = lib.paraexp_direct(arr, n, None, None, ctypes.c_void_p(16), None, 0, None)
    assert st == _lib.PXP_EWORKSPACE
    # missing output
    st = lib.paraexp_direct(arr, n, None, None, None, ctypes.c_void_p(256), 1 << 30, None)
    assert st == _lib.PXP_EINVAL
    # bad method
    st = lib.pxp_gradient(arr, n, 7, None, None, None, None, None, None, None, None,
                          None, 0, None)
    assert st == _lib.PXP_EINVAL
    # empty batch is a no-op
    st = lib.pxp_gradient(arr, 0, 0, None, None, None, None, None, None, None, None,
                          None, 0, None)
    assert st == _lib.PXP_OK
