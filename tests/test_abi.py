"""The C-ABI library loads and exports every entry point the header declares,
and rejects malformed problems on the host before anything is enqueued
(no GPU needed: these paths make no HIP call)."""
import ctypes
import os
import re

import numpy as np
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


def test_header_declares_the_three_boundary_calls():
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
    # 14 int32, 1 int64, 9 doubles, then twice 2 int32 and a double
    assert ctypes.sizeof(_lib.pxp_problem) == 14 * 4 + 8 + 9 * 8 + 2 * (2 * 4 + 8)


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


def test_2d_shape_and_precision_rules():
    """2D problems: power-of-two rows of 64..256 points, whole 16-row bands,
    2048-point multiples, non-negative velocities, FP64; shift-and-invert on
    power-of-two grids;
    the Paraexp path takes at most four RK4 steps per slice (checked when a
    call names the method)."""
    import math
    base = dict(op="advdiff2d_upwind", control="forcing", nx=64, ny=32,
                L=2 * math.pi, vx=1.0, vy=0.5, nu=0.02, T=0.5, n_steps=64, P=16,
                m=30, basis=np.zeros((1, 64 * 32)))
    ok = api.make_problem(base, krylov="poly")
    assert _lib.pxp_workspace_size([ok]) > 0
    for change, code in [(dict(nx=96), _lib.PXP_EUNSUPPORTED),
                         (dict(nx=512, basis=np.zeros((1, 512 * 32))), _lib.PXP_EUNSUPPORTED),
                         (dict(ny=24), _lib.PXP_EUNSUPPORTED),
                         (dict(nx=64, ny=16, basis=np.zeros((1, 1024))), _lib.PXP_EUNSUPPORTED),
                         (dict(vx=-1.0), _lib.PXP_EUNSUPPORTED),
                         (dict(T=50.0), _lib.PXP_EUNSTABLE_DT)]:
        p = api.make_problem(dict(base, **change), krylov="poly")
        with pytest.raises(_lib.PxpError) as e:
            _lib.pxp_workspace_size([p])
        assert e.value.code == code, change
    for kw, code in [(dict(krylov="poly", prec="fp32_bulk"), _lib.PXP_EUNSUPPORTED)]:
        with pytest.raises(_lib.PxpError) as e:
            _lib.pxp_workspace_size([api.make_problem(base, **kw)])
        assert e.value.code == code, kw
    # shift-and-invert (the Fourier solve): power-of-two grids of at most
    # 256 x 256, a Krylov dimension whose LDS layout (the FFT buffers share
    # the small dense scratch) fits in 160 KB, terminal cost only
    assert _lib.pxp_workspace_size([api.make_problem(base, krylov="shift_invert")]) > 0
    assert _lib.pxp_workspace_size([api.make_problem(dict(base, m=50),
                                                     krylov="shift_invert")]) > 0
    for change in [dict(ny=48, basis=np.zeros((1, 64 * 48))), dict(m=60)]:
        with pytest.raises(_lib.PxpError) as e:
            _lib.pxp_workspace_size([api.make_problem(dict(base, **change),
                                                      krylov="shift_invert")])
        assert e.value.code == _lib.PXP_EUNSUPPORTED, change
    with pytest.raises(_lib.PxpError) as e:
        _lib.pxp_workspace_size([api.make_problem(dict(base, cost="integral"),
                                                  krylov="shift_invert", sched="tree")])
    assert e.value.code == _lib.PXP_EUNSUPPORTED
    # eight steps per slice: sized and accepted, refused by the Paraexp call
    p8 = api.make_problem(dict(base, P=8), krylov="poly")
    assert _lib.pxp_workspace_size([p8]) > 0


def test_tune_workspace_covers_every_candidate():
    """The tuner's workspace holds the largest candidate's workspace plus the
    gradient scratch; it is a host-only computation."""
    inst = workloads.make("advdiff1d_n128")[0]
    p = api.make_problem(inst, krylov="poly")
    plain = _lib.pxp_workspace_size([p])
    tuned = _lib.pxp_tune_workspace_size([p], 4, 64)
    assert tuned >= plain
    # a larger slice range needs at least as much
    assert _lib.pxp_tune_workspace_size([p], 4, 500) >= tuned


def test_problem_flags():
    """Unknown flag bits are refused; the absorbed adjoint is for the 1D
    linear problems and sizes extra workspace for its integrals."""
    inst = workloads.make("advdiff1d_n128")[0]
    plain = api.make_problem(inst, krylov="poly")
    absorbed = api.make_problem(inst, krylov="poly", absorbed=True)
    assert _lib.pxp_workspace_size([absorbed]) > _lib.pxp_workspace_size([plain])
    bad = api.make_problem(inst, krylov="poly")
    bad.flags = 8
    with pytest.raises(_lib.PxpError) as e:
        _lib.pxp_workspace_size([bad])
    assert e.value.code == _lib.PXP_EINVAL
    # the integral cost is a 2D path
    ic1d = api.make_problem(dict(inst, cost="integral"), krylov="poly")
    assert ic1d.flags == _lib.FLAG_INTEGRAL_COST
    with pytest.raises(_lib.PxpError) as e:
        _lib.pxp_workspace_size([ic1d])
    assert e.value.code == _lib.PXP_EUNSUPPORTED
    burg = api.make_problem(workloads.make("burgers1d_n2048")[0], krylov="poly", absorbed=True)
    with pytest.raises(_lib.PxpError) as e:
        _lib.pxp_workspace_size([burg])
    assert e.value.code == _lib.PXP_EUNSUPPORTED


def test_noalloc_rejects_oversize_on_host(lib):
    # the size check runs before any HIP call: no GPU needed
    inst = workloads.make("advdiff1d_n4096")[0]
    p = api.make_problem(inst)
    assert _lib.pxp_workspace_size([p]) > _lib.NOALLOC_SCRATCH_BYTES
    arr, n = _lib.problems_array([p])
    code = lib.pxp_gradient_noalloc(arr, n, 0, None, None, None, None, None, None,
                                    None, None, None, None)
    assert code == _lib.PXP_EWORKSPACE


def test_adjoint_rejects_integral_cost_source_on_host(lib):
    """Step sources are taken only by 2D problems that carry the integral-cost
    flag (their workspace holds the adjoint slices' buffers): a 1D problem
    with a non-null source is refused before any HIP call."""
    inst = workloads.make("advdiff1d_n128")[0]
    p = api.make_problem(inst)
    arr, n = _lib.problems_array([p])
    fake = ctypes.c_void_p(4096)  # never dereferenced: refused first
    code = lib.paraexp_adjoint(arr, n, fake, fake, None, None, fake, 1 << 30, None)
    assert code == _lib.PXP_EUNSUPPORTED


def test_report_struct_layout():
    assert ctypes.sizeof(_lib.pxp_report) == 4 * 4 + 2 * 8 + 2 * 8


def _icost2d(**kw):
    import math
    base = dict(op="advdiff2d_upwind", control="forcing", cost="integral", nx=64, ny=32,
                L=2 * math.pi, vx=1.0, vy=1.0, nu=0.02, T=0.5, n_steps=64, P=16, m=30,
                basis=np.zeros((2, 64 * 32)))
    base.update(kw)
    return base


def test_integral_cost_rules_on_host(lib):
    """The integral cost runs on the uniformised tree schedule of the 2D
    problems; the largest adjoint piece is bounded; its workspace holds the
    (n_steps + 1) n step sources; pxp_cost (terminal cost only) refuses it
    before any HIP call."""
    ok = api.make_problem(_icost2d(), krylov="uniform", sched="tree")
    plain = api.make_problem(dict(_icost2d(), cost="terminal"), krylov="uniform", sched="tree")
    n = 64 * 32
    grow = _lib.pxp_workspace_size([ok]) - _lib.pxp_workspace_size([plain])
    assert grow >= (64 + 1) * n * 8 + (2 * 16 - 1) * n * 8
    assert _lib.pxp_workspace_size([api.make_problem(_icost2d(), krylov="auto",
                                                     sched="tree")]) > 0
    for kw, code in [(dict(krylov="uniform", sched="chain"), _lib.PXP_EUNSUPPORTED),
                     (dict(krylov="poly", sched="chain"), _lib.PXP_EUNSUPPORTED),
                     (dict(krylov="taylor", sched="classic"), _lib.PXP_EUNSUPPORTED)]:
        with pytest.raises(_lib.PxpError) as e:
            _lib.pxp_workspace_size([api.make_problem(_icost2d(), **kw)])
        assert e.value.code == code, kw
    # mu T/2 beyond the bound of one adjoint piece: T = 500 on a grid where
    # mu is about 20 (the step of the accepted case keeps RK4 stable)
    long = api.make_problem(_icost2d(T=500.0, n_steps=65536, P=16384), krylov="uniform",
                            sched="tree")
    with pytest.raises(_lib.PxpError) as e:
        _lib.pxp_workspace_size([long])
    assert e.value.code == _lib.PXP_EUNSUPPORTED
    arr, nb = _lib.problems_array([ok])
    fake = ctypes.c_void_p(4096)  # never dereferenced: refused first
    assert lib.pxp_cost(arr, nb, fake, fake, fake, fake, None, None) == _lib.PXP_EUNSUPPORTED


def test_integral_cost_workload_accepted(lib):
    """The section 4.2 stand-in: four diffusivities on 128^2, T = 10, 2048
    steps in 512 slices; every instance passes the host checks (RK4
    stability, tree bound)."""
    insts = workloads.make("advdiff2d_icost")
    assert [i["nu"] for i in insts] == [0.01, 0.02, 0.05, 0.1]
    probs = [api.make_problem(i, krylov="uniform", sched="tree", tol=1e-9) for i in insts]
    assert all(p.flags == _lib.FLAG_INTEGRAL_COST for p in probs)
    assert _lib.pxp_workspace_size(probs) > 4 * 2049 * 128 * 128 * 8


def test_burgers_integral_cost_rules_on_host(lib):
    """The Burgers integral cost (hybrid scheme) is FP64 only; the hybrid
    fields must be non-negative; the workspace grows by the adjoint slices'
    end states and segment scratch."""
    inst = dict(workloads.make("burgers1d_n2048")[0], cost="integral")
    ok = api.make_problem(inst, krylov="poly")
    plain = api.make_problem(dict(inst, cost="terminal"), krylov="poly")
    assert _lib.pxp_workspace_size([ok]) > _lib.pxp_workspace_size([plain])
    with pytest.raises(_lib.PxpError) as e:
        _lib.pxp_workspace_size([api.make_problem(inst, krylov="poly", prec="fp32_bulk")])
    assert e.value.code == _lib.PXP_EUNSUPPORTED
    for bad in (dict(hyb_slices=-1), dict(hyb_group=-2), dict(hyb_k=-0.5)):
        with pytest.raises(_lib.PxpError) as e:
            _lib.pxp_workspace_size([api.make_problem(dict(inst, **bad), krylov="poly")])
        assert e.value.code == _lib.PXP_EINVAL, bad


def test_nl_paraexp_rules_on_host(lib):
    """The iterative nonlinear direct (section 3.2) is a Burgers FP64 path
    with the terminal cost; its workspace holds two generations of stage
    states (8 n_steps n doubles) and the slices' states; negative iteration
    counts and tolerances are refused."""
    base = workloads.make("burgers1d_n2048")[0]
    inst = dict(base, nl_paraexp=True)
    ok = api.make_problem(inst, krylov="auto")
    assert ok.flags == _lib.FLAG_NL_PARAEXP
    plain = api.make_problem(base, krylov="auto")
    n, nt = 2048, 8192
    assert _lib.pxp_workspace_size([ok]) - _lib.pxp_workspace_size([plain]) >= 8 * nt * n * 8
    for bad, code in [(dict(prec="fp32_bulk"), _lib.PXP_EUNSUPPORTED)]:
        with pytest.raises(_lib.PxpError) as e:
            _lib.pxp_workspace_size([api.make_problem(inst, krylov="auto", **bad)])
        assert e.value.code == code, bad
    for bad, code in [(dict(cost="integral"), _lib.PXP_EUNSUPPORTED),
                      (dict(nl_iters=-1), _lib.PXP_EINVAL),
                      (dict(nl_slices=-2), _lib.PXP_EINVAL),
                      (dict(nl_slices=3), _lib.PXP_EINVAL),
                      (dict(nl_tol=-1.0), _lib.PXP_EINVAL)]:
        with pytest.raises(_lib.PxpError) as e:
            _lib.pxp_workspace_size([api.make_problem(dict(inst, **bad), krylov="auto")])
        assert e.value.code == code, bad
    lin = dict(workloads.make("advdiff1d_n128")[0], nl_paraexp=True)
    with pytest.raises(_lib.PxpError) as e:
        _lib.pxp_workspace_size([api.make_problem(lin, krylov="poly")])
    assert e.value.code == _lib.PXP_EUNSUPPORTED


def test_chebyshev_flavour_rules_on_host(lib):
    """The Chebyshev flavour is the Burgers chains' (its own chain kernel):
    named for a linear problem it is refused, for the Burgers workload's
    grid accepted."""
    lin = workloads.make("advdiff1d_n128")[0]
    with pytest.raises(_lib.PxpError) as e:
        _lib.pxp_workspace_size([api.make_problem(lin, krylov="chebyshev")])
    assert e.value.code == _lib.PXP_EUNSUPPORTED
    burg = workloads.make("burgers1d_n2048")[0]
    assert _lib.pxp_workspace_size([api.make_problem(burg, krylov="chebyshev")]) > 0
