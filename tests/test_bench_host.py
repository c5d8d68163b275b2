"""Host-side checks of bench.py that need no GPU: the one-GPU contract, the
algorithmic-bytes formula of an Arnoldi space, and the rule that counter
traffic is reported only for the kernel source it was measured on."""
import hashlib
import math
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("m", [1, 2, 7, 40])
@pytest.mark.parametrize("passes", [1.0, 1.5, 2.0])
def test_krylov_space_bytes_closed_form(m, passes):
    """Step j reads j+1 basis vectors twice per pass and writes one; the
    recombination reads m and writes one; the start vector is read and
    written: in total passes*m*(m+1) + 2m + 3 vectors of 8n bytes."""
    n = 4096
    want = 8.0 * n * (passes * m * (m + 1) + 2 * m + 3)
    assert bench.krylov_space_bytes(n, m, passes) == pytest.approx(want, rel=1e-15)


def _fake_tree(tmp_path, src_text, line_sha):
    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_2004_00546_amd" / "csrc").mkdir(parents=True)
    (tmp_path / "paper_2004_00546_amd" / "csrc" / "pxp_krylov.hip").write_text(src_text)
    (tmp_path / "profiles" / "advdiff1d_n4096_kernels.md").write_text(
        "text\ntraffic k_direct bytes_per_launch=1234.5 source_sha256_prefix=%s\n" % line_sha)


def test_profiled_traffic_only_for_the_profiled_source(tmp_path, monkeypatch):
    src = "// kernel source\n"
    sha = hashlib.sha256(src.encode()).hexdigest()[:16]
    _fake_tree(tmp_path, src, sha)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profiled_traffic("k_direct") == 1234.5
    assert bench.profiled_traffic("k_other") is None
    # the kernel changed after the counters were taken: no traffic figure
    (tmp_path / "paper_2004_00546_amd" / "csrc" / "pxp_krylov.hip").write_text(src + "x")
    assert bench.profiled_traffic("k_direct") is None


def test_tree_jobs_counts_pairs():
    """A pairwise tree over P slices has P - 1 pairs; ceil(log2 P) levels;
    the right-hand ranges of level l are 2^(l-1) slices (power of two P)."""
    for P in (1, 2, 6, 13, 64, 256):
        lv = bench.tree_jobs(P)
        assert sum(len(x) for x in lv) == max(P - 1, 0)
        assert len(lv) == (0 if P == 1 else math.ceil(math.log2(P)))
    lv = bench.tree_jobs(256)
    assert all(set(x) == {2 ** l} for l, x in enumerate(lv))


def test_pois_terms_tail_rule():
    """The smallest D whose Poisson tail is below tol: the tail at D is below,
    the tail at D - 1 above (checked against a direct sum)."""
    for lam in (0.13, 0.53, 8.5, 68.0, 136.0):
        for tol in (1e-10, 1e-12):
            D = bench.pois_terms(lam, tol)
            pk = [math.exp(k * math.log(lam) - lam - math.lgamma(k + 1)) for k in range(D + 200)]
            tail = lambda d: sum(pk[d:])  # noqa: E731
            assert tail(D) <= tol * (1 + 1e-9)
            assert tail(D - 1) > tol


def test_hybrid_bounds_follow_eq_nonequip():
    """The hybrid scheme's adjoint slices (the library's rule, restated for
    the bench model): equal slices for k = 0; for k > 0 the lengths shrink
    toward T by about k / (k + 1) per slice (eq. paritionRatio), on the grid
    of lcm(macro step, checkpoint interval)."""
    import bench
    from paper_2004_00546_amd import workloads
    inst = workloads.make("burgers1d_icost")[0]
    b = bench.hyb_bounds(inst)
    assert b[0] == 0 and b[-1] == inst["n_steps"] and len(b) == 129
    assert len(set(b[i + 1] - b[i] for i in range(len(b) - 1))) == 1
    b = bench.hyb_bounds(dict(inst, hyb_slices=16, hyb_k=2.0))
    L = 64
    assert all(x % L == 0 for x in b) and b == sorted(set(b))
    d = [b[i + 1] - b[i] for i in range(len(b) - 1)]
    for i in range(3):
        assert abs(d[i + 1] / d[i] - 2.0 / 3.0) < 0.1


def test_burgers_class_models():
    """The Burgers models: the serial march's flop, the Chebyshev chains'
    flop from the term counters (direct class: the nonlinear chain), and
    the nonlinear iteration's marches as HBM bytes, scaled by the measured
    iterations per call."""
    from paper_2004_00546_amd import api, workloads
    inst = workloads.make("burgers1d_nl")[0]
    n, nt = inst["nx"], inst["n_steps"]
    prob = api.make_problem(inst)
    m = bench.class_models([inst], [prob], None, {0: (64, 1000.0, 0), 1: (256, 6000.0, 0)},
                           nl_k=5.0)
    assert m["serial_direct"][1] == 4 * nt * n * bench.BURGERS_FLOPS
    assert m["krylov_direct"][1] == 1000.0 * n * bench.CHEB_FLOPS
    assert m["ltv_adjoint"][1] == 6000.0 * n * bench.CHEB_FLOPS
    st = 4 * nt * n * 8
    assert m["nl_iter"] == ("hbm", 5.0 * 2 * st, "B", m["nl_iter"][3])
    assert m["slices"][1] == 5.0 * (st + nt * n * 8)
    # without the measured iteration count the marches have no model
    assert "nl_iter" not in bench.class_models([inst], [prob], None, {}, nl_k=None)


def test_nl_model_formulas():
    """eq. nonLinSpeedup on measured class times: the predicted time is
    K (S tau_I + (n_t - S) tau_H + S tau_F) + the adjoint; s > 1 exactly
    when N exceeds the bound solved from it; the ceiling is the N -> oo
    limit."""
    inst = dict(n_steps=8192, P=128, nl_slices=64)
    S, Sa, nt = 128, 64, 8192
    steps = 2
    kern = {"slices": {"per_step_ms": 5 * 0.4}, "krylov_direct": {"per_step_ms": 5 * 1.6},
            "nl_iter": {"per_step_ms": 5 * 0.6}, "ltv_adjoint": {"per_step_ms": 4.3},
            "ltv_nodes": {"per_step_ms": 0.05}, "ltv_check": {"per_step_ms": 0.3}}
    kern_ser = {"serial_direct": 7.66, "serial_reverse": 24.9}
    report = [{"nl_iterations": 10}]
    m = bench.nl_model(inst, kern, kern_ser, 0.018, 0.0327, report, steps)
    assert m["iterations"] == 5.0 and m["slices"] == 64 and m["adjoint_slices"] == 128
    ti, th, tf = 0.4 / S, 1.6 / (nt - S), 0.6 / S
    adj = 4.3 + 0.05 + 0.3
    assert m["predicted_ms"] == pytest.approx(5 * (S * ti + (nt - S) * th + S * tf) + adj)
    tds, tas = 7.66 / nt, 24.9 / nt
    tia, tha = 0.05 / Sa, 4.3 / (nt - Sa)
    n_min = (5 * (ti + tf - th) + tia - tha) / (tds + tas - 5 * th - tha)
    assert m["min_slices_for_speedup"] == pytest.approx(n_min)

    # the bound is where the modelled speedup crosses one: eq. nonLinSpeedup
    # with the measured per-step times at N slices of the horizon
    def speedup(N):
        ser = nt * (tds + tas)
        par = 5 * (nt / N * (ti + tf) + nt * (N - 1) / N * th) + nt / N * tia + nt * (N - 1) / N * tha
        return ser / par
    assert speedup(n_min * 1.01) > 1.0 > speedup(n_min * 0.99)
    assert m["ceiling_speedup"] == pytest.approx((tds + tas) / (5 * th + tha))
