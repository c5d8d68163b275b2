"""Benchmark: gradient evaluations per second on one MI355X, Paraexp vs serial
RK4 stepping, at the FP64 accuracy gate (rel err <= 1e-8 against the CPU
oracle).

Workload (default): 1D periodic advection-diffusion, N = 4096, T = 4,
dt = 1e-4 (40 000 RK4 steps), 64 time slices, Krylov dimension 40,
64 forcing amplitudes; one full direct-adjoint gradient per step.

Prints one JSON line (see --help for options).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "gradient evals/s, Paraexp vs serial stepping on 1 GPU at rel err ≤1e-8"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(x, ref):
    return float(np.linalg.norm(np.asarray(x) - ref) / np.linalg.norm(ref))


def rk4_slice_flops(n, n_steps):
    # per point and stage: stencil 9, source 3, accumulation 2, stage state 2
    return 64.0 * n * n_steps


def krylov_space_bytes(n, m):
    """Algorithmic bytes of one Arnoldi space of dimension m on n points:
    step j reads V_0..V_j four times (two Gram-Schmidt passes, each a dot
    pass and an update pass) and writes V_{j+1}; the recombination reads m
    vectors and writes one; the start vector is read and written once."""
    vecs = sum(4 * (j + 1) + 1 for j in range(m)) + (m + 1) + 2
    return 8.0 * n * vecs


def profiled_traffic(kernel_key):
    """HBM bytes per launch from the committed counter summary, only while
    the Krylov kernel source is the one that was profiled."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "advdiff1d_n4096_kernels.md")
    src = os.path.join(ROOT, "paper_2004_00546_amd", "csrc", "pxp_krylov.hip")
    try:
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
        for line in open(prof):
            if line.startswith("traffic " + kernel_key + " "):
                f = dict(kv.split("=") for kv in line.split()[2:])
                if f.get("source_sha256_prefix") == sha:
                    return float(f["bytes_per_launch"])
    except OSError:
        pass
    return None


def m_is_full(inst):
    # shift-and-invert spaces always run to the full dimension m
    return True


def time_runner(torch, r, steps, warmup):
    for _ in range(warmup):
        r.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r.run()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="advdiff1d_n4096")
    ap.add_argument("--krylov", default=None, choices=["poly", "shift_invert"])
    ap.add_argument("--sched", default="classic", choices=["classic", "chain"])
    ap.add_argument("--serial-steps", type=int, default=5)
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32_bulk"])
    ap.add_argument("--tol", type=float, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle", action="store_true",
                    help="skip the CPU accuracy check (profiler runs only; "
                         "the JSON line then reports value 0)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy five times (scale "
                         "for the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the time slices are a "
              "batch dimension inside each launch); --gpus %d is not supported"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2004_00546_amd import _lib, api, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        nbytes = 1 << 30
        a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_launch": nbytes,
                          "launches": 5}), flush=True)
        return
    inst = workloads.make(args.workload)[0]
    n, n_steps, P, m = inst["nx"] * inst.get("ny", 1), inst["n_steps"], inst["P"], inst["m"]
    log("workload %s: N=%d steps=%d P=%d m=%d" % (args.workload, n, n_steps, P, m))

    if args.krylov is None:
        # shift-and-invert needs a constant-coefficient tridiagonal operator
        args.krylov = "shift_invert" if inst["op"] == "advdiff1d" else "poly"
    tol = args.tol if args.tol is not None else (1e-10 if args.prec == "fp64" else 1e-6)
    pxp = api.GradientRunner([inst], method="paraexp", krylov=args.krylov,
                             sched=args.sched, prec=args.prec, tol=tol)
    ser = api.GradientRunner([inst], method="serial", prec=args.prec)

    # timed Paraexp region, with per-kernel events on the library's stream
    for _ in range(args.warmup):
        pxp.run()
    torch.cuda.synchronize()
    pxp.status()
    _lib.pxp_device_counters(pxp.ws)
    _lib.pxp_profile_enable(True)
    for k in _lib.KCLASS:
        _lib.pxp_profile_read(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pxp.run()
    torch.cuda.synchronize()
    t_pxp = (time.perf_counter() - t0) / args.steps
    _lib.pxp_profile_enable(False)
    kern = {}
    for k in _lib.KCLASS:
        ms, cnt = _lib.pxp_profile_read(k)
        if cnt:
            kern[k] = dict(avg_ms=ms / cnt, launches=cnt)
    substeps, iters = _lib.pxp_device_counters(pxp.ws)
    code, est = pxp.status()
    res_pxp = pxp.results()[0]
    log("paraexp %.3f ms/gradient  kernels %s  status %d est %.1e"
        % (t_pxp * 1e3, kern, code, est))

    t_ser = time_runner(torch, ser, args.serial_steps, 1)
    res_ser = ser.results()[0]
    log("serial %.3f ms/gradient" % (t_ser * 1e3))

    # accuracy against the oracle; the same run is the CPU baseline timing
    if args.no_oracle:
        nan = float("nan")
        ref = dict(grad=res_pxp["grad"] * nan, qT=res_pxp["qT"] * nan,
                   lam0=res_pxp["lam"] * nan, Lambda=res_pxp["lam"] * nan)
        t_orc = nan
        args.no_cpu_baseline = True
    else:
        import oracle
        oracle.build()
        t0 = time.perf_counter()
        ref = oracle.gradient(inst)
        t_orc = time.perf_counter() - t0
    lam_key = "Lambda" if inst["control"] == "forcing" else "lam0"
    err = dict(paraexp_grad=rel(res_pxp["grad"], ref["grad"]),
               paraexp_adjoint=rel(res_pxp["lam"], ref[lam_key]),
               paraexp_qT=rel(res_pxp["qT"], ref["qT"]),
               serial_grad=rel(res_ser["grad"], ref["grad"]),
               serial_qT=rel(res_ser["qT"], ref["qT"]))
    log("rel errors", err, "oracle %.2f s" % t_orc)

    # Roofline of the HBM-streaming kernel: the direct homogeneous pieces
    # (P-1 Arnoldi spaces in one launch); the register-resident RK4 slices
    # are reported against the FP64 vector peak.
    roof = None
    if "krylov_direct" in kern and args.sched == "classic" and m_is_full(inst):
        byts = (P - 1) * krylov_space_bytes(n, m)
        sec = kern["krylov_direct"]["avg_ms"] * 1e-3
        ach = byts / sec / 1e9
        tr = profiled_traffic("k_krylov1d_direct_classic")
        roof = dict(kernel="k_krylov1d, direct pieces (classic, %d workgroups)" % (P - 1),
                    bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=ach / HBM_PEAK_GBS, traffic=tr,
                    algorithmic_bytes_per_launch=byts,
                    avg_launch_ms=kern["krylov_direct"]["avg_ms"])
    elif "slices" in kern:
        ach = rk4_slice_flops(n, n_steps) / (kern["slices"]["avg_ms"] * 1e-3) / 1e12
        roof = dict(kernel="k_rk4_lin1d (inhomogeneous slices)", bound="alu",
                    achieved=ach, peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=ach / FP64_PEAK_TFLOPS, traffic=None)
    elif "ltv_adjoint" in kern:
        sp = substeps / max(1, args.steps)
        byts = sp * krylov_space_bytes(n, max(1, int(round(iters / max(sp, 1) / max(1, args.steps) * args.steps))))
        ach = byts / (kern["ltv_adjoint"]["avg_ms"] * 1e-3) / 1e9
        roof = dict(kernel="k_krylov1d, time-varying Magnus chain (1 workgroup)",
                    bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=ach / HBM_PEAK_GBS, traffic=None)

    gate = 1e-8 if args.prec == "fp64" else 1e-5
    ok = err["paraexp_grad"] <= gate and err["paraexp_qT"] <= gate and code == 0
    line = {
        "metric": METRIC,
        "value": (1.0 / t_pxp) if ok else 0.0,
        "unit": "gradient evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_pxp * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "N": n, "T": inst["T"],
                   "n_steps": n_steps, "slices": P, "krylov_m": m,
                   "krylov": args.krylov, "schedule": args.sched,
                   "precision": args.prec, "gate": gate,
                   "controls": int(inst["basis"].shape[0])},
        "serial_gpu": {"value": 1.0 / t_ser, "ms_per_step": t_ser * 1e3},
        "speedup_vs_serial": t_ser / t_pxp,
        "rel_err_vs_oracle": err,
        "krylov": {"spaces_per_gradient": substeps / max(1, args.steps),
                   "iters_per_gradient": iters / max(1, args.steps),
                   "max_est": est, "status": code},
        "kernels_ms": {k: v["avg_ms"] for k, v in kern.items()},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = {"value": 1.0 / t_orc, "unit": "gradient evals/s",
                                "cores": 1, "kind": "oracle",
                                "sample": "one full gradient of the workload "
                                          "(serial FP64 RK4 + exact discrete adjoint)"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
