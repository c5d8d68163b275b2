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
FP32_PEAK_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(x, ref):
    return float(np.linalg.norm(np.asarray(x) - ref) / np.linalg.norm(ref))


def rk4_slice_flops(n, n_steps):
    # per point and stage: stencil 9, source 3, accumulation 2, stage state 2
    return 64.0 * n * n_steps


def krylov_space_bytes(n, m, passes=2.0):
    """Algorithmic bytes of one Arnoldi space of dimension m on n points:
    step j reads V_0..V_j twice per Gram-Schmidt pass (a dot pass and an
    update pass; `passes` = average passes per step, 1 to 2) and writes
    V_{j+1}; the recombination reads m vectors and writes one; the start
    vector is read and written once."""
    vecs = sum(2 * passes * (j + 1) + 1 for j in range(m)) + (m + 1) + 2
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


def warm(torch, r, count, seconds):
    """Untimed calls: at least `count`, and until `seconds` have passed."""
    t0 = time.perf_counter()
    k = 0
    while k < count or time.perf_counter() - t0 < seconds:
        r.run()
        torch.cuda.synchronize()
        k += 1


def time_runner(torch, r, steps, warmup, seconds=1.0):
    warm(torch, r, warmup, seconds)
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
    ap.add_argument("--warmup-seconds", type=float, default=2.0,
                    help="keep warming up (untimed gradients) for at least this long, so "
                         "the timed region runs at steady-state clocks")
    ap.add_argument("--workload", default="advdiff1d_n4096")
    ap.add_argument("--krylov", default="auto", choices=["poly", "shift_invert", "auto", "taylor", "uniform"])
    ap.add_argument("--sched", default=None, choices=["classic", "chain", "tree"],
                    help="schedule of the direct pieces (default: tree in 2D, classic in 1D)")
    ap.add_argument("--serial-steps", type=int, default=5)
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32_bulk"])
    ap.add_argument("--tol", type=float, default=None)
    ap.add_argument("--block", type=int, default=0,
                    help="threads per workgroup of the RK4 marches (0 = default)")
    ap.add_argument("--kblock", type=int, default=0,
                    help="threads per workgroup of the Krylov kernels (0 = default)")
    ap.add_argument("--graph", action="store_true",
                    help="also time replays of the gradient captured in a hipGraph")
    ap.add_argument("--absorbed", action="store_true",
                    help="adjoint in the absorbed form (batch of adjoint slices "
                         "plus classic pieces; 1D linear problems)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick P, Krylov flavour, schedule and workgroup size with the "
                         "library's autotuner before timing")
    ap.add_argument("--p-range", default="8,256",
                    help="slice counts the autotuner may choose (lo,hi)")
    ap.add_argument("--instances", type=int, default=0,
                    help="use only the first K instances of a batch workload (0 = all)")
    ap.add_argument("--oracle-budget", type=float, default=2.5e8,
                    help="point-steps of the oracle accuracy sample for batch workloads")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle", action="store_true",
                    help="skip the CPU accuracy check (profiler runs only; "
                         "the JSON line then reports value 0)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy five times (scale "
                         "for the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the time slices are a "
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
    insts = workloads.make(args.workload)
    if args.instances > 0:
        insts = insts[:args.instances]
    inst = insts[0]
    B = len(insts)
    n, n_steps, P, m = inst["nx"] * inst.get("ny", 1), inst["n_steps"], inst["P"], inst["m"]
    work = [int(x["nx"]) * int(x.get("ny", 1)) * int(x["n_steps"]) for x in insts]
    log("workload %s: %d instance(s); first N=%d steps=%d P=%d m=%d; point-steps %.3g"
        % (args.workload, B, n, n_steps, P, m, sum(work)))

    if args.sched is None:
        args.sched = "tree" if inst["op"] == "advdiff2d_upwind" else "classic"
    tol = args.tol if args.tol is not None else (1e-9 if args.prec == "fp64" else 1e-6)
    kw = dict(prec=args.prec, block=args.block, kblock=args.kblock)
    pkw = dict(kw, absorbed=args.absorbed)
    tuned = None
    if args.autotune:
        lo, hi = (int(v) for v in args.p_range.split(","))
        t0 = time.perf_counter()
        probs, rep = api.autotune(insts, p_min=lo, p_max=hi,
                                  rtol=1e-9 if args.prec == "fp64" else 5e-6,
                                  krylov=args.krylov, sched=args.sched, tol=tol, **pkw)
        names = {v: k for k, v in _lib.KRYLOV.items()}
        tuned = {"seconds": time.perf_counter() - t0,
                 "P": sorted({int(p.P) for p in probs}),
                 "krylov": sorted({names[int(p.krylov)] for p in probs}),
                 "sched": sorted({"classic" if p.sched == 0 else "chain" for p in probs}),
                 "kblock": sorted({int(p.kblock) for p in probs}),
                 "groups": len({r["group"] for r in rep})}
        log("autotune", tuned, rep[:4])
        pxp = api.GradientRunner(insts, method="paraexp", problems=probs)
    else:
        pxp = api.GradientRunner(insts, method="paraexp", krylov=args.krylov,
                                 sched=args.sched, tol=tol, **pkw)
    ser = api.GradientRunner(insts, method="serial", krylov="auto", **kw)

    # timed Paraexp region, with per-kernel events on the library's stream
    warm(torch, pxp, args.warmup, args.warmup_seconds)
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
            kern[k] = dict(avg_ms=ms / cnt, launches=cnt, per_step_ms=ms / args.steps)
    substeps, iters, reorth = _lib.pxp_device_counters(pxp.ws)
    code, est = pxp.status()
    res_pxp = pxp.results()
    log("paraexp %.3f ms/step  kernels %s  status %d est %.1e"
        % (t_pxp * 1e3, kern, code, est))

    t_graph = None
    if args.graph:
        t_graph = time_graph(torch, pxp, args.steps)
        log("paraexp, hipGraph replay %.3f ms/step" % (t_graph * 1e3))

    t_ser = time_runner(torch, ser, args.serial_steps, 1)
    res_ser = ser.results()
    log("serial %.3f ms/step" % (t_ser * 1e3))

    # accuracy against the oracle on a bounded sample of the instances (all
    # of them for single-instance workloads); the same runs time the CPU
    # baseline
    sample = oracle_sample(insts, work, args.oracle_budget)
    err = None
    t_orc = float("nan")
    if not args.no_oracle:
        import oracle
        oracle.build()
        err = dict(paraexp_grad=0.0, paraexp_adjoint=0.0, paraexp_qT=0.0,
                   serial_grad=0.0, serial_qT=0.0)
        t0 = time.perf_counter()
        for i in sample:
            ref = oracle.gradient(insts[i])
            lam_key = "Lambda" if insts[i]["control"] == "forcing" else "lam0"
            e = dict(paraexp_grad=rel(res_pxp[i]["grad"], ref["grad"]),
                     paraexp_adjoint=rel(res_pxp[i]["lam"], ref[lam_key]),
                     paraexp_qT=rel(res_pxp[i]["qT"], ref["qT"]),
                     serial_grad=rel(res_ser[i]["grad"], ref["grad"]),
                     serial_qT=rel(res_ser[i]["qT"], ref["qT"]))
            err = {k: max(err[k], v) for k, v in e.items()}
        t_orc = time.perf_counter() - t0
        log("rel errors (max over %d sampled instance(s))" % len(sample), err,
            "oracle %.2f s" % t_orc)
    else:
        args.no_cpu_baseline = True

    roof = roofline(kern, insts, args, substeps, iters, pxp.problems, reorth)

    gate = 1e-8 if args.prec == "fp64" else 1e-5
    ok = (err is not None and err["paraexp_grad"] <= gate and err["paraexp_qT"] <= gate
          and code == 0)
    cfg = {"workload": args.workload, "instances": B, "N": n, "T": inst["T"],
           "n_steps": n_steps, "slices": P, "krylov_m": m, "krylov": args.krylov,
           "schedule": args.sched, "precision": args.prec, "gate": gate,
           "controls": int(np.asarray(inst["basis"]).shape[0]),
           "block": args.block, "kblock": args.kblock,
           "adjoint_form": "absorbed" if args.absorbed else "unabsorbed"}
    if B > 1:
        cfg.update(N=sorted({int(x["nx"]) * int(x.get("ny", 1)) for x in insts}),
                   n_steps=[min(int(x["n_steps"]) for x in insts),
                            max(int(x["n_steps"]) for x in insts)],
                   T=[min(x["T"] for x in insts), max(x["T"] for x in insts)],
                   point_steps=sum(work))
    line = {
        "metric": METRIC,
        "value": (B / t_pxp) if ok else 0.0,
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
        "config": cfg,
        "serial_gpu": {"value": B / t_ser, "ms_per_step": t_ser * 1e3},
        "speedup_vs_serial": t_ser / t_pxp,
        "rel_err_vs_oracle": err,
        "oracle_sample": sample,
        "krylov": {"spaces_per_step": substeps / max(1, args.steps),
                   "iters_per_step": iters / max(1, args.steps),
                   "reorth_per_step": reorth / max(1, args.steps),
                   "max_est": est, "status": code},
        "kernels_ms": {k: v["avg_ms"] for k, v in kern.items()},
        "roofline": roof,
    }
    if t_graph is not None:
        line["graph"] = {"value": B / t_graph, "ms_per_step": t_graph * 1e3}
    if tuned is not None:
        line["config"]["autotune"] = tuned
    if not args.no_cpu_baseline:
        w_s = sum(work[i] for i in sample)
        t_all = t_orc * sum(work) / w_s
        line["cpu_baseline"] = {
            "value": B / t_all, "unit": "gradient evals/s", "cores": 1, "kind": "oracle",
            "sample": ("one full gradient of the workload (serial FP64 RK4 + exact "
                       "discrete adjoint)" if B == 1 else
                       "full gradients of instances %s (%.3g of %.3g point-steps, %.1f s), "
                       "scaled by point-steps to the %d-instance batch"
                       % (sample, w_s, sum(work), t_orc, B))}
    print(json.dumps(line), flush=True)


def oracle_sample(insts, work, budget):
    """Instances the oracle checks: all of a single-instance workload; for a
    batch, the cheapest instance of each grid size, then the cheapest others
    while the point-step budget lasts."""
    if len(insts) == 1:
        return [0]
    order = sorted(range(len(insts)), key=lambda i: work[i])
    pick, seen, used = [], set(), 0
    for i in order:
        nn = int(insts[i]["nx"]) * int(insts[i].get("ny", 1))
        if nn not in seen:
            pick.append(i)
            seen.add(nn)
            used += work[i]
    for i in order:
        if i not in pick and used + work[i] <= budget:
            pick.append(i)
            used += work[i]
    return sorted(pick)


def time_graph(torch, r, steps):
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        r.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        r.run()
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def roofline(kern, insts, args, substeps, iters, problems, reorth=0):
    """Roofline object for the kernel class that takes the most time per step."""
    if not kern:
        return None
    top = max(kern, key=lambda k: kern[k]["per_step_ms"])
    inst = insts[0]
    n = inst["nx"] * inst.get("ny", 1)
    P, m = int(problems[0].P), int(problems[0].m)
    sec = kern[top]["avg_ms"] * 1e-3
    if top == "krylov_direct" and int(problems[0].sched) == 0 and len(insts) == 1:
        # spaces may stop before dimension m: count the average dimension
        # reached (Arnoldi iterations / spaces, all launches), rounded down
        m_eff = min(m, int(iters / max(substeps, 1))) if substeps else m
        passes = 1.0 + reorth / iters if iters else 2.0
        byts = (P - 1) * krylov_space_bytes(n, m_eff, passes)
        ach = byts / sec / 1e9
        return dict(kernel="k_krylov1d, direct pieces (classic, %d workgroups)" % (P - 1),
                    bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=ach / HBM_PEAK_GBS,
                    traffic=profiled_traffic("k_krylov1d_direct_classic"),
                    algorithmic_bytes_per_launch=byts, krylov_dim=m_eff,
                    gram_schmidt_passes=passes,
                    avg_launch_ms=kern[top]["avg_ms"])
    if top == "slices" and len(insts) == 1:
        ach = rk4_slice_flops(n, inst["n_steps"]) / sec / 1e12
        return dict(kernel="k_rk4_lin1d (inhomogeneous slices)", bound="alu",
                    achieved=ach, peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=ach / FP64_PEAK_TFLOPS, traffic=None, avg_launch_ms=kern[top]["avg_ms"])
    if top == "serial_direct" and all(x["op"] == "burgers1d" for x in insts):
        # one launch marches every instance; 48 flop per point and step
        per_step = kern[top]["launches"] / args.steps
        fl = sum(48.0 * x["nx"] * x["n_steps"] for x in insts) / per_step
        peak = FP64_PEAK_TFLOPS if args.prec == "fp64" else FP32_PEAK_TFLOPS
        ach = fl / sec / 1e12
        return dict(kernel="k_burgers_direct_batch (serial Burgers RK4 marches)",
                    bound="alu", achieved=ach, peak=peak, unit="TFLOP/s",
                    frac=ach / peak, traffic=None, avg_launch_ms=kern[top]["avg_ms"])
    if top in ("ltv_adjoint", "krylov_adjoint", "krylov_direct"):
        # bytes streamed by the Arnoldi steps actually taken (device counters):
        # step j of a space reads j+1 basis vectors twice per Gram-Schmidt
        # pass (passes from the device's second-pass counter) and writes one
        sp = substeps / max(1, args.steps)
        it = iters / max(1, args.steps)
        mm = it / max(sp, 1.0)
        nbar = sum(x["nx"] * x.get("ny", 1) for x in insts) / len(insts)
        passes = 1.0 + reorth / iters if iters else 2.0
        byts = sp * krylov_space_bytes(nbar, max(1, int(round(mm))), passes)
        launches = kern[top]["launches"] / args.steps
        ach = byts / launches / sec / 1e9
        return dict(kernel="k_krylov1d (%s)" % top, bound="hbm", achieved=ach,
                    peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS, traffic=None,
                    avg_launch_ms=kern[top]["avg_ms"])
    return dict(kernel=top, bound=None, achieved=None, peak=None, unit=None, frac=None,
                traffic=None, avg_launch_ms=kern[top]["avg_ms"])


if __name__ == "__main__":
    main()
