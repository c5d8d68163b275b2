"""Benchmark: gradient evaluations per second on one MI355X, Paraexp vs serial
RK4 stepping, at the FP64 accuracy gate (rel err <= 1e-8 against the CPU
oracle).

Workload (default): 16 independent instances of the 2D periodic upwind
advection-diffusion problem on 256 x 256 grids, horizons T uniform in
[0.5, 2] (256 to 1024 RK4 steps), 256 time slices, 8 forcing blob
amplitudes each; one step = one full direct-adjoint gradient of every
instance; value = 16 / seconds per step.  A secondary measurement on the
1D N = 4096 problem (40 000 steps, 64 slices) rides in the same JSON line.

Prints one JSON line (see --help for options).
"""
from __future__ import annotations

import argparse
import functools
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "gradient evals/s, Paraexp vs serial stepping on 1 GPU at rel err ≤1e-8"
DEFAULT_WORKLOAD = "advdiff2d_256"
SECONDARY_WORKLOAD = "advdiff1d_n4096"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
# flops per grid point and stencil application (multiply-add = 2 flops):
# 2D RK4 step as its polynomial, Horner level: 5-point stencil (5 FMA) +
# r_j y + f_j F (2 FMA)
RK2D_FLOPS = 14.0
# 2D uniformised exponential, one term: 4-point N (4 FMA) + weighted sum (1)
POIS_FLOPS = 10.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(x, ref):
    return float(np.linalg.norm(np.asarray(x) - ref) / np.linalg.norm(ref))


def krylov_space_bytes(n, m, passes=2.0):
    """Algorithmic bytes of one Arnoldi space of dimension m on n points:
    step j reads V_0..V_j twice per Gram-Schmidt pass (a dot pass and an
    update pass; `passes` = average passes per step, 1 to 2) and writes
    V_{j+1}; the recombination reads m vectors and writes one; the start
    vector is read and written once."""
    vecs = sum(2 * passes * (j + 1) + 1 for j in range(m)) + (m + 1) + 2
    return 8.0 * n * vecs


@functools.lru_cache(maxsize=None)
def pois_terms(lam, tol):
    """Terms of a uniformised exponential: the smallest D with the Poisson
    tail P(X >= D) <= tol (the library's rule)."""
    if lam <= 0.0:
        return 1
    K = int(lam + 40.0 * math.sqrt(lam) + 80.0)
    logp = [k * math.log(lam) - lam - math.lgamma(k + 1.0) for k in range(K + 1)]
    tail, D = 0.0, K + 1
    for k in range(K, 0, -1):
        tail += math.exp(logp[k])
        if tail > tol:
            break
        D = k
    return D


def tree_jobs(P):
    """(left-range length of each pair) for the pairwise tree of P slices:
    a list per level of the right-hand range sizes of its pairs."""
    size = [1] * P
    levels = []
    while len(size) > 1:
        pairs = len(size) // 2
        levels.append([size[2 * j + 1] for j in range(pairs)])
        ns = [size[2 * j] + size[2 * j + 1] for j in range(pairs)]
        if len(size) % 2:
            ns.append(size[-1])
        size = ns
    return levels


def tree_pairs(P):
    """(left, right) range lengths of every pair, per level, of the pairwise
    tree of P slices (an odd last range carried up alone)."""
    size = [1] * P
    levels = []
    while len(size) > 1:
        pairs = len(size) // 2
        levels.append([(size[2 * j], size[2 * j + 1]) for j in range(pairs)])
        ns = [size[2 * j] + size[2 * j + 1] for j in range(pairs)]
        if len(size) % 2:
            ns.append(size[-1])
        size = ns
    return levels


def sten2d_mu(inst):
    """Diagonal magnitude of the 2D upwind five-point operator."""
    hx, hy = inst["L"] / inst["nx"], inst["L"] / inst["ny"]
    nu = inst["nu"]
    return (inst["vx"] / hx + inst["vy"] / hy + 2 * nu / hx ** 2 + 2 * nu / hy ** 2)


def profiled_traffic(kernel_key, prof_name="advdiff1d_n4096_kernels.md",
                     src_name="pxp_krylov.hip"):
    """HBM bytes per launch from a committed counter summary, only while the
    kernel source is the one that was profiled."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", prof_name)
    src = os.path.join(ROOT, "paper_2004_00546_amd", "csrc", src_name)
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


def host_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return dict(nproc=os.cpu_count(), usable_cpus=usable, cpu_model=model)


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


def profile_classes(torch, _lib, r, steps):
    """Per-class kernel time (ms per call) over `steps` calls of r, from the
    library's events."""
    _lib.pxp_profile_enable(True)
    for k in _lib.KCLASS:
        _lib.pxp_profile_read(k)
    for _ in range(steps):
        r.run()
    torch.cuda.synchronize()
    _lib.pxp_profile_enable(False)
    out = {}
    for k in _lib.KCLASS:
        ms, cnt = _lib.pxp_profile_read(k)
        if cnt:
            out[k] = ms / steps
    return out


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


def oracle_sample(insts, work, budget):
    """Instances the oracle checks: all of a single-instance workload; for a
    batch, the longest one, the cheapest of each grid size, then the
    cheapest others while the point-step budget lasts."""
    if len(insts) == 1:
        return [0]
    order = sorted(range(len(insts)), key=lambda i: work[i])
    pick, seen, used = [order[-1]], set(), work[order[-1]]
    for i in order:
        nn = int(insts[i]["nx"]) * int(insts[i].get("ny", 1))
        if nn not in seen:
            seen.add(nn)
            if i not in pick:
                pick.append(i)
                used += work[i]
    for i in order:
        if i not in pick and used + work[i] <= budget:
            pick.append(i)
            used += work[i]
    return sorted(pick)


def run_oracle(insts, sample, threads):
    """Oracle gradients of the sampled instances, `threads` at a time (the
    oracle is a C library called through ctypes, which releases the GIL).
    Returns (results by index, wall seconds, summed per-instance seconds)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    oracle.build()

    def one(i):
        t0 = time.perf_counter()
        out = oracle.gradient(insts[i])
        return i, out, time.perf_counter() - t0

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(one, sample))
    wall = time.perf_counter() - t0
    return {i: o for i, o, _ in res}, wall, {i: dt for i, _, dt in res}


# ---- roofline models of the kernel classes ------------------------------------

# Burgers: flop per point per RK4 stage (central advection and diffusion,
# the stage update and the step sum) and per Chebyshev term (stencil
# coefficients from W, the 3-point stencil, the shift and scale, the
# three-term recurrence and the weighted sum)
BURGERS_FLOPS = 14.0
CHEB_FLOPS = 18.0


def class_models(insts, problems, args, counters, nl_k=None):
    """Per kernel class: (bound, algorithmic quantity per class launch, unit
    word, description).  counters: {cls: (substeps, iters, reorth)} per step
    of the direct (0) and adjoint (1) exponentials."""
    out = {}
    two_d = all(x["op"] == "advdiff2d_upwind" for x in insts)
    one_lin = all(x["op"] == "advdiff1d" for x in insts)
    tol = problems[0].krylov_tol * 1e-2
    if two_d:
        n = [x["nx"] * x["ny"] for x in insts]
        flops = sum(x["n_steps"] * 4 * nn * RK2D_FLOPS for x, nn in zip(insts, n))
        out["slices"] = ("alu", flops, "flop",
                         "k_band2d_fwd: every slice of every instance, 4 stencil "
                         "applications per RK4 step at %g flop per point" % RK2D_FLOPS)
        sched = {0: "classic", 1: "chain", 2: "tree"}[int(problems[0].sched)]
        if sched == "tree":
            byts = sum(3 * (int(p.P) - 1) * 8 * nn for p, nn in zip(problems, n))
            terms = 0
            for x, p, nn in zip(insts, problems, n):
                mu, dT = sten2d_mu(x), x["T"] / int(p.P)
                for lv in tree_jobs(int(p.P)):
                    terms += sum(pois_terms(mu * dT * r, tol) for r in lv) * nn
            out["krylov_direct"] = (
                "hbm", byts, "B",
                "k_pois2d, tree of uniformised exponentials: every pair reads its two "
                "partial sums and writes one (3 vectors per pair, P-1 pairs per "
                "instance); %.3g term-points (%.3g flop) beside it" %
                (terms, terms * POIS_FLOPS))
        icost = all(x.get("cost") == "integral" for x in insts)
        if icost and sched == "tree":
            # integral cost: the tree is walked back down (each pair with a
            # start state reads it and the left sum and writes the state at
            # its middle; the leftmost pairs copy), the sources are written
            # by a second march of every slice and read by the adjoint slices,
            # whose pieces combine pairwise with two sums (state and Lambda
            # share, the halves' shares added)
            dn, st, rs, adj, adj_terms = 0.0, 0.0, 0.0, 0.0, 0.0
            for x, p, nn in zip(insts, problems, n):
                P, nt = int(p.P), int(x["n_steps"])
                mu, dT = sten2d_mu(x), x["T"] / P
                for lv in tree_pairs(P):
                    for j, (ls, rs_) in enumerate(lv):
                        first = j == 0
                        dn += (2 if first else 3) * 8 * nn
                        adj += 6 * 8 * nn
                        adj_terms += pois_terms(mu * dT * ls, tol) * nn
                st += (nt + 1) * 8 * nn + (P - 1) * 8 * nn
                rs += (nt + 1) * 8 * nn + 2 * P * 8 * nn
            bd, bq, wd, dd = out["krylov_direct"]
            out["krylov_direct"] = (bd, bq + dn, wd,
                                    dd + "; plus the walk back down for the slice-start "
                                    "states (3 vectors per pair, 2 for the leftmost)")
            out["sources"] = (
                "hbm", st, "B",
                "k_band2d_src: every slice again from its corrected start state "
                "(read once), writing the n_t + 1 step sources dJ/dq_n; %.3g flop of "
                "RK4 beside it" % flops)
            out["adj_slices"] = (
                "hbm", rs, "B",
                "k_band2d_rsrc: the adjoint slices read every step source once and "
                "write each slice's end state and Lambda share")
            out["krylov_adjoint"] = (
                "hbm", adj, "B",
                "k_pois2d, adjoint tree of the integral cost: every pair reads its "
                "halves' states and Lambda shares and writes its state and share (6 "
                "vectors per pair; the root's share is Lambda); %.3g term-points "
                "beside it" % adj_terms)
        elif all(int(p.krylov) in (2, 4) for p in problems):
            # the adjoint piece by uniformisation (AUTO or named)
            lam = [sten2d_mu(x) * x["T"] for x in insts]
            adj_terms = sum(pois_terms(min(l, 600.0), tol) * math.ceil(l / 600.0) * nn
                            for l, nn in zip(lam, n))
            out["krylov_adjoint"] = (
                "alu", adj_terms * (POIS_FLOPS + 2.0), "flop",
                "k_pois2d, the adjoint piece with its time integral: terms x points x "
                "%g flop" % (POIS_FLOPS + 2.0))
    burgers = all(x["op"] == "burgers1d" for x in insts)
    if burgers:
        # one workgroup per march or chain: FP64 work on one CU, latency
        # bound; the nonlinear iteration's marches stream the stage states
        n = [int(x["nx"]) for x in insts]
        nt = [int(x["n_steps"]) for x in insts]
        flops = sum(4 * s * nn * BURGERS_FLOPS for s, nn in zip(nt, n))
        out["serial_direct"] = ("alu", flops, "flop",
                                "k_rk4_burgers_direct: the serial march, 4 stages per step at "
                                "%g flop per point, one workgroup per instance" % BURGERS_FLOPS)
        for cls, name in ((1, "ltv_adjoint"), (0, "krylov_direct")):
            if counters.get(cls) and counters[cls][1]:
                terms = counters[cls][1]
                out[name] = ("alu", terms * n[0] * CHEB_FLOPS if len(n) == 1 else
                             terms * sum(n) / len(n) * CHEB_FLOPS, "flop",
                             "k_cheb_chain: %.0f series terms per step (device counter) x "
                             "points x %g flop (stencil coefficients, stencil, recurrence, "
                             "sum); one workgroup per chain" % (terms, CHEB_FLOPS))
        if all(x.get("nl_paraexp") for x in insts) and len(insts) == 1 and nl_k:
            # per iteration (nl_k of them per call, measured): the zero-start
            # march reads every stage state, the second march reads and
            # writes them, the averages read the step states
            st = 4 * nt[0] * n[0] * 8
            out["nl_iter"] = ("hbm", nl_k * 2 * st, "B",
                              "k_burgers_nl_march from the corrected starts: reads the "
                              "previous stage states and writes the new ones (%.3g B per "
                              "iteration, %.1f iterations)" % (2 * st, nl_k))
            out["slices"] = ("hbm", nl_k * (st + nt[0] * n[0] * 8), "B",
                             "k_burgers_nl_march from zero (reads the stage states) and "
                             "k_nl_slice_mean (reads the step states), %.1f iterations"
                             % nl_k)
    if one_lin and len(insts) == 1 and counters.get(0):
        inst, p = insts[0], problems[0]
        n = inst["nx"]
        sub, it, re = counters[0]
        if int(p.sched) == 0 and sub:
            m_eff = min(int(p.m), int(it / sub))
            passes = 1.0 + re / it if it else 2.0
            byts = (int(p.P) - 1) * krylov_space_bytes(n, m_eff, passes)
            out["krylov_direct"] = (
                "hbm", byts, "B",
                "k_krylov1d, direct pieces (classic, %d workgroups): P-1 Arnoldi spaces "
                "at the measured mean dimension %d and %.3f Gram-Schmidt passes per "
                "step" % (int(p.P) - 1, m_eff, passes))
    return out


def roofline(kern, models, steps, traffic=None):
    objs = {}
    for k, (bound, q, word, desc) in models.items():
        if k not in kern:
            continue
        per_launch = kern[k]["launches"] / steps
        sec = kern[k]["avg_ms"] * 1e-3
        q_launch = q / per_launch
        if bound == "hbm":
            ach, peak, unit = q_launch / sec / 1e9, HBM_PEAK_GBS, "GB/s"
        else:
            ach, peak, unit = q_launch / sec / 1e12, FP64_PEAK_TFLOPS, "TFLOP/s"
        objs[k] = dict(kernel=desc, bound=bound, achieved=ach, peak=peak, unit=unit,
                       frac=ach / peak, traffic=(traffic or {}).get(k),
                       algorithmic_per_launch=q_launch, algorithmic_unit=word,
                       avg_launch_ms=kern[k]["avg_ms"])
    if not kern:
        return None, objs
    top = max(kern, key=lambda k: kern[k]["per_step_ms"])
    main = objs.get(top, dict(kernel=top, bound=None, achieved=None, peak=None, unit=None,
                              frac=None, traffic=None, avg_launch_ms=kern[top]["avg_ms"]))
    return main, objs


# ---- one workload ---------------------------------------------------------------

def measure(args, name, torch, _lib, api, workloads, steps, serial_steps, with_oracle,
            cpu_baseline):
    insts = workloads.make(name)
    if args.instances > 0 and name == args.workload:
        insts = insts[:args.instances]
    if args.pick and name == args.workload:
        insts = [insts[int(i)] for i in args.pick.split(",")]
    if name == args.workload:
        for key, v in (("hyb_slices", args.hyb_slices), ("hyb_k", args.hyb_k),
                       ("hyb_group", args.hyb_group), ("nl_iters", args.nl_iters),
                       ("nl_tol", args.nl_tol), ("nl_slices", args.nl_slices),
                       ("P", args.slices)):
            if v is not None:
                insts = [dict(x, **{key: v}) for x in insts]
    inst = insts[0]
    B = len(insts)
    n = inst["nx"] * inst.get("ny", 1)
    work = [int(x["nx"]) * int(x.get("ny", 1)) * int(x["n_steps"]) for x in insts]
    log("workload %s: %d instance(s); first N=%d steps=%d P=%d; point-steps %.3g"
        % (name, B, n, inst["n_steps"], inst["P"], sum(work)))
    sched = args.sched or ("tree" if inst["op"] == "advdiff2d_upwind" else "classic")
    tol = args.tol if args.tol is not None else (1e-9 if args.prec == "fp64" else 1e-6)
    kw = dict(prec=args.prec, block=args.block, kblock=args.kblock)
    pkw = dict(kw, absorbed=args.absorbed)
    tuned = None
    if args.autotune and name == args.workload:
        lo, hi = (int(v) for v in args.p_range.split(","))
        t0 = time.perf_counter()
        probs, rep = api.autotune(insts, p_min=lo, p_max=hi,
                                  rtol=1e-9 if args.prec == "fp64" else 5e-6,
                                  krylov=args.krylov, sched=sched, tol=tol, **pkw)
        names = {v: k for k, v in _lib.KRYLOV.items()}
        tuned = {"seconds": time.perf_counter() - t0,
                 "P": sorted({int(p.P) for p in probs}),
                 "krylov": sorted({names[int(p.krylov)] for p in probs}),
                 "sched": sorted({{0: "classic", 1: "chain", 2: "tree"}[int(p.sched)]
                                  for p in probs}),
                 "kblock": sorted({int(p.kblock) for p in probs}),
                 "groups": len({r["group"] for r in rep})}
        log("autotune", tuned, rep[:4])
        pxp = api.GradientRunner(insts, method="paraexp", problems=probs)
    else:
        pxp = api.GradientRunner(insts, method="paraexp", krylov=args.krylov, sched=sched,
                                 tol=tol, **pkw)
    # (the integral cost is validated on the tree schedule also for the
    # serial method, which uses neither)
    ser = api.GradientRunner(insts, method="serial", krylov=args.krylov, sched=sched, **kw)

    # timed Paraexp region, with per-kernel events on the library's stream
    warm(torch, pxp, args.warmup, args.warmup_seconds)
    pxp.status()
    _lib.pxp_last_report(pxp.problems, pxp.ws)
    c0 = {c: _lib.pxp_device_counters_class(pxp.ws, c) for c in (0, 1)}
    _lib.pxp_profile_enable(True)
    for k in _lib.KCLASS:
        _lib.pxp_profile_read(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pxp.run()
    torch.cuda.synchronize()
    t_pxp = (time.perf_counter() - t0) / steps
    _lib.pxp_profile_enable(False)
    kern = {}
    for k in _lib.KCLASS:
        ms, cnt = _lib.pxp_profile_read(k)
        if cnt:
            kern[k] = dict(avg_ms=ms / cnt, launches=cnt, per_step_ms=ms / steps)
    c1 = {c: _lib.pxp_device_counters_class(pxp.ws, c) for c in (0, 1)}
    counters = {c: tuple((b - a) / steps for a, b in zip(c0[c], c1[c])) for c in (0, 1)}
    code, est = pxp.status()
    report = _lib.pxp_last_report(pxp.problems, pxp.ws)
    res_pxp = pxp.results()
    log("paraexp %.3f ms/step  kernels %s  status %d est %.1e" % (t_pxp * 1e3, kern, code, est))

    t_graph = None
    if args.graph and name == args.workload:
        t_graph = time_graph(torch, pxp, steps)
        log("paraexp, hipGraph replay %.3f ms/step" % (t_graph * 1e3))

    t_ser, res_ser, kern_ser = None, None, {}
    if serial_steps > 0:
        t_ser = time_runner(torch, ser, serial_steps, 1)
        res_ser = ser.results()
        kern_ser = profile_classes(torch, _lib, ser, serial_steps)
        log("serial %.3f ms/step  kernels %s" % (t_ser * 1e3, kern_ser))

    # accuracy against the oracle on a bounded sample of the instances, run
    # instance-parallel; the same runs time the CPU baseline
    sample = oracle_sample(insts, work, args.oracle_budget)
    err, orc = None, None
    if with_oracle:
        hi = host_info()
        threads = max(1, min(len(sample), hi["usable_cpus"] or 1, args.oracle_threads))
        refs, wall, per = run_oracle(insts, sample, threads)
        err = dict(paraexp_grad=0.0, paraexp_grad_maxabs=0.0, paraexp_adjoint=0.0,
                   paraexp_qT=0.0, serial_grad=0.0, serial_qT=0.0)
        for i in sample:
            ref = refs[i]
            lam_key = "Lambda" if insts[i]["control"] == "forcing" else "lam0"
            g = res_pxp[i]["grad"]
            e = dict(paraexp_grad=rel(g, ref["grad"]),
                     paraexp_grad_maxabs=float(np.max(np.abs(g - ref["grad"])) /
                                               np.max(np.abs(ref["grad"]))),
                     paraexp_adjoint=rel(res_pxp[i]["lam"], ref[lam_key]),
                     paraexp_qT=rel(res_pxp[i]["qT"], ref["qT"]),
                     serial_grad=rel(res_ser[i]["grad"], ref["grad"]) if res_ser else 0.0,
                     serial_qT=rel(res_ser[i]["qT"], ref["qT"]) if res_ser else 0.0)
            err = {k: max(err[k], v) for k, v in e.items()}
        w_s = sum(work[i] for i in sample)
        orc = dict(wall=wall, cpu=sum(per.values()), threads=threads, point_steps=w_s,
                   host=hi)
        log("rel errors (max over %d sampled instance(s))" % len(sample), err,
            "oracle %.2f s wall on %d thread(s), %.2f s summed" % (wall, threads, orc["cpu"]))

    nl_k = (sum(r.get("nl_iterations", 0) for r in report) / steps) if report else None
    models = class_models(insts, pxp.problems, args, counters, nl_k)
    traffic = {}
    if inst["op"] == "advdiff2d_upwind":
        tr = profiled_traffic("k_pois2d_tree", "%s_kernels.md" % name, "pxp_expo2d.hip")
        if tr is not None:
            traffic["krylov_direct"] = tr
    elif name == SECONDARY_WORKLOAD:
        tr = profiled_traffic("k_krylov1d_direct_classic")
        if tr is not None:
            traffic["krylov_direct"] = tr
    roof, roof_all = roofline(kern, models, steps, traffic)

    gate = 1e-8 if args.prec == "fp64" else 1e-5
    ok = (err is not None and err["paraexp_grad"] <= gate and err["paraexp_qT"] <= gate
          and code == 0)
    out = dict(name=name, B=B, P=sorted({int(p.P) for p in pxp.problems}), t_pxp=t_pxp,
               t_ser=t_ser, t_graph=t_graph, ok=ok, gate=gate, kern_ser=kern_ser, steps=steps,
               err=err, sample=sample, kern=kern, counters=counters, est=est, code=code,
               roof=roof, roof_all=roof_all, tuned=tuned, report=report, sched=sched,
               insts=insts, work=work, orc=orc)
    return out


def hyb_bounds(inst):
    """Adjoint slice bounds of the hybrid scheme (the library's rule: eq.
    nonEquiP rounded to multiples of lcm(macro step, checkpoint interval))."""
    nt, P, c = int(inst["n_steps"]), int(inst["P"]), int(inst["ckpt_every"])
    S = nt // P
    L = S // math.gcd(S, c) * c
    U = nt // L
    N = min(int(inst.get("hyb_slices", 0)) or P, U)
    k = float(inst.get("hyb_k", 0.0))
    r = k / (k + 1.0)
    b = [0]
    for i in range(1, N):
        f = (1 - r ** i) / (1 - r ** N) if k > 0 else i / N
        a = int(round(f * U)) * L
        if b[-1] < a < nt:
            b.append(a)
    b.append(nt)
    return b


def hybrid_model(inst, kern, t_ser):
    """The hybrid scheme's times against eq. hybridSpeedup: tau_I (march,
    per RK4 step), tau_I^dagger (adjoint slices, per step of one slice: the
    batches run their slices concurrently), the chain (tau_H^dagger T_H) and
    the check; predicted T_L = n_t tau_I + (last slice) tau_I^dagger +
    chain; the ceiling (tau_I + tau_I^dagger) / (tau_I + tau_H^dagger)."""
    nt = int(inst["n_steps"])
    b = hyb_bounds(inst)
    G = int(inst.get("hyb_group", 0)) or 4
    d = kern.get("serial_direct", {}).get("per_step_ms")
    a = kern.get("adj_slices", {}).get("per_step_ms")
    ch = kern.get("ltv_adjoint", {}).get("per_step_ms", 0.0)
    ck = kern.get("ltv_check", {}).get("per_step_ms", 0.0)
    if not d or not a:
        return None
    tau_i = d / nt
    tau_a = a * G / nt  # equal slices: each batch runs G slices at once
    pred = nt * tau_i + (b[-1] - b[-2]) * tau_a + ch + ck
    serial_model = nt * (tau_i + tau_a)
    return {"slices": len(b) - 1, "group": G, "k": float(inst.get("hyb_k", 0.0)),
            "tau_I_us_per_step": tau_i * 1e3, "tau_I_adj_us_per_step": tau_a * 1e3,
            "k_measured": tau_a / tau_i, "chain_ms": ch, "check_ms": ck,
            "predicted_ms": pred,
            "predicted_speedup_vs_serial": (t_ser * 1e3 / pred) if t_ser else None,
            "ceiling_speedup": serial_model / (nt * tau_i + ch)}


def nl_model(inst, kern, kern_ser, t_pxp, t_ser, report, steps):
    """The iterative nonlinear direct's times against eq. nonLinSpeedup,
    per RK4 step of one slice or of the horizon: tau_I (the slices' Jacobians
    and the slices from zero, S steps per iteration), tau_H (the chain of
    slice exponentials, n_t - S steps of time per iteration), tau_F (the
    slices marched again from their corrected starts and the change check,
    S steps: the iterate at the stage points, a step the paper's sum
    formulation does not have), tau_D^S and tau_A^S (serial march and
    serial discrete adjoint, per step).  Predicted T_L = K (S tau_I +
    (n_t - S) tau_H + S tau_F) + the parallel adjoint as measured; the
    speedup condition of eq. speedupCond and the ceiling (N -> infinity)
    follow from eq. nonLinSpeedup with the adjoint's parallel cost split the
    same way (tau_I^dagger: the Magnus node states over a slice, tau_H^dagger:
    the Magnus chain per step)."""
    nt, Pa = int(inst["n_steps"]), int(inst["P"])
    P = int(inst.get("nl_slices", 0)) or Pa  # the iteration's slices
    S, Sa = nt // P, nt // Pa  # ... and the adjoint's Magnus steps
    if not report or not t_ser:
        return None
    K = sum(r["nl_iterations"] for r in report) / steps
    if K <= 0:
        return None
    sl = kern.get("slices", {}).get("per_step_ms", 0.0) / K
    ch = kern.get("krylov_direct", {}).get("per_step_ms", 0.0) / K
    fm = kern.get("nl_iter", {}).get("per_step_ms", 0.0) / K
    adj = sum(kern.get(k, {}).get("per_step_ms", 0.0)
              for k in ("ltv_adjoint", "ltv_nodes", "ltv_check", "serial_reverse"))
    tau_i, tau_h, tau_f = sl / S, ch / (nt - S), fm / S
    tau_ds = kern_ser.get("serial_direct", 0.0) / nt
    tau_as = kern_ser.get("serial_reverse", 0.0) / nt
    tau_ia = kern.get("ltv_nodes", {}).get("per_step_ms", 0.0) / Sa
    tau_ha = kern.get("ltv_adjoint", {}).get("per_step_ms", 0.0) / (nt - Sa)
    pred = K * (S * tau_i + (nt - S) * tau_h + S * tau_f) + adj
    # s > 1 iff N (tau_D^S + tau_A^S - K tau_H - tau_H^dagger)
    #           > K (tau_I + tau_F - tau_H) + tau_I^dagger - tau_H^dagger
    den = tau_ds + tau_as - K * tau_h - tau_ha
    num = K * (tau_i + tau_f - tau_h) + tau_ia - tau_ha
    return {"iterations": K, "slices": P, "adjoint_slices": Pa,
            "per_iteration_ms": {"jacobians_and_slices": sl, "chain": ch,
                                 "iterate_and_change": fm},
            "adjoint_ms": adj, "serial_direct_ms": kern_ser.get("serial_direct"),
            "serial_adjoint_ms": kern_ser.get("serial_reverse"),
            "tau_us_per_step": {"I": tau_i * 1e3, "H": tau_h * 1e3, "F": tau_f * 1e3,
                                "D_serial": tau_ds * 1e3, "A_serial": tau_as * 1e3,
                                "I_adj": tau_ia * 1e3, "H_adj": tau_ha * 1e3},
            "predicted_ms": pred, "measured_ms": t_pxp * 1e3,
            "speedup_vs_serial": t_ser / t_pxp,
            "min_slices_for_speedup": (num / den) if den > 0 else None,
            "ceiling_speedup": (tau_ds + tau_as) / (K * tau_h + tau_ha)}


def summary_report(report):
    """Per-instance report condensed to ranges."""
    if not report:
        return None
    keys = ("substeps", "iterations")
    return dict(krylov_direct=sorted({str(r["krylov_direct"]) for r in report}),
                krylov_adjoint=sorted({str(r["krylov_adjoint"]) for r in report}),
                P=sorted({r["P"] for r in report}),
                **{k: [min(r[k] for r in report), max(r[k] for r in report)] for k in keys},
                max_est=max(r["max_est"] for r in report))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--warmup-seconds", type=float, default=2.0,
                    help="keep warming up (untimed gradients) for at least this long, so "
                         "the timed region runs at steady-state clocks")
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--krylov", default="auto",
                    choices=["poly", "shift_invert", "auto", "taylor", "uniform", "chebyshev"])
    ap.add_argument("--sched", default=None, choices=["classic", "chain", "tree"],
                    help="schedule of the direct pieces (default: tree in 2D, classic in 1D)")
    ap.add_argument("--serial-steps", type=int, default=5,
                    help="timed serial-method gradients (0: none, for profiler runs)")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32_bulk"])
    ap.add_argument("--tol", type=float, default=None)
    ap.add_argument("--block", type=int, default=0,
                    help="threads per workgroup of the 1D RK4 marches (0 = default)")
    ap.add_argument("--kblock", type=int, default=0,
                    help="threads per workgroup of the 1D Krylov kernels (0 = default)")
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
    ap.add_argument("--hyb-slices", type=int, default=None,
                    help="Burgers integral cost: adjoint slices of the hybrid scheme")
    ap.add_argument("--hyb-k", type=float, default=None,
                    help="Burgers integral cost: k of eq. nonEquiP (0 = equal slices)")
    ap.add_argument("--hyb-group", type=int, default=None,
                    help="Burgers integral cost: adjoint slices per launch")
    ap.add_argument("--nl-iters", type=int, default=None,
                    help="iterative nonlinear direct: most iterations")
    ap.add_argument("--nl-tol", type=float, default=None,
                    help="iterative nonlinear direct: change of q(T) that ends it")
    ap.add_argument("--nl-slices", type=int, default=None,
                    help="iterative nonlinear direct: slices of the iteration")
    ap.add_argument("--slices", type=int, default=None,
                    help="override the workload's slice count P")
    ap.add_argument("--pick", default="",
                    help="comma-separated instance indices of the workload to run "
                         "(e.g. one diffusivity of advdiff2d_icost)")
    ap.add_argument("--instances", type=int, default=0,
                    help="use only the first K instances of a batch workload (0 = all)")
    ap.add_argument("--oracle-budget", type=float, default=2.5e8,
                    help="point-steps of the oracle accuracy sample for batch workloads")
    ap.add_argument("--oracle-threads", type=int, default=16,
                    help="oracle instances run at once (at most the usable host cores)")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the secondary 1D N=4096 measurement")
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

    m = measure(args, args.workload, torch, _lib, api, workloads, args.steps,
                args.serial_steps, not args.no_oracle, not args.no_cpu_baseline)
    insts, B = m["insts"], m["B"]
    inst = insts[0]
    cfg = {"workload": args.workload, "instances": B,
           "N": sorted({int(x["nx"]) * int(x.get("ny", 1)) for x in insts}),
           "grid": sorted({"%dx%d" % (x["nx"], x.get("ny", 1)) for x in insts}),
           "T": [min(x["T"] for x in insts), max(x["T"] for x in insts)],
           "n_steps": [min(int(x["n_steps"]) for x in insts),
                       max(int(x["n_steps"]) for x in insts)],
           "slices": m["P"],
           "krylov": args.krylov, "schedule": m["sched"], "precision": args.prec,
           "gate": m["gate"], "controls": int(np.asarray(inst["basis"]).shape[0]),
           "adjoint_form": "absorbed" if args.absorbed else "unabsorbed",
           "point_steps": sum(m["work"])}
    if m["tuned"] is not None:
        cfg["autotune"] = m["tuned"]
    if inst.get("cost") == "integral":
        cfg["cost"] = "integral"
        if inst["op"] == "burgers1d":
            cfg["hybrid"] = {"adjoint_slices": int(inst.get("hyb_slices", 0)) or int(inst["P"]),
                             "k": float(inst.get("hyb_k", 0.0)),
                             "group": int(inst.get("hyb_group", 0)) or 4}
    line = {
        "metric": METRIC,
        "value": (B / m["t_pxp"]) if m["ok"] else 0.0,
        "unit": "gradient evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["t_pxp"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": cfg,
        "serial_gpu": ({"value": B / m["t_ser"], "ms_per_step": m["t_ser"] * 1e3}
                       if m["t_ser"] else None),
        "speedup_vs_serial": m["t_ser"] / m["t_pxp"] if m["t_ser"] else None,
        "rel_err_vs_oracle": m["err"],
        "oracle_sample": m["sample"],
        "krylov_counters_per_step": {"direct": m["counters"][0], "adjoint": m["counters"][1],
                                     "fields": ["substeps", "iterations or terms",
                                                "second Gram-Schmidt passes"],
                                     "max_est": m["est"], "status": m["code"]},
        "instance_report": summary_report(m["report"]),
        "kernels_ms": {k: v["avg_ms"] for k, v in m["kern"].items()},
        "roofline": m["roof"],
        "roofline_classes": m["roof_all"],
    }
    if m["t_graph"] is not None:
        line["graph"] = {"value": B / m["t_graph"], "ms_per_step": m["t_graph"] * 1e3}
    if inst["op"] == "burgers1d" and inst.get("cost") == "integral" and B == 1:
        line["hybrid_model"] = hybrid_model(inst, m["kern"], m["t_ser"])
    if inst.get("nl_paraexp") and B == 1:
        cfg["direct"] = "iterative nonlinear Paraexp (at most %d iterations)" % int(
            inst.get("nl_iters", 8))
        line["nl_model"] = nl_model(inst, m["kern"], m["kern_ser"], m["t_pxp"], m["t_ser"],
                                    m["report"], m["steps"])
    if m["orc"] is not None and not args.no_cpu_baseline:
        o = m["orc"]
        work = m["work"]
        # the whole batch at the sample's measured rates
        t_par = o["wall"] * sum(work) / o["point_steps"]
        t_one = o["cpu"] * sum(work) / o["point_steps"]
        line["cpu_baseline"] = {
            "value": B / t_par, "unit": "gradient evals/s", "cores": o["threads"],
            "kind": "oracle",
            "single_core_value": B / t_one,
            "host": o["host"],
            "sample": ("full gradients (serial FP64 RK4 + exact discrete adjoint) of "
                       "instances %s, %.3g of %.3g point-steps, run %d at a time: %.1f s "
                       "wall, %.1f s summed over instances; scaled by point-steps to the "
                       "%d-instance batch" % (m["sample"], o["point_steps"], sum(work),
                                              o["threads"], o["wall"], o["cpu"], B))}
    if not args.no_secondary and args.workload == DEFAULT_WORKLOAD:
        s = measure(args, SECONDARY_WORKLOAD, torch, _lib, api, workloads,
                    max(5, args.steps // 2), 2, not args.no_oracle, False)
        line["secondary"] = {
            "workload": SECONDARY_WORKLOAD, "value": (s["B"] / s["t_pxp"]) if s["ok"] else 0.0,
            "ms_per_step": s["t_pxp"] * 1e3, "serial_ms_per_step": s["t_ser"] * 1e3,
            "speedup_vs_serial": s["t_ser"] / s["t_pxp"], "rel_err_vs_oracle": s["err"],
            "kernels_ms": {k: v["avg_ms"] for k, v in s["kern"].items()},
            "roofline": s["roof"], "instance_report": summary_report(s["report"])}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
