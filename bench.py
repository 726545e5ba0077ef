#!/usr/bin/env python3
"""Benchmark of the butterfly manifold harmonic transform apply on one MI355X.

One step = one FP32 synthesis f = Phi~ c plus one FP32 analysis g = Phi~^T f
on a block of nrhs right-hand sides, inputs resident in HBM.  The metric is
RHS*points per second over both directions: 2 * n * nrhs / seconds_per_step.
The same inputs are also run through the plain FP64 GPU apply for the speedup
figure.  The workload is the nonuniform periodic square: 65536 i.i.d. points,
16384 real Fourier modes, leaf 128 (L = 9), ID tolerance 1e-8, 64 RHS with
coefficients N(0,1) / (1 + |k|^2).  Factors are built on the host in FP64
before timing (not timed).

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"f64": ("mfma", 78.6, "TFLOP/s"), "f32": ("mfma", 157.3, "TFLOP/s")}
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_memory():
    """Resident size of this process and the host memory still available, GB."""
    try:
        import psutil
        return {"rss_GB": round(psutil.Process().memory_info().rss / 1e9, 1),
                "avail_GB": round(psutil.virtual_memory().available / 1e9, 1)}
    except Exception:
        return {}


def _counter_record(workload):
    """The committed rocprofv3 counter summary of a workload
    (profiles/hbm_traffic_<workload>.json), or None when it is missing or any
    source it lists (the kernels and the host code that lays out their work)
    has changed since its counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_%s.json" % workload)
    try:
        with open(path) as f:
            d = json.load(f)
        src = d.get("sources_sha1") or {}
        for rel, sha in src.items():
            with open(os.path.join(ROOT, rel), "rb") as f:
                if hashlib.sha1(f.read()).hexdigest() != sha:
                    return None
    except (OSError, ValueError):
        return None
    return d if src else None


def measured_traffic(workload, part="fwd", per="launch"):
    """HBM bytes per stage launch (or per apply) of one measured part (e.g. the
    forward FP32 apply): FETCH_SIZE and WRITE_SIZE scaled by what the same
    counters read for a plain copy of known size.  None without a current record."""
    d = _counter_record(workload)
    if not d or part not in d:
        return None
    return d[part]["hbm_bytes_per_launch" if per == "launch" else "hbm_bytes_per_apply"]


def measured_mfma_busy(workload, part="fwd"):
    """MfmaUtil (matrix-core busy percent, duration-weighted over the part's
    stage launches) from the same record, or None."""
    d = _counter_record(workload)
    if not d or part + "_mfma" not in d:
        return None
    return d[part + "_mfma"]["mfma_busy_pct"]


# MI355X spec-sheet peaks: dense MFMA TFLOP/s per arithmetic type and HBM GB/s.
MFMA_PEAK = {"f64": 78.6, "f32": 157.3, "bf16x2": 2500.0, "bf16x3": 2500.0}
HBM_PEAK = 8000.0
SPLIT_PRODUCTS = {"f64": 1, "f32": 1, "bf16x2": 3, "bf16x3": 6}
# factor bytes streamed per stored entry: the split precisions keep FP32 factors and split them on load
FACTOR_BYTES = {"f64": 8, "f32": 4, "bf16x2": 4, "bf16x3": 4}


def roofline_for(prec, F, n, m, b, apply_ms, launches):
    """Roofline of one apply: the binding one of the MFMA time (executed flops,
    split products counted, at the type's peak) and the HBM time (algorithmic
    bytes: stored factors plus inputs and outputs).  `achieved` is that
    quantity per launch over the average launch duration.  F is the number of
    factor entries the timed apply reads (the forward pool keeps only T of the
    compact ID blocks)."""
    io = (8 if prec == "f64" else 4) * (n + m) * b
    alg_bytes = FACTOR_BYTES[prec] * F + io
    exec_flops = 2.0 * F * b * SPLIT_PRODUCTS[prec]
    t_mfma = exec_flops / (MFMA_PEAK[prec] * 1e12)
    t_hbm = alg_bytes / (HBM_PEAK * 1e9)
    t = apply_ms * 1e-3
    if t_mfma >= t_hbm:
        r = {"bound": "mfma", "achieved": exec_flops / t / 1e12, "peak": MFMA_PEAK[prec], "unit": "TFLOP/s",
             "per_launch_flops": exec_flops / launches, "flops_counted": "2 F b x split products"}
    else:
        r = {"bound": "hbm", "achieved": alg_bytes / t / 1e9, "peak": HBM_PEAK, "unit": "GB/s",
             "per_launch_alg_bytes": alg_bytes / launches}
    r["frac"] = r["achieved"] / r["peak"]
    r["traffic"] = None
    r["avg_launch_ms"] = apply_ms / launches
    r["t_roof_ms"] = max(t_mfma, t_hbm) * 1e3
    return r


def folded_levels(fs):
    """Leading all-identity levels, which the forward apply folds into its first
    stage (no launch of their own)."""
    ident, L = np.asarray(fs["ident"]), int(fs["L"])
    k = 0
    while k <= L and ident[k].all():
        k += 1
    return k


def level_bytes(fs, b, s_x, merged=False):
    """Implementation bytes of one forward apply: every level vector it writes
    (sum of the ranks of a level, b columns; folded levels have none, and a plan
    that merges the leaf bases into the last level does not form y_L) written
    once and read once."""
    rank = np.asarray(fs["rank"], dtype=np.int64)
    last = int(fs["L"]) if merged else int(fs["L"]) + 1
    return 2.0 * float(rank[folded_levels(fs):last].sum()) * b * s_x


def stage_launches(plan, fs):
    """Stage launches of one apply in either direction: the plan's stages (L + 2,
    or L + 1 with merged leaf blocks) less the folded identity levels (the
    transposed apply sums their copies in one gather-sum launch instead)."""
    from paper_2605_21828_amd import bfmht as B
    return B.bfmht_plan_num_stages(plan.handle) - folded_levels(fs)


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return int(max([d.get("num_threads", 1) for d in threadpool_info()] or [1]))
    except Exception:
        return int(os.cpu_count() or 1)


def event_time(fn, reps, torch):
    """Average milliseconds of fn() over reps, measured with HIP events on the current stream."""
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    e.synchronize()
    return s.elapsed_time(e) / reps


def cpu_baseline(fs, pts, c_host, f_host, out32, g32, rows, cols, lam, variant_outputs=None):
    """The oracle as it stands, timed on the host cores, plus the accuracy check.

    Times the oracle's butterfly apply and its transpose (O2, NumPy) on a
    bounded sample of whole passes over the same factors and RHS; reports
    RHS*points/s over both directions.  Then measures the GPU FP32 results
    (and any precision variant's) against the dense FP64 transform (O1) on
    sampled rows and columns.
    """
    from oracle import butterfly as ob
    from oracle import dense as od
    from oracle import modes as om
    cores = _blas_threads()
    # Bounded sample: whole passes over all RHS until about 10 s of host work.
    b_s = c_host.shape[1]
    t0 = time.time()
    passes = 0
    while passes == 0 or (time.time() - t0 < 10.0 and passes < 16):
        ob.apply(fs, c_host[:, :b_s])
        ob.apply_transpose(fs, f_host[:, :b_s])
        passes += 1
    dt = time.time() - t0
    n = int(fs["n"])
    md = om.fourier_modes(int(fs["m"]))
    ref_f = od.fourier_synthesis_rows(pts, md, rows, c_host)
    ref_g = od.fourier_analysis_cols(pts, md, cols, f_host)
    err_f = od.rel_err_cols(out32[rows], ref_f)[0]
    err_g = od.rel_err_cols(g32[cols], ref_g)[0]
    base = {"value": 2.0 * n * b_s * passes / dt, "unit": "RHS*points/s", "cores": int(cores), "kind": "oracle",
            "sample": "oracle butterfly apply + transpose (NumPy FP64) of the same factors, %d pass(es) over all %d "
                      "RHS, %.1f s" % (passes, b_s, dt)}
    acc = {"synthesis_rows_sampled": len(rows), "synthesis_rel_err": err_f,
           "analysis_cols_sampled": len(cols), "analysis_rel_err": err_g}
    for prec, (yv, gv) in (variant_outputs or {}).items():
        acc["%s_synthesis_rel_err" % prec] = od.rel_err_cols(yv[rows], ref_f)[0]
        acc["%s_analysis_rel_err" % prec] = od.rel_err_cols(gv[cols], ref_g)[0]
    return base, acc


def dense_context(pts, modes, c32, f32, reps, torch):
    """Context only: the same products with the dense transform matrix formed on
    the GPU (closed-form Fourier entries) and multiplied by the vendor GEMM
    (torch.matmul: rocBLAS / hipBLASLt), FP64 and FP32, both directions.  Not a
    path of this library; it shows what the butterfly saves at this size."""
    dev = c32.device
    x = torch.tensor(pts, dtype=torch.float64, device=dev)
    md = torch.tensor(modes, dtype=torch.int64, device=dev)
    kmax = int(md[:, :2].max())
    k = torch.arange(kmax + 1, dtype=torch.float64, device=dev)
    tabs = []
    for a in range(2):
        arg = x[:, a:a + 1] * k[None, :]
        tabs.append(torch.stack([torch.cos(arg), torch.sin(arg)], dim=2).reshape(x.shape[0], -1))
    Phi = tabs[0][:, 2 * md[:, 0] + md[:, 2]] * tabs[1][:, 2 * md[:, 1] + md[:, 3]]
    del tabs
    out = {"dense_GB_fp64": Phi.numel() * 8 / 1e9}
    for name, dt in (("f64", torch.float64), ("f32", torch.float32)):
        A = Phi if dt == torch.float64 else Phi.float()
        c, f = c32.to(dt), f32.to(dt)
        ft = f.t().contiguous()
        A @ c
        torch.matmul(ft, A)
        out[name + "_apply_ms"] = event_time(lambda: A @ c, reps, torch)
        out[name + "_apply_transpose_ms"] = event_time(lambda: torch.matmul(ft, A), reps, torch)
        del A, c, f, ft
    del Phi
    torch.cuda.empty_cache()
    out["note"] = "dense Phi formed on the GPU, vendor GEMM via torch.matmul; context only, not this library"
    return out


def bench_batched(args):
    """Multi-instance workload: 32 uniform-grid instances of uneven size, FP32."""
    import torch

    from paper_2605_21828_amd import workloads as wl
    from paper_2605_21828_amd.autotune import tune_batch
    from paper_2605_21828_amd.bfmht import Batch, Plan
    from paper_2605_21828_amd.factor import io as fio

    spec = wl.BATCHED
    inst = wl.batched_instances(spec)
    dev = torch.device("cuda:0")
    built = {}
    for side in sorted({s for s, _ in inst}):
        n = side * side
        log("building factors: grid side %d (n=%d, m=%d)" % (side, n, n // 4))
        built[side] = fio.fourier_factors(wl.grid_points(side), n // 4, spec["leaf"], spec["tol"],
                                          workers=args.workers, cache=args.cache)[0]
    by_side = {side: Plan(fs, "f32", max_nrhs=spec["max_nrhs"], device=dev) for side, fs in built.items()}
    plans, xs, fvs, cs_host = [], [], [], []
    for i, (side, b) in enumerate(inst):
        p = by_side[side]   # instances of one side share one uploaded factor set
        c = wl.coefficients(spec["wid"] * 100 + i, p.m, b)
        cs_host.append(c)
        plans.append(p)
        xs.append(torch.tensor(c, dtype=torch.float32, device=dev))
        fvs.append(torch.tensor(wl.values(spec["wid"] * 100 + i, p.n, b), dtype=torch.float32, device=dev))
    batch = Batch(plans)
    outs = [torch.empty((p.n, x.shape[1]), dtype=torch.float32, device=dev) for p, x in zip(plans, xs)]
    outs_t = [torch.empty((p.m, x.shape[1]), dtype=torch.float32, device=dev) for p, x in zip(plans, xs)]
    tune_batch(batch, xs, transpose=False, log=log)
    tune_batch(batch, fvs, transpose=True, log=log)

    def step():
        batch.launch(xs, outs, False)
        batch.launch(fvs, outs_t, True)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    reps = max(args.steps, 5)
    ms_fwd = event_time(lambda: batch.launch(xs, outs, False), reps, torch)

    def one_by_one():
        for p, x, y in zip(plans, xs, outs):
            p.apply(x, out=y)
    ms_seq = event_time(one_by_one, reps, torch)
    rhs_points = sum(p.n * int(x.shape[1]) for p, x in zip(plans, xs))
    # roofline of the batch: each instance at its own bound (small RHS counts are
    # HBM-bound, large ones MFMA-bound), summed over the instances
    t_mfma = t_hbm = t_roof = 0.0
    for s, b in inst:
        Fi = by_side[s].stored_fwd   # forward pool entries (compact ID blocks)
        n_i = s * s
        tm = 2.0 * Fi * b / (MFMA_PEAK["f32"] * 1e12)
        th = (4.0 * Fi + 4.0 * (n_i + n_i // 4) * b) / (HBM_PEAK * 1e9)
        t_roof += max(tm, th)
        if tm >= th:
            t_mfma += tm
        else:
            t_hbm += th
    frac = t_roof / (ms_fwd * 1e-3)
    bound = "mfma" if t_mfma >= t_hbm else "hbm"
    peak = MFMA_PEAK["f32"] if bound == "mfma" else HBM_PEAK
    errs, base = None, None
    if not args.no_cpu_baseline:
        from oracle import butterfly as ob
        from oracle import dense as od
        from oracle import modes as om
        errs = []
        torch.cuda.synchronize()
        for (side, b), y, c in zip(inst, outs, cs_host):
            ref = om.grid_synthesis_ifft2(side, om.fourier_modes(side * side // 4), c)
            errs.append(od.rel_err_cols(y.double().cpu().numpy(), ref)[0])
        # the oracle's butterfly apply + transpose of every instance, whole
        # passes over the batch, bounded to about 15 s of host work
        fvs_host = [fv.double().cpu().numpy() for fv in fvs]
        t0 = time.time()
        passes = done = 0
        while passes == 0 or (time.time() - t0 < 15.0 and passes < 8):
            for (side, b), c, fv in zip(inst, cs_host, fvs_host):
                ob.apply(built[side], c)
                ob.apply_transpose(built[side], fv)
                done += side * side * b
            passes += 1
        dt_cpu = time.time() - t0
        base = {"value": 2.0 * done / dt_cpu, "unit": "RHS*points/s", "cores": _blas_threads(), "kind": "oracle",
                "sample": "oracle butterfly apply + transpose (NumPy FP64) of every instance's factors and RHS, "
                          "%d pass(es) over the 32 instances, %.1f s" % (passes, dt_cpu)}
    res = {
        "metric": "butterfly apply RHS*points/s (FP32 batched synthesis + analysis)",
        "value": 2.0 * rhs_points / (ms * 1e-3), "unit": "RHS*points/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched32", "instances": [[s, b] for s, b in inst], "m": "n/4",
                   "leaf": spec["leaf"], "tol": spec["tol"], "step": "batched apply + batched apply_transpose"},
        "roofline": {"bound": bound, "achieved": frac * peak, "peak": peak,
                     "unit": "TFLOP/s" if bound == "mfma" else "GB/s", "frac": frac,
                     "traffic": measured_traffic("batched32", "fwd"), "traffic_unit": "bytes per stage launch",
                     "t_roof_ms": t_roof * 1e3, "t_roof_mfma_bound_ms": t_mfma * 1e3,
                     "t_roof_hbm_bound_ms": t_hbm * 1e3,
                     "note": "sum over instances of max(HBM time, MFMA time); achieved = frac x peak of the "
                             "dominant bound; traffic: counter bytes per stage launch of one batched forward call",
                     "traffic_per_batched_apply": measured_traffic("batched32", "fwd", per="apply"),
                     "mfma_busy_pct_counter": measured_mfma_busy("batched32", "fwd"),
                     "kernel": "batched_stage_kernel<1> (all launches of one batched FP32 apply)"},
        "cpu_baseline": base,
        "extra": {"batched_apply_ms": ms_fwd, "one_by_one_apply_ms": ms_seq,
                  "batching_speedup": ms_seq / ms_fwd,
                  "max_instance_rel_err_vs_inverse_dft":
                  max(errs) if errs else None, "instance_rel_err": errs},
    }
    print(json.dumps(res), flush=True)


def bench_sphere(args):
    """Perturbed-sphere workload: BF16 split applies with 256 RHS (FP32 and FP64 beside them)."""
    import torch

    from paper_2605_21828_amd import workloads as wl
    from paper_2605_21828_amd.bfmht import Plan
    from paper_2605_21828_amd.factor import io as fio

    spec = wl.SPHERE
    log("building sphere problem and factors: level %d, m=%d" % (spec["level"], spec["m"]))
    fs, prob = fio.sphere_factors(spec["level"], spec["wid"], spec["m"], spec["leaf"], spec["tol"],
                                  workers=args.workers, log=lambda s: log("  ", s), cache=args.cache)
    Phi = prob["Phi"]
    n, m, b = Phi.shape[0], Phi.shape[1], spec["nrhs"]
    F = fio.stored_entries(fs)
    c = wl.coefficients(spec["wid"], m, b)
    fv = wl.values(spec["wid"], n, b)
    dev = torch.device("cuda:0")
    main = args.precision or "bf16x3"
    rec = {}
    outs = {}
    for prec in [main] + [p for p in ("bf16x3", "bf16x2", "f32", "f64") if p != main]:
        dt = torch.float64 if prec == "f64" else torch.float32
        p = Plan(fs, prec, max_nrhs=b, device=dev)
        ct, ft = torch.tensor(c, dtype=dt, device=dev), torch.tensor(fv, dtype=dt, device=dev)
        y = torch.empty((n, b), dtype=dt, device=dev)
        g = torch.empty((m, b), dtype=dt, device=dev)
        shapes = None
        if not args.no_tune:
            from paper_2605_21828_amd.autotune import tune_plan
            shapes = tune_plan(p, fs, b, use_cache=args.cache, log=log)

        def step():
            p.apply(ct, out=y)
            p.apply_t(ft, out=g)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        reps = max(args.steps, 5)
        t_f = event_time(lambda: p.apply(ct, out=y), reps, torch)
        t_b = event_time(lambda: p.apply_t(ft, out=g), reps, torch)
        outs[prec] = (y.double().cpu().numpy(), g.double().cpu().numpy())
        rec[prec] = {"ms_per_step": ms, "apply_ms": t_f, "apply_transpose_ms": t_b, "tile_shapes": shapes,
                     "forward_factor_entries": p.stored_fwd, "stage_launches": stage_launches(p, fs),
                     "leaf_merged": p.leaf_merged}
        log("%s step %.3f ms" % (prec, ms))
        del p, ct, ft, y, g
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        from oracle import butterfly as ob
        from oracle import dense as od
        t0 = time.time()
        passes = 0
        while passes == 0 or (time.time() - t0 < 10.0 and passes < 16):
            ob.apply(fs, c)
            ob.apply_transpose(fs, fv)
            passes += 1
        dt_cpu = time.time() - t0
        ref_y, ref_g = Phi @ c, Phi.T @ fv
        for prec, (y, g) in outs.items():
            rec[prec]["synthesis_rel_err_vs_dense_fp64"] = od.rel_err_cols(y, ref_y)[0]
            rec[prec]["analysis_rel_err_vs_dense_fp64"] = od.rel_err_cols(g, ref_g)[0]
        base = {"value": 2.0 * n * b * passes / dt_cpu, "unit": "RHS*points/s", "cores": _blas_threads(),
                "kind": "oracle",
                "sample": "oracle butterfly apply + transpose (NumPy FP64) of the same factors, %d pass(es) over "
                          "all %d RHS, %.1f s" % (passes, b, dt_cpu)}
    else:
        base = None
    t_main = rec[main]["apply_ms"]
    launches = rec[main]["stage_launches"]
    roof = roofline_for(main, rec[main]["forward_factor_entries"], n, m, b, t_main, launches=launches)
    part = "fwd" if main == "bf16x3" else main + "_fwd"   # the counter record's headline part is BF16X3
    roof["traffic"] = measured_traffic("sphere40962", part)
    roof["traffic_unit"] = "bytes per launch"
    roof["mfma_busy_pct_counter"] = measured_mfma_busy("sphere40962", part)
    roof["level_vector_bytes_per_launch"] = level_bytes(fs, b, 4, rec[main]["leaf_merged"]) / launches
    res = {
        "metric": "butterfly apply RHS*points/s (%s synthesis + analysis)" % main,
        "value": 2.0 * n * b / (rec[main]["ms_per_step"] * 1e-3), "unit": "RHS*points/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": rec[main]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": main, "data": "synthetic",
        "config": {"workload": "sphere40962", "n": n, "m": m, "nrhs": b, "leaf": spec["leaf"], "tol": spec["tol"],
                   "L": int(fs["L"]), "step": "apply + apply_transpose"},
        "roofline": roof,
        "cpu_baseline": base,
        "extra": {"stored_factor_entries": F, "compression_vs_dense": n * m / F, "precisions": rec},
    }
    print(json.dumps(res), flush=True)


def lsq_checks(fs, pts, c_np, f, grad_np, lam_rows):
    """Oracle leg of the least-squares workload: the autograd gradient at c
    against central differences of the oracle's FP64 butterfly loss on 64
    coordinates and against the dense FP64 2 Phi^T (Phi c - f) of the exact
    transform on 256 sampled columns; also times the oracle's apply pair."""
    from oracle import butterfly as ob
    from oracle import dense as od
    from oracle import modes as om
    md_oracle = om.fourier_modes(int(fs["m"]))
    coords = lam_rows["fd"]
    cols = lam_rows["cols"]
    h = 1.0
    t0 = time.time()
    E = np.zeros((c_np.size, len(coords)))
    E[coords, np.arange(len(coords))] = h
    Yp = ob.apply(fs, c_np[:, None] + E)
    Ym = ob.apply(fs, c_np[:, None] - E)
    fd = (np.sum((Yp - f[:, None]) ** 2, axis=0) - np.sum((Ym - f[:, None]) ** 2, axis=0)) / (2 * h)
    t_fd = time.time() - t0
    fd_err = float(np.linalg.norm(grad_np[coords] - fd) / np.linalg.norm(fd))
    t1 = time.time()
    r = od.fourier_synthesis_all(pts, md_oracle, c_np) - f
    dense = 2.0 * od.fourier_analysis_cols(pts, md_oracle, cols, r)
    dense_err = float(np.linalg.norm(grad_np[cols] - dense) / np.linalg.norm(dense))
    t_dense = time.time() - t1
    # oracle timing: apply + transpose pairs at b = 1, about 10 s of host work
    t2 = time.time()
    passes = 0
    while passes == 0 or (time.time() - t2 < 10.0 and passes < 32):
        ob.apply(fs, c_np[:, None])
        ob.apply_transpose(fs, f[:, None])
        passes += 1
    t_pair = time.time() - t2
    base = {"value": 2.0 * int(fs["n"]) * passes / t_pair, "unit": "RHS*points/s", "cores": _blas_threads(),
            "kind": "oracle",
            "sample": "oracle butterfly apply + transpose (NumPy FP64) of the same factors, one RHS, %d pass(es), "
                      "%.1f s" % (passes, t_pair)}
    return base, {"gradient_check_point": "random N(0,1) coefficients",
                  "fd_coordinates": len(coords), "fd_rel_err": fd_err, "fd_seconds": t_fd,
                  "dense_cols_sampled": len(cols), "dense_grad_rel_err": dense_err, "dense_seconds": t_dense}


def bench_lsq(args):
    """Differentiable least-squares fit: 262144 i.i.d. points, 65536 modes, FP32 autograd, 100 GD steps."""
    import torch

    from paper_2605_21828_amd import workloads as wl
    from paper_2605_21828_amd.autograd import least_squares_step
    from paper_2605_21828_amd.bfmht import Plan
    from paper_2605_21828_amd.factor import io as fio
    from paper_2605_21828_amd.factor.fourier import FourierBlocks, real_modes

    w = wl.WORKLOADS["iid" + args.workload[len("lsq"):]]
    n, m, wid = w["n"], w["m"], w["wid"]
    pts = wl.points_for(w)
    log("building factors: n=%d m=%d leaf=%d tol=%g workers=%d" % (n, m, w["leaf"], w["tol"], args.workers),
        host_memory())
    t0 = time.time()
    fs, _ = fio.fourier_factors(pts, m, w["leaf"], w["tol"], workers=args.workers, cache=args.cache,
                                log=lambda s: log("  factor", s, host_memory()), device=_build_device(args))
    t_build = time.time() - t0
    F = fio.stored_entries(fs)
    modes = real_modes(m)
    lam = (modes[:, 0] ** 2 + modes[:, 1] ** 2).astype(np.float64)
    c_star = wl.coefficients(wid, m, 1, lam=lam, kind="decay")[:, 0]
    log("exact right-hand side f = Phi c* + 1e-3 noise")
    f = FourierBlocks(pts, modes).synthesis(c_star) + 1e-3 * wl.values(wid, n, 1)[:, 0]
    dev = torch.device("cuda:0")
    log("uploading FP32 plan (%d stored entries)" % F, host_memory())
    t_plan = time.time()
    plan = Plan(fs, "f32", max_nrhs=1, device=dev)
    t_plan = time.time() - t_plan
    log("plan created and uploaded in %.1f s" % t_plan, host_memory())
    ft = torch.tensor(f, dtype=torch.float32, device=dev)
    # step size 0.5 / sigma_max^2, sigma_max^2 from 20 power iterations on Phi~^T Phi~
    v = torch.tensor(wl.coefficients(wid, m, 1, stream=5)[:, 0], dtype=torch.float32, device=dev)
    for _ in range(20):
        v = plan.apply_t(plan.apply(v))
        s2 = torch.linalg.norm(v)
        v = v / s2
    lr = 0.5 / float(s2)
    c = torch.zeros(m, dtype=torch.float32, device=dev)
    for _ in range(args.warmup):
        least_squares_step(plan, c, ft, lr)
    torch.cuda.synchronize()
    losses = []
    t1 = time.perf_counter()
    for _ in range(args.steps):
        c, loss = least_squares_step(plan, c, ft, lr)
        losses.append(loss)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t1) * 1e3 / args.steps
    losses = [float(x) for x in losses]
    log("gd step %.3f ms, loss %.4g -> %.4g" % (ms, losses[0], losses[-1]))
    # gradient through autograd at a generic point (random N(0,1) coefficients):
    # near the minimiser the residual is tiny and FP32 cancellation, not the
    # transform, would decide the comparison
    c_chk = torch.tensor(wl.coefficients(wid, m, 1, stream=5)[:, 0], dtype=torch.float32, device=dev)
    cg = c_chk.detach().requires_grad_(True)
    from paper_2605_21828_amd.autograd import BFApply
    r = BFApply.apply(cg, plan) - ft
    (r * r).sum().backward()
    grad_np = cg.grad.double().cpu().numpy()
    c_np = c_chk.double().cpu().numpy()
    reps = 5
    ms_fwd = event_time(lambda: plan.apply(c), reps, torch)
    ms_bwd = event_time(lambda: plan.apply_t(ft), reps, torch)
    roof = roofline_for("f32", plan.stored_fwd, n, m, 1, ms_fwd, launches=stage_launches(plan, fs))
    roof["traffic"] = measured_traffic(w_key := "iid" + args.workload[len("lsq"):], "fwd")
    roof["traffic_unit"] = "bytes per launch"
    roof["traffic_transposed"] = measured_traffic(w_key, "bwd")
    base, acc = None, {}
    if not args.no_cpu_baseline:
        log("oracle checks: finite differences and dense gradient")
        sel = {"fd": wl.sample_indices(wid, m, 64, stream=4), "cols": wl.sample_indices(wid, m, 256, stream=3)}
        base, acc = lsq_checks(fs, pts, c_np, f, grad_np, sel)
    res = {
        "metric": "gradient-descent steps/s (FP32 autograd least squares: apply + transposed apply per step)",
        "value": 1e3 / ms, "unit": "steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m, "nrhs": 1, "leaf": w["leaf"], "tol": w["tol"],
                   "L": int(fs["L"]), "step": "forward apply + autograd backward (transposed apply) + update"},
        "roofline": roof,
        "cpu_baseline": base,
        "extra": {"stored_factor_entries": F, "compression_vs_dense": n * m / F, "factor_build_seconds": t_build,
                  "factor_build_on": "gpu" if args.device_build else "host (NumPy/SciPy, %d workers)" % args.workers,
                  "plan_create_upload_seconds": t_plan, "host_memory_at_end": host_memory(),
                  "fp32_apply_ms": ms_fwd, "fp32_apply_transpose_ms": ms_bwd, "step_size": lr,
                  "loss_first": losses[0], "loss_last": losses[-1],
                  "loss_monotone": all(b <= a * (1 + 1e-6) for a, b in zip(losses, losses[1:])), **acc},
    }
    print(json.dumps(res), flush=True)


def lsqr_checks(Phi, X, c):
    """Oracle leg of the inverse-transform workload: dense FP64 least squares of
    the same coordinates (and its time on the host cores)."""
    t0 = time.time()
    ref = np.linalg.lstsq(Phi, X, rcond=None)[0]
    dt = time.time() - t0
    from oracle import dense as od
    base = {"value": 1.0 / dt, "unit": "solves/s", "cores": _blas_threads(), "kind": "oracle",
            "sample": "dense FP64 least squares (numpy lstsq) of the %d coordinate columns, %.1f s" % (X.shape[1], dt)}
    return base, {"coef_rel_err_vs_dense_lstsq": od.rel_err_cols(c, ref)[0]}


def bench_inverse(args):
    """Inverse transform of the perturbed sphere's vertex coordinates by LSQR (Sec. 7.1)."""
    import torch

    from paper_2605_21828_amd import workloads as wl
    from paper_2605_21828_amd.bfmht import Plan
    from paper_2605_21828_amd.factor import io as fio

    spec = wl.SPHERE
    prec = args.precision or "f32"
    log("building sphere problem and factors: level %d, m=%d" % (spec["level"], spec["m"]))
    fs, prob = fio.sphere_factors(spec["level"], spec["wid"], spec["m"], spec["leaf"], spec["tol"],
                                  workers=args.workers, log=lambda s: log("  ", s), cache=args.cache)
    X = np.asarray(prob["v"], dtype=np.float64)
    n, m, b = X.shape[0], spec["m"], X.shape[1]
    F = fio.stored_entries(fs)
    dev = torch.device("cuda:0")
    dt = torch.float64 if prec == "f64" else torch.float32
    p = Plan(fs, prec, max_nrhs=b, device=dev)
    Xt = torch.tensor(X, dtype=dt, device=dev)
    iters = args.steps
    for _ in range(max(1, args.warmup)):
        p.lsqr(Xt, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c, rn = p.lsqr(Xt, iters)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    per_iter = ms / max(1, iters)
    c_np = c.double().cpu().numpy()
    # algorithmic bytes of one step: both applies' factor bytes (the forward one
    # reads the compact ID blocks) plus their inputs and outputs
    # stage launches of both applies, the input gather and copy sum, and the six vector kernels
    launches = 2 * stage_launches(p, fs) + 2 + 6
    step_bytes = (FACTOR_BYTES[prec] * (p.stored_fwd + p.stored_t)
                  + 2 * (8 if prec == "f64" else 4) * (n + m) * b)
    achieved = step_bytes / (per_iter * 1e-3) / 1e9
    base, acc = (None, {})
    if not args.no_cpu_baseline:
        base, acc = lsqr_checks(prob["Phi"], X, c_np)
    res = {
        "metric": "LSQR steps/s (inverse transform of the vertex coordinates, %s)" % prec,
        "value": 1e3 / per_iter, "unit": "steps/s",
        "n_gpus": 1, "steps": iters, "warmup": args.warmup, "ms_per_step": per_iter,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": prec, "data": "synthetic",
        "config": {"workload": "inverse_sphere40962", "n": n, "m": m, "nrhs": b, "leaf": spec["leaf"],
                   "tol": spec["tol"], "L": int(fs["L"]), "step": "one LSQR step: apply + apply_transpose + vector kernels"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK, "traffic": None, "avg_launch_ms": per_iter / launches,
                     "per_step_alg_bytes": step_bytes},
        "cpu_baseline": base,
        "extra": {"stored_factor_entries": F, "lsqr_steps": iters, "solve_ms": ms,
                  "residual_estimate": rn.double().cpu().numpy().tolist(), **acc},
    }
    print(json.dumps(res), flush=True)


def bench_latency(args):
    """Uniform 64 x 64 grid, 1024 modes, one RHS: a latency-bound apply whose
    factors stay in L2/MALL.  Times the FP64 (and FP32) synthesis and analysis
    eagerly and as HIP graph replays (torch CUDA graphs capture the library's
    kernel launches on the capturing stream), and checks FP64 against the oracle
    and the inverse DFT."""
    import torch

    from paper_2605_21828_amd import workloads as wl
    from paper_2605_21828_amd.bfmht import Plan
    from paper_2605_21828_amd.factor import io as fio

    w = wl.WORKLOADS["grid64"]
    pts = wl.points_for(w)
    fs, _ = fio.fourier_factors(pts, w["m"], w["leaf"], w["tol"], workers=args.workers, cache=args.cache)
    n, m, b = w["n"], w["m"], w["nrhs"]
    c_host = wl.coefficients(w["wid"], m, b)
    f_host = wl.values(w["wid"], n, b)
    dev = torch.device("cuda:0")
    reps = max(200, args.steps)
    rec, outs = {}, {}
    for prec in ("f64", "f32"):
        dt = torch.float64 if prec == "f64" else torch.float32
        p = Plan(fs, prec, max_nrhs=b, device=dev)
        x = torch.tensor(c_host, dtype=dt, device=dev)
        fv = torch.tensor(f_host, dtype=dt, device=dev)
        y = torch.empty((n, b), dtype=dt, device=dev)
        g = torch.empty((m, b), dtype=dt, device=dev)
        for _ in range(max(3, args.warmup)):
            p.apply(x, out=y)
            p.apply_t(fv, out=g)
        torch.cuda.synchronize()
        eager_f = event_time(lambda: p.apply(x, out=y), reps, torch)
        eager_b = event_time(lambda: p.apply_t(fv, out=g), reps, torch)
        graphs = []
        for fn in (lambda: p.apply(x, out=y), lambda: p.apply_t(fv, out=g)):
            gr = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gr):
                fn()
            graphs.append(gr)
        graph_f = event_time(graphs[0].replay, reps, torch)
        graph_b = event_time(graphs[1].replay, reps, torch)
        torch.cuda.synchronize()
        outs[prec] = (y.double().cpu().numpy(), g.double().cpu().numpy())
        rec[prec] = {"apply_us": eager_f * 1e3, "apply_transpose_us": eager_b * 1e3,
                     "graph_apply_us": graph_f * 1e3, "graph_apply_transpose_us": graph_b * 1e3}
        log("%s: apply %.1f us (graph %.1f), transpose %.1f us (graph %.1f)" % (
            prec, eager_f * 1e3, graph_f * 1e3, eager_b * 1e3, graph_b * 1e3))
    checks, base = None, None
    if not args.no_cpu_baseline:
        from oracle import butterfly as ob
        from oracle import dense as od
        from oracle import modes as om
        # the oracle's FP64 synthesis of the same factors and RHS, bounded to about 10 s
        t0 = time.time()
        passes = 0
        while passes == 0 or (time.time() - t0 < 10.0 and passes < 2000):
            ob.apply(fs, c_host)
            passes += 1
        us_cpu = (time.time() - t0) * 1e6 / passes
        base = {"value": us_cpu, "unit": "us", "cores": _blas_threads(), "kind": "oracle",
                "sample": "oracle butterfly synthesis (NumPy FP64) of the same factors and RHS, %d pass(es), %.1f s"
                          % (passes, us_cpu * passes * 1e-6)}
        md = om.fourier_modes(m)
        y64, g64 = outs["f64"]
        checks = {"f64_vs_oracle_butterfly": od.rel_err_cols(y64, ob.apply(fs, c_host))[0],
                  "f64_transpose_vs_oracle_butterfly": od.rel_err_cols(g64, ob.apply_transpose(fs, f_host))[0],
                  "f64_vs_inverse_dft": od.rel_err_cols(y64, om.grid_synthesis_ifft2(w["N"], md, c_host))[0],
                  "f32_vs_inverse_dft": od.rel_err_cols(outs["f32"][0], om.grid_synthesis_ifft2(w["N"], md, c_host))[0]}
    F = fio.stored_entries(fs)
    # the faster of eager launches and graph replay (graph replay measured slower here)
    t = min(rec["f64"]["apply_us"], rec["f64"]["graph_apply_us"])
    plan_f = Plan(fs, "f64", max_nrhs=b, device=dev)
    res = {
        "metric": "FP64 synthesis latency (one RHS)",
        "value": t, "unit": "us", "n_gpus": 1, "steps": reps, "warmup": args.warmup, "ms_per_step": t * 1e-3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "grid64", "n": n, "m": m, "nrhs": b, "leaf": w["leaf"], "tol": w["tol"],
                   "L": int(fs["L"]), "step": "one apply"},
        "roofline": dict(roofline_for("f64", plan_f.stored_fwd, n, m, b, t * 1e-3, launches=stage_launches(plan_f, fs)),
                         traffic=measured_traffic("grid64", "f64_fwd"), traffic_unit="bytes per launch",
                         note="latency-bound: the factors are L2/MALL-resident; reported, not a target"),
        "cpu_baseline": base,
        "extra": {"stored_factor_entries": F, "precisions": rec, "checks": checks},
    }
    print(json.dumps(res), flush=True)


def _qr_flops(fs):
    """Algorithmic flops of the column IDs of a factor set: a Householder QR
    stopped after k = rank steps costs sum_{j<k} 4 (M - j)(K - j) on an M x K
    block (the reflector's dot product and update of every remaining column);
    blocks without rows or columns cost nothing."""
    L, nb = int(fs["L"]), 2 ** int(fs["L"])
    xoff, koff, rank = fs["xoff"], fs["koff"], fs["rank"]
    tot = 0.0
    for lvl in range(L + 1):
        nf = 2 ** (L - lvl)
        for q in range(nb):
            i, j = divmod(q, nf)
            M = int(xoff[(i + 1) * nf] - xoff[i * nf]) if lvl else int(xoff[-1])
            K = int(koff[j + 1] - koff[j]) if lvl == 0 else int(rank[lvl - 1][(i // 2) * 2 * nf + 2 * j] +
                                                                 rank[lvl - 1][(i // 2) * 2 * nf + 2 * j + 1])
            k = np.arange(int(rank[lvl][q]), dtype=np.float64)
            if M and K:
                tot += float(np.sum(4.0 * (M - k) * (K - k)))
    return tot


def _id_stream_bytes(fs):
    """Bytes the column IDs of a factor set must stream at the least: an exactly
    pivoted step reads every remaining column below the step's row once (it needs
    every updated norm), 8 (M - j)(K - j) bytes at step j < k; a block with more than
    twice as many rows as columns pivots on its K x K triangle after a blocked
    reduction that reads and writes every trailing column once per 16-column panel."""
    L, nb = int(fs["L"]), 2 ** int(fs["L"])
    xoff, koff, rank = fs["xoff"], fs["koff"], fs["rank"]
    tot = 0.0
    for lvl in range(L + 1):
        nf = 2 ** (L - lvl)
        for q in range(nb):
            i, j = divmod(q, nf)
            M = int(xoff[(i + 1) * nf] - xoff[i * nf]) if lvl else int(xoff[-1])
            K = int(koff[j + 1] - koff[j]) if lvl == 0 else int(rank[lvl - 1][(i // 2) * 2 * nf + 2 * j] +
                                                                 rank[lvl - 1][(i // 2) * 2 * nf + 2 * j + 1])
            if not (M and K):
                continue
            Mp = M
            if M > 2 * K:
                p0 = np.arange(0, K, 16, dtype=np.float64)
                tot += float(np.sum(16.0 * (M - p0) * np.maximum(K - p0 - 16, 0)))
                Mp = K
            k = np.arange(int(rank[lvl][q]), dtype=np.float64)
            tot += float(np.sum(8.0 * (Mp - k) * (K - k)))
    return tot


def _block_skeletons(fs):
    """Per level, per block: (input columns, local skeleton) read back from a
    stored factor set (the unit columns of P; every column of an identity block)."""
    L, nb = int(fs["L"]), 2 ** int(fs["L"])
    koff = fs["koff"]
    skel, out = [None] * nb, []
    for lvl in range(L + 1):
        nf = 2 ** (L - lvl)
        new, cur = [None] * nb, []
        for q in range(nb):
            i, j = divmod(q, nf)
            cols = np.arange(koff[j], koff[j + 1]) if lvl == 0 else \
                np.concatenate([skel[(i // 2) * 2 * nf + 2 * j], skel[(i // 2) * 2 * nf + 2 * j + 1]])
            r = int(fs["rank"][lvl][q])
            if fs["ident"][lvl][q]:
                Jl = np.arange(cols.size)
            elif r == 0:
                Jl = np.zeros(0, np.int64)
            else:
                o = int(fs["P_off"][lvl][q])
                P = fs["P"][o:o + r * cols.size].reshape(r, cols.size)
                unit = (P == 1.0) & (np.abs(P).sum(axis=0) == 1.0)[None, :]
                Jl = np.array([int(np.flatnonzero(unit[t])[0]) for t in range(r)], np.int64)
            new[q] = cols[Jl]
            cur.append((cols, Jl))
        out.append(cur)
        skel = new
    return out


def bench_build(args):
    """The butterfly factorization on the GPU (FP64 column IDs: block formation,
    pivoted QR and interpolation matrices in HIP kernels) on the i.i.d. square:
    seconds per build, against the host builder (NumPy/SciPy on the host's
    cores) and the oracle's column ID timed on sampled blocks."""
    import torch

    from oracle import dense as od
    from oracle import interp as oi
    from oracle import modes as om
    from paper_2605_21828_amd import workloads as wl
    from paper_2605_21828_amd.bfmht import Plan
    from paper_2605_21828_amd.factor import io as fio
    from paper_2605_21828_amd.factor import trees
    from paper_2605_21828_amd.factor.device_build import build_factors_device, fourier_tables
    from paper_2605_21828_amd.factor.fourier import real_modes

    wname = args.workload[len("build_"):]
    w = wl.WORKLOADS[wname]
    n, m, leaf, tol = w["n"], w["m"], w["leaf"], w["tol"]
    pts = wl.points_for(w)
    L = trees.depth_for(n, leaf)
    perm, xoff = trees.box_bisection_tree(pts, L)
    koff = trees.frequency_tree(m, L)
    modes = real_modes(m)
    dev = torch.device("cuda:0")
    # warm-up: a small build loads the kernels and grows no buffer of the timed one
    sw = wl.iid_points(99, 2048)
    sL = trees.depth_for(2048, 64)
    sp, sx = trees.box_bisection_tree(sw, sL)
    build_factors_device(fourier_tables(sw, real_modes(512), sp, dev), 2048, 512, sp, sx,
                         trees.frequency_tree(512, sL), sL, tol)
    torch.cuda.synchronize()
    log("device build: n=%d m=%d leaf=%d tol=%g L=%d" % (n, m, leaf, tol, L), host_memory())
    events = []
    t0 = time.perf_counter()
    tabs = fourier_tables(pts, modes, perm, dev)
    torch.cuda.synchronize()
    t_tab = time.perf_counter() - t0
    fs = build_factors_device(tabs, n, m, perm, xoff, koff, L, tol, events=events,
                              log=lambda s: log("  build", s))
    torch.cuda.synchronize()
    t_dev = time.perf_counter() - t0
    id_ms = sum(a.elapsed_time(b) for a, b in events)
    flops = _qr_flops(fs)
    log("device build %.2f s (column-ID kernels %.1f ms, %.3g flop)" % (t_dev, id_ms, flops), host_memory())
    del tabs
    # accuracy: FP64 synthesis of the device-built set on sampled rows against the dense transform
    b = 2
    c = wl.coefficients(w["wid"], m, b)
    p64 = Plan(fs, "f64", max_nrhs=b, device=dev)
    y = p64.apply(torch.tensor(c, dtype=torch.float64, device=dev)).cpu().numpy()
    rows = wl.sample_indices(w["wid"], n, 256)
    omodes = om.fourier_modes(m)
    synth_err = od.rel_err_cols(y[rows], od.fourier_synthesis_rows(pts, omodes, rows, c))[0]
    del p64
    host = None
    if args.host_build:
        log("host build (%d workers)" % args.workers)
        t1 = time.perf_counter()
        fh, _ = fio.fourier_factors(pts, m, leaf, tol, workers=args.workers, cache=False)
        t_host = time.perf_counter() - t1
        same_rank = float(np.mean(fh["rank"] == fs["rank"]))
        same_skel = bool(np.array_equal(fh["skel_L"], fs["skel_L"]))
        host = {"seconds": t_host, "workers": args.workers, "blocks_with_equal_rank": same_rank,
                "final_skeletons_equal": same_skel, "stored_entries_host": fio.stored_entries(fh),
                "speedup_device_vs_host": t_host / t_dev}
        log("host build %.1f s: %.1fx the device build; equal ranks on %.4f of the blocks" % (
            t_host, t_host / t_dev, same_rank))
        del fh
    base, sample_check = None, None
    if not args.no_cpu_baseline:
        # oracle column IDs of sampled blocks of every level (about 20 s), scaled
        # to all blocks of each level; the sampled blocks also check the device's
        # skeletons and interpolation matrices
        rng = wl.rng(w["wid"], 5)
        per = _block_skeletons(fs)
        nb = 2 ** L
        t_or, t_est, checked, agree, p_err = 0.0, 0.0, 0, 0, 0.0
        for lvl in range(L + 1):
            nf = 2 ** (L - lvl)
            qs = rng.choice(nb, 2, replace=False)
            tl = 0.0
            for q in qs:
                i, j = divmod(int(q), nf)
                cols, Jl = per[lvl][q]
                if not cols.size:
                    continue
                blk_rows = perm[xoff[i * nf]:xoff[(i + 1) * nf]]
                A = om.phi(pts[blk_rows], omodes[cols])
                t1 = time.perf_counter()
                Jo, Po, ido = oi.column_id(A, tol)
                tl += time.perf_counter() - t1
                checked += 1
                agree += int(np.array_equal(Jo, Jl))
                if Po is not None and Po.size and not fs["ident"][lvl][q]:
                    r = int(fs["rank"][lvl][q])
                    o = int(fs["P_off"][lvl][q])
                    Pd = fs["P"][o:o + r * cols.size].reshape(r, cols.size)
                    if Pd.shape == Po.shape:
                        p_err = max(p_err, float(np.abs(Pd - Po).max() / max(1.0, np.abs(Po).max())))
            t_or += tl
            t_est += tl * nb / len(qs)
        base = {"value": t_est, "unit": "s", "cores": _blas_threads(), "kind": "oracle",
                "sample": "oracle column ID (SciPy pivoted QR, FP64) of 2 blocks per level, %.1f s, scaled to "
                          "all %d blocks of each level (block formation not counted)" % (t_or, nb)}
        sample_check = {"blocks": checked, "same_skeleton": agree, "max_rel_P_diff": p_err}
    peak = 78.6   # FP64 vector FMA, TFLOP/s
    tf = flops / (id_ms * 1e-3) / 1e12 if id_ms > 0 else 0.0
    sbytes = _id_stream_bytes(fs)
    gbs = sbytes / (id_ms * 1e-3) / 1e9 if id_ms > 0 else 0.0
    res = {
        "metric": "butterfly factorization time on the device (FP64 column IDs)",
        "value": t_dev, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": t_dev * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m, "leaf": leaf, "tol": tol, "L": L,
                   "step": "tables, every level's blocks formed and decomposed, leaf bases, factor set packed"},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s", "frac": gbs / 8000.0,
                     "traffic": measured_traffic(args.workload, "id", per="apply"),
                     "traffic_unit": "bytes per build (every column-ID launch)",
                     "kernel": "hqr_panel/hqr_trail + cpqr_kernel (every bfmht_column_id launch)",
                     "alg_bytes": sbytes,
                     "note": "least streamed bytes of exactly pivoted column IDs (one read of the remaining "
                             "columns per pivot step; tall blocks: their blocked reduction reads and writes each "
                             "trailing column once per 16-column panel) over the column-ID launches' event time"},
        "cpu_baseline": base,
        "extra": {"column_id_kernel_ms": id_ms, "tables_seconds": t_tab, "qr_flops": flops,
                  "qr_tflops_fp64": tf, "qr_frac_of_fp64_vector_peak": tf / peak,
                  "stored_entries": fio.stored_entries(fs),
                  "levels": [[s[0], s[1], s[2], s[3], s[4], s[5]] for s in fs["build_stats"].tolist()],
                  "fp64_synthesis_rel_err_256_rows": synth_err, "host_build": host,
                  "oracle_sample_check": sample_check, "host_memory_at_end": host_memory()},
    }
    print(json.dumps(res), flush=True)


def bench_copy(args):
    """Calibration: a plain device copy of a known number of bytes (for HBM byte counters)."""
    import torch
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    ms = event_time(lambda: dst.copy_(src), 5, torch)
    print(json.dumps({"workload": "copy", "bytes_read_per_copy": nbytes, "bytes_written_per_copy": nbytes,
                      "ms_per_copy": ms, "GBps_read_plus_write": 2 * nbytes / (ms * 1e-3) / 1e9}), flush=True)


def _build_device(args):
    """The GPU that builds the factor sets with --device-build (column IDs on
    the device), else None (the host builder)."""
    if not getattr(args, "device_build", False):
        return None
    import torch
    return torch.device("cuda:0")


def counter_run(args):
    """A fixed number of applies of one direction and precision and nothing
    else (no timing, no oracle), for hardware-counter passes under rocprofv3:
    the counter totals divided by the printed apply count give per-apply
    figures.  Workloads: iid65536, iid131072 (one RHS, the least-squares fit's
    shape), sphere40962 (256 RHS) and batched32 (one batched call per apply).
    Tile shapes come from the autotuner's cache when --cache is given."""
    import torch

    from paper_2605_21828_amd import workloads as wl
    from paper_2605_21828_amd.bfmht import Batch, Plan
    from paper_2605_21828_amd.factor import io as fio

    prec, fwd, count = args.counter_precision, args.counter_direction == "fwd", args.counter_applies
    dev = torch.device("cuda:0")
    if args.workload.startswith("build_"):
        # one factorization on the GPU and nothing else (the counters of its column-ID launches)
        from paper_2605_21828_amd.factor import trees
        from paper_2605_21828_amd.factor.device_build import build_factors_device, fourier_tables
        from paper_2605_21828_amd.factor.fourier import real_modes
        w = wl.WORKLOADS[args.workload[len("build_"):]]
        pts = wl.points_for(w)
        L = trees.depth_for(w["n"], w["leaf"])
        perm, xoff = trees.box_bisection_tree(pts, L)
        build_factors_device(fourier_tables(pts, real_modes(w["m"]), perm, dev), w["n"], w["m"], perm, xoff,
                             trees.frequency_tree(w["m"], L), L, w["tol"])
        torch.cuda.synchronize()
        print(json.dumps({"counter_run": args.workload, "precision": "f64", "direction": "build", "applies": 1,
                          "stage_launches_per_apply": None}), flush=True)
        return
    dt = torch.float64 if prec == "f64" else torch.float32
    if args.workload == "batched32":
        spec = wl.BATCHED
        inst = wl.batched_instances(spec)
        plans = {}
        for side in sorted({s for s, _ in inst}):
            fs = fio.fourier_factors(wl.grid_points(side), side * side // 4, spec["leaf"], spec["tol"],
                                     workers=args.workers, cache=args.cache)[0]
            plans[side] = Plan(fs, prec, max_nrhs=spec["max_nrhs"], device=dev)
        ps = [plans[s] for s, _ in inst]
        xs = [torch.randn(((p.m if fwd else p.n), b), dtype=dt, device=dev) for p, (_, b) in zip(ps, inst)]
        batch = Batch(ps)
        outs = [torch.empty(((p.n if fwd else p.m), b), dtype=dt, device=dev) for p, (_, b) in zip(ps, inst)]
        if args.cache and not args.no_tune:
            from paper_2605_21828_amd.autotune import tune_batch
            tune_batch(batch, xs, transpose=not fwd, log=log)
        run = lambda: batch.launch(xs, outs, not fwd)   # noqa: E731
        launches = None
    else:
        if args.workload == "sphere40962":
            spec = wl.SPHERE
            fs, _ = fio.sphere_factors(spec["level"], spec["wid"], spec["m"], spec["leaf"], spec["tol"],
                                       workers=args.workers, cache=args.cache)
            b = spec["nrhs"]
        else:
            w = wl.WORKLOADS[args.workload]
            fs, _ = fio.fourier_factors(wl.points_for(w), w["m"], w["leaf"], w["tol"], workers=args.workers,
                                        cache=args.cache, arity=args.arity, device=_build_device(args))
            b = w["nrhs"]
        p = Plan(fs, prec, max_nrhs=b, device=dev)
        if args.cache and not args.no_tune:
            from paper_2605_21828_amd.autotune import tune_plan
            tune_plan(p, fs, b, use_cache=True, log=log)
        x = torch.randn(((p.m if fwd else p.n), b), dtype=dt, device=dev)
        y = torch.empty(((p.n if fwd else p.m), b), dtype=dt, device=dev)
        run = (lambda: p.apply(x, out=y)) if fwd else (lambda: p.apply_t(x, out=y))
        launches = stage_launches(p, fs)
    run()
    torch.cuda.synchronize()
    for _ in range(count):
        run()
    torch.cuda.synchronize()
    print(json.dumps({"counter_run": args.workload, "precision": prec, "direction": args.counter_direction,
                      "applies": count + 1, "stage_launches_per_apply": launches}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="iid65536")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dense-context", action="store_true",
                    help="skip the dense-matrix vendor-GEMM timing reported as context")
    ap.add_argument("--variants", default="f64,bf16x2,bf16x3",
                    help="comma list of other precisions timed on the same inputs")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--cache", action="store_true", help="reuse a factor file cached under $BFMHT_CACHE")
    ap.add_argument("--no-tune", action="store_true", help="keep the default tile widths")
    ap.add_argument("--no-leaf-compare", action="store_true",
                    help="skip the comparison plan with a separate leaf stage (kernel traces of the headline apply)")
    ap.add_argument("--precision", default=None, help="headline precision of the sphere workload")
    ap.add_argument("--arity", type=int, default=2, choices=(2, 4),
                    help="tree arity of the nonuniform-square workloads (4: quadtree and 4-ary mode tree)")
    ap.add_argument("--device-build", action="store_true",
                    help="build the factor sets of the least-squares and counter workloads on the GPU")
    ap.add_argument("--host-build", action="store_true",
                    help="build_* workloads: also time the host builder on the same inputs")
    ap.add_argument("--counter-applies", type=int, default=0,
                    help="counter run: this many applies (plus one) of one direction and precision, nothing else")
    ap.add_argument("--counter-direction", default="fwd", choices=("fwd", "bwd"))
    ap.add_argument("--counter-precision", default="f32", choices=("f64", "f32", "bf16x2", "bf16x3"))
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.counter_applies > 0:
        return counter_run(args)
    if args.workload == "batched32":
        return bench_batched(args)
    if args.workload == "copy":
        return bench_copy(args)
    if args.workload == "grid64":
        return bench_latency(args)
    if args.workload == "inverse_sphere40962":
        return bench_inverse(args)
    if args.workload in ("lsq262144", "lsq131072"):
        return bench_lsq(args)
    if args.workload == "sphere40962":
        return bench_sphere(args)
    if args.workload.startswith("build_"):
        return bench_build(args)

    import torch

    from paper_2605_21828_amd import workloads as wl
    from paper_2605_21828_amd.bfmht import Plan
    from paper_2605_21828_amd.factor import io as fio
    from paper_2605_21828_amd.factor.fourier import real_modes

    w = wl.WORKLOADS[args.workload]
    n, m, b = w["n"], w["m"], w["nrhs"]
    counter_key = args.workload if args.arity == 2 else "%s_arity%d" % (args.workload, args.arity)
    pts = wl.points_for(w)
    log("building factors: n=%d m=%d leaf=%d tol=%g arity=%d" % (n, m, w["leaf"], w["tol"], args.arity))
    fs, _ = fio.fourier_factors(pts, m, w["leaf"], w["tol"], workers=args.workers, cache=args.cache,
                                log=lambda s: log("  factor", s), arity=args.arity)
    F = fio.stored_entries(fs)
    modes = real_modes(m)
    lam = (modes[:, 0] ** 2 + modes[:, 1] ** 2).astype(np.float64)
    c_host = wl.coefficients(w["wid"], m, b, lam=lam, kind=w["coef"])
    f_host = wl.values(w["wid"], n, b)

    dev = torch.device("cuda:0")
    log("uploading FP32 plan")
    p32 = Plan(fs, "f32", max_nrhs=b, device=dev)
    c32 = torch.tensor(c_host, dtype=torch.float32, device=dev)
    f32 = torch.tensor(f_host, dtype=torch.float32, device=dev)
    y32 = torch.empty((n, b), dtype=torch.float32, device=dev)
    g32 = torch.empty((m, b), dtype=torch.float32, device=dev)

    tuned = None
    if not args.no_tune:
        from paper_2605_21828_amd.autotune import tune_plan
        tuned = tune_plan(p32, fs, b, use_cache=args.cache, log=log)

    def step():
        p32.apply(c32, out=y32)
        p32.apply_t(f32, out=g32)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    log("fp32 step %.3f ms" % ms)

    # per-direction timings with HIP events (torch's current stream is the one the library launches on)
    reps = max(args.steps, 5)
    ms_fwd = event_time(lambda: p32.apply(c32, out=y32), reps, torch)
    ms_bwd = event_time(lambda: p32.apply_t(f32, out=g32), reps, torch)
    launches = stage_launches(p32, fs)   # stage launches of one forward apply
    # the forward apply reads the compact ID blocks (T only): its algorithmic
    # factor entries are the forward pool's, not the full factor count F
    F_fwd = p32.stored_fwd
    flops = 2.0 * F_fwd * b
    alg_bytes32 = 4.0 * F_fwd + 4.0 * (n + m) * b
    achieved = flops / (ms_fwd * 1e-3) / 1e12
    result_extra = {
        "fp32_apply_ms": ms_fwd, "fp32_apply_transpose_ms": ms_bwd,
        "fp32_apply_alg_GBps": alg_bytes32 / (ms_fwd * 1e-3) / 1e9,
        "stored_factor_entries": F, "compression_vs_dense": n * m / F,
        "forward_factor_entries": F_fwd,
        "stage_launches_per_apply": launches,
        "tile_shapes": tuned,
        "leaf_merged": p32.leaf_merged,
    }
    if p32.leaf_merged and not args.no_leaf_compare:
        # the same factors with the leaf bases as a stage of their own (comparison)
        log("uploading FP32 plan with a separate leaf stage")
        ps = Plan(fs, "f32", max_nrhs=b, device=dev, leaf_stage=True)
        if not args.no_tune:
            tune_plan(ps, fs, b, use_cache=args.cache, log=log)
        ys, gs = torch.empty_like(y32), torch.empty_like(g32)
        result_extra["separate_leaf_stage"] = {
            "apply_ms": event_time(lambda: ps.apply(c32, out=ys), reps, torch),
            "apply_transpose_ms": event_time(lambda: ps.apply_t(f32, out=gs), reps, torch),
            "stage_launches_per_apply": stage_launches(ps, fs), "forward_factor_entries": ps.stored_fwd}
        del ps, ys, gs
    variants_out = {}

    # Precision variants on the same inputs: the plain FP64 apply (speedup
    # reference and accuracy anchor) and the BF16 split products.
    variants = [v for v in args.variants.split(",") if v]
    y64 = None
    variant_outputs = {}
    for prec in variants:
        log("uploading %s plan" % prec)
        pv = Plan(fs, prec, max_nrhs=b, device=dev)
        dt = torch.float64 if prec == "f64" else torch.float32
        cv = c32.to(dt) if prec != "f64" else torch.tensor(c_host, dtype=dt, device=dev)
        fv = f32.to(dt) if prec != "f64" else torch.tensor(f_host, dtype=dt, device=dev)
        yv = torch.empty((n, b), dtype=dt, device=dev)
        gv = torch.empty((m, b), dtype=dt, device=dev)
        shapes = None
        if not args.no_tune:
            from paper_2605_21828_amd.autotune import tune_plan
            shapes = tune_plan(pv, fs, b, use_cache=args.cache, log=log)
        for _ in range(2):
            pv.apply(cv, out=yv)
            pv.apply_t(fv, out=gv)
        t_f = event_time(lambda: pv.apply(cv, out=yv), reps, torch)
        t_b = event_time(lambda: pv.apply_t(fv, out=gv), reps, torch)
        rec = {"apply_ms": t_f, "apply_transpose_ms": t_b,
               "speedup_vs_fp32": (ms_fwd + ms_bwd) / (t_f + t_b),
               "plan_device_GB": pv.device_bytes / 1e9, "tile_shapes": shapes,
               "roofline": dict(roofline_for(prec, pv.stored_fwd, n, m, b, t_f, launches),
                                traffic=measured_traffic(counter_key, prec + "_fwd"),
                                mfma_busy_pct_counter=measured_mfma_busy(counter_key, prec + "_fwd"))}
        if prec == "f64":
            y64 = yv.clone()
        else:
            if y64 is not None:
                rec["rel_err_vs_fp64_gpu"] = float(torch.linalg.norm(yv.double() - y64) / torch.linalg.norm(y64))
            variant_outputs[prec] = (yv.double().cpu().numpy(), gv.double().cpu().numpy())
        variants_out[prec] = rec
        del pv, cv, fv, yv, gv
        torch.cuda.empty_cache()
    if y64 is not None:
        result_extra["fp32_vs_fp64_gpu_rel_err"] = float(torch.linalg.norm(y32.double() - y64) / torch.linalg.norm(y64))
        result_extra["speedup_fp32_vs_fp64_plain"] = ((variants_out["f64"]["apply_ms"] + variants_out["f64"]["apply_transpose_ms"])
                                                      / (ms_fwd + ms_bwd))
    result_extra["variants"] = variants_out
    if not args.no_dense_context:
        result_extra["dense_context"] = dense_context(pts, modes, c32, f32, reps, torch)

    base = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        rows = wl.sample_indices(w["wid"], n, 2048)
        cols = wl.sample_indices(w["wid"], m, 2048, stream=4)
        out_np = y32.double().cpu().numpy()
        g_np = g32.double().cpu().numpy()
        base, acc = cpu_baseline(fs, pts, c_host, f_host, out_np, g_np, rows, cols, lam, variant_outputs)
        result_extra.update(acc)

    bound, peak, unit = PEAK["f32"]
    res = {
        "metric": "butterfly apply RHS*points/s (FP32 synthesis + analysis)",
        "value": 2.0 * n * b / (ms * 1e-3),
        "unit": "RHS*points/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m, "nrhs": b, "leaf": w["leaf"], "tol": w["tol"],
                   "L": int(fs["L"]), "arity": args.arity, "step": "apply + apply_transpose"},
        "roofline": {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                     "frac": achieved / peak, "traffic": measured_traffic(counter_key),
                     "traffic_unit": "bytes per launch",
                     "mfma_busy_pct_counter": measured_mfma_busy(counter_key),
                     "alg_bytes_per_launch": alg_bytes32 / launches,
                     # level vectors written by one stage and read by the next: not
                     # algorithmic (intermediate), reported beside it
                     "impl_bytes_per_launch": level_bytes(fs, b, 4, p32.leaf_merged) / launches,
                     "kernel": "stage_kernel<P_F32, forward> (all stage launches of one FP32 apply)",
                     "per_launch_alg_flops": flops / launches,
                     "avg_launch_ms": ms_fwd / launches},
        "cpu_baseline": base,
        "extra": result_extra,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
