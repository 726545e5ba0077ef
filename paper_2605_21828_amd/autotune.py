"""Tile-width autotuner for the butterfly apply.

The tunable is the workgroup tile shape of each stage (`bfmht_plan_set_tile`):
64 or 128 output rows by 16, 32 or 64 right-hand-side columns.  Narrower tiles
read each factor row more than once but give a small stage more workgroups;
taller tiles halve the LDS traffic and right-hand-side re-reads per flop but
waste more rows on ragged blocks and leave fewer workgroups.  Which wins
depends on the stage's shape, the precision and the RHS count, so it is
measured.  The search is greedy over stages in order: every stage keeps the
shape that gives the fastest full apply, timed with HIP events on the current
stream, the others held at their current choice.  Results are cached in a JSON file keyed by the
plan's shape (sizes, ranks, precision) and the RHS count.
"""
import hashlib
import json
import os

import numpy as np

from . import bfmht as B

WIDTHS = (16, 32, 64)
HEIGHTS = (64, 128)
SHAPES = [(r, c) for r in HEIGHTS for c in WIDTHS]
CACHE = os.environ.get("BFMHT_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "bfmht", "tune.json"))


def signature(fs, precision, nrhs, stored_fwd=0, stages=0):
    """Cache key: the tree shape, the precision, the RHS count, the forward
    pool size and the stage count (compact, full-block and merged-leaf plans of
    one factor set tune apart)."""
    h = hashlib.sha1()
    for k in ("rank", "ident", "xoff", "koff"):
        h.update(np.ascontiguousarray(fs[k]).tobytes())
    return "%s|%d|%d|%d|%s|%d|F%d|S%d" % (precision, int(fs["n"]), int(fs["m"]), int(fs["L"]), h.hexdigest()[:16],
                                          nrhs, int(stored_fwd), int(stages))


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(path, cache):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def _time(fn, reps, torch):
    fn()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    e.synchronize()
    return s.elapsed_time(e) / reps


def apply_config(plan, config):
    for d, key in ((0, "fwd"), (1, "bwd")):
        for k, (r, c) in enumerate(config.get(key, [])):
            B.bfmht_plan_set_tile(plan.handle, d, k, r, c)


def tune_plan(plan, fs, nrhs, reps=10, cache_path=CACHE, use_cache=True, log=None):
    """Choose per-stage tile widths for `plan` at this RHS count; returns the config dict."""
    torch = plan.torch
    key = signature(fs, plan.precision, nrhs, getattr(plan, "stored_fwd", 0), B.bfmht_plan_num_stages(plan.handle))
    cache = _load_cache(cache_path) if use_cache else {}
    if key in cache:
        apply_config(plan, cache[key])
        return cache[key]
    x = torch.randn((plan.m, nrhs), dtype=plan.dtype, device=plan.device)
    y = torch.randn((plan.n, nrhs), dtype=plan.dtype, device=plan.device)
    out_f = torch.empty((plan.n, nrhs), dtype=plan.dtype, device=plan.device)
    out_b = torch.empty((plan.m, nrhs), dtype=plan.dtype, device=plan.device)
    S = B.bfmht_plan_num_stages(plan.handle)
    config = {}
    for d, key_d, fn in ((0, "fwd", lambda: plan.apply(x, out=out_f)), (1, "bwd", lambda: plan.apply_t(y, out=out_b))):
        choice = [(64, 0)] * S
        for k in range(S):
            B.bfmht_plan_set_tile(plan.handle, d, k, 64, 0)
        base = _time(fn, reps, torch)
        for k in range(S):
            best, best_t = choice[k], base
            for r, c in SHAPES:
                if c > 16 and nrhs <= c // 2:
                    continue  # wider than twice the RHS count only adds idle columns
                B.bfmht_plan_set_tile(plan.handle, d, k, r, c)
                t = _time(fn, reps, torch)
                if t < best_t * 0.995:
                    best, best_t = (r, c), t
            choice[k] = best
            B.bfmht_plan_set_tile(plan.handle, d, k, *best)
            base = min(base, best_t)
        config[key_d] = [list(c) for c in choice]
        config[key_d + "_ms"] = base
        if log:
            log("autotune %s: %s -> %.3f ms" % (key_d, choice, base))
    if use_cache:
        cache = _load_cache(cache_path)
        cache[key] = config
        _store_cache(cache_path, cache)
    return config


def tune_batch(batch, inputs, transpose=False, reps=5, log=None):
    """Choose one uniform tile shape per distinct plan of a batch by greedy
    search over plans, timing the whole batched apply."""
    torch = batch.torch
    outs = [torch.empty(((p.m if transpose else p.n), int(x.shape[1])), dtype=p.dtype, device=batch.device)
            for p, x in zip(batch.plans, inputs)]
    d = 1 if transpose else 0

    def set_all(p, shape):
        for k in range(B.bfmht_plan_num_stages(p.handle)):
            B.bfmht_plan_set_tile(p.handle, d, k, *shape)

    def fn():
        batch.launch(inputs, outs, transpose)

    distinct, widest = [], {}
    for p, x in zip(batch.plans, inputs):
        if id(p) not in widest:
            distinct.append(p)
            widest[id(p)] = 0
        widest[id(p)] = max(widest[id(p)], int(x.shape[1]))
    for p in distinct:
        set_all(p, (64, 0))
    base = _time(fn, reps, torch)
    choice = []
    for p in distinct:
        best, best_t = (64, 0), base
        for r, c in SHAPES:
            if c > 16 and widest[id(p)] <= c // 2:
                continue  # wider than twice the largest RHS count only adds idle columns
            set_all(p, (r, c))
            t = _time(fn, reps, torch)
            if t < best_t * 0.995:
                best, best_t = (r, c), t
        set_all(p, best)
        choice.append(best)
        base = min(base, best_t)
    if log:
        log("autotune batch (%s): shapes %s -> %.3f ms" % ("transpose" if transpose else "forward", choice, base))
    return choice, base
