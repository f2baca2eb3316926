"""Autotuner for the solver's launch shapes.

For a shape class (device, block size, N, number of right-hand sides, number
of shifts, precision, carry) it times short trial solves of the real problem
for each candidate option set and keeps the fastest per outer iteration.
Every trial runs the library itself (gsc_solve / gsc_solve_batched); the
per-iteration time is the difference of two trial lengths, so the set-up
(pair upload, first CG solve, interval estimate) does not bias the choice.
Results are cached as JSON (``GSC_AUTOTUNE_CACHE`` or
``~/.cache/gsc_autotune.json``).
"""
from __future__ import annotations

import json
import math
import os
import sys

from . import api

KNOBS_FULL = [
    dict(fuse_steps=16, spmm_kernel=1, inner_method=2),
    dict(fuse_steps=12, spmm_kernel=1, inner_method=2),
    dict(fuse_steps=8, spmm_kernel=1, inner_method=2),
    dict(fuse_steps=16, spmm_kernel=1, inner_method=1),
]
KNOBS_PROJECTED = [
    dict(spmm_kernel=1, inner_method=2),
    dict(spmm_kernel=1, inner_method=1),
]
KNOBS_BATCHED = [
    dict(graph_iters=4), dict(graph_iters=1), dict(graph_iters=8),
]


def _cache_path():
    return os.environ.get("GSC_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "gsc_autotune.json"))


def _load():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(cache):
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    except OSError:
        pass


def shape_key(block, n, nrhs, nshift, precision, carry, tag="solve"):
    b2 = lambda v: int(round(math.log2(max(v, 1))))  # noqa: E731
    return f"{tag}|gfx950|B{block}|N2^{b2(n)}|R2^{b2(nrhs)}|K2^{b2(nshift)}|{precision}|{carry}"


def _wall(fn, reps=2):
    import time
    best = float("inf")
    out = None
    for _ in range(reps):
        t = time.perf_counter()
        out = fn()
        best = min(best, time.perf_counter() - t)
    return best, out


def _per_iter(ctx, pair, z, rhs, opts, t1, t2):
    base = dict(opts)
    extra = {"proj": rhs[:, None]} if base.get("carry") == "projected" else {}

    def run(mi):
        return lambda: api.solve(ctx, pair, z, rhs=rhs, out="device", want_cols=False, max_iter=mi,
                                 **base, **extra)
    ta, a = _wall(run(t1))
    tb, b = _wall(run(t2))
    di = b.outer_iters - a.outer_iters
    if di <= 0 or tb <= ta:
        raise RuntimeError(f"trial did not separate: {a.outer_iters}/{b.outer_iters} iters, {ta:.4f}/{tb:.4f} s")
    return (tb - ta) / di


def tune_solve(ctx, pair, z, rhs, precision="fp64", carry="full", tol=1e-10, t1=8, t2=32,
               candidates=None, force=False, verbose=False):
    """Best option dict for this problem's shape class (trial solves run on
    the given problem).  Cached per shape class."""
    import numpy as np
    rhs = np.ascontiguousarray(rhs, dtype=np.int64)
    key = shape_key(pair.block, pair.n, len(rhs), len(z), precision, carry)
    cache = _load()
    if key in cache and not force:
        return dict(cache[key]["opts"])
    cands = candidates or (KNOBS_FULL if carry == "full" else KNOBS_PROJECTED)
    best, best_t, table = None, float("inf"), []
    for c in cands:
        opts = dict(c, precision=precision, carry=carry, tol=tol)
        try:
            t = _per_iter(ctx, pair, z, rhs, opts, t1, t2)
        except Exception as e:  # a candidate the library rejects is skipped
            table.append((c, float("inf")))
            if verbose:
                print("autotune: skip", c, repr(e), file=sys.stderr)
            continue
        table.append((c, t))
        if verbose:
            print(f"autotune {key}: {c} -> {t * 1e3:.3f} ms/iter", file=sys.stderr)
        if t < best_t:
            best, best_t = c, t
    cache[key] = dict(opts=best, ms_per_iter=best_t * 1e3,
                      trials=[dict(opts=c, ms_per_iter=t * 1e3) for c, t in table])
    _store(cache)
    return dict(best)


def tune_batched(ctx, problems, precision="mixed", tol=1e-6, t1=8, t2=24, candidates=None,
                 force=False, verbose=False):
    """Best graph chunk / product kernel for a batch (keyed by its size)."""
    tot = sum(p["pair"].n * len(p["rhs"]) for p in problems)
    key = shape_key(4, tot, len(problems), max(len(p["z"]) for p in problems), precision,
                    "projected", tag="batched")
    cache = _load()
    if key in cache and not force:
        return dict(cache[key]["opts"])
    best, best_t, table = None, float("inf"), []
    for c in candidates or KNOBS_BATCHED:
        opts = dict(c, precision=precision, tol=tol)
        ta, _ = _wall(lambda: api.solve_batched(ctx, problems, max_iter=t1, **opts), reps=1)
        tb, _ = _wall(lambda: api.solve_batched(ctx, problems, max_iter=t2, **opts), reps=1)
        t = max(1e-9, tb - ta) / (t2 - t1)
        table.append((c, t))
        if verbose:
            print(f"autotune {key}: {c} -> {t * 1e3:.3f} ms/iter")
        if t < best_t:
            best, best_t = c, t
    cache[key] = dict(opts=best, ms_per_iter=best_t * 1e3,
                      trials=[dict(opts=c, ms_per_iter=t * 1e3) for c, t in table])
    _store(cache)
    return dict(best)
