"""Autotuner for the solver's launch and tile shapes.

For a shape class (device, block size, N, number of right-hand sides, number
of shifts, precision, carry) it times short trial solves of the real problem
and keeps the fastest option set per outer iteration.  The search is
coordinate-wise over a space of tile and launch shapes -- the rhs tile R_t,
the workgroup rows of the product launches, the Chebyshev column block, the
fused shift-update depth, the inner method, and for batches the graph chunk
and the number of concurrent jobs: starting from the library's automatic
choices, each knob in turn takes the value that is fastest with the others
held at their best so far.  Every trial runs the library itself (gsc_solve /
gsc_solve_batched); the per-iteration time is the difference of two trial
lengths, so the set-up (pair upload, first CG solve, interval estimate) does
not bias the choice.  Results are cached as JSON (``GSC_AUTOTUNE_CACHE`` or
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

# coordinate search spaces: knob -> candidate values, the first being the
# library's automatic choice (0 = auto)
SPACE_FULL = {
    "fuse_steps": [0, 12, 8],
    "inner_method": [0, 1],
    "cheb_block": [0, 64, 128, 256],
    "row_groups": [0, 256, 1024, 4096],
}
SPACE_PROJECTED = {
    "inner_method": [0, 1],
    "cheb_block": [0, 64, 128, 256],
    "row_groups": [0, 256, 1024, 4096],
    "rhs_tile": [0, 128, 256],
}
SPACE_BATCHED = {
    "graph_iters": [0, 1, 8],
    "batch_streams": [0, 2, 4, 16],
    "rhs_tile": [0, 64, 256],
    "cheb_block": [0, 64, 128],
    "row_groups": [0, 256, 1024],
}


def coordinate_search(space, measure, verbose=None):
    """Coordinate-wise minimisation of ``measure(opts) -> seconds`` over
    ``space`` (knob -> candidate values, the first the default): each knob
    in turn keeps the fastest of its values with the other knobs at their
    best so far.  A value whose trial raises (the library rejects it) counts
    as infinitely slow.  Returns (best options without default values,
    best time, [(options, time), ...] of every trial)."""
    cur = {k: v[0] for k, v in space.items()}
    trials = {}

    def timed(opts):
        key = tuple(sorted(opts.items()))
        if key not in trials:
            try:
                t = float(measure({k: v for k, v in opts.items() if v != space[k][0]}))
            except Exception as e:  # noqa: BLE001 - a rejected candidate
                if verbose:
                    verbose(f"skip {opts}: {e!r}")
                t = float("inf")
            trials[key] = t
            if verbose:
                verbose(f"{opts} -> {t * 1e3:.3f} ms")
        return trials[key]

    best_t = timed(cur)
    for knob, values in space.items():
        for v in values:
            if v == cur[knob]:
                continue
            cand = dict(cur, **{knob: v})
            t = timed(cand)
            if t < best_t:
                cur, best_t = cand, t
    best = {k: v for k, v in cur.items() if v != space[k][0]}
    table = [({k: v for k, v in key if v != space[k][0]}, t) for key, t in trials.items()]
    return best, best_t, table


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
               candidates=None, space=None, force=False, verbose=False):
    """Best option dict for this problem's shape class (trial solves run on
    the given problem): a coordinate search over ``space`` (default
    SPACE_FULL or SPACE_PROJECTED), or the fastest of an explicit list of
    ``candidates``.  Cached per shape class."""
    import numpy as np
    rhs = np.ascontiguousarray(rhs, dtype=np.int64)
    key = shape_key(pair.block, pair.n, len(rhs), len(z), precision, carry)
    cache = _load()
    if key in cache and not force:
        return dict(cache[key]["opts"])
    say = (lambda m: print(f"autotune {key}: {m}", file=sys.stderr)) if verbose else None

    def measure(c):
        return _per_iter(ctx, pair, z, rhs, dict(c, precision=precision, carry=carry, tol=tol), t1, t2)
    if candidates is not None:
        table = []
        for c in candidates:
            try:
                t = measure(c)
            except Exception as e:  # noqa: BLE001 - a candidate the library rejects is skipped
                t = float("inf")
                if say:
                    say(f"skip {c}: {e!r}")
            table.append((dict(c), t))
        best, best_t = min(table, key=lambda ct: ct[1])
    else:
        best, best_t, table = coordinate_search(space or (SPACE_FULL if carry == "full" else SPACE_PROJECTED),
                                                measure, say)
    cache[key] = dict(opts=best, ms_per_iter=best_t * 1e3,
                      trials=[dict(opts=c, ms_per_iter=t * 1e3) for c, t in table])
    _store(cache)
    return dict(best)


def batch_key(problems, precision):
    """Shape class of a batch: its largest system, its total N x R, its
    number of systems and its largest shift count (log2 bins)."""
    nmax = max(p["pair"].n for p in problems)
    tot = sum(p["pair"].n * len(p["rhs"]) for p in problems)
    b2 = lambda v: int(round(math.log2(max(v, 1))))  # noqa: E731
    return (f"batched|gfx950|Nmax2^{b2(nmax)}|NR2^{b2(tot)}|S2^{b2(len(problems))}"
            f"|K2^{b2(max(len(p['z']) for p in problems))}|{precision}|projected")


def tune_batched(ctx, problems, precision="mixed", tol=1e-6, t1=8, t2=24, candidates=None, space=None,
                 force=False, verbose=False):
    """Best tile and launch shapes for a batch (keyed by batch_key): a
    coordinate search over ``space`` (default SPACE_BATCHED: graph chunk,
    concurrent jobs, rhs tile, Chebyshev column block, row groups), or the
    fastest of an explicit list of ``candidates``.  Cached per class."""
    key = batch_key(problems, precision)
    cache = _load()
    if key in cache and not force:
        return dict(cache[key]["opts"])
    say = (lambda m: print(f"autotune {key}: {m}", file=sys.stderr)) if verbose else None

    def measure(c):
        opts = dict(c, precision=precision, tol=tol)
        ta, a = _wall(lambda: api.solve_batched(ctx, problems, max_iter=t1, **opts), reps=1)
        tb, b = _wall(lambda: api.solve_batched(ctx, problems, max_iter=t2, **opts), reps=1)
        di = max(o["outer_iters"] for o in b) - max(o["outer_iters"] for o in a)
        if di <= 0 or tb <= ta:
            raise RuntimeError(f"trial did not separate ({ta:.4f}/{tb:.4f} s)")
        return (tb - ta) / di
    if candidates is not None:
        table = []
        for c in candidates:
            try:
                t = measure(c)
            except Exception as e:  # noqa: BLE001
                t = float("inf")
                if say:
                    say(f"skip {c}: {e!r}")
            table.append((dict(c), t))
        best, best_t = min(table, key=lambda ct: ct[1])
    else:
        best, best_t, table = coordinate_search(space or SPACE_BATCHED, measure, say)
    cache[key] = dict(opts=best, ms_per_iter=best_t * 1e3,
                      trials=[dict(opts=c, ms_per_iter=t * 1e3) for c, t in table])
    _store(cache)
    return dict(best)
