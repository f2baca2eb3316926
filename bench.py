"""Throughput of the generalized shifted COCG hot path on one MI355X.

One step = ASED pair build on the device (eq. Hap-1) + the shifted solve of
(z_k S - H) x = e_j for every shift and right-hand side (seed COCG, pi
recurrence, fused shift updates, inner CG for S^{-1} r, seed switching),
with the Green's-function columns left in HBM.  The default workload is
si4096: Si diamond 8x8x8 cells (4096 atoms, N = 16384, 69,632 4x4 blocks),
Gaussian displacements 0.05 A, 256 shifts on [-20, 5] eV with eta 0.05 eV,
256 right-hand sides (all orbitals of 64 random atoms), FP64, tol 1e-10.

Prints one JSON line.  The roofline object reports the dominant kernel's
algorithmic bytes (counted on the device per launch) over its HIP-event time
measured live on the library's stream during the timed steps.  The CPU
baseline times the step-by-step oracle model of the same method on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "shift·RHS·iterations/s + HBM GB/s; mixed-batched vs plain FP64 at 1e-6"
UNIT = "shift·RHS·iterations/s"


def workload(name):
    from synth import configs
    if name == "si4096":
        return configs.si4096()
    if name == "si64":
        return configs.si64()
    raise SystemExit(f"unknown workload {name}")


def describe(cfg, args):
    s = cfg["system"]
    return {
        "workload": cfg["name"],
        "system": f"{s.n_atoms} atoms, N={s.n}, nnzb={s.nnzb}, block={s.block}",
        "shifts": int(len(cfg["z"])),
        "rhs": int(len(cfg["rhs"])),
        "eta": float(cfg["z"][0].imag),
        "tol": args.tol,
        "carry": "full",
        "fuse_steps": args.fuse,
        "spmm_kernel": args.spmm,
        "inner_method": args.inner,
        "precision": args.precision,
        "parallelism": "1 GPU",
    }


def host_cpu():
    """CPU model and the cores this process may use (for the oracle timings)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline(cfg, iters):
    """Oracle model of the method (oracle/shifted_cocg.py) on one rhs and all
    shifts of the workload, for a fixed number of outer iterations."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import ased, green, shifted_cocg

    s = cfg["system"]
    Sb, Hb, _ = ased.pair_blocks(s)
    S, H = green.sparse_matrices(s, Sb, Hb)
    b = np.zeros(s.n)
    b[int(cfg["rhs"][0])] = 1.0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        r = shifted_cocg.solve(H, S, cfg["z"], b, tol=1e-10, max_iter=iters)
        dt = time.perf_counter() - t0
    return {"value": r.active_shift_iters / dt, "unit": UNIT, "cores": 1, "kind": "oracle", "host": host_cpu(),
            "sample": f"oracle step-by-step model (numpy/scipy, 1 thread), workload {cfg['name']}, "
                      f"1 rhs x {len(cfg['z'])} shifts x {r.iters} outer iterations "
                      f"({r.active_shift_iters} active shift-iterations, {r.inner_iters} inner CG "
                      f"steps) in {dt:.1f} s"}


def cpu_dense_lu(cfg, n_shifts=1):
    """The plain definition of the result, timed the way a dense solver would
    run it: dense z S - H and LAPACK LU (oracle/green.py) for every right-hand
    side of the workload at ``n_shifts`` shifts, on all BLAS threads of the
    host; reported per shift and extrapolated to all shifts."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import ased, green

    s = cfg["system"]
    S, H, _ = ased.dense_pair(s)
    z = cfg["z"][:n_shifts]
    t0 = time.perf_counter()
    green.solve_dense(H, S, z, cfg["rhs"])
    dt = (time.perf_counter() - t0) / n_shifts
    threads = max([p.get("num_threads", 1) for p in threadpool_info() if p.get("user_api") == "blas"] or [1])
    return {"kind": "oracle dense LU (numpy/scipy LAPACK)", "threads": threads, "host": host_cpu(),
            "seconds_per_shift": dt, "extrapolated_seconds_all_shifts": dt * len(cfg["z"]),
            "sample": f"{n_shifts} shift(s) x {len(cfg['rhs'])} rhs of {cfg['name']} (N={s.n}, dense "
                      f"{s.n}x{s.n} complex LU per shift)"}


def forces_measure(name, n_slices=8, precision=None, inner_relax=False):
    """One MD-style step at full size: the band energy over every orbital,
    its gradients on the stored H, S entries (one shifted solve with the
    z-derivative carry) and the forces through the ASED pair.  slab8192: FP64,
    tol 1e-10, 512 shifts on [-20, E_F]; water3000: complex64 products, FP64
    recurrences, tol 1e-6, 1024 shifts on [-40, 5] eV weighted up to the
    mid-gap Fermi level of a small box of the same model."""
    import numpy as np
    import torch

    from paper_1002_1202_amd import api
    from synth import configs
    from synth.grids import trapezoid_weights

    if name == "slab8192":
        cfg = configs.slab8192()
        w, ef = cfg["w"], cfg["e_fermi"]
    elif name == "water3000":
        from oracle import ased as oased, spectral as ospec
        cfg = configs.water3000()
        small = configs.water_small(n_mol=8, n_rhs=4)["system"]
        S, H0, _ = oased.dense_pair(small)
        ev, _ = ospec.eig_pencil(H0, S)
        nocc = int(round(small.valence.sum() / 2))
        ef = float(0.5 * (ev[nocc - 1] + ev[nocc]))
        w = trapezoid_weights(cfg["z"]) * (cfg["z"].real <= ef)
    else:
        raise SystemExit(f"unknown forces workload {name}")
    if precision is not None:
        cfg["precision"] = precision
    s, z = cfg["system"], cfg["z"]
    ctx = api.Context(0)
    pair, scale = api.pair_from_system(ctx, s)
    shape = (pair.nnzb, pair.block, pair.block)
    dH = torch.zeros(shape, dtype=torch.float64, device="cuda:0")
    dS = torch.zeros_like(dH)
    print(f"forces {name}: N={s.n} K={len(z)} precision={cfg['precision']} tol={cfg['tol']}",
          file=sys.stderr, flush=True)
    # the gradient's columns split over slices of orbitals (each slice one
    # call; the slices add up to the full band energy and its gradient)
    slices = np.array_split(np.arange(s.n, dtype=np.int64), n_slices)
    E, iters, inner, work, conv = 0.0, 0, 0, 0, []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, orbs in enumerate(slices):
        _, _, e, info = api.band_energy_vjp(ctx, pair, z, w, 1.0, dH, dS, orbs=orbs, tol=cfg["tol"],
                                            precision=cfg["precision"], inner_relax=inner_relax)
        E += e
        iters = max(iters, info["outer_iters"])
        inner += info["inner_iters"]
        work += info["shift_rhs_iters"]
        conv.append(info["converged"])
        print(f"forces {name}: slice {i + 1}/{len(slices)} ({len(orbs)} orbitals) done at "
              f"{time.perf_counter() - t0:.1f} s, {info['outer_iters']} outer iterations", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    F = api.ased_vjp(ctx, pair, s, scale, dH, dS)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return {"metric": "band energy + forces, all orbitals", "workload": name,
            "system": f"{s.n_atoms} atoms, N={s.n}, nnzb={s.nnzb}, block={s.block}", "shifts": int(len(z)),
            "rhs": int(s.n), "slices": len(slices), "precision": cfg["precision"], "tol": cfg["tol"],
            "inner_relax": bool(inner_relax),
            "e_fermi": ef, "seconds_solve_with_gradients": t1 - t0, "seconds_forces_from_gradients": t2 - t1,
            "outer_iters": iters, "inner_iters": inner, "shift_rhs_iters": work,
            "value": work / (t1 - t0), "unit": UNIT,
            "converged_frac": float(np.mean(np.concatenate([c.ravel() for c in conv]))), "E_band": E,
            "max_abs_force": float(np.abs(F).max()), "abs_sum_force": float(np.abs(F.sum(0)).max())}


def copy_bandwidth(reps=10):
    """Measured device-to-device copy rate (GB/s, bytes read + written) of a
    1 GiB FP64 tensor, best of ``reps`` launches timed with events on torch's
    stream: the achievable streaming rate the roofline is also quoted
    against."""
    import torch
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    nbytes = 2 * a.numel() * 8
    del a, b
    torch.cuda.empty_cache()
    return nbytes / best / 1e9


def mixed_compare(ctx, pair, s, z, rhs, Gc, tol, knobs, fp64_result):
    """The timed step in mixed precision (FP64 seed process, complex64 inner
    rounds refined in FP64), fixed and relaxed inner tolerance, best of 2
    steps each, with every G element compared to the FP64 step's result."""
    import torch

    from paper_1002_1202_amd import api
    ref = Gc.clone()
    out = {"fp64_solve_ms": fp64_result.seconds * 1e3}
    for name, relax in (("fixed", False), ("inner_relax", True)):
        best = None
        for _ in range(2):
            api.ased_build(ctx, pair, s)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = api.solve(ctx, pair, z, rhs=rhs, out="device", out_cols=Gc, tol=tol, precision="mixed",
                           inner_relax=relax, **knobs)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if best is None or dt < best[0]:
                best = (dt, r)
        dt, r = best
        diff = float((Gc - ref).abs().max() / ref.abs().max())
        out[name] = {"ms_per_step": dt * 1e3, "value": r.shift_rhs_iters / dt, "outer_iters": r.outer_iters,
                     "inner_iters": r.inner_iters, "G_rel_diff_vs_fp64": diff,
                     "converged_frac": float(r.converged.mean())}
    Gc.copy_(ref)
    del ref
    torch.cuda.empty_cache()
    return out


def relax_compare(ctx, pair, s, z, rhs, Gc, tol, knobs):
    """The timed step again with the relaxed inner tolerance (option
    inner_relax, not the method's fixed inner tolerance): best of 2 steps,
    iterations, and the largest difference of any G element from the
    fixed-tolerance result of the last timed step (still in Gc)."""
    import numpy as np
    import torch

    from paper_1002_1202_amd import api

    Gr = torch.empty_like(Gc)
    best, r = float("inf"), None
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        api.ased_build(ctx, pair, s)
        r = api.solve(ctx, pair, z, rhs=rhs, out="device", out_cols=Gr, tol=tol, inner_relax=True, **knobs)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    d = g = 0.0
    for k in range(Gc.shape[0]):
        d = max(d, float((Gr[k] - Gc[k]).abs().max()))
        g = max(g, float(Gc[k].abs().max()))
    del Gr
    return {"ms_per_step": best * 1e3, "value": r.shift_rhs_iters / best, "unit": UNIT,
            "outer_iters": r.outer_iters, "inner_iters": r.inner_iters,
            "converged_frac": float(np.mean(r.converged)), "rel_diff_vs_fixed_inner_tol": d / g}


def host_output_step(ctx, pair, s, z, rhs, tol, knobs):
    """One step with G returned in host memory (GSC_MEM_HOST): the copy of
    every G column over PCIe is inside the timed region.  Reported beside
    the headline, which keeps its outputs in HBM."""
    import torch

    from paper_1002_1202_amd import api

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    api.ased_build(ctx, pair, s)
    r = api.solve(ctx, pair, z, rhs=rhs, out="host", tol=tol, **knobs)
    dt = time.perf_counter() - t0
    nbytes = r.G_cols.nbytes
    del r
    return {"ms_per_step": dt * 1e3, "value": None, "bytes_to_host": nbytes,
            "note": "G columns (complex128, K x R x N) copied to pageable host memory"}


def lanczos_compare(ctx, cfg):
    """G_jj of every right-hand side of the workload at every shift by the
    generalised Lanczos process + continued fraction (Sec. 3.2) and by the
    projected shifted COCG solver, same tolerance; best of 2 runs each."""
    import numpy as np
    import torch

    from paper_1002_1202_amd import api

    s, z, rhs, tol = cfg["system"], cfg["z"], cfg["rhs"], cfg["tol"]
    pair, _ = api.pair_from_system(ctx, s)
    best = {}
    for name in ("lanczos", "cocg_projected"):
        t_best, out = float("inf"), None
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if name == "lanczos":
                out = api.lanczos_green(ctx, pair, z, rhs, m_max=4000, tol=tol, check_every=16, out="device")
            else:
                out = api.solve(ctx, pair, z, rhs=rhs, tol=tol, carry="projected", proj=rhs[:, None], out="device")
            torch.cuda.synchronize()
            t_best = min(t_best, time.perf_counter() - t0)
        best[name] = (t_best, out)
    tl, lz = best["lanczos"]
    tc, co = best["cocg_projected"]
    # one more Lanczos run with every kernel timed (algorithmic bytes / time)
    api.profile_enable(ctx, True)
    api.lanczos_green(ctx, pair, z, rhs, m_max=4000, tol=tol, check_every=16, out="device")
    prof = api.profile_read(ctx)
    api.profile_enable(ctx, False)
    kernels = {k: {"ms": round(v[0], 3), "launches": v[1], "GB": round(v[2] / 1e9, 3),
                   "GB/s": round(v[2] / (v[0] * 1e-3) / 1e9, 1) if v[0] > 0 else None}
               for k, v in prof.items() if v[1] > 0}
    g1 = lz.G_diag.cpu().numpy()
    g2 = co.G_proj[:, :, 0].cpu().numpy()
    return {"workload": f"{cfg['name']} G_jj: {len(rhs)} rhs x {len(z)} shifts, tol {tol:g}",
            "lanczos": {"seconds": tl, "steps_min": int(lz.steps.min()), "steps_max": int(lz.steps.max()),
                        "inner_iters": int(lz.inner_iters),
                        "value": lz.shift_rhs_iters / tl, "unit": "shift·RHS·steps/s",
                        "kernels": kernels},
            "cocg_projected": {"seconds": tc, "outer_iters": int(co.outer_iters),
                               "value": co.shift_rhs_iters / tc, "unit": UNIT},
            "speedup_lanczos_vs_cocg": tc / tl,
            "rel_diff_G_jj": float(np.abs(g1 - g2).max() / np.abs(g2).max())}


def scc_measure(ctx):
    """Charge self-consistency (eq. Hap-CSC) end to end on small water boxes:
    8 molecules with a fixed integration window (E_F mid-gap of the neutral
    system, from the oracle's spectrum) and 24 molecules with E_F set each
    iteration by charge neutrality; both converge to 1e-9 e.  The oracle's
    loops (dense LU per shift, 1 thread) are timed beside them."""
    import numpy as np
    import torch
    from threadpoolctl import threadpool_limits

    from oracle import ased as oased, csc as ocsc, spectral as ospec
    from paper_1002_1202_amd import api
    from synth import configs
    from synth.csc import hubbard_u
    from synth.grids import shift_grid, trapezoid_weights

    out = {}
    small = configs.water_small(n_mol=8, n_rhs=4)["system"]
    S8, H8, _ = oased.dense_pair(small)
    ev, _ = ospec.eig_pencil(H8, S8)
    nocc = int(round(small.valence.sum() / 2))
    ef = 0.5 * (ev[nocc - 1] + ev[nocc])
    z_fixed = shift_grid(-60.0, ef, 128, 0.5)
    z_neutral = shift_grid(-60.0, 5.0, 128, 0.5)
    runs = (("water8_fixed_window", 8, z_fixed, trapezoid_weights(z_fixed), False, 4),
            ("water24_neutral", 24, z_neutral, None, True, 6))
    for name, n_mol, z, w, neutral, hist in runs:
        s = small if n_mol == 8 else configs.water_small(n_mol=n_mol, n_rhs=4)["system"]
        pair, _ = api.pair_from_system(ctx, s)
        cs = api.Csc(ctx, pair, s, hubbard_u(s))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = cs.scc(pair, z, w, s.valence, beta=0.2, history=hist, scc_tol=1e-9, max_iter=300, tol=1e-10,
                   neutral=neutral)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rec = {"atoms": int(s.n_atoms), "N": int(s.n), "shifts": int(len(z)), "neutral": neutral,
               "iterations": r["iterations"], "residual": r["residual"], "seconds": dt,
               "seconds_per_iteration": dt / r["iterations"], "converged": r["status"] == 0}
        if neutral:
            rec["e_fermi"] = r["e_fermi"]
        S, H0, _ = oased.dense_pair(s)
        gamma = ocsc.gamma_matrix(s, hubbard_u(s))
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            ref = ocsc.scc(s, S, H0, gamma, z, w, beta=0.2, tol=1e-9, max_iter=300, history=hist,
                           neutral=neutral)
            t_or = time.perf_counter() - t0
        rec["dq_max_diff_vs_oracle"] = float(np.abs(r["dq"] - ref[0]).max())
        rec["cpu_oracle"] = {"kind": "oracle", "cores": 1, "seconds": t_or, "iterations": ref[3]}
        out[name] = rec
    return out


def charge_vjp_measure(ctx):
    """Gradient of a charge loss on every orbital of a 64-molecule water box
    (two full-carry solves per orbital + the pattern contraction), next to
    the band-energy backward on the same system (z-derivative carry); with
    qbar = 1 and weights w E the two give the same gradient."""
    import numpy as np
    import torch

    from paper_1002_1202_amd import api
    from synth import configs

    c = configs.water_small(n_mol=64, n_rhs=4, n_shift=64, eta=0.2)
    s, z = c["system"], c["z"]
    w = np.full(len(z), (z[-1].real - z[0].real) / (len(z) - 1))
    pair, _ = api.pair_from_system(ctx, s)
    orbs = np.arange(s.n)
    out = {"workload": f"water64: N={s.n}, {len(z)} shifts, all orbitals, tol 1e-10"}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dH, dS, _ = api.charge_vjp(ctx, pair, z, w * z.real, orbs, np.ones(s.n))
    torch.cuda.synchronize()
    out["charge_vjp_seconds"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    eH, eS, _, _ = api.band_energy_vjp(ctx, pair, z, w)
    torch.cuda.synchronize()
    out["band_energy_vjp_seconds"] = time.perf_counter() - t0
    out["rel_diff"] = float(max(np.abs(dH - eH).max() / np.abs(eH).max(), np.abs(dS - eS).max() / np.abs(eS).max()))
    # the oracle's dense form of the same gradient, 1 thread
    from threadpoolctl import threadpool_limits

    from oracle import ased as oased, green as ogreen
    S, H, _ = oased.dense_pair(s)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        ogreen.charge_grad_dense(H, S, z, w * z.real, orbs, np.ones(s.n))
        out["cpu_oracle_seconds"] = time.perf_counter() - t0
    out["cpu_oracle"] = "oracle/green.py charge_grad_dense (dense inverses per shift), 1 thread"
    return out


def batched_compare(ctx, copy_gbs=None, tune=False):
    """The 32-system batched workload (projected carry: G_jj, charges and
    band-energy terms) at the workloads' tol 1e-6, timed for the mixed and
    the plain FP64 solver, each with and without the relaxed inner
    tolerance, and for the all-complex64 seed process.  Every run's error is
    measured against an FP64 reference at tol 1e-10 over all 32 systems
    (G_jj relative to max|G_jj|, charges in e); the reference itself against
    the dense-LU oracle on sampled shifts of the systems with N <= 8192.
    Speed-ups are stated only between runs that meet 1e-6 on G_jj and
    1e-5 e on the charges.  Algorithmic bytes come from the library's count
    of column-iterations (no events inside the captured graphs).  With
    ``tune`` the autotuner first searches the batch's tile and launch shapes
    for the mixed solver, and the mixed runs are repeated with them."""
    import numpy as np
    import torch

    from oracle import ased as oased, green as ogreen
    from paper_1002_1202_amd import api
    from synth import configs
    from synth.grids import trapezoid_weights

    b = configs.batch32()
    probs = []
    for it in b["items"]:
        pair, _ = api.pair_from_system(ctx, it["system"])
        probs.append(dict(pair=pair, z=it["z"], rhs=it["rhs"], w=trapezoid_weights(it["z"])))
    ns = [p["pair"].n for p in probs]
    out = {"workload": f"batch32: 32 Si systems (N {min(ns)}..{max(ns)}, K 128..1024, R 64..512), "
                       "tol 1e-6, projected carry, graph chunks of 4 iterations"}
    if copy_gbs is None:
        copy_gbs = copy_bandwidth()

    def run(prec, tol=1e-6, relax=False, shapes=None):
        shapes = dict(shapes or {})
        shapes.setdefault("graph_iters", 4)
        api.solve_batched(ctx, probs[:2], tol=tol, precision=prec, max_iter=4, inner_relax=relax)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o = api.solve_batched(ctx, probs, tol=tol, precision=prec, inner_relax=relax, **shapes)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        work = sum(x["shift_rhs_iters"] for x in o)
        by = sum(x["alg_bytes"] for x in o)
        bi = sum(x["alg_bytes_inner"] for x in o)
        rec = {"precision": prec, "tol": tol, "inner_relax": relax, "shapes": shapes, "seconds": dt,
               "value": work / dt,
               "unit": UNIT, "max_outer_iters": max(x["outer_iters"] for x in o),
               "inner_steps": sum(x["inner_iters"] for x in o),
               "converged_frac": float(np.mean([x["converged"].mean() for x in o])),
               "alg_GB": by / 1e9, "inner_share": bi / by if by > 0 else None,
               "roofline_whole_path": {"achieved": by / dt / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                       "frac": by / dt / 1e9 / HBM_PEAK_GBS,
                                       "frac_of_copy": by / dt / 1e9 / copy_gbs}}
        print(f"batched {prec} tol {tol:g} relax={relax}: {dt:.2f} s, {work / dt:.3e} shift-rhs-it/s, "
              f"{by / dt / 1e9:.0f} GB/s algorithmic", file=sys.stderr, flush=True)
        return rec, [(x["G_jj"].cpu().numpy(), x["q"].cpu().numpy(), x["e"].cpu().numpy()) for x in o]

    runs = {}
    plan = [("mixed", "mixed", False, None), ("mixed_relax", "mixed", True, None),
            ("fp64", "fp64", False, None), ("fp64_relax", "fp64", True, None), ("c64", "c64", False, None)]
    if tune:
        from paper_1002_1202_amd import autotune
        t0 = time.perf_counter()
        best = autotune.tune_batched(ctx, probs, precision="mixed", tol=1e-6, force=True, verbose=True)
        out["autotune"] = {"shapes": best, "seconds": time.perf_counter() - t0,
                           "space": autotune.SPACE_BATCHED}
        print(f"batched autotune: {best}", file=sys.stderr, flush=True)
        plan += [("mixed_tuned", "mixed", False, best), ("mixed_relax_tuned", "mixed", True, best)]
    for name, prec, relax, shapes in plan:
        runs[name] = run(prec, relax=relax, shapes=shapes)
    ref_rec, ref = run("fp64", tol=1e-10)
    out["reference"] = ref_rec
    # the reference against the dense-LU oracle on 4 sampled shifts of the
    # systems small enough for a dense factorisation
    small = [i for i in np.argsort(ns) if ns[i] <= 8192][:3]
    errs = []
    for i in small:
        it = b["items"][i]
        S, H, _ = oased.dense_pair(it["system"])
        ks = np.linspace(0, len(it["z"]) - 1, 4).astype(int)
        X = ogreen.solve_dense(H, S, it["z"][ks], it["rhs"])
        g0 = X[:, np.arange(len(it["rhs"])), it["rhs"]]
        errs.append(float(np.abs(ref[i][0][ks] - g0).max() / np.abs(g0).max()))
    out["reference"]["err_vs_oracle_sampled"] = {"G_jj_rel": max(errs), "systems_N": [int(ns[i]) for i in small],
                                                 "shifts_per_system": 4}
    for name, (rec, res) in runs.items():
        rec["err_vs_reference"] = {
            "G_jj_rel": max(float(np.abs(g - gr).max() / np.abs(gr).max()) for (g, _, _), (gr, _, _) in zip(res, ref)),
            "charge_abs_e": max(float(np.abs(q - qr).max()) for (_, q, _), (_, qr, _) in zip(res, ref)),
            "band_energy_term_abs_eV": max(float(np.abs(e - er).max()) for (_, _, e), (_, _, er) in zip(res, ref))}
        rec["meets_1e-6"] = bool(rec["err_vs_reference"]["G_jj_rel"] <= 1e-6
                                 and rec["err_vs_reference"]["charge_abs_e"] <= 1e-5)
        out[name] = rec
    sec = {k: out[k]["seconds"] for k in runs}
    ok = {k: out[k]["meets_1e-6"] for k in runs}
    out["speedup_at_1e-6"] = {
        "mixed_vs_fp64": sec["fp64"] / sec["mixed"] if ok["mixed"] and ok["fp64"] else None,
        "mixed_relax_vs_fp64_relax": (sec["fp64_relax"] / sec["mixed_relax"]
                                      if ok["mixed_relax"] and ok["fp64_relax"] else None),
        "mixed_relax_vs_plain_fp64": sec["fp64"] / sec["mixed_relax"] if ok["mixed_relax"] and ok["fp64"] else None}
    if tune:
        out["speedup_at_1e-6"].update({
            "mixed_tuned_vs_fp64": sec["fp64"] / sec["mixed_tuned"] if ok["mixed_tuned"] and ok["fp64"] else None,
            "mixed_relax_tuned_vs_plain_fp64": (sec["fp64"] / sec["mixed_relax_tuned"]
                                                if ok["mixed_relax_tuned"] and ok["fp64"] else None)})
    return out


def member_measure(ctx, index, precision, tol=1e-6, relax=False):
    """One member of the 32-system batch alone (projected carry, G_jj and
    the S e_j projection, tol 1e-6), one warm-up and one timed solve with
    every kernel timed by HIP events on the library's stream: per-kernel
    algorithmic GB/s and the dominant kernel's roofline.  The largest
    member (index 31, N = 131072) has streamed vectors far beyond the 256 MB
    infinity cache."""
    import torch

    from paper_1002_1202_amd import api
    from synth import configs

    it = configs.batch32()["items"][index]
    s, z, rhs = it["system"], it["z"], it["rhs"]
    pair, _ = api.pair_from_system(ctx, s)
    kw = dict(tol=tol, precision=precision, carry="projected", proj=rhs[:, None], inner_relax=relax)
    api.solve(ctx, pair, z, rhs=rhs, max_iter=3, **kw)
    api.profile_enable(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = api.solve(ctx, pair, z, rhs=rhs, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    p = api.profile_read(ctx)
    api.profile_enable(ctx, False)
    dom = max(p, key=lambda k: p[k][0])
    ms, n, by = p[dom]
    copy_gbs = copy_bandwidth()
    achieved = by / (ms * 1e-3) / 1e9
    from paper_1002_1202_amd import rocprof_summary
    traffic = None
    if dom in rocprof_summary.KERNEL_SOURCES:
        traffic = rocprof_summary.read_traffic(
            os.path.join(ROOT, "profiles", f"batch32_member{index}_{dom}_traffic.md"), dom)
    return {"workload": f"batch32 member {index}: N={s.n}, K={len(z)}, R={len(rhs)}, projected carry",
            "precision": precision, "tol": tol, "inner_relax": relax, "seconds": dt,
            "value": r.shift_rhs_iters / dt, "unit": UNIT, "outer_iters": r.outer_iters,
            "inner_iters": r.inner_iters,
            "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "copy_gbs_measured": copy_gbs,
                         "frac_of_copy": achieved / copy_gbs, "bytes_per_launch": by / max(n, 1),
                         "avg_launch_ms": ms / max(n, 1), "traffic": traffic},
            "kernels": {k: {"ms": round(v[0], 3), "launches": v[1], "GB": round(v[2] / 1e9, 3),
                            "GB/s": round(v[2] / (v[0] * 1e-3) / 1e9, 1) if v[0] > 0 else None}
                        for k, v in p.items() if v[1] > 0}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="si4096")
    ap.add_argument("--fuse", type=int, default=16)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed", "c64"])
    ap.add_argument("--tol", type=float, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=300)
    ap.add_argument("--spmm", type=int, default=0,
                    help="0 auto, 1 row kernel (the only layout)")
    ap.add_argument("--inner", type=int, default=0, help="0 auto, 1 CG, 2 Chebyshev")
    ap.add_argument("--autotune", action="store_true",
                    help="time the candidate launch shapes on this problem first and use the fastest")
    ap.add_argument("--member", type=int, default=31,
                    help="with --only member: the batch32 member (default 31, the largest)")
    ap.add_argument("--only", default=None, choices=["batched", "lanczos", "member"],
                    help="instead of the throughput line: only the batched mixed-vs-FP64 comparison or only "
                         "the Lanczos-vs-COCG comparison (its own JSON line; for per-workload profiles)")
    ap.add_argument("--forces", default=None, choices=["slab8192", "water3000"],
                    help="instead of the throughput line: one band energy + forces step over every "
                         "orbital of a full-size workload (its own JSON line)")
    ap.add_argument("--forces-precision", default=None, choices=["fp64", "mixed", "c64"],
                    help="override the forces workload's precision (slab8192: fp64, water3000: mixed)")
    ap.add_argument("--forces-inner-relax", action="store_true",
                    help="run the forces workload with the relaxed inner tolerance (option inner_relax)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the timed step in mixed precision on the same workload")
    ap.add_argument("--extras", action="store_true",
                    help="also time the Lanczos comparison, the SCC loop, the charge-loss adjoint and the "
                         "step with G returned to host memory")
    ap.add_argument("--no-dense-lu", action="store_true",
                    help="skip timing the dense-LU oracle on the host (one shift, all BLAS threads)")
    ap.add_argument("--no-lanczos", action="store_true")
    ap.add_argument("--no-host-output", action="store_true",
                    help="skip the step that returns G in host memory (PCIe-inclusive)")
    ap.add_argument("--no-relax", action="store_true",
                    help="skip the timed step with the relaxed inner tolerance")
    ap.add_argument("--no-scc", action="store_true")
    ap.add_argument("--no-charge-vjp", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a copy-like kernel over 1 GiB first (torch.neg: 1 GiB read, 1 GiB written), "
                         "which calibrates the HBM byte counters of a --pmc run")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU only (no collectives, no sharding); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1002_1202_amd import api

    if args.copy_probe:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        torch.neg(a, out=b)
        torch.cuda.synchronize()
        print(f"copy probe: {a.numel() * 8} bytes read and written", file=sys.stderr, flush=True)
        del a, b
    if args.forces:
        print(json.dumps(forces_measure(args.forces, precision=args.forces_precision,
                                        inner_relax=args.forces_inner_relax)), flush=True)
        return
    if args.only == "batched":
        print(json.dumps(batched_compare(api.Context(0), tune=args.autotune)), flush=True)
        return
    if args.only == "member":
        print(json.dumps(member_measure(api.Context(0), args.member, args.precision, tol=args.tol or 1e-6)),
              flush=True)
        return
    if args.only == "lanczos":
        print(json.dumps(lanczos_compare(api.Context(0), workload(args.workload))), flush=True)
        return
    cfg = workload(args.workload)
    if args.tol is None:
        args.tol = cfg["tol"]
    s = cfg["system"]
    z, rhs = cfg["z"], cfg["rhs"]
    K, R, N = len(z), len(rhs), s.n
    ctx = api.Context(0)
    pair = api.Pair(ctx, s.block, s.rowptr, s.colidx)
    Gc = torch.empty((K, R, N), dtype=torch.complex128, device="cuda:0")

    knobs = dict(fuse_steps=args.fuse, spmm_kernel=args.spmm, inner_method=args.inner)
    tuned = None
    if args.autotune:
        from paper_1002_1202_amd import autotune
        api.ased_build(ctx, pair, s)
        tuned = autotune.tune_solve(ctx, pair, z, rhs, precision=args.precision, carry="full", tol=args.tol,
                                    verbose=True, force=True)
        knobs.update(tuned)
        print(f"autotuned: {tuned}", file=sys.stderr, flush=True)

    def step():
        api.ased_build(ctx, pair, s)
        return api.solve(ctx, pair, z, rhs=rhs, out="device", out_cols=Gc, tol=args.tol,
                         precision=args.precision, **knobs)

    # warmup; the first warmup step times every kernel to find the dominant one
    dom = None
    for i in range(max(args.warmup, 1)):
        if i == 0:
            api.profile_enable(ctx, True)
        r = step()
        if i == 0:
            pw = api.profile_read(ctx)
            dom = max(pw, key=lambda k: pw[k][0])
            api.profile_enable(ctx, False)
        print(f"warmup {i}: iters={r.outer_iters} switches={r.switches} "
              f"inner={r.inner_iters} conv={r.converged.mean():.3f} dev_s={r.seconds:.3f}",
              file=sys.stderr, flush=True)
    print("warmup kernel split (ms): " + ", ".join(f"{k}={v[0]:.1f}" for k, v in pw.items() if v[1]),
          file=sys.stderr, flush=True)
    # timed steps: HIP events around the dominant kernel only
    api.profile_enable(ctx, True, only=dom)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results, step_s = [], []
    for i in range(args.steps):
        ts = time.perf_counter()
        r = step()
        torch.cuda.synchronize()
        step_s.append(time.perf_counter() - ts)
        results.append(r)
        print(f"step {i}: iters={r.outer_iters} switches={r.switches} dev_s={r.seconds:.3f}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = api.profile_read(ctx)
    api.profile_enable(ctx, False)

    work = sum(r.shift_rhs_iters for r in results)
    value = work / dt
    total_bytes = sum(v[2] for v in prof.values())
    ms, launches, byts = prof[dom]
    achieved = (byts / (ms * 1e-3)) / 1e9 if ms > 0 else 0.0
    from paper_1002_1202_amd import rocprof_summary
    traffic = None
    if dom in rocprof_summary.KERNEL_SOURCES:
        traffic = rocprof_summary.read_traffic(
            os.path.join(ROOT, "profiles", f"{cfg['name']}_{dom}_traffic.md"), dom)
    copy_gbs = copy_bandwidth()
    kernels = {k: {"warmup_ms": round(v[0], 3), "launches": v[1], "GB": round(v[2] / 1e9, 3),
                   "GB/s": round(v[2] / (v[0] * 1e-3) / 1e9, 1) if v[0] > 0 else None,
                   "frac_of_copy": round(v[2] / (v[0] * 1e-3) / 1e9 / copy_gbs, 3) if v[0] > 0 else None}
               for k, v in pw.items() if v[1] > 0}
    line = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "ms_per_step_median": float(np.median(step_s)) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "mixed": "f64 seed process, c64 inner rounds refined in f64",
                  "c64": "c64 vectors and products, f64 recurrences"}[args.precision],
        "data": "synthetic",
        "config": describe(cfg, args),
        "hbm_gbs_algorithmic": total_bytes / dt / 1e9,
        "outer_iters": results[-1].outer_iters,
        "shift_rhs_iters_per_step": results[-1].shift_rhs_iters,
        "nominal_K_R_iters_per_step": K * R * results[-1].outer_iters,
        "switches": results[-1].switches,
        "inner_iters": results[-1].inner_iters,
        "converged_frac": float(np.mean(results[-1].converged)),
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "copy_gbs_measured": copy_gbs, "frac_of_copy": achieved / copy_gbs,
                     "bytes_per_launch": byts / max(launches, 1),
                     "avg_launch_ms": ms / max(launches, 1), "traffic": traffic},
        "kernels": kernels,
    }
    line["config"].update({k: v for k, v in knobs.items()})
    line["config"]["autotuned"] = tuned is not None
    if not args.no_relax and args.precision == "fp64":
        line["inner_relax"] = relax_compare(ctx, pair, s, z, rhs, Gc, args.tol, knobs)
        print(f"inner_relax: {line['inner_relax']}", file=sys.stderr, flush=True)
    if not args.no_mixed and args.precision == "fp64":
        line["mixed"] = mixed_compare(ctx, pair, s, z, rhs, Gc, args.tol, knobs, results[-1])
        print(f"mixed: {line['mixed']}", file=sys.stderr, flush=True)
    if args.extras and not args.no_host_output:
        line["host_output"] = host_output_step(ctx, pair, s, z, rhs, args.tol, knobs)
        line["host_output"]["value"] = results[-1].shift_rhs_iters / (line["host_output"]["ms_per_step"] * 1e-3)
        print(f"host output: {line['host_output']['ms_per_step']:.0f} ms per step", file=sys.stderr, flush=True)
    del Gc
    torch.cuda.empty_cache()
    if args.extras and not args.no_lanczos:
        line["lanczos"] = lanczos_compare(ctx, cfg)
        print(f"lanczos: {line['lanczos']['lanczos']['seconds']:.3f} s vs projected COCG "
              f"{line['lanczos']['cocg_projected']['seconds']:.3f} s", file=sys.stderr, flush=True)
    if args.extras and not args.no_scc:
        line["scc"] = scc_measure(ctx)
        print(f"scc: {line['scc']}", file=sys.stderr, flush=True)
    if args.extras and not args.no_charge_vjp:
        line["charge_vjp"] = charge_vjp_measure(ctx)
        print(f"charge_vjp: {line['charge_vjp']}", file=sys.stderr, flush=True)
    if not args.no_batched:
        line["batched"] = batched_compare(ctx, copy_gbs, tune=args.autotune)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_iters)
        print(f"cpu baseline: {line['cpu_baseline']['sample']}", file=sys.stderr, flush=True)
        if not args.no_dense_lu:
            line["cpu_dense_lu"] = cpu_dense_lu(cfg)
            print(f"cpu dense LU: {line['cpu_dense_lu']}", file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
