"""Benchmark of the grid-embedded FFT BEM operator on one MI355X.

Workload: 3D Laplace, FP32 transforms, unit-cube surface with 100 grid points
per edge (58,808 nodes) voxelised on a 128^3 grid, FFT padded to 256^3.  One
step = one apply r = c u + D[u] - S[q] (all four kernels) on device-resident
inputs; value = applies per second.  Also reported: per-stage HIP-event
times and the roofline of the dominant stage, the sphere (R = 0.35) and FP64
variants, GMRES time-to-solve at relative true residual 1e-6 for the mixed
problem (Dirichlet above the centre, Neumann below), and the CPU oracle on a
bounded sample of targets.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import math
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "BEM matvecs/s + GMRES time-to-solve @1e-6 rel. residual; HBM roofline fraction"
HBM_PEAK_GBS = 8000.0


def model_bytes(info, b):
    """The byte model of one apply (b = bytes per stored real): per field
    f = Hx Ny Nz 2b (the x-pass half spectrum), g = Hx Py Nz 2b (after the
    y pass); forward x, y: F (2f + g); fused z pass with the products:
    F g + K Hx Hy Hz b + O g; inverse y, x: O (g + 2f).  It credits the
    zero padding, the half spectrum, the octant spectra and the fused scatter
    and gather, not the occupancy of the boundary."""
    px, py, pz = info["pad"]
    hx, hy, hz = px // 2 + 1, py // 2 + 1, pz // 2 + 1
    ny, nz = info["n"][1], info["n"][2]
    F, K, O = info["nfields"], info["nspectra"], info["noutputs"]
    f = hx * ny * nz * 2 * b
    g = hx * py * nz * 2 * b
    return {"forward_xy": F * (2 * f + g), "zpass": F * g + K * hx * hy * hz * b + O * g,
            "inverse_yx": O * (g + 2 * f)}


def zpass_roofline(info, b, ms, kernel):
    """Roofline object of the z pass: the model's bytes (model_bytes) over
    its measured time, and the bytes the design must move (occupied planes
    only) beside it."""
    mb = model_bytes(info, b)["zpass"]
    moved = stage_bytes(info, b)["zpass"]
    gbs = mb / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": kernel, "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "model_bytes": mb, "ms": ms,
            "occupied_planes_bytes": moved, "frac_occupied_planes_bytes": moved / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}


def stage_bytes(info, prec_bytes, arith_bytes=None):
    """Bytes of each stage of this design for one apply (the bytes each
    kernel must read or write once, occupied planes only; node data O(M)
    included).  prec_bytes: stored real (Y, Z, spectra); arith_bytes: real
    of the inverse-y rows and the node fields (default prec_bytes)."""
    ab = arith_bytes or prec_bytes
    px, py, pz = info["pad"]
    hx, hy, hz = px // 2 + 1, py // 2 + 1, pz // 2 + 1
    nzo = info["z_count"]
    F, K, O, m = info["nfields"], info["nspectra"], info["noutputs"], info["m"]
    cb = 2 * prec_bytes
    g = hx * nzo * py * cb                     # one complex field after the y transform
    spec = info["spectra_bytes"]               # octant spectra as stored
    nodes_in = m * (8 * 2 * info["ncomp"] + 4 * 4 + 8 * 4)
    ny = info["n"][1]
    w = O * hx * ny * nzo * 2 * ab             # inverse-y rows y < ny, kx contiguous
    return {
        "fwd_xy": F * g + nodes_in,
        "zpass": F * g + spec + O * g,
        "inv_y": O * g + w,
        # each row read once; per node: indices, c and self-term blocks, u, q, r
        "gather": w + m * (4 * 4 + 8 * 2 * O * O + 8 * 3 * O),
    }


def measured_traffic(workload, kernel):
    """HBM bytes per launch of 'kernel' from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by its copy-kernel
    calibration factor), or None when the sources of the apply kernels have
    changed since the counters were taken."""
    from paper_1809_00845_amd.profile_summary import apply_sources_sha256

    path = os.path.join(ROOT, "profiles", "apply_laplace3d_cube128_fp32_counters.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("workload") != workload or rec.get("csrc_sha256") != apply_sources_sha256():
        return None
    k = rec["kernels"].get("k_" + kernel)
    return None if k is None else k["read_bytes"] + k["write_bytes"]


def zpass_alu_view(info, ms):
    """The z pass against the FP32 vector units: 5 P log2 P flops per complex
    transform (4 forward, 1 inverse per pencil for Laplace 3D) plus 4 flops
    per spectral product, over Hx * Py pencils.  Packed FP32 instructions are
    not used, so the peak is half the chip's 157.3 TFLOP/s."""
    P = info["pad"][2]
    hx, py = info["pad"][0] // 2 + 1, info["pad"][1]
    per_pencil = 5 * 5 * P * math.log2(P) + 4 * info["nspectra"] * P
    flops = per_pencil * hx * py
    tf = flops / (ms * 1e-3) / 1e12
    return {"flops": flops, "achieved_tflops": tf, "peak_tflops_unpacked_fp32": 78.65, "frac": tf / 78.65}


def bench_grid_eval(plan, q, u, info, steps):
    """S[q] - D[u] over the whole grid box (the representation formula
    inside the boundary), FP64 out.  The evaluation shares the apply's
    forward passes, z pass and inverse y pass; its own last stage is the
    inverse x transform of two grid rows per pencil (k_vol_x), whose
    kernel time is in the rocprofv3 summary."""
    import torch

    out = None
    for _ in range(3):
        out = plan.eval_grid(q, u, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.eval_grid(q, u, out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    nx, ny, nzo, O = info["n"][0], info["n"][1], info["z_count"], info["noutputs"]
    return {"ms_per_eval": ms, "grid_points": nx * ny * nzo, "points_per_s": nx * ny * nzo * O / (ms * 1e-3)}


def bench_dirichlet_cg(B, I, dev):
    """The paper's solver (end of Sec. 4): CG on the symmetrised Dirichlet
    single-layer system, against GMRES on the same problem, both FP64 to a
    1e-6 relative residual.  The 2D square is the paper's Fig. 6 setting:
    500 grid points per side on a 500^2 grid (1024-point transforms); the
    sphere is the 128^3 one."""
    import torch

    res = {}
    for name, g, kind, harm in (("square2d_500_per_side_500sq", I.square2d(500, 500), B.LAPLACE2D,
                                 I.harmonic_2d_x2y2),
                                ("sphere_128cubed", I.sphere3d(128, 0.35), B.LAPLACE3D, I.harmonic_3d_xyz)):
        u = torch.tensor(harm(g)[0], device=dev)
        plan = B.Plan(g, kind, precision=B.FP64)
        bc = torch.zeros(g.m, dtype=torch.uint8, device=dev)
        row = {"nodes": g.m}
        for tag, fn in (("cg_jacobi", lambda: plan.solve_cg(u, tol=1e-6, precond=1)),
                        ("cg_plain", lambda: plan.solve_cg(u, tol=1e-6, precond=0)),
                        ("gmres_jacobi", lambda: plan.solve(bc, u, tol=1e-6))):
            fn()  # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, inf = fn()
            torch.cuda.synchronize()
            row[tag] = {"seconds": time.perf_counter() - t0, "iters": inf["iters"],
                        "true_relres": inf["true_relres"], "status": inf["status"]}
        plan.close()
        res[name] = row
    return res


def bench_halfspace(B, I, dev, steps):
    """The elastic half-space of eq. (9) on the 256^2 surface (P = 512): the
    convolution the paper starts from, run on the same engine.  Applies
    with loads on every grid point (FP32, FP64), and the frictionless Hertz
    contact on a disc of radius 0.3 (normal displacement given, shear
    traction zero) solved to 1e-6."""
    import torch

    nu, mu = 0.3, 1.0
    out = {}
    g = I.halfspace_patch(256)
    rng = np.random.default_rng(0)
    q = torch.tensor(rng.uniform(-1, 1, (3, g.m)), device=dev)
    u = torch.zeros_like(q)
    r = torch.empty_like(q)
    for tag, prec in (("fp32", B.FP32), ("fp64", B.FP64)):
        pl = B.Plan(g, B.HALFSPACE, precision=prec, nu=nu, mu=mu)
        out[f"full_surface_{tag}_matvec_s"] = steps / timed_applies(pl, q, u, r, steps, 5)
        pl.close()
    a, p0, E = 0.3, 1.0, 2 * mu * (1 + nu)
    gd = I.halfspace_patch(256, a)
    rr = np.sum((gd.nodes - gd.center) ** 2, axis=1)
    bc = np.zeros((3, gd.m), dtype=np.uint8)
    bc[:2] = 1
    known = np.zeros((3, gd.m))
    known[2] = np.pi * (1 - nu ** 2) * p0 * (2 * a ** 2 - rr) / (4 * a * E)
    bct = torch.tensor(bc.reshape(-1), device=dev)
    kt = torch.tensor(known.reshape(-1), device=dev)
    pl = B.Plan(gd, B.HALFSPACE, precision=B.FP64, nu=nu, mu=mu)
    pl.solve(bct, kt, tol=1e-6)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, inf = pl.solve(bct, kt, tol=1e-6)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pz = x.cpu().numpy().reshape(3, gd.m)[2]
    ex = p0 * np.sqrt(np.clip(1 - rr / a ** 2, 0, None))
    inner = rr < (0.8 * a) ** 2
    out["hertz_disc_solve_fp64"] = {"nodes": gd.m, "seconds": dt, "iters": inf["iters"],
                                    "true_relres": inf["true_relres"],
                                    "pressure_err_inner": float(np.abs(pz[inner] - ex[inner]).max() / p0),
                                    "force_ratio": float(np.sum(pz * gd.weights) / (2 * np.pi * a * a * p0 / 3))}
    pl.close()
    out["nodes_full_surface"] = g.m
    return out


def median_apply_ms(plan, q, u, r, n=100):
    """Median of n single applies, each bracketed by HIP events on the
    stream the apply is queued on."""
    import torch

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for _ in range(5):
        plan.apply(q, u, r)
    for a, b in evs:
        a.record()
        plan.apply(q, u, r)
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in evs]))


def timed_applies(plan, q, u, r, steps, warmup):
    import torch

    for _ in range(warmup):
        plan.apply(q, u, r)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.apply(q, u, r)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def cpu_baseline(geom, q, u, budget_s=12.0):
    import oracle as O

    p = O.problem(geom, O.LAPLACE3D)
    t = time.perf_counter()
    O.apply(p, q, u, targets=(0, 200))
    per = (time.perf_counter() - t) / 200.0
    nt = int(max(200, min(geom.m, budget_s / max(per, 1e-9))))
    t = time.perf_counter()
    O.apply(p, q, u, targets=(0, nt))
    dt = time.perf_counter() - t
    full = dt / nt * geom.m
    return {"value": 1.0 / full, "unit": "matvec/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"direct-sum FP64 oracle on targets 0..{nt} of {geom.m} (all sources), "
                      f"{dt:.1f} s, scaled to one full apply ({full:.1f} s)"}


def bench_batched(B, I, dev, steps=20, count=64, nrhs=4):
    """64 star surfaces (seed 2) on grids drawn from {64, 96, 128, 160}^3,
    4 right-hand sides each (Dirichlet data from random harmonic polynomials
    of degree <= 3): batched FP32 apply (graph replay) against per-plan
    applies, and batched lockstep GMRES to 1e-6 against the same members
    solved one at a time, at equal precision (FP32 and FP64)."""
    import tempfile

    import torch

    t0 = time.perf_counter()
    items = I.draw_batch(2, count)
    geoms = I.star_batch(items)
    t_geom = time.perf_counter() - t0
    tune = tempfile.NamedTemporaryFile(prefix="bemfft_tune_", delete=False)
    tune.close()
    os.environ["BEMFFT_TUNE_CACHE"] = tune.name
    t0 = time.perf_counter()
    plans = [B.Plan(g, B.LAPLACE3D, precision=B.FP32, autotune=1) for g in geoms]
    t_plan = time.perf_counter() - t0
    t0 = time.perf_counter()
    batch = B.Batch(plans, nrhs=nrhs, use_graph=True)
    t_batch = time.perf_counter() - t0
    rng = np.random.default_rng(20)
    known, bcs = [], []
    for g in geoms:
        for _ in range(nrhs):
            u, _ = I.random_harmonic_3d(g, rng)
            known.append(u)
            bcs.append(np.zeros(g.m, dtype=np.uint8))
    known = torch.tensor(np.concatenate(known), device=dev)
    bcs = torch.tensor(np.concatenate(bcs), device=dev)
    q = torch.zeros_like(known)
    r = torch.empty_like(known)
    nm = len(batch.offsets)
    for _ in range(3):
        batch.apply(q, known, r)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.apply(q, known, r)
    torch.cuda.synchronize()
    dt_b = (time.perf_counter() - t0) / steps
    # the same members one plan call at a time
    views = [(p, batch.offsets[k], batch.lengths[k]) for k, p in
             enumerate([pl for pl in plans for _ in range(nrhs)])]
    qv = [q[o:o + n] for _, o, n in views]
    uv = [known[o:o + n] for _, o, n in views]
    rv = [r[o:o + n] for _, o, n in views]
    for (p, _, _), a, b_, c in zip(views, qv, uv, rv):
        p.apply(a, b_, c)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = max(2, steps // 5)
    for _ in range(reps):
        for (p, _, _), a, b_, c in zip(views, qv, uv, rv):
            p.apply(a, b_, c)
    torch.cuda.synchronize()
    dt_s = (time.perf_counter() - t0) / reps
    # solves at equal precision: batched lockstep GMRES against the same
    # members solved one at a time, in FP32 and in FP64
    def seq_solves(plan_list):
        total, iters = 0.0, []
        for p_ in plan_list:
            o, n = batch.offsets[len(iters)], batch.lengths[len(iters)]
            p_.solve(bcs[o:o + n].contiguous(), known[o:o + n].contiguous(), tol=1e-6, restart=100,
                     maxit=1000)  # warm: the plan's solve workspace
            for _ in range(nrhs):
                kk = len(iters)
                o, n = batch.offsets[kk], batch.lengths[kk]
                bck = bcs[o:o + n].contiguous()
                knk = known[o:o + n].contiguous()
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                _, si = p_.solve(bck, knk, tol=1e-6, restart=100, maxit=1000)
                torch.cuda.synchronize()
                total += time.perf_counter() - t1
                iters.append(si["iters"])
        return total, iters

    def batched_solve(bt):
        x = torch.zeros_like(known)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st_, info_ = bt.solve(bcs, known, x, tol=1e-6, restart=100, maxit=1000)
        torch.cuda.synchronize()
        return time.perf_counter() - t1, st_, info_

    batched_solve(batch)  # warm: workspace of the batch
    t_bsolve, st, sinfo = batched_solve(batch)
    its = [i["iters"] for i in sinfo]
    t_seq32, seq32_its = seq_solves(plans)
    p64s = [B.Plan(g, B.LAPLACE3D, precision=B.FP64) for g in geoms]
    batch64 = B.Batch(p64s, nrhs=nrhs, use_graph=True)
    batched_solve(batch64)  # warm: workspace of the FP64 batch
    t_b64, st64, sinfo64 = batched_solve(batch64)
    t_seq, seq_its = seq_solves(p64s)
    batch64.close()
    for p_ in p64s:
        p_.close()
    os.unlink(tune.name)
    sizes = sorted(set(n for n, _ in items))
    out = {
        "workload": "64 star surfaces (seed 2), grids {64,96,128,160}^3 padded 2N, 4 Dirichlet RHS each",
        "members": nm, "nodes_total": int(sum(g.m for g in geoms)),
        "grid_counts": {str(n): sum(1 for m_, _ in items if m_ == n) for n in sizes},
        "groups_by_pad_and_schedule": len(set((p.info()["pad"][0], p.info()["zsched"]) for p in plans)),
        "batched_apply_ms": dt_b * 1e3, "batched_rhs_matvec_s": nm / dt_b,
        "per_plan_apply_ms": dt_s * 1e3, "per_plan_rhs_matvec_s": nm / dt_s,
        "batched_solve_fp32_s": t_bsolve, "batched_solve_status": st,
        "batched_solve_iters_max": int(max(its)), "batched_solve_iters_mean": float(np.mean(its)),
        "batched_solve_relres_max": float(max(i["true_relres"] for i in sinfo)),
        "sequential_fp32_solves_s": t_seq32, "sequential_fp32_iters_mean": float(np.mean(seq32_its)),
        "batched_vs_sequential_fp32": t_seq32 / t_bsolve,
        "batched_solve_fp64_s": t_b64, "batched_solve_fp64_status": st64,
        "batched_solve_fp64_iters_mean": float(np.mean([i["iters"] for i in sinfo64])),
        "batched_solve_fp64_relres_max": float(max(i["true_relres"] for i in sinfo64)),
        "sequential_fp64_solves_s": t_seq, "sequential_fp64_iters_mean": float(np.mean(seq_its)),
        "batched_vs_sequential_fp64": t_seq / t_b64,
        "setup_s": {"voxelise": t_geom, "plans": t_plan, "batch_and_graph": t_batch},
    }
    batch.close()
    for p in plans:
        p.close()
    return out


def bench_navier_star(B, I, dev, steps, mixed=True):
    """Navier (Kelvin, nu = 0.3, mu = 1) on the star surface of seed 1 on a
    192^3 grid padded to 384^3: FP32, FP64 and 16-bit (BF16 storage, z
    transforms on the matrix cores) applies with the z pass against the HBM
    roofline, and time to solve for the traction under a given linear
    displacement field, to 1e-6 (plan + solve and solve alone)."""
    import torch

    t0 = time.perf_counter()
    g = I.star3d(192, I.draw_stars(1, 1)[0])
    t_geom = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    q = torch.tensor(rng.uniform(-1, 1, (3, g.m)), device=dev)
    u = torch.tensor(rng.uniform(-1, 1, (3, g.m)), device=dev)
    r = torch.empty_like(u)
    out = {"nodes": g.m, "grid": 192, "pad": 384, "voxelise_s": t_geom}
    names = ["fwd_xy", "zpass", "inv_y", "gather"]
    plans = {}
    for tag, prec, b in (("fp32", B.FP32, 4), ("fp64", B.FP64, 8), ("bf16_mfma", B.BF16_MFMA, 2)):
        pl = B.Plan(g, B.NAVIER3D, precision=prec, nu=0.3, mu=1.0, keep_fp64=prec != B.FP64,
                    autotune=1 if prec != B.BF16_MFMA else 0)
        plans[tag] = pl
        inf = pl.info()
        n = max(10, steps // (10 if prec == B.FP64 else 4))
        st = B.bemfft_apply_profile(pl.handle, q, u, r, reps=20)
        kern = "k_zpass16" if prec == B.BF16_MFMA else "k_zpass"
        out[tag] = {"matvec_s": n / timed_applies(pl, q, u, r, n, 3),
                    "apply_ms_median": median_apply_ms(pl, q, u, r, 50),
                    "stage_ms": dict(zip(names, st)),
                    "plan_seconds": inf["plan_seconds"],
                    "z_schedule": inf["zsched"], "forward_kx_per_thread": inf["fwd_xg"],
                    "roofline": zpass_roofline(inf, b, st[1], kern),
                    "apply_model_bytes": sum(model_bytes(inf, b).values())}
    out["roofline"] = out["fp32"]["roofline"]
    E = np.random.default_rng(11).normal(size=(3, 3))
    uu = (g.rel() @ E.T).T
    bct = torch.zeros((3, g.m), dtype=torch.uint8, device=dev)
    known = torch.tensor(np.ascontiguousarray(uu), device=dev)
    solves = {}
    for tag, pl, kw in (("fp64", plans["fp64"], {}), ("fp32", plans["fp32"], {}),
                        ("fp32_refined_fp64", plans["fp32"], {"refine": 1, "inner_tol": 1e-3}),
                        ("bf16_mfma_refined_fp64", plans["bf16_mfma"], {"refine": 1, "inner_tol": 1e-2})):
        pl.solve(bct, known, tol=1e-6, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, si = pl.solve(bct, known, tol=1e-6, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        solves[tag] = {"seconds": dt, "plan_plus_solve_s": dt + pl.info()["plan_seconds"], "iters": si["iters"],
                       "outer": si["outer"], "true_relres": si["true_relres"], "status": si["status"],
                       "residual_precision": "fp32" if tag == "fp32" else "fp64"}
    out["time_to_solve_1e-6"] = solves
    for pl in plans.values():
        pl.close()
    if mixed:
        out["mixed_bc_preconditioners"] = bench_navier_mixed(B, I, dev)
    return out


def bench_navier_mixed(B, I, dev):
    """The mixed Navier problem (displacement given above the centre,
    traction below) on a 64^3 sphere, FP64 to 1e-6: scalar Jacobi against
    the 3x3 block Jacobi of each node (the 192^3 star's mixed problem stalls
    near 1e-5 with both; only its Dirichlet problem is timed above)."""
    import torch

    nu, mu = 0.3, 1.0
    g = I.sphere3d(64, 0.35)
    lam = 2 * mu * nu / (1 - 2 * nu)
    E = np.random.default_rng(5).normal(size=(3, 3))
    Es = 0.5 * (E + E.T)
    uu = (g.rel() @ E.T).T
    tt = (g.normals @ (lam * np.trace(Es) * np.eye(3) + 2 * mu * Es).T).T
    bc = np.tile(I.mixed_bc_upper(g), (3, 1))
    bct = torch.tensor(bc, device=dev)
    known = torch.tensor(np.where(bc == 0, uu, tt), device=dev)
    pl = B.Plan(g, B.NAVIER3D, precision=B.FP64, nu=nu, mu=mu)
    res = {"workload": "Navier sphere 64^3 (%d nodes), mixed BC, FP64, GMRES(100) to 1e-6" % g.m}
    for tag, pc in (("jacobi", 1), ("block_jacobi_3x3", 2)):
        pl.solve(bct, known, tol=1e-6, precond=pc, maxit=3000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, si = pl.solve(bct, known, tol=1e-6, precond=pc, maxit=3000)
        torch.cuda.synchronize()
        res[tag] = {"seconds": time.perf_counter() - t0, "iters": si["iters"], "true_relres": si["true_relres"],
                    "status": si["status"]}
    pl.close()
    return res


def bench_cube_bf16(B, I, dev, cube, q, u, steps):
    """The 16-bit form on the headline cube: applies (z pass on the matrix
    cores) with its roofline, and mixed-problem solves to 1e-6 with FP64
    refinement."""
    import torch

    r = torch.empty_like(u)
    pl = B.Plan(cube, B.LAPLACE3D, precision=B.BF16_MFMA, keep_fp64=True)
    inf = pl.info()
    names = ["fwd_xy", "zpass", "inv_y", "gather"]
    st = B.bemfft_apply_profile(pl.handle, q, u, r, reps=max(20, steps // 4))
    out = {"matvec_s": steps / timed_applies(pl, q, u, r, steps, 5),
           "apply_ms_median": median_apply_ms(pl, q, u, r, 100),
           "stage_ms": dict(zip(names, st)),
           "roofline": zpass_roofline(inf, 2, st[1], "k_zpass16"),
           "apply_model_bytes": sum(model_bytes(inf, 2).values()),
           "plan_seconds": inf["plan_seconds"]}
    uu, qq = I.harmonic_3d_xyz(cube)
    bc = I.mixed_bc_upper(cube)
    known = torch.tensor(np.where(bc == 0, uu, qq), device=dev)
    bct = torch.tensor(bc, device=dev)
    pl.solve(bct, known, tol=1e-6, refine=1, inner_tol=1e-2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, si = pl.solve(bct, known, tol=1e-6, refine=1, inner_tol=1e-2)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["refined_solve_1e-6"] = {"seconds": dt, "plan_plus_solve_s": dt + inf["plan_seconds"],
                                 "iters": si["iters"], "outer": si["outer"], "true_relres": si["true_relres"],
                                 "status": si["status"], "residual_precision": "fp64"}
    pl.close()
    return out


def bench_learned(B, args):
    """Learned start: a 4-layer, 16-channel dilated conv net on the G^3 grid,
    trained on the GPU with the library's kernels on star problems (seed 3)
    solved by the library's FP64 GMRES, then GMRES to 1e-6 from the learned
    start (use_x0 = 2) against GMRES from zero on held-out problems."""
    import torch

    from paper_1809_00845_amd import learned as LS

    G, ntr, nte = args.learned_grid, args.learned_train, args.learned_test
    quiet = getattr(args, "quiet", False)
    t0 = time.perf_counter()
    probs = LS.problem_set(G, ntr + nte, seed=3)
    t_geom = time.perf_counter() - t0
    print(f"  voxelised {ntr + nte} stars at {G}^3 in {t_geom:.1f} s", file=sys.stderr, flush=True)
    net = B.Net(G, (1, 2, 4, 8), seed=0)
    t0 = time.perf_counter()
    train = LS.make_samples(net, probs[:ntr], progress=None if quiet else 200)
    test_s = LS.make_samples(net, probs[ntr:], progress=None if quiet else 100)
    t_data = time.perf_counter() - t0
    e0 = LS.relative_error(net, test_s)
    # one training step, timed alone
    s = train[0]
    for _ in range(3):
        net.gradients(s.x, s.vox, s.tgt, s.wt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        net.gradients(s.x, s.vox, s.tgt, s.wt)
    t_grad = (time.perf_counter() - t0) / 10
    t0 = time.perf_counter()
    hist = LS.train(net, train, epochs=args.learned_epochs, lr=2e-3, progress_s=0 if quiet else 30.0)
    t_train = time.perf_counter() - t0
    e1 = LS.relative_error(net, test_s)
    del train, test_s
    # inference alone
    xb = torch.empty((6, net.V), dtype=torch.float32, device="cuda:0")
    yb = torch.empty(net.V, dtype=torch.float32, device="cuda:0")
    for _ in range(3):
        net.forward(xb.zero_(), yb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        net.forward(xb, yb)
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t0) / 20
    for _ in range(3):
        net.infer(xb, yb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(50):
        net.infer(xb, yb)
    torch.cuda.synchronize()
    t_inf = (time.perf_counter() - t0) / 50
    t0 = time.perf_counter()
    rows = LS.evaluate(net, probs[ntr:])
    t_eval = time.perf_counter() - t0
    sm = LS.summary(rows)
    net.close()
    return {
        "workload": f"learned start: star surfaces (seed 3) on {G}^3, pad {2 * G}^3, Laplace Dirichlet, "
                    f"{ntr} train / {nte} held-out, GMRES(100) right Jacobi to 1e-6, FP64",
        "network": "conv3d 3x3x3 dilations 1,2,4,8; 6->16->16->16->1; ReLU; trained in FP32, "
                   "inference FP16 on the matrix cores with FP32 accumulation",
        "params": net.nparam,
        "epochs": args.learned_epochs,
        "test_rel_sq_error_before": e0, "test_rel_sq_error_after": e1,
        "train_loss_per_epoch": hist,
        "ms_per_train_step": 1e3 * t_grad,
        "ms_per_forward_fp32": 1e3 * t_fwd,
        "ms_per_inference_fp16_mfma": 1e3 * t_inf,
        "seconds": {"voxelise": t_geom, "solve_and_inputs": t_data, "train": t_train, "evaluate": t_eval},
        **sm,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--quick", action="store_true", help="apply timing only (for profilers)")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-shape batched workload")
    ap.add_argument("--batched-only", action="store_true", help="only the 64-shape batched workload")
    ap.add_argument("--no-navier", action="store_true", help="skip the 192^3 Navier star workload")
    ap.add_argument("--navier-only", action="store_true", help="only the 192^3 Navier star workload (for profilers)")
    ap.add_argument("--no-navier-mixed", action="store_true",
                    help="skip the Navier mixed-problem preconditioner comparison (for profilers)")
    ap.add_argument("--bf16-only", action="store_true",
                    help="only the 16-bit cube applies (z pass on the matrix cores; for profilers)")
    ap.add_argument("--solve-only", action="store_true",
                    help="only the mixed cube solves to 1e-6 (FP64 and FP32 plans), 3 each (for profilers)")
    ap.add_argument("--halfspace-only", action="store_true",
                    help="only the elastic half-space workload (256^2 surface, Hertz contact)")
    ap.add_argument("--cg-only", action="store_true",
                    help="only the Dirichlet CG vs GMRES solves (2D square, 3D sphere)")
    ap.add_argument("--grid-eval-only", action="store_true",
                    help="only the grid-box evaluation on the FP32 cube plan (for profilers)")
    ap.add_argument("--learned", action="store_true",
                    help="only the learned-start workload: train on GPU-solved star problems, then compare solves")
    ap.add_argument("--no-learned", action="store_true", help="skip the reduced learned-start workload")
    ap.add_argument("--learned-grid", type=int, default=96)
    ap.add_argument("--learned-train", type=int, default=2000)
    ap.add_argument("--learned-test", type=int, default=200)
    ap.add_argument("--learned-epochs", type=int, default=4)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB read + 256 MiB write kernel (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the operator is not sharded",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_probe:
        x = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda:0")  # 256 MiB
        for _ in range(5):
            y = x * 1.0
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": x.numel() * 8, "copy_probe_bytes_written": y.numel() * 8,
                          "launches": 5}), flush=True)
        return

    from paper_1809_00845_amd import binding as B
    from paper_1809_00845_amd import inputs as I

    B.load()  # raises if the HIP library is missing
    dev = torch.device("cuda:0")
    if args.batched_only:
        print(json.dumps(bench_batched(B, I, dev)), flush=True)
        return
    if args.learned:
        print(json.dumps(bench_learned(B, args)), flush=True)
        return
    if args.halfspace_only:
        print(json.dumps(bench_halfspace(B, I, dev, args.steps)), flush=True)
        return
    if args.cg_only:
        print(json.dumps(bench_dirichlet_cg(B, I, dev)), flush=True)
        return
    if args.navier_only:
        print(json.dumps(bench_navier_star(B, I, dev, args.steps, mixed=not args.no_navier_mixed)), flush=True)
        return
    if args.solve_only:
        g = I.cube3d(128, 100)
        uu, qq = I.harmonic_3d_xyz(g)
        bc = I.mixed_bc_upper(g)
        known = torch.tensor(np.where(bc == 0, uu, qq), device=dev)
        bct = torch.tensor(bc, device=dev)
        res = {}
        for tag, prec in (("fp64", B.FP64), ("fp32", B.FP32)):
            pl = B.Plan(g, B.LAPLACE3D, precision=prec)
            ts = []
            for _ in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, si = pl.solve(bct, known, tol=1e-6)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            res[tag] = {"seconds": ts, "iters": si["iters"], "true_relres": si["true_relres"]}
            pl.close()
        print(json.dumps({"workload": "laplace3d cube 128^3 mixed solve to 1e-6", **res}), flush=True)
        return
    cube = I.cube3d(128, 100)
    uh, qh = I.harmonic_3d_xyz(cube)
    noise = I.uniform_noise(cube.m, 0, 2)
    qn, un = qh + noise[0], uh + noise[1]
    q = torch.tensor(qn, device=dev)
    u = torch.tensor(un, device=dev)
    r = torch.empty_like(u)

    if args.bf16_only:
        pl = B.Plan(cube, B.LAPLACE3D, precision=B.BF16_MFMA)
        dt = timed_applies(pl, q, u, r, args.steps, args.warmup)
        print(json.dumps({"workload": "laplace3d cube 128^3 16-bit applies", "matvec_s": args.steps / dt}), flush=True)
        return
    plan = B.Plan(cube, B.LAPLACE3D, precision=B.FP32, keep_fp64=True, autotune=1)
    info = plan.info()
    if args.grid_eval_only:
        print(json.dumps({"workload": "laplace3d cube 128^3 grid-box evaluation, fp32",
                          **bench_grid_eval(plan, q, u, info, args.steps)}), flush=True)
        return
    dt = timed_applies(plan, q, u, r, args.steps, args.warmup)
    value = args.steps / dt
    stage_ms = B.bemfft_apply_profile(plan.handle, q, u, r, reps=max(20, args.steps // 4))
    sb = stage_bytes(info, 4)
    names = ["fwd_xy", "zpass", "inv_y", "gather"]
    stages = {n: {"ms": ms, "gbs": sb[n] / (ms * 1e-3) / 1e9, "bytes": sb[n]} for n, ms in zip(names, stage_ms)}
    dom = max(names, key=lambda n: stages[n]["ms"])
    apply_bytes = sum(sb.values())
    model = model_bytes(info, 4)
    zroof = zpass_roofline(info, 4, stages["zpass"]["ms"], "k_zpass")
    workload = "laplace3d_cube_surface_128cubed_pad256_fp32"
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "matvec/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "nodes": cube.m, "grid": 128,
                   "pad": 256, "edge_points": 100, "occupied_planes": info["z_count"],
                   "z_schedule": info["zsched"], "autotune_us": info["tune_us"],
                   "forward_kx_per_thread": info["fwd_xg"], "autotune_forward_us": info["fwd_tune_us"]},
        # the dominant kernel is the z pass; achieved = the model's z-pass bytes
        # (F g + K Hx Hy Hz b + O g) over its mean event time
        "roofline": {"bound": "hbm", "kernel": "k_zpass", "achieved": zroof["achieved"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": zroof["frac"], "traffic": measured_traffic(workload, "zpass"),
                     "model_bytes": zroof["model_bytes"],
                     "frac_occupied_planes_bytes": zroof["frac_occupied_planes_bytes"]},
        "apply_ms_median": median_apply_ms(plan, q, u, r, max(50, args.steps // 2)),
        "stages": stages,
        "apply_gbs": apply_bytes / (sum(stage_ms) * 1e-3) / 1e9,
        "apply_model_bytes": sum(model.values()),
        "apply_model_frac": sum(model.values()) / (sum(stage_ms) * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "zpass_alu_view": zpass_alu_view(info, stages["zpass"]["ms"]),
    }
    if not args.quick:
        extra = {}
        # the field over the grid box (representation formula), same plan
        extra["cube_grid_eval_fp32"] = bench_grid_eval(plan, q, u, info, max(20, args.steps // 4))
        # FP64 apply, same cube
        plan64 = B.Plan(cube, B.LAPLACE3D, precision=B.FP64, autotune=1)
        dt64 = timed_applies(plan64, q, u, r, max(20, args.steps // 4), 5)
        extra["cube_fp64_matvec_s"] = max(20, args.steps // 4) / dt64
        # sphere
        sph = I.sphere3d(128, 0.35)
        us, qs = I.harmonic_3d_xyz(sph)
        ns = I.uniform_noise(sph.m, 0, 2)
        qsd = torch.tensor(qs + ns[0], device=dev)
        usd = torch.tensor(us + ns[1], device=dev)
        rs = torch.empty_like(usd)
        psph = B.Plan(sph, B.LAPLACE3D, precision=B.FP32, keep_fp64=True)
        dts = timed_applies(psph, qsd, usd, rs, args.steps, 5)
        extra["sphere_nodes"] = sph.m
        extra["sphere_fp32_matvec_s"] = args.steps / dts
        extra["sphere_stage_ms"] = dict(zip(names, B.bemfft_apply_profile(psph.handle, qsd, usd, rs, reps=50)))
        extra["cube_fp64_stage_ms"] = dict(zip(names, B.bemfft_apply_profile(plan64.handle, q, u, r, reps=20)))
        # time to solve, mixed BC, 1e-6 true relative residual
        solves = {}
        for name, g, pl32, pl64 in (("cube", cube, plan, plan64), ("sphere", sph, psph, None)):
            uu, qq = I.harmonic_3d_xyz(g)
            bc = I.mixed_bc_upper(g)
            known = torch.tensor(np.where(bc == 0, uu, qq), device=dev)
            bct = torch.tensor(bc, device=dev)
            if pl64 is None:
                pl64 = B.Plan(g, B.LAPLACE3D, precision=B.FP64)
            for tag, pl, kw in (("fp64", pl64, {}), ("fp32", pl32, {}),
                                ("fp32_refined_fp64", pl32, {"refine": 1, "inner_tol": 1e-4})):
                pl.solve(bct, known, tol=1e-6, **kw)  # warm (workspace allocation)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, si = pl.solve(bct, known, tol=1e-6, **kw)
                torch.cuda.synchronize()
                dts = time.perf_counter() - t0
                solves[f"{name}_{tag}"] = {"seconds": dts, "plan_plus_solve_s": dts + pl.info()["plan_seconds"],
                                           "iters": si["iters"],
                                           "outer": si["outer"], "true_relres": si["true_relres"],
                                           "residual_precision": "fp64" if tag != "fp32" else "fp32",
                                           "status": si["status"]}
        extra["time_to_solve_1e-6"] = solves
        extra["dirichlet_cg_vs_gmres"] = bench_dirichlet_cg(B, I, dev)
        extra["halfspace_256sq"] = bench_halfspace(B, I, dev, max(20, args.steps // 4))
        extra["plan_seconds_cube_fp32"] = info["plan_seconds"]
        extra["cube_bf16_mfma"] = bench_cube_bf16(B, I, dev, cube, q, u, args.steps)
        if not args.no_navier:
            print("  navier star 192^3 ...", file=sys.stderr, flush=True)
            extra["navier_star_192"] = bench_navier_star(B, I, dev, args.steps)
        if not args.no_batched:
            plan64.close()
            extra["batched_64_stars_4rhs"] = bench_batched(B, I, dev)
        if not args.no_learned:
            # the learned-start workload at reduced size (64^3 grid, 300
            # training and 40 held-out stars); --learned runs the full one
            print("  learned start, reduced ...", file=sys.stderr, flush=True)
            la = argparse.Namespace(learned_grid=64, learned_train=300, learned_test=40, learned_epochs=3,
                                    quiet=True)
            extra["learned_start_reduced"] = bench_learned(B, la)
        out["extra"] = extra
        if not args.no_cpu:
            out["cpu_baseline"] = cpu_baseline(cube, qn, un)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
