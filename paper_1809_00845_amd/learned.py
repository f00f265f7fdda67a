"""Learned initial guess for the Dirichlet solve: problem sets, training and
evaluation, all driving the library's network calls (bemfft_net_*).

A problem is a star-shaped surface voxelised on a G^3 grid with Dirichlet
data u from a random harmonic polynomial of degree <= 3 (the seeded
generators of ``inputs``).  Its training target is the flux q that the
library's own FP64 GMRES finds (Sec. 4: u given, q sought), scaled to
s h q with s = 1/rms(u).  The network, its training and its inference run
on the GPU; this module only loops over problems and keeps statistics.
"""

from __future__ import annotations

import math
import sys
import time

import numpy as np

from . import binding as B
from . import inputs


def problem_set(G: int, count: int, seed: int, quad_per_cell: int = 8, workers: int | None = None):
    """``count`` (geometry, u) pairs: star shapes and harmonic data drawn
    from one seed."""
    specs = inputs.draw_stars(seed, count)
    geoms = inputs.star_batch([(G, s) for s in specs], quad_per_cell=quad_per_cell, workers=workers)
    rng = np.random.default_rng(seed)
    return [(g, inputs.random_harmonic_3d(g, rng)[0]) for g in geoms]


class Sample:
    """One training or test problem held on the device."""

    def __init__(self, x, vox, tgt, wt, iters, geom=None, u=None):
        self.x, self.vox, self.tgt, self.wt = x, vox, tgt, wt
        self.iters = iters
        self.geom, self.u = geom, u


def make_samples(net, problems, tol=1e-8, keep_problem=False, progress=None):
    """Solve every problem with the FP64 plan, build the network input and
    the target on the device.  Returns a list of Sample."""
    import torch

    dev = torch.device("cuda")
    out = []
    xbuf = torch.empty((6, net.V), dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    for i, (g, u) in enumerate(problems):
        plan = B.Plan(g, B.LAPLACE3D, precision=B.FP64)
        try:
            bc = torch.zeros(g.m, dtype=torch.uint8, device=dev)
            known = torch.from_numpy(np.ascontiguousarray(u)).to(dev)
            q, info = plan.solve(bc, known, tol=tol, restart=100, maxit=1000)
            if info["status"] != 0:
                raise RuntimeError(f"training solve {i} did not converge: {info}")
            s = 1.0 / math.sqrt(float(np.mean(u * u)))
            net.input(plan, bc, known, s, xbuf)
            vox, w = B.plan_node_voxels(plan.handle, g.m)
            tgt = (s * g.h) * q
            wt = torch.from_numpy(w).to(dev) / torch.sum(torch.from_numpy(w).to(dev) * tgt * tgt)
            out.append(Sample(xbuf.clone(), torch.from_numpy(vox).to(dev), tgt.float().contiguous(),
                              wt.float().contiguous(), info["iters"],
                              g if keep_problem else None, u if keep_problem else None))
        finally:
            plan.close()
        if progress and (i + 1) % progress == 0:
            print(f"  samples {i + 1}/{len(problems)} ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    return out


def train(net, samples, epochs: int, lr: float = 1e-3, seed: int = 0, progress_s: float = 30.0):
    """Adam over the samples, one problem per step, cosine learning rate.
    Returns the mean loss of each epoch."""
    rng = np.random.default_rng(seed)
    total = epochs * len(samples)
    step, hist = 0, []
    t0 = last = time.perf_counter()
    for ep in range(epochs):
        ls = []
        for i in rng.permutation(len(samples)):
            s = samples[i]
            lr_t = 0.5 * lr * (1.0 + math.cos(math.pi * step / total))
            ls.append(net.train_step(s.x, s.vox, s.tgt, s.wt, max(lr_t, 1e-3 * lr)))
            step += 1
            if progress_s and time.perf_counter() - last > progress_s:
                last = time.perf_counter()
                print(f"  train step {step}/{total} loss {np.mean(ls):.4f} ({last - t0:.0f} s)", file=sys.stderr,
                      flush=True)
        hist.append(float(np.mean(ls)))
    return hist


def relative_error(net, samples):
    """Mean of sum wt (y - t)^2 over the samples (wt is normalised so that
    this is the squared relative error of the scaled flux)."""
    errs = []
    for s in samples:
        L, _ = net.gradients(s.x, s.vox, s.tgt, s.wt)
        errs.append(L)
    return float(np.mean(errs))


def evaluate(net, problems, tol=1e-6):
    """Plain FP64 GMRES from zero against the learned start (use_x0 = 2, the
    guess kept only if its residual beats x = 0), per problem."""
    import torch

    dev = torch.device("cuda")
    xbuf = torch.empty((6, net.V), dtype=torch.float32, device=dev)
    rows = []
    for g, u in problems:
        plan = B.Plan(g, B.LAPLACE3D, precision=B.FP64)
        try:
            bc = torch.zeros(g.m, dtype=torch.uint8, device=dev)
            known = torch.from_numpy(np.ascontiguousarray(u)).to(dev)
            _, i0 = plan.solve(bc, known, tol=tol)  # warm-up of the plan's solve workspace
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, i0 = plan.solve(bc, known, tol=tol)
            t0 = time.perf_counter() - t
            x0 = torch.zeros(g.m, dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            t = time.perf_counter()
            net.guess(plan, bc, known, xbuf, x0)
            _, i1 = plan.solve(bc, known, x0, tol=tol, use_x0=2)
            t1 = time.perf_counter() - t
            rows.append({"m": g.m, "iters0": i0["iters"], "iters1": i1["iters"], "t0": t0, "t1": t1,
                         "relres0": i0["true_relres"], "relres1": i1["true_relres"], "x0_used": i1["x0_used"],
                         "x0_relres": i1["x0_relres"], "status0": i0["status"], "status1": i1["status"]})
        finally:
            plan.close()
    return rows


def summary(rows):
    a = lambda k: np.array([r[k] for r in rows], dtype=float)
    return {
        "problems": len(rows),
        "iters_plain_mean": float(a("iters0").mean()),
        "iters_learned_mean": float(a("iters1").mean()),
        "time_plain_ms_mean": 1e3 * float(a("t0").mean()),
        "time_learned_ms_mean": 1e3 * float(a("t1").mean()),
        "guess_relres_median": float(np.median(a("x0_relres"))),
        "guess_kept": int(a("x0_used").sum()),
        "relres_max": float(max(a("relres0").max(), a("relres1").max())),
        "all_converged": bool(all(r["status0"] == 0 and r["status1"] == 0 for r in rows)),
    }
