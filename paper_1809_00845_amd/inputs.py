"""Seeded synthetic inputs: voxelised boundaries and boundary data.

This module only builds geometry and data; it holds none of the operator's
arithmetic (no kernels, no sums, no transforms).  Both the HIP path and the
CPU oracle are fed from it, so that they see the same inputs.

Recipe (the paper's own example is a grid-aligned closed boundary, Sec. 4,
Fig. 3; curved shapes need a node definition the paper does not give):

* The unit box [0,1)^d carries a uniform grid with ``n`` points per axis,
  spacing ``h = 1/n``, origin 0.  Grid point ``g`` sits at ``h*g``.
* One node per grid point whose half-open cell ``[p - h/2, p + h/2)^d`` holds
  a part of the boundary.  The node's position is that grid point, its weight
  ``w`` is the boundary measure inside the cell (arc length in 2D, area in 3D)
  and its normal is the mean outward normal ``(1/w) * integral of n dS`` over
  that piece (unit on smooth pieces, shorter at cube edges and corners).
* Circle: piecewise-exact arcs.  Cube faces lie on grid planes: exact.
  Sphere and star-shaped surfaces: the measure is binned from a fine
  midpoint quadrature in (theta, phi).

Every random draw uses ``numpy.random.default_rng(seed)``.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Geometry:
    """A voxelised closed boundary.

    ``nodes``/``normals`` are ``(m, dim)`` float64, ``weights`` is ``(m,)``.
    ``n`` is the grid size per axis (three entries; ``n[2] == 1`` in 2D).
    """

    dim: int
    n: tuple
    h: float
    origin: tuple
    nodes: np.ndarray
    normals: np.ndarray
    weights: np.ndarray
    center: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.weights.shape[0])

    def grid_index(self) -> np.ndarray:
        """Integer grid coordinates of the nodes (they sit on grid points)."""
        return np.rint((self.nodes - np.asarray(self.origin[: self.dim])) / self.h).astype(np.int64)

    def rel(self) -> np.ndarray:
        """Node positions relative to the shape's centre."""
        return self.nodes - self.center[None, :]

    def permuted(self, seed: int) -> "Geometry":
        """Same boundary with the node order shuffled (the plan must not care)."""
        p = np.random.default_rng(seed).permutation(self.m)
        return Geometry(self.dim, self.n, self.h, self.origin, self.nodes[p].copy(),
                        self.normals[p].copy(), self.weights[p].copy(), self.center,
                        self.name + f"_perm{seed}", dict(self.meta, perm=p))


# --------------------------------------------------------------------------- 2D


def circle2d(n: int = 128, radius: float = 0.4, center=(0.5, 0.5)) -> Geometry:
    """Circle of ``radius`` on an ``n x n`` unit grid, exact arcs per cell."""
    h = 1.0 / n
    cx, cy = center
    cuts = [0.0, 2.0 * math.pi]
    for i in range(-1, n + 1):
        line = (i + 0.5) * h
        cval = (line - cx) / radius
        if abs(cval) < 1.0:
            a = math.acos(cval)
            cuts += [a, 2.0 * math.pi - a]
        sval = (line - cy) / radius
        if abs(sval) < 1.0:
            a = math.asin(sval)
            cuts += [a % (2.0 * math.pi), (math.pi - a) % (2.0 * math.pi)]
    cuts = np.unique(np.asarray(cuts))
    acc: dict = {}
    order = []
    for a, b in zip(cuts[:-1], cuts[1:]):
        if b - a <= 0.0:
            continue
        mid = 0.5 * (a + b)
        px, py = cx + radius * math.cos(mid), cy + radius * math.sin(mid)
        g = (int(math.floor(px / h + 0.5)), int(math.floor(py / h + 0.5)))
        w = radius * (b - a)
        nx = radius * (math.sin(b) - math.sin(a))
        ny = -radius * (math.cos(b) - math.cos(a))
        if g not in acc:
            acc[g] = [0.0, 0.0, 0.0]
            order.append(g)
        acc[g][0] += w
        acc[g][1] += nx
        acc[g][2] += ny
    gs = np.asarray(order, dtype=np.int64)
    vals = np.asarray([acc[g] for g in order])
    w = vals[:, 0]
    nrm = vals[:, 1:] / w[:, None]
    return Geometry(2, (n, n, 1), h, (0.0, 0.0, 0.0), gs * h, nrm, w,
                    np.asarray(center, dtype=np.float64), f"circle{n}_R{radius}")


def square2d(n: int = 128, side_points: int = 100) -> Geometry:
    """Grid-aligned square with ``side_points`` grid points per side (the
    paper's Sec. 4 example shape).  Each side node carries arc length ``h``;
    corner nodes carry ``h`` (two half cells) with the mean of the two normals.
    """
    h = 1.0 / n
    lo = (n - side_points) // 2
    hi = lo + side_points - 1
    nodes, nrms, ws = [], [], []
    for gy in range(lo, hi + 1):
        for gx in range(lo, hi + 1):
            on_x = gx in (lo, hi)
            on_y = gy in (lo, hi)
            if not (on_x or on_y):
                continue
            nv = np.zeros(2)
            cnt = 0
            if on_x:
                nv[0] += -1.0 if gx == lo else 1.0
                cnt += 1
            if on_y:
                nv[1] += -1.0 if gy == lo else 1.0
                cnt += 1
            nodes.append((gx * h, gy * h))
            nrms.append(nv / cnt)
            ws.append(h)
    c = (lo + hi) * 0.5 * h
    return Geometry(2, (n, n, 1), h, (0.0, 0.0, 0.0), np.asarray(nodes), np.asarray(nrms),
                    np.asarray(ws), np.asarray([c, c]), f"square{n}_{side_points}")


# --------------------------------------------------------------------------- 3D


def cube3d(n: int = 128, edge_points: int = 100) -> Geometry:
    """Cube surface with ``edge_points`` grid points per edge, faces on grid
    planes, centred in the ``n^3`` box.  Face nodes: area ``h^2``; edge nodes:
    two half cells (``h^2``) with the mean of two face normals; corners: three
    quarter cells (``3h^2/4``) with the mean of three face normals.
    """
    h = 1.0 / n
    lo = (n - edge_points) // 2
    hi = lo + edge_points - 1
    r = np.arange(lo, hi + 1)
    gx, gy, gz = np.meshgrid(r, r, r, indexing="ij")
    gx, gy, gz = gx.ravel(), gy.ravel(), gz.ravel()
    onx = (gx == lo) | (gx == hi)
    ony = (gy == lo) | (gy == hi)
    onz = (gz == lo) | (gz == hi)
    keep = onx | ony | onz
    gx, gy, gz, onx, ony, onz = gx[keep], gy[keep], gz[keep], onx[keep], ony[keep], onz[keep]
    cnt = onx.astype(np.int64) + ony + onz
    nv = np.zeros((gx.size, 3))
    nv[:, 0] = np.where(onx, np.where(gx == lo, -1.0, 1.0), 0.0)
    nv[:, 1] = np.where(ony, np.where(gy == lo, -1.0, 1.0), 0.0)
    nv[:, 2] = np.where(onz, np.where(gz == lo, -1.0, 1.0), 0.0)
    nv /= cnt[:, None]
    # one face: a full cell; an edge: two halves; a corner: three quarters
    w = np.where(cnt == 1, h * h, np.where(cnt == 2, h * h, 0.75 * h * h))
    nodes = np.stack([gx, gy, gz], axis=1) * h
    c = (lo + hi) * 0.5 * h
    return Geometry(3, (n, n, n), h, (0.0, 0.0, 0.0), nodes, nv, w,
                    np.asarray([c, c, c]), f"cube{n}_{edge_points}")


def _bin_surface(n, surf, ntheta, nphi, center, name, rows_per_chunk=64, oversample=1, project=None):
    """Bin a parametric closed surface ``surf(theta, phi) -> (x, x_theta, x_phi)``
    into half-open grid cells: weight = area, normal = mean outward normal.

    oversample = s > 1: the pieces are the surface inside the half-open
    cells of the coarser grid of spacing s h (n / s cells per axis), and each
    node sits at its piece's area-weighted centroid, moved onto the surface
    by ``project`` -- not on a grid point.  The geometry keeps the fine grid
    (spacing h), so a plan snaps every node to within h/2 of its surface
    point while the node count follows the coarse spacing."""
    if n % oversample:
        raise ValueError("the grid size must be a multiple of the oversampling factor")
    h = 1.0 / n
    nc = n // oversample
    hc = oversample * h
    dth = math.pi / ntheta
    dph = 2.0 * math.pi / nphi
    th_all = (np.arange(ntheta) + 0.5) * dth
    ph = (np.arange(nphi) + 0.5) * dph
    ncell = nc * nc * nc
    acc_w = np.zeros(ncell)
    acc_n = np.zeros((3, ncell))
    acc_x = np.zeros((3, ncell)) if oversample > 1 else None
    for s in range(0, ntheta, rows_per_chunk):
        th = th_all[s:s + rows_per_chunk]
        T, Ph = np.meshgrid(th, ph, indexing="ij")
        x, xt, xp = surf(T, Ph)
        cr = np.cross(xt, xp)  # outward for (theta, phi) ordering
        da = np.linalg.norm(cr, axis=-1) * dth * dph
        nrm = cr / np.linalg.norm(cr, axis=-1, keepdims=True)
        g = np.floor(x / hc + 0.5).astype(np.int64)
        if g.min() < 0 or g.max() >= nc:
            raise ValueError("surface leaves the grid")
        lin = (g[..., 0] * nc + g[..., 1]) * nc + g[..., 2]
        lin = lin.ravel()
        acc_w += np.bincount(lin, weights=da.ravel(), minlength=ncell)
        for k in range(3):
            acc_n[k] += np.bincount(lin, weights=(nrm[..., k] * da).ravel(), minlength=ncell)
            if acc_x is not None:
                acc_x[k] += np.bincount(lin, weights=(x[..., k] * da).ravel(), minlength=ncell)
    sel = np.nonzero(acc_w > 0.0)[0]
    w = acc_w[sel]
    nv = (acc_n[:, sel] / w[None, :]).T
    meta = {}
    if acc_x is None:
        gx, rem = np.divmod(sel, n * n)
        gy, gz = np.divmod(rem, n)
        nodes = np.stack([gx, gy, gz], axis=1) * h
    else:
        nodes = (acc_x[:, sel] / w[None, :]).T
        if project is not None:
            nodes = project(nodes)
        if nodes.min() < 0.0 or nodes.max() >= 1.0 - 0.5 * h:
            raise ValueError("surface leaves the grid")
        meta = {"oversample": oversample, "node_spacing": hc}
    return Geometry(3, (n, n, n), h, (0.0, 0.0, 0.0), nodes, nv, w,
                    np.asarray(center, dtype=np.float64), name, meta)


def _default_quadrature(n):
    nt = max(1024, 16 * n)
    return nt, 2 * nt


def sphere3d(n: int = 128, radius: float = 0.35, center=(0.5, 0.5, 0.5), ntheta=None, nphi=None,
             oversample: int = 1) -> Geometry:
    """Sphere of ``radius`` voxelised on an ``n^3`` unit grid; with
    ``oversample`` = s the nodes follow the grid of spacing s/n and sit on
    the sphere (see _bin_surface)."""
    nt, npf = _default_quadrature(n)
    ntheta, nphi = ntheta or nt, nphi or npf
    c = np.asarray(center, dtype=np.float64)

    def surf(T, Ph):
        st, ct, sp, cp = np.sin(T), np.cos(T), np.sin(Ph), np.cos(Ph)
        er = np.stack([st * cp, st * sp, ct], axis=-1)
        et = np.stack([ct * cp, ct * sp, -st], axis=-1)
        ep = np.stack([-sp, cp, np.zeros_like(sp)], axis=-1)
        return c + radius * er, radius * et, radius * st[..., None] * ep

    def project(p):
        d = p - c[None, :]
        return c[None, :] + radius * d / np.linalg.norm(d, axis=1, keepdims=True)

    name = f"sphere{n}_R{radius}" + (f"_os{oversample}" if oversample > 1 else "")
    return _bin_surface(n, surf, ntheta, nphi, c, name, oversample=oversample, project=project)


def real_sph_harm(l: int, m: int, theta, phi):
    """Orthonormal real spherical harmonic Y_lm (polar angle theta)."""
    from scipy.special import sph_harm_y

    y = sph_harm_y(l, abs(m), theta, phi)
    if m == 0:
        return np.real(y)
    if m > 0:
        return math.sqrt(2.0) * (-1) ** m * np.real(y)
    return math.sqrt(2.0) * (-1) ** m * np.imag(y)


_LM = [(l, m) for l in range(5) for m in range(-l, l + 1)]  # 25 harmonics, l <= 4


@dataclass
class StarSpec:
    lm: list
    coef: np.ndarray
    base: float = 0.3
    amp: float = 0.2

    def radius(self, theta, phi):
        s = np.zeros(np.broadcast(theta, phi).shape)
        for (l, m), c in zip(self.lm, self.coef):
            s = s + c * real_sph_harm(l, m, theta, phi)
        return self.base * (1.0 + self.amp * s)


def draw_stars(seed: int, count: int, rmin=0.1, rmax=0.45):
    """``count`` star-shaped radius functions r = 0.3(1 + 0.2 sum_6 c_i Y_i),
    six distinct real Y_lm with l <= 4, c_i ~ N(0, 1), redrawn from the same
    stream while min r <= rmin or max r >= rmax."""
    rng = np.random.default_rng(seed)
    tt, pp = np.meshgrid(np.linspace(0, math.pi, 91), np.linspace(0, 2 * math.pi, 181), indexing="ij")
    out = []
    while len(out) < count:
        idx = rng.choice(25, 6, replace=False)
        coef = rng.standard_normal(6)
        spec = StarSpec([_LM[i] for i in idx], coef)
        r = spec.radius(tt, pp)
        if r.min() <= rmin or r.max() >= rmax:
            continue
        out.append(spec)
    return out


def _theta_part(l, m, theta):
    """theta factor of the real Y_lm (its phi factor is cos(m phi), 1 or
    sin(|m| phi)); real_sph_harm = _theta_part * _phi_part."""
    from scipy.special import sph_harm_y

    v = np.real(sph_harm_y(l, abs(m), theta, np.zeros_like(theta)))
    return v if m == 0 else math.sqrt(2.0) * (-1) ** m * v


def _phi_part(m, phi, deriv=False):
    if m == 0:
        return np.zeros_like(phi) if deriv else np.ones_like(phi)
    if m > 0:
        return -m * np.sin(m * phi) if deriv else np.cos(m * phi)
    k = -m
    return k * np.cos(k * phi) if deriv else np.sin(k * phi)


def draw_batch(seed: int, count: int, sizes=(64, 96, 128, 160), rmin=0.1, rmax=0.45):
    """``count`` (grid size, star) pairs: the grid size uniform over
    ``sizes``, then the star drawn as in draw_stars, all from one stream."""
    rng = np.random.default_rng(seed)
    tt, pp = np.meshgrid(np.linspace(0, math.pi, 91), np.linspace(0, 2 * math.pi, 181), indexing="ij")
    out = []
    while len(out) < count:
        n = int(sizes[rng.integers(len(sizes))])
        while True:
            idx = rng.choice(25, 6, replace=False)
            coef = rng.standard_normal(6)
            spec = StarSpec([_LM[i] for i in idx], coef)
            r = spec.radius(tt, pp)
            if rmin < r.min() and r.max() < rmax:
                break
        out.append((n, spec))
    return out


def _star_job(args):
    n, spec, q = args
    return star3d(n, spec, ntheta=q * n, nphi=2 * q * n)


def star_batch(items, quad_per_cell: int = 8, workers: int | None = None):
    """Voxelise many (n, spec) pairs in parallel processes; quadrature of
    quad_per_cell*n x 2*quad_per_cell*n points per shape."""
    import multiprocessing as mp
    import os

    if workers is None:
        workers = max(1, min(16, len(os.sched_getaffinity(0))))
    jobs = [(n, spec, quad_per_cell) for n, spec in items]
    if workers == 1:
        return [_star_job(j) for j in jobs]
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_star_job, jobs, chunksize=1)


def star3d(n: int, spec: StarSpec, center=(0.5, 0.5, 0.5), ntheta=None, nphi=None) -> Geometry:
    """Star-shaped surface ``r(theta, phi)`` voxelised on an ``n^3`` grid.
    Each real Y_lm factors into a theta part and a phi part, so r and its
    derivatives on the quadrature grid are small matrix products."""
    nt, npf = _default_quadrature(n)
    ntheta, nphi = ntheta or nt, nphi or npf
    c = np.asarray(center, dtype=np.float64)
    d = 1e-6
    ph_all = (np.arange(nphi) + 0.5) * (2.0 * math.pi / nphi)
    Pphi = np.stack([_phi_part(m, ph_all) for (l, m) in spec.lm])          # (6, nphi)
    Pphi_d = np.stack([_phi_part(m, ph_all, True) for (l, m) in spec.lm])
    coef = np.asarray(spec.coef)

    def surf(T, Ph):
        th = T[:, 0]
        Th = np.stack([_theta_part(l, m, th) for (l, m) in spec.lm], 1)    # (nt, 6)
        Th_d = np.stack([(_theta_part(l, m, th + d) - _theta_part(l, m, th - d)) / (2 * d)
                         for (l, m) in spec.lm], 1)
        s = (Th * coef) @ Pphi
        r = spec.base * (1.0 + spec.amp * s)
        rt = spec.base * spec.amp * ((Th_d * coef) @ Pphi)
        rp = spec.base * spec.amp * ((Th * coef) @ Pphi_d)
        st, ct, sp, cp = np.sin(T), np.cos(T), np.sin(Ph), np.cos(Ph)
        er = np.stack([st * cp, st * sp, ct], axis=-1)
        et = np.stack([ct * cp, ct * sp, -st], axis=-1)
        ep = np.stack([-sp, cp, np.zeros_like(sp)], axis=-1)
        x = c + r[..., None] * er
        xt = rt[..., None] * er + r[..., None] * et
        xp = rp[..., None] * er + (r * st)[..., None] * ep
        return x, xt, xp

    return _bin_surface(n, surf, ntheta, nphi, c, f"star{n}")


# --------------------------------------------------------------------------- data


def halfspace_patch(n: int = 256, radius: float | None = None, center=(0.5, 0.5)) -> Geometry:
    """Surface nodes of an elastic half-space on an ``n^2`` unit grid: every
    grid point (radius None) or those within ``radius`` of ``center`` (a
    circular contact patch).  Weight = cell area h^2; normals are unused."""
    h = 1.0 / n
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    pts = np.stack([x.ravel(), y.ravel()], axis=1) * h
    if radius is not None:
        pts = pts[np.linalg.norm(pts - np.asarray(center)[None, :], axis=1) <= radius]
    m = pts.shape[0]
    return Geometry(2, (n, n, 1), h, (0.0, 0.0), pts, np.zeros((m, 2)), np.full(m, h * h),
                    np.asarray(center, dtype=np.float64), f"halfspace{n}" + (f"_a{radius}" if radius else ""))


def harmonic_2d_x2y2(geom: Geometry):
    """u = x^2 - y^2 (relative to the centre) at the nodes and its flux
    q = n . grad u with the node's mean normal."""
    x, y = geom.rel().T
    u = x * x - y * y
    q = 2.0 * x * geom.normals[:, 0] - 2.0 * y * geom.normals[:, 1]
    return u, q


def harmonic_3d_xyz(geom: Geometry):
    """u = x*y*z (relative to the centre) and q = n . grad u."""
    x, y, z = geom.rel().T
    u = x * y * z
    nx, ny, nz = geom.normals.T
    q = y * z * nx + x * z * ny + x * y * nz
    return u, q


_SOLID = None


def solid_harmonics_deg3():
    """The 16 real harmonic polynomials of degree <= 3, each as a callable
    returning (value, gradient) for points of shape (m, 3)."""
    def mk(f, g):
        return (f, g)

    hs = [
        mk(lambda x, y, z: np.ones_like(x), lambda x, y, z: (0 * x, 0 * x, 0 * x)),
        mk(lambda x, y, z: x, lambda x, y, z: (1 + 0 * x, 0 * x, 0 * x)),
        mk(lambda x, y, z: y, lambda x, y, z: (0 * x, 1 + 0 * x, 0 * x)),
        mk(lambda x, y, z: z, lambda x, y, z: (0 * x, 0 * x, 1 + 0 * x)),
        mk(lambda x, y, z: x * y, lambda x, y, z: (y, x, 0 * x)),
        mk(lambda x, y, z: y * z, lambda x, y, z: (0 * x, z, y)),
        mk(lambda x, y, z: x * z, lambda x, y, z: (z, 0 * x, x)),
        mk(lambda x, y, z: x * x - y * y, lambda x, y, z: (2 * x, -2 * y, 0 * x)),
        mk(lambda x, y, z: 2 * z * z - x * x - y * y, lambda x, y, z: (-2 * x, -2 * y, 4 * z)),
        mk(lambda x, y, z: x * y * z, lambda x, y, z: (y * z, x * z, x * y)),
        mk(lambda x, y, z: x * (x * x - 3 * y * y), lambda x, y, z: (3 * x * x - 3 * y * y, -6 * x * y, 0 * x)),
        mk(lambda x, y, z: y * (3 * x * x - y * y), lambda x, y, z: (6 * x * y, 3 * x * x - 3 * y * y, 0 * x)),
        mk(lambda x, y, z: z * (x * x - y * y), lambda x, y, z: (2 * x * z, -2 * y * z, x * x - y * y)),
        mk(lambda x, y, z: x * (4 * z * z - x * x - y * y),
           lambda x, y, z: (4 * z * z - 3 * x * x - y * y, -2 * x * y, 8 * x * z)),
        mk(lambda x, y, z: y * (4 * z * z - x * x - y * y),
           lambda x, y, z: (-2 * x * y, 4 * z * z - x * x - 3 * y * y, 8 * y * z)),
        mk(lambda x, y, z: z * (2 * z * z - 3 * x * x - 3 * y * y),
           lambda x, y, z: (-6 * x * z, -6 * y * z, 6 * z * z - 3 * x * x - 3 * y * y)),
    ]
    return hs


def random_harmonic_3d(geom: Geometry, rng: np.random.Generator):
    """Random combination of the 16 solid harmonics of degree <= 3 with N(0,1)
    coefficients; returns (u, q) at the nodes."""
    coef = rng.standard_normal(16)
    x, y, z = geom.rel().T
    u = np.zeros(geom.m)
    gx, gy, gz = np.zeros(geom.m), np.zeros(geom.m), np.zeros(geom.m)
    for c, (f, g) in zip(coef, solid_harmonics_deg3()):
        u += c * f(x, y, z)
        a, b, d = g(x, y, z)
        gx += c * a
        gy += c * b
        gz += c * d
    q = gx * geom.normals[:, 0] + gy * geom.normals[:, 1] + gz * geom.normals[:, 2]
    return u, q


def mixed_bc_upper(geom: Geometry) -> np.ndarray:
    """Boundary-condition flags: 0 = u known (Dirichlet) where the node lies
    above the centre (z > 0, or y > 0 in 2D), 1 = q known (Neumann) elsewhere."""
    zrel = geom.rel()[:, geom.dim - 1]
    return np.where(zrel > 0.0, 0, 1).astype(np.uint8)


def uniform_noise(m: int, seed: int, ncomp: int = 1):
    """U(-1, 1) noise, shape (ncomp, m)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(ncomp, m))
