"""CPU FP64 oracle for the grid-embedded BEM operator (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
and never imports it.

The arithmetic lives in ``bem_oracle.c`` (plain C, FP64, OpenMP over targets):
a direct O(M^2) summation of the discrete operator that the FFT convolution of
the paper (Sec. 3, eqs. 14-16) evaluates.  This module only marshals arrays and
adds textbook steps on top, for the mixed boundary-value problem of eq. (4)/(8)
and the paper's Dirichlet problem (end of Sec. 4):

* a dense LU solve of the assembled system (``numpy.linalg.solve``), for
  problems whose dense matrix fits (``solve_lu``);
* a plain restarted GMRES written from its definition (Saad and Schultz,
  1986: Arnoldi with modified Gram-Schmidt, Givens rotations, restart), with
  the direct-sum operator applied matrix-free, for problems beyond LU sizes
  (``gmres``, ``solve_gmres``);
* conjugate gradients on the symmetrised Dirichlet system (``dirichlet_cg``).
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bem_oracle.c")
_LIB = os.path.join(_HERE, "libbem_oracle.so")

LAPLACE2D, LAPLACE3D, NAVIER3D, HALFSPACE = 0, 1, 2, 3
C_HALF, C_USER, C_IMPLICIT = 0, 1, 2

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, strict IEEE: no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_long)
        L.orc_laplace2d.argtypes = [dp, dp]
        L.orc_laplace3d.argtypes = [dp, dp]
        L.orc_kelvin_u.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp]
        L.orc_kelvin_t.argtypes = [dp, dp, ctypes.c_double, dp]
        L.orc_self_laplace2d.argtypes = [ctypes.c_double]
        L.orc_self_laplace2d.restype = ctypes.c_double
        L.orc_self_laplace3d.argtypes = [ctypes.c_double]
        L.orc_self_laplace3d.restype = ctypes.c_double
        L.orc_self_kelvin.argtypes = [ctypes.c_double, dp, ctypes.c_double, ctypes.c_double, dp]
        L.orc_grid_k0.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.orc_snap.argtypes = [ctypes.c_int, ctypes.c_long, dp, ctypes.c_double, dp, lp, lp]
        L.orc_snap.restype = ctypes.c_long
        L.orc_apply.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_long, lp, dp, dp, ctypes.c_int, dp, dp, dp,
                                ctypes.c_long, ctypes.c_long, dp, dp, dp, ctypes.c_int, dp, dp]
        L.orc_assemble.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_long, lp, dp, dp, dp, dp, dp, ctypes.c_int, dp, dp]
        L.orc_volume.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_long, lp, dp, dp, dp, dp, ctypes.c_long, lp, dp, dp,
                                 ctypes.c_int, dp, dp]
        L.orc_halfspace.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp]
        L.orc_self_halfspace.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _l(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_long))


def num_threads() -> int:
    return int(lib().orc_num_threads())


# ----------------------------------------------------------------- kernels


def laplace2d(xi):
    """(u*, du*/dx, du*/dy) at displacement xi = field - target, eqs. (3), (12)."""
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    out = np.zeros(3)
    lib().orc_laplace2d(_d(xi), _d(out))
    return out


def laplace3d(xi):
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    out = np.zeros(4)
    lib().orc_laplace3d(_d(xi), _d(out))
    return out


def kelvin_u(xi, nu, mu):
    """Kelvin displacement tensor of eq. (7), 3x3."""
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    out = np.zeros(9)
    lib().orc_kelvin_u(_d(xi), nu, mu, _d(out))
    return out.reshape(3, 3)


def kelvin_t(xi, n, nu):
    """Kelvin traction kernel T[k, j] (force direction k, component j)."""
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.float64)
    out = np.zeros(9)
    lib().orc_kelvin_t(_d(xi), _d(n), nu, _d(out))
    return out.reshape(3, 3)


def halfspace(d, nu, mu):
    """Boussinesq-Cerruti tensor K[a][b] at the surface offset d = target -
    source (eq. 9)."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    out = np.zeros(9)
    lib().orc_halfspace(_d(d), nu, mu, _d(out))
    return out.reshape(3, 3)


def self_halfspace(w, nu, mu):
    out = np.zeros(9)
    lib().orc_self_halfspace(float(w), nu, mu, _d(out))
    return out.reshape(3, 3)


def self_laplace2d(w):
    return float(lib().orc_self_laplace2d(float(w)))


def self_laplace3d(w):
    return float(lib().orc_self_laplace3d(float(w)))


def self_kelvin(w, n, nu, mu):
    n = np.ascontiguousarray(n, dtype=np.float64)
    out = np.zeros(9)
    lib().orc_self_kelvin(float(w), _d(n), nu, mu, _d(out))
    return out.reshape(3, 3)


def grid_k0(kernel, h, nu=0.3, mu=1.0):
    out = np.zeros(9)
    lib().orc_grid_k0(kernel, h, nu, mu, _d(out))
    return out.reshape(3, 3)


# ----------------------------------------------------------------- operator


@dataclass
class Problem:
    """Geometry handed to the oracle: plain arrays, nothing else."""

    kernel: int
    h: float
    origin: np.ndarray
    n: np.ndarray
    nodes: np.ndarray
    normals: np.ndarray
    weights: np.ndarray
    nu: float = 0.3
    mu: float = 1.0
    cell_quad: int = 0  # 0: kernels point-sampled at offsets m != 0; q >= 2: cell means

    @property
    def dim(self):
        return 2 if self.kernel in (LAPLACE2D, HALFSPACE) else 3

    @property
    def ncomp(self):
        return 3 if self.kernel in (NAVIER3D, HALFSPACE) else 1

    @property
    def m(self):
        return int(self.weights.shape[0])


def problem(geom, kernel, nu=0.3, mu=1.0, cell_quad=0) -> Problem:
    """Build an oracle Problem from any object with dim/n/h/origin/nodes/
    normals/weights attributes (the shared input generators make those)."""
    d = geom.dim
    return Problem(kernel, float(geom.h), np.asarray(geom.origin[:d], dtype=np.float64),
                   np.asarray(geom.n[:d], dtype=np.int64),
                   np.ascontiguousarray(geom.nodes, dtype=np.float64),
                   np.ascontiguousarray(geom.normals, dtype=np.float64),
                   np.ascontiguousarray(geom.weights, dtype=np.float64), nu, mu, int(cell_quad))


def cell_rule(q: int):
    """The per-axis rule of the cell means (constant elements, Sec. 4 /
    Fig. 5): q Gauss-Legendre points on [-1/2, 1/2] (numpy's ``leggauss``,
    rescaled) with weights summing to 1.  q = 0: point values."""
    if q <= 0:
        return np.zeros(1), np.zeros(1)
    x, w = np.polynomial.legendre.leggauss(int(q))
    return np.ascontiguousarray(0.5 * x), np.ascontiguousarray(0.5 * w)


def _rule_args(p: Problem):
    x, w = cell_rule(p.cell_quad)
    return (int(max(p.cell_quad, 0)), x, w)


def snap(p: Problem) -> np.ndarray:
    """Grid index of every node: floor((x - origin)/h + 1/2)."""
    g = np.zeros((p.m, p.dim), dtype=np.int64)
    bad = lib().orc_snap(p.dim, p.m, _d(p.nodes), p.h, _d(p.origin), _l(p.n.astype(np.int64)), _l(g))
    if bad >= 0:
        raise ValueError(f"node {bad} lies outside the grid")
    return g


def apply(p: Problem, q, u, cmode=C_IMPLICIT, cuser=None, targets=None, with_scale=False,
          with_c=False):
    """r = c u + D[u] - S[q] at the targets (a contiguous range ``(t0, t1)`` or
    None for all nodes).  ``q``/``u``: (ncomp, m) or (m,) for Laplace."""
    g = snap(p)
    nc = p.ncomp
    q = np.ascontiguousarray(np.reshape(q, (nc, p.m)), dtype=np.float64)
    u = np.ascontiguousarray(np.reshape(u, (nc, p.m)), dtype=np.float64)
    t0, t1 = (0, p.m) if targets is None else targets
    nt = t1 - t0
    r = np.zeros((nc, nt))
    sc = np.zeros((nc, nt))
    cbuf = np.zeros((nt, nc * nc))
    if cmode == C_USER:
        cu = np.ascontiguousarray(np.reshape(cuser, (p.m, nc * nc)), dtype=np.float64)
        cptr = _d(cu)
    else:
        cu = None
        cptr = None
    cq, cx, cw = _rule_args(p)
    lib().orc_apply(p.kernel, p.nu, p.mu, p.h, p.m, _l(g), _d(p.normals), _d(p.weights), cmode,
                    cptr, _d(q), _d(u), t0, t1, _d(r), _d(sc), _d(cbuf), cq, _d(cx), _d(cw))
    out = [r if nc > 1 else r[0]]
    if with_scale:
        out.append(sc if nc > 1 else sc[0])
    if with_c:
        out.append(cbuf.reshape(nt, nc, nc) if nc > 1 else cbuf[:, 0])
    return out[0] if len(out) == 1 else tuple(out)


def volume(p: Problem, q, u, pts, with_scale=False):
    """The representation formula at grid points (c = 1 inside, 0 outside):
    v(p) = S[q](p) - D[u](p), the plain grid sum at points that hold nodes.
    ``pts``: (npts, dim) integer grid indices.  Returns (ncomp, npts), or
    (npts,) for Laplace; with_scale adds the sum of the terms' magnitudes."""
    g = snap(p)
    nc = p.ncomp
    q = np.ascontiguousarray(np.reshape(q, (nc, p.m)), dtype=np.float64)
    u = np.ascontiguousarray(np.reshape(u, (nc, p.m)), dtype=np.float64)
    pts = np.ascontiguousarray(np.reshape(pts, (-1, p.dim)), dtype=np.int64)
    out = np.zeros((nc, pts.shape[0]))
    sc = np.zeros((nc, pts.shape[0]))
    cq, cx, cw = _rule_args(p)
    lib().orc_volume(p.kernel, p.nu, p.mu, p.h, p.m, _l(g), _d(p.normals), _d(p.weights), _d(q), _d(u),
                     pts.shape[0], _l(pts), _d(out), _d(sc), cq, _d(cx), _d(cw))
    if nc == 1:
        out, sc = out[0], sc[0]
    return (out, sc) if with_scale else out


def assemble(p: Problem):
    """Dense S, D ((nc m) x (nc m), component-major) and the implicit c blocks."""
    g = snap(p)
    n = p.ncomp * p.m
    S = np.zeros((n, n))
    D = np.zeros((n, n))
    c = np.zeros((p.m, p.ncomp * p.ncomp))
    cq, cx, cw = _rule_args(p)
    lib().orc_assemble(p.kernel, p.nu, p.mu, p.h, p.m, _l(g), _d(p.normals), _d(p.weights),
                       _d(S), _d(D), _d(c), cq, _d(cx), _d(cw))
    return S, D, c


def c_matrix(p: Problem, cmode, cuser=None, c_implicit=None):
    """The free-term operator as a dense (nc m)^2 matrix (component-major)."""
    nc, m = p.ncomp, p.m
    if p.kernel == HALFSPACE:  # r = K[sigma] - u whatever the mode
        blocks = np.tile(-np.eye(nc).reshape(1, nc * nc), (m, 1))
    elif cmode == C_HALF:
        blocks = np.tile(0.5 * np.eye(nc).reshape(1, nc * nc), (m, 1))
    elif cmode == C_USER:
        blocks = np.reshape(cuser, (m, nc * nc))
    else:
        blocks = c_implicit
    C = np.zeros((nc * m, nc * m))
    idx = np.arange(m)
    for a in range(nc):
        for b in range(nc):
            C[a * m + idx, b * m + idx] = blocks[:, a * nc + b]
    return C


def mixed_system(p: Problem, bc, known, cmode=C_IMPLICIT, cuser=None):
    """Dense A, b of the mixed boundary-value problem: unknown x holds q where
    u is given (bc == 0) and u where q is given (bc == 1); A x = b is
    "r = 0" (eq. 4 / 8) with the known values moved to the right."""
    S, D, cimp = assemble(p)
    C = c_matrix(p, cmode, cuser, cimp)
    bc = np.reshape(bc, -1).astype(bool)          # True: q known
    known = np.reshape(known, -1)
    # r = (C + D) u - S q ;  columns of unknowns
    Au = C + D
    As = -S
    A = np.where(bc[None, :], Au, As)
    Bk = np.where(bc[None, :], As, Au)
    b = -Bk @ known
    return A, b


def solve_lu(p: Problem, bc, known, cmode=C_IMPLICIT, cuser=None):
    """Textbook dense LU solve of the mixed system (small problems)."""
    A, b = mixed_system(p, bc, known, cmode, cuser)
    x = np.linalg.solve(A, b)
    return x.reshape(p.ncomp, p.m) if p.ncomp > 1 else x


def dirichlet_cg(p: Problem, u, tol=1e-10, maxit=1000, precond=True, cmode=C_IMPLICIT, cuser=None, x0=None):
    """The paper's solver (end of Sec. 4): conjugate gradients for q in
    S q = c u + D u (eq. 4 with r = 0, u given everywhere, Laplace).

    S = G W with G symmetric, so CG (Hestenes-Stiefel, with an optional
    diagonal preconditioner) runs on the symmetrised matrix
    A = W^1/2 S W^-1/2 and right-hand side W^1/2 (c u + D u); q = W^-1/2 y.
    Stops when ||r|| <= tol ||b|| for the recursive residual r.  Returns
    (q, iterations)."""
    S, D, cimp = assemble(p)
    C = c_matrix(p, cmode, cuser, cimp)
    sw = np.sqrt(p.weights)
    A = sw[:, None] * S / sw[None, :]
    b = sw * ((C + D) @ np.reshape(u, -1))
    minv = 1.0 / np.diag(A) if precond else np.ones(p.m)
    y = np.zeros(p.m) if x0 is None else sw * np.reshape(x0, -1)
    r = b - A @ y
    z = minv * r
    d = z.copy()
    rz = r @ z
    bn = np.linalg.norm(b)
    it = 0
    while np.linalg.norm(r) > tol * bn and it < maxit:
        ad = A @ d
        alpha = rz / (d @ ad)
        y = y + alpha * d
        r = r - alpha * ad
        z = minv * r
        rz_new = r @ z
        d = z + (rz_new / rz) * d
        rz = rz_new
        it += 1
    return y / sw, it


# ----------------------------------------------------------------- GMRES


def gmres(matvec, b, tol=1e-10, restart=50, maxit=1000, minv=None, x0=None):
    """Restarted GMRES(restart) for A x = b, written from its definition.

    Right preconditioning by the diagonal ``minv`` (A M y = b, x = M y).  Each
    cycle starts from the true residual r0 = b - A x; the Arnoldi process with
    modified Gram-Schmidt builds V and the Hessenberg matrix H, Givens
    rotations reduce H to triangular form, and the residual norm of the
    least-squares problem min ||beta e1 - H y|| is the last rotated entry of
    beta e1.  A cycle ends at ``restart`` steps or when that norm falls to
    tol ||b||; x += M V y.  Stops when the true residual ||b - A x|| <= tol
    ||b|| or after ``maxit`` iterations.

    Returns (x, iterations, true relative residual, per-iteration estimated
    relative residuals)."""
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    M = np.ones(n) if minv is None else np.asarray(minv, dtype=np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    history = []
    if bnorm == 0.0:
        return np.zeros(n), 0, 0.0, history
    iters = 0
    while True:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta <= tol * bnorm or iters >= maxit:
            return x, iters, beta / bnorm, history
        m = min(restart, maxit - iters)
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        while k < m:
            w = matvec(M * V[k])
            for i in range(k + 1):  # modified Gram-Schmidt
                H[i, k] = V[i] @ w
                w = w - H[i, k] * V[i]
            H[k + 1, k] = np.linalg.norm(w)
            for i in range(k):  # earlier rotations on the new column
                t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
                H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
                H[i, k] = t
            rr = math.hypot(H[k, k], H[k + 1, k])
            cs[k], sn[k] = (H[k, k] / rr, H[k + 1, k] / rr) if rr > 0 else (1.0, 0.0)
            hnext = H[k + 1, k]
            H[k, k], H[k + 1, k] = rr, 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            iters += 1
            k += 1
            history.append(abs(g[k]) / bnorm)
            if abs(g[k]) <= tol * bnorm or hnext == 0.0:
                break
            V[k] = w / hnext
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        x = x + M * (V[:k].T @ y)


def mixed_parts(p: Problem, bc, known):
    """(q, u) of the known values placed in their slots, and a function that
    places an unknown vector x in the other slots (bc == 0: u known, q
    unknown; bc == 1: q known, u unknown)."""
    nc, m = p.ncomp, p.m
    bc = np.reshape(bc, (nc, m)).astype(bool)
    known = np.reshape(known, (nc, m))
    qk = np.where(bc, known, 0.0)
    uk = np.where(bc, 0.0, known)

    def place(x):
        x = np.reshape(x, (nc, m))
        return np.where(bc, 0.0, x), np.where(bc, x, 0.0)

    return qk, uk, place


def mixed_diagonal(p: Problem, bc, cmode=C_IMPLICIT, cuser=None):
    """Diagonal of the mixed operator: -S_jj (the node's flat-panel self
    integral) where q is unknown, c_jj + D_jj = c_jj where u is unknown
    (the double-layer self term is zero)."""
    nc, m = p.ncomp, p.m
    bc = np.reshape(bc, (nc, m)).astype(bool)
    _, cblk = apply(p, np.zeros((nc, m)), np.zeros((nc, m)), cmode=cmode, cuser=cuser, with_c=True)
    cblk = np.reshape(cblk, (m, nc, nc))
    sdiag = np.zeros((nc, m))
    for j in range(m):
        w = p.weights[j]
        if p.kernel == LAPLACE2D:
            sdiag[0, j] = self_laplace2d(w)
        elif p.kernel == LAPLACE3D:
            sdiag[0, j] = self_laplace3d(w)
        elif p.kernel == NAVIER3D:
            sdiag[:, j] = np.diag(self_kelvin(w, p.normals[j], p.nu, p.mu))
        else:
            raise ValueError("mixed_diagonal: boundary families only")
    cdiag = np.stack([cblk[:, k, k] for k in range(nc)])
    return np.where(bc, cdiag, -sdiag).reshape(-1)


def solve_gmres(p: Problem, bc, known, tol=1e-10, restart=50, maxit=2000, precond=True, cmode=C_IMPLICIT,
                cuser=None):
    """The mixed problem A x = b with A x = apply(x in the unknown slots) and
    b = -apply(known values), by ``gmres`` with the direct-sum operator
    applied matrix-free (each product is one O(M^2) ``apply``).  Jacobi
    (right) scaling with ``mixed_diagonal`` if precond.  Returns (x,
    iterations, true relative residual), x shaped like ``known``."""
    nc, m = p.ncomp, p.m
    qk, uk, place = mixed_parts(p, bc, known)
    b = -np.reshape(apply(p, qk, uk, cmode=cmode, cuser=cuser), -1)

    def matvec(x):
        q, u = place(x)
        return np.reshape(apply(p, q, u, cmode=cmode, cuser=cuser), -1)

    minv = None
    if precond:
        d = mixed_diagonal(p, bc, cmode, cuser)
        minv = np.where((d != 0) & np.isfinite(d), 1.0 / np.where(d != 0, d, 1.0), 1.0)
    x, it, rel, _ = gmres(matvec, b, tol=tol, restart=restart, maxit=maxit, minv=minv)
    return (x.reshape(nc, m) if nc > 1 else x), it, rel
