"""Pins of the oracle parts added for solves beyond LU sizes and for nodes
that share a grid cell (CPU only).

* The Navier grid value at offset 0 (used whenever two nodes share a cell)
  is the orientation average of the flat-panel integral of Kelvin's tensor
  (eq. 7) over an h x h panel.  It is checked against a scipy quadrature of
  the tensor over panels in the three grid planes, computed here without the
  oracle's self-term code, and against the average of the oracle's own panel
  integral over the six axis normals and over the 12 icosahedron vertices.
* The plain restarted GMRES is checked against closed forms (a rank-one
  update of the identity is solved in two steps; any n x n system in n),
  against LU, and on the mixed problems of eq. (4) and eq. (8) against the
  dense LU solution of the same discrete system.
"""

import math

import numpy as np
import pytest
from scipy import integrate

import oracle as O
from paper_1809_00845_amd import inputs as I


def _square_polar(f, a):
    """Integral of f(x, y) over the square [-a, a]^2 in polar coordinates
    around the weakly singular origin."""

    def inner(t):
        c, s = math.cos(t), math.sin(t)
        rmax = a / max(abs(c), abs(s))
        v, _ = integrate.quad(lambda r: f(r * c, r * s) * r, 0.0, rmax, epsabs=1e-15, epsrel=1e-12, limit=200)
        return v

    pts = [math.pi / 4, 3 * math.pi / 4, 5 * math.pi / 4, 7 * math.pi / 4]
    v, _ = integrate.quad(inner, 0.0, 2 * math.pi, points=pts, limit=200, epsabs=1e-14, epsrel=1e-12)
    return v


def _kelvin_u(xi, nu, mu):
    """Kelvin's displacement tensor, eq. (7), typed here from the formula."""
    r = np.linalg.norm(xi)
    return ((3 - 4 * nu) * np.eye(3) / r + np.outer(xi, xi) / r ** 3) / (16 * math.pi * mu * (1 - nu))


def test_navier_grid_value_is_orientation_averaged_panel_by_quadrature(orc):
    nu, mu, h = 0.3, 1.7, 1.0 / 48
    a = 0.5 * h
    mean = np.zeros((3, 3))
    for axis in range(3):  # panel in the plane normal to e_axis
        t1, t2 = [b for b in range(3) if b != axis]
        blk = np.zeros((3, 3))
        for k in range(3):
            for j in range(3):
                def f(x, y, k=k, j=j):
                    xi = np.zeros(3)
                    xi[t1], xi[t2] = x, y
                    return _kelvin_u(xi, nu, mu)[k, j]
                blk[k, j] = _square_polar(f, a)
        mean += blk / 3
    k0w = orc.grid_k0(O.NAVIER3D, h, nu, mu) * h * h
    assert np.abs(k0w - mean).max() < 1e-9 * np.abs(mean).max()
    # off-diagonal entries vanish in the average, the diagonal is isotropic
    assert np.abs(k0w - np.diag(np.diag(k0w))).max() == 0.0
    assert np.ptp(np.diag(k0w)) < 1e-15 * k0w[0, 0]


@pytest.mark.parametrize("h", [1.0 / 16, 1.0 / 192])
def test_navier_grid_value_equals_mean_of_panel_blocks(orc, h):
    nu, mu = 0.25, 0.8
    k0w = orc.grid_k0(O.NAVIER3D, h, nu, mu) * h * h
    axes = [s * e for e in np.eye(3) for s in (1.0, -1.0)]
    mean_axes = sum(orc.self_kelvin(h * h, n, nu, mu) for n in axes) / 6
    assert np.abs(k0w - mean_axes).max() < 1e-14 * np.abs(k0w).max()
    # the icosahedron's 12 vertices are a spherical 2-design: <n n> = I/3
    p = (1 + math.sqrt(5)) / 2
    ico = []
    for s1 in (1, -1):
        for s2 in (1, -1):
            ico += [(0, s1, s2 * p), (s1, s2 * p, 0), (s2 * p, 0, s1)]
    ico = [np.array(v, dtype=float) / np.linalg.norm(v) for v in ico]
    mean_ico = sum(orc.self_kelvin(h * h, n, nu, mu) for n in ico) / 12
    assert np.abs(k0w - mean_ico).max() < 1e-14 * np.abs(k0w).max()


def test_laplace_grid_values_are_panel_integrals(orc):
    h = 1.0 / 40
    # 2D: int_{-h/2}^{h/2} -ln|x| / (2 pi) dx, divided by h
    seg, _ = integrate.quad(lambda x: -math.log(abs(x)) / (2 * math.pi), -h / 2, h / 2, points=[0.0])
    assert abs(orc.grid_k0(O.LAPLACE2D, h)[0, 0] * h - seg) < 1e-12 * abs(seg)
    sq = _square_polar(lambda x, y: 1.0 / (4 * math.pi * math.hypot(x, y)), h / 2)
    assert abs(orc.grid_k0(O.LAPLACE3D, h)[0, 0] * h * h - sq) < 1e-9 * sq


def test_navier_same_cell_pair_uses_grid_value(orc):
    """Two Navier nodes in one cell, with different normals and weights: the
    single-layer block between them is the grid value times the source
    weight, each diagonal block is the node's own panel integral, and the
    double layer between them vanishes."""

    class G:
        pass

    h = 1.0 / 16
    g = G()
    g.dim, g.n, g.h, g.origin = 3, (16, 16, 16), h, (0.0, 0.0, 0.0)
    g.nodes = np.array([[0.5, 0.5, 0.5], [0.5 + 0.3 * h, 0.5 - 0.2 * h, 0.5 + 0.1 * h]])
    n1 = np.array([0.3, -0.4, 0.866])
    n1 /= np.linalg.norm(n1)
    g.normals = np.array([[0.0, 0.0, 1.0], n1])
    g.weights = np.array([0.7 * h * h, 1.3 * h * h])
    p = O.problem(g, O.NAVIER3D, 0.3, 1.0)
    S, D, _ = O.assemble(p)
    k0 = O.grid_k0(O.NAVIER3D, h, 0.3, 1.0)
    for k in range(3):
        for j in range(3):
            assert S[k * 2 + 0, j * 2 + 1] == pytest.approx(k0[k, j] * g.weights[1], rel=1e-14, abs=1e-300)
            assert S[k * 2 + 1, j * 2 + 0] == pytest.approx(k0[k, j] * g.weights[0], rel=1e-14, abs=1e-300)
            for a in range(2):
                for b in range(2):
                    assert D[k * 2 + a, j * 2 + b] == 0.0
    for a in range(2):
        blk = np.array([[S[k * 2 + a, j * 2 + a] for j in range(3)] for k in range(3)])
        ref = O.self_kelvin(g.weights[a], g.normals[a], 0.3, 1.0)
        assert np.abs(blk - ref).max() < 1e-14 * np.abs(ref).max()


# ------------------------------------------------------------------ GMRES


def test_gmres_rank_one_update_takes_two_steps():
    """A = I + u v^T has minimal polynomial of degree 2, so the Krylov space
    holds the solution after two steps (exact arithmetic)."""
    rng = np.random.default_rng(5)
    n = 60
    u, v = rng.normal(size=n), rng.normal(size=n) / n
    A = np.eye(n) + np.outer(u, v)
    b = rng.normal(size=n)
    x, it, rel, hist = O.gmres(lambda z: A @ z, b, tol=1e-13, restart=50)
    assert it == 2
    assert rel < 1e-13
    assert np.abs(x - np.linalg.solve(A, b)).max() < 1e-12 * np.abs(x).max()


def test_gmres_full_krylov_space_and_monotone_residual():
    rng = np.random.default_rng(6)
    n = 30
    A = 3 * np.eye(n) + rng.normal(size=(n, n)) / math.sqrt(n)
    b = rng.normal(size=n)
    x, it, rel, hist = O.gmres(lambda z: A @ z, b, tol=1e-12, restart=n)
    assert it <= n and rel <= 1e-12
    assert np.all(np.diff(hist) <= 1e-15)  # minimal residual over growing spaces
    assert np.abs(x - np.linalg.solve(A, b)).max() < 1e-10 * np.abs(x).max()


def test_gmres_restarted_with_diagonal_scaling_matches_lu():
    rng = np.random.default_rng(7)
    n = 80
    d = 10.0 ** rng.uniform(-2, 2, n)
    A = np.diag(d) @ (np.eye(n) + 0.3 * rng.normal(size=(n, n)) / math.sqrt(n))
    b = rng.normal(size=n)
    x, it, rel, _ = O.gmres(lambda z: A @ z, b, tol=1e-12, restart=7, maxit=2000, minv=1.0 / d)
    assert rel <= 1e-12
    assert np.linalg.norm(x - np.linalg.solve(A, b)) < 1e-9 * np.linalg.norm(x)


def test_gmres_mixed_laplace_sphere_matches_lu(orc):
    g = I.sphere3d(16, 0.35)
    p = O.problem(g, O.LAPLACE3D)
    uh, qh = I.harmonic_3d_xyz(g)
    bc = I.mixed_bc_upper(g)
    known = np.where(bc == 0, uh, qh)
    xl = O.solve_lu(p, bc, known)
    for restart in (100, 10):
        xg, it, rel = O.solve_gmres(p, bc, known, tol=1e-11, restart=restart)
        assert rel <= 1e-11
        assert np.linalg.norm(xg - xl) < 1e-8 * np.linalg.norm(xl), restart


def test_gmres_mixed_navier_matches_lu(orc):
    g = I.sphere3d(10, 0.35)
    p = O.problem(g, O.NAVIER3D, 0.3, 1.0)
    rng = np.random.default_rng(11)
    bc = (g.rel()[:, 2] < 0).astype(np.uint8)
    bc = np.stack([bc] * 3)
    known = rng.uniform(-1, 1, (3, g.m))
    xl = O.solve_lu(p, bc, known)
    xg, it, rel = O.solve_gmres(p, bc, known, tol=1e-11, restart=60)
    assert rel <= 1e-11
    assert np.linalg.norm(xg - xl) < 1e-8 * np.linalg.norm(xl)
    # Jacobi is what makes it converge in a few dozen steps; without it the
    # same answer, more iterations
    xn, itn, reln = O.solve_gmres(p, bc, known, tol=1e-11, restart=60, precond=False)
    assert reln <= 1e-11 and itn > it
    assert np.linalg.norm(xn - xl) < 1e-8 * np.linalg.norm(xl)
