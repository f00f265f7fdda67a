"""Pins of the oracle's cell-mean kernels (constant elements, Sec. 4 / Fig. 5).

With a cell rule the oracle replaces each kernel value at a grid offset
m != 0 by its mean over the grid cell centred on the offset.  These tests
hold that step against things the oracle does not compute itself:

* the closed-form integral of 1/r over a box (the antiderivative
  yz ln(x+r) + xz ln(y+r) + xy ln(z+r) - x^2/2 atan(yz/(xr)) - ...) for the
  3D single layer, and the closed-form face integrals of 1/r for the mean of
  its gradient (divergence theorem: the mean of d/dx_a over a box is the
  difference of the two a-faces' integrals over the volume);
* scipy's adaptive quadrature of the pair kernels for Laplace 2D, Kelvin
  (both tensors) and the half-space, at offsets where the Gauss rule has
  converged far below the tolerance;
* special cases: a one-point rule is the point value, and offset 0 keeps its
  self and same-cell values whatever the rule.

Each pin runs the oracle's whole apply (or volume) on two nodes, so the
offset, sign, scaling by h and weighting of the rule are all in the path.
"""

import numpy as np
import pytest
from scipy import integrate

import oracle

pytestmark = pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")

H = 0.125
ORIGIN = np.zeros(3)


def _two_nodes(kernel, m, normal1=(0.6, 0.0, 0.8), w=(0.011, 0.023), q=8, nu=0.3, mu=1.0):
    dim = 2 if kernel in (oracle.LAPLACE2D, oracle.HALFSPACE) else 3
    g0 = np.full(dim, 4)
    g1 = g0 + np.asarray(m[:dim])
    nodes = np.stack([g0, g1]).astype(np.float64) * H
    n1 = np.asarray(normal1[:dim], dtype=np.float64)
    n1 = n1 / np.linalg.norm(n1)
    normals = np.stack([n1, n1])
    return oracle.Problem(kernel, H, ORIGIN[:dim].copy(), np.full(dim, 12, dtype=np.int64),
                          np.ascontiguousarray(nodes), np.ascontiguousarray(normals),
                          np.asarray(w, dtype=np.float64), nu, mu, q)


def _single_col(p):
    """-r_0 for q = (0, 1), u = 0: the single-layer entry G_01 (per component)."""
    nc = p.ncomp
    out = np.zeros((nc, nc))
    for b in range(nc):
        qv = np.zeros((nc, 2))
        qv[b, 1] = 1.0
        r = oracle.apply(p, qv, np.zeros((nc, 2)), cmode=oracle.C_HALF)
        out[:, b] = -np.reshape(r, (nc, 2))[:, 0]
    return out


def _double_col(p):
    """r_0 for u = (0, e_b), q = 0 and c = 1/2: the double-layer entry H_01."""
    nc = p.ncomp
    out = np.zeros((nc, nc))
    for b in range(nc):
        uv = np.zeros((nc, 2))
        uv[b, 1] = 1.0
        r = oracle.apply(p, np.zeros((nc, 2)), uv, cmode=oracle.C_HALF)
        out[:, b] = np.reshape(r, (nc, 2))[:, 0]
    return out


def _box_inv_r(lo, hi):
    """Integral of 1/r over the box [lo, hi] (closed form)."""
    def f(x, y, z):
        r = np.sqrt(x * x + y * y + z * z)
        return (y * z * np.log(x + r) + x * z * np.log(y + r) + x * y * np.log(z + r)
                - 0.5 * x * x * np.arctan(y * z / (x * r)) - 0.5 * y * y * np.arctan(x * z / (y * r))
                - 0.5 * z * z * np.arctan(x * y / (z * r)))
    s = 0.0
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                s += (-1) ** (a + b + c) * f((hi, lo)[a][0], (hi, lo)[b][1], (hi, lo)[c][2])
    return s


def _face_inv_r(x, lo, hi):
    """Integral of 1/r over the rectangle [lo, hi] of the plane at distance x."""
    def g(y, z):
        r = np.sqrt(x * x + y * y + z * z)
        return y * np.log(z + r) + z * np.log(y + r) - x * np.arctan(y * z / (x * r))
    return g(hi[0], hi[1]) - g(lo[0], hi[1]) - g(hi[0], lo[1]) + g(lo[0], lo[1])


@pytest.mark.parametrize("m", [(1, 0, 0), (1, 1, 0), (-1, 2, 1), (3, -2, 5)])
def test_laplace3d_single_layer_cell_mean_closed_form(m):
    p = _two_nodes(oracle.LAPLACE3D, m)
    lo = (np.asarray(m, float) - 0.5) * H
    hi = lo + H
    mean = _box_inv_r(lo, hi) / H**3 / (4 * np.pi)
    got = _single_col(p)[0, 0]
    assert got == pytest.approx(p.weights[1] * mean, rel=5e-8)  # 8-point rule next to the source


# tolerance: the 8-point rule's own error, largest in the cells next to the source
@pytest.mark.parametrize("m,rel", [((1, 0, 0), 1e-6), ((0, -1, 1), 1e-7), ((2, 1, -3), 1e-9)])
def test_laplace3d_double_layer_cell_mean_closed_form(m, rel):
    p = _two_nodes(oracle.LAPLACE3D, m, normal1=(0.48, -0.6, 0.64))
    lo = (np.asarray(m, float) - 0.5) * H
    hi = lo + H
    grad = np.zeros(3)
    for a in range(3):
        o = [b for b in range(3) if b != a]
        upper = _face_inv_r(hi[a], lo[o], hi[o])
        lower = _face_inv_r(lo[a], lo[o], hi[o])
        grad[a] = (upper - lower) / H**3 / (4 * np.pi)  # mean of d/dx_a (1/(4 pi r))
    want = p.weights[1] * grad @ p.normals[1]
    got = _double_col(p)[0, 0]
    assert got == pytest.approx(want, rel=rel, abs=rel * abs(p.weights[1] * grad).max())


def test_laplace3d_q4_error_far_from_the_source():
    # the 4-point rule the plans use: converged to ~1e-7 two cells out
    m = (2, 1, 0)
    p = _two_nodes(oracle.LAPLACE3D, m, q=4)
    lo = (np.asarray(m, float) - 0.5) * H
    mean = _box_inv_r(lo, lo + H) / H**3 / (4 * np.pi)
    assert _single_col(p)[0, 0] == pytest.approx(p.weights[1] * mean, rel=1e-6)
    # and it differs from the point value by far more than that
    p0 = _two_nodes(oracle.LAPLACE3D, m, q=0)
    assert abs(_single_col(p0)[0, 0] / _single_col(p)[0, 0] - 1) > 1e-4


def _dbl(fn, m):
    lo = (np.asarray(m[:2], float) - 0.5) * H
    val, _ = integrate.dblquad(lambda y, x: fn(np.array([x, y])), lo[0], lo[0] + H, lo[1], lo[1] + H,
                               epsabs=0, epsrel=1e-12)
    return val / H**2


@pytest.mark.parametrize("m,rel", [((1, 0), 1e-8), ((2, -3), 1e-10)])
def test_laplace2d_cell_mean_vs_adaptive_quadrature(m, rel):
    p = _two_nodes(oracle.LAPLACE2D, m, normal1=(0.8, -0.6))
    g = _single_col(p)[0, 0] / p.weights[1]
    want = _dbl(lambda xi: oracle.laplace2d(xi)[0], m)
    assert g == pytest.approx(want, rel=rel)
    d = _double_col(p)[0, 0] / p.weights[1]
    n = p.normals[1]
    want_d = _dbl(lambda xi: oracle.laplace2d(xi)[1] * n[0] + oracle.laplace2d(xi)[2] * n[1], m)
    assert d == pytest.approx(want_d, rel=100 * rel)


def _tpl(fn, m):
    lo = (np.asarray(m, float) - 0.5) * H
    val, _ = integrate.tplquad(lambda z, y, x: fn(np.array([x, y, z])), lo[0], lo[0] + H, lo[1], lo[1] + H,
                               lo[2], lo[2] + H, epsabs=0, epsrel=1e-11)
    return val / H**3


def test_kelvin_cell_means_vs_adaptive_quadrature():
    m = (2, -1, 1)
    nu, mu = 0.27, 1.3
    p = _two_nodes(oracle.NAVIER3D, m, normal1=(0.36, 0.48, 0.8), nu=nu, mu=mu)
    G = _single_col(p) / p.weights[1]
    Hm = _double_col(p) / p.weights[1]
    n = p.normals[1]
    for a in range(3):
        for b in range(3):
            gu = _tpl(lambda xi: oracle.kelvin_u(xi, nu, mu)[a, b], m)
            gt = _tpl(lambda xi: oracle.kelvin_t(xi, n, nu)[a, b], m)
            assert G[a, b] == pytest.approx(gu, rel=1e-9, abs=1e-11 * abs(G).max())
            assert Hm[a, b] == pytest.approx(gt, rel=1e-9, abs=1e-11 * abs(Hm).max())


def test_halfspace_cell_means_vs_adaptive_quadrature():
    m = (1, -2)
    nu, mu = 0.3, 0.8
    p = _two_nodes(oracle.HALFSPACE, m, nu=nu, mu=mu)
    G = _single_col(p) / p.weights[1]
    # apply gives K[sigma] at target 0 from node 1: K at d = p_0 - p_1
    for a in range(3):
        for b in range(3):
            want = _dbl(lambda xi: oracle.halfspace(-xi, nu, mu)[a, b], m)
            assert -G[a, b] == pytest.approx(want, rel=1e-9, abs=1e-11 * abs(G).max())


@pytest.mark.parametrize("kernel", [oracle.LAPLACE2D, oracle.LAPLACE3D, oracle.NAVIER3D, oracle.HALFSPACE])
def test_one_point_rule_is_the_point_value(kernel):
    m = (1, 2, -1)
    a = _two_nodes(kernel, m, q=1)
    b = _two_nodes(kernel, m, q=0)
    np.testing.assert_array_equal(_single_col(a), _single_col(b))
    np.testing.assert_array_equal(_double_col(a), _double_col(b))


@pytest.mark.parametrize("kernel", [oracle.LAPLACE3D, oracle.NAVIER3D])
def test_offset_zero_unchanged_by_the_rule(kernel):
    # two nodes in one cell plus the self terms: the rule does not touch them
    p4 = _two_nodes(kernel, (0, 0, 0), q=4)
    p0 = _two_nodes(kernel, (0, 0, 0), q=0)
    S4, D4, c4 = oracle.assemble(p4)
    S0, D0, c0 = oracle.assemble(p0)
    np.testing.assert_array_equal(S4, S0)
    np.testing.assert_array_equal(D4, D0)


def test_volume_uses_the_same_cell_means():
    # the grid field of one source at a node-free grid point two cells away
    m = (2, 0, -1)
    p = _two_nodes(oracle.LAPLACE3D, (5, 5, 5), q=8)
    target = np.array([[4 - m[0], 4 - m[1], 4 - m[2]]])  # source node 0 sits at (4,4,4)
    qv = np.array([1.0, 0.0])
    v = oracle.volume(p, qv, np.zeros(2), target)
    lo = (np.asarray(m, float) - 0.5) * H
    mean = _box_inv_r(lo, lo + H) / H**3 / (4 * np.pi)
    assert v[0] == pytest.approx(p.weights[0] * mean, rel=2e-9)


def test_assemble_and_apply_agree_with_the_rule():
    rng = np.random.default_rng(7)
    g = rng.integers(0, 12, size=(40, 3))
    nodes = g * H
    nr = rng.normal(size=(40, 3))
    nr /= np.linalg.norm(nr, axis=1, keepdims=True)
    p = oracle.Problem(oracle.LAPLACE3D, H, ORIGIN.copy(), np.full(3, 12, dtype=np.int64),
                       np.ascontiguousarray(nodes, dtype=np.float64), np.ascontiguousarray(nr),
                       rng.uniform(0.5, 1.5, 40) * H * H, 0.3, 1.0, 4)
    S, D, c = oracle.assemble(p)
    q = rng.normal(size=40)
    u = rng.normal(size=40)
    r = oracle.apply(p, q, u)
    want = c[:, 0] * u + D @ u - S @ q
    np.testing.assert_allclose(r, want, rtol=0, atol=1e-12 * np.abs(want).max())
