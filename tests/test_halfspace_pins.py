"""Pins of the oracle's elastic half-space (eq. 9, the surface convolution of
contact mechanics) against closed forms it does not compute itself:

* reciprocity K_ab(d) = K_ba(-d) of the Boussinesq-Cerruti tensor;
* uniform pressure p on a disc of radius a: the surface inside sinks by
  4 (1 - nu^2) p a E(r/a) / (pi E) (E(k) the complete elliptic integral of
  the second kind; 2 (1 - nu^2) p a / E at the centre);
* Hertz pressure p0 sqrt(1 - r^2/a^2): the surface inside the disc is the
  paraboloid u_z = pi (1 - nu^2) p0 (2 a^2 - r^2) / (4 a E);
* uniform tangential traction q on a disc: the centre moves by
  (2 - nu) q a / (2 mu) (the disc integrals of 1/r and x^2/r^3);
* the normal part equals 2 (1 - nu) / mu times the Laplace 3D single layer
  of the same patch laid in a plane of a 3D grid (a separate code path);
* the frictionless solve for the Hertz displacement reaches the Hertz
  pressure and force.

(E = 2 mu (1 + nu).)  Sign errors in the coupling terms fail reciprocity; a
wrong self term or normalisation fails the disc values.
"""

import numpy as np
import pytest

from paper_1809_00845_amd import inputs as I

NU, MU = 0.3, 1.0
E = 2 * MU * (1 + NU)


def _vol(orc, g, sigma, pts):
    """Surface displacement K[sigma] at grid points (the oracle's volume
    form returns S[q] - D[u] = -K[sigma] for this kernel)."""
    p = orc.problem(g, orc.HALFSPACE, NU, MU)
    return -orc.volume(p, sigma, np.zeros_like(sigma), pts)


def test_reciprocity_and_parity(orc):
    rng = np.random.default_rng(0)
    for _ in range(20):
        d = rng.normal(size=2)
        K = orc.halfspace(d, NU, MU)
        Km = orc.halfspace(-d, NU, MU)
        assert np.allclose(K, Km.T, rtol=1e-14, atol=0)
        # the in-plane block is symmetric and even; the coupling terms are odd
        assert np.allclose(K[:2, :2], K[:2, :2].T, rtol=1e-14, atol=0)
        assert np.allclose(K[:2, :2], Km[:2, :2], rtol=1e-14, atol=0)
        assert np.allclose(K[:2, 2], -Km[:2, 2], rtol=1e-14, atol=0)


def test_uniform_pressure_on_a_disc(orc):
    from scipy.special import ellipe

    n, a, pr = 128, 0.3, 1.0
    g = I.halfspace_patch(n, a)
    sigma = np.zeros((3, g.m))
    sigma[2] = pr
    c = np.rint(np.asarray(g.center) / g.h).astype(np.int64)
    u0 = _vol(orc, g, sigma, c[None, :])
    assert abs(u0[2, 0] / (2 * (1 - NU ** 2) * pr * a / E) - 1) < 1e-2
    # inside the disc u_z = 4 (1 - nu^2) p a E(r/a) / (pi E), E(k) the complete
    # elliptic integral of the second kind (it gives the rim value at r = a)
    idx = np.arange(0, g.m, 53)
    r = np.linalg.norm(g.nodes[idx] - g.center, axis=1)
    u = _vol(orc, g, sigma, np.rint(g.nodes[idx] / g.h).astype(np.int64))
    ex = 4 * (1 - NU ** 2) * pr * a / (np.pi * E) * ellipe((r / a) ** 2)
    inner = r < 0.9 * a
    assert np.abs(u[2][inner] / ex[inner] - 1).max() < 5e-3
    # the normal load pulls the surface radially inwards
    out = r > 0.5 * a
    radial = np.sum(u[:2, out] * (g.nodes[idx][out] - g.center).T, axis=0)
    assert np.all(radial < 0)


def test_hertz_pressure_gives_a_paraboloid(orc):
    n, a, p0 = 128, 0.3, 1.0
    g = I.halfspace_patch(n, a)
    rel = g.nodes - g.center
    rr = np.sum(rel ** 2, axis=1)
    sigma = np.zeros((3, g.m))
    sigma[2] = p0 * np.sqrt(np.clip(1 - rr / a ** 2, 0, None))
    idx = np.arange(0, g.m, 97)
    u = _vol(orc, g, sigma, np.rint(g.nodes[idx] / g.h).astype(np.int64))
    ex = np.pi * (1 - NU ** 2) * p0 * (2 * a ** 2 - rr[idx]) / (4 * a * E)
    assert np.abs(u[2] - ex).max() / ex.max() < 1e-2


def test_uniform_shear_on_a_disc(orc):
    n, a, qx = 128, 0.3, 1.0
    g = I.halfspace_patch(n, a)
    sigma = np.zeros((3, g.m))
    sigma[0] = qx
    c = np.rint(np.asarray(g.center) / g.h).astype(np.int64)
    u = _vol(orc, g, sigma, c[None, :])
    assert abs(u[0, 0] / ((2 - NU) * qx * a / (2 * MU)) - 1) < 1e-2
    assert abs(u[1, 0]) < 1e-12 and abs(u[2, 0]) < 1e-12


def test_normal_part_is_a_scaled_laplace_single_layer(orc):
    g = I.halfspace_patch(32, 0.4)
    rng = np.random.default_rng(1)
    pz = rng.uniform(-1, 1, g.m)
    sigma = np.zeros((3, g.m))
    sigma[2] = pz
    p = orc.problem(g, orc.HALFSPACE, NU, MU)
    r = orc.apply(p, sigma, np.zeros((3, g.m)))  # K[sigma] - 0
    # the same patch as a flat plate in the plane z = 5 of a 32^3 grid
    nodes3 = np.concatenate([g.nodes, np.full((g.m, 1), 5 * g.h)], axis=1)
    plate = type(g)(3, (32, 32, 32), g.h, (0.0, 0.0, 0.0), nodes3, np.tile([0.0, 0.0, 1.0], (g.m, 1)),
                    g.weights, np.r_[g.center, 5 * g.h])
    p3 = orc.problem(plate, orc.LAPLACE3D)
    s = -orc.apply(p3, pz, np.zeros(g.m), cmode=orc.C_USER, cuser=np.zeros(g.m))  # S[pz]
    assert np.abs(r[2] - 2 * (1 - NU) / MU * s).max() <= 1e-12 * np.abs(r[2]).max()


@pytest.mark.parametrize("n", [48, 64])
def test_displacement_solve_reaches_hertz(orc, n):
    # frictionless contact: the Hertz paraboloid given for u_z, zero shear
    # traction given for x and y; the solved pressure approaches
    # p0 sqrt(1 - r^2/a^2) and the force 2 pi a^2 p0 / 3
    a, p0 = 0.3, 1.0
    g = I.halfspace_patch(n, a)
    rel = g.nodes - g.center
    rr = np.sum(rel ** 2, axis=1)
    p = orc.problem(g, orc.HALFSPACE, NU, MU)
    bc = np.zeros((3, g.m), dtype=np.uint8)
    bc[:2] = 1
    known = np.zeros((3, g.m))
    known[2] = np.pi * (1 - NU ** 2) * p0 * (2 * a ** 2 - rr) / (4 * a * E)
    sol = orc.solve_lu(p, bc, known)
    ex = p0 * np.sqrt(np.clip(1 - rr / a ** 2, 0, None))
    inner = rr < (0.8 * a) ** 2
    assert np.abs(sol[2][inner] - ex[inner]).max() < 1e-2 * p0
    force = np.sum(sol[2] * g.weights)
    assert abs(force / (2 * np.pi * a ** 2 * p0 / 3) - 1) < 1e-2
