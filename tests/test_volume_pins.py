"""Pins of the oracle's grid evaluation (the representation formula at grid
points: c = 1 inside the boundary, 0 outside, Sec. 2; the convolution over
the whole grid, Sec. 4) against facts it does not compute itself:

* Gauss: the double layer of a constant density is -1 inside a closed
  surface and 0 outside, so u = 1, q = 0 gives 1 inside and 0 outside;
* harmonic data u with its flux q reproduce u inside and 0 outside;
* Navier: a rigid translation (t = 0) and a linear field with its Hooke
  traction are reproduced inside, 0 outside;
* at a node's own grid point the value differs from the pinned boundary
  operator only by the (grid - exact) self term of the single layer.

A sign error in either layer, a swapped offset (the odd kernels change
sign) or a missing term fails one of these.  Targets keep at least three
cells from the boundary, where the snapped discretisation is accurate.
"""

import numpy as np
import pytest

from paper_1809_00845_amd import inputs as I


def _targets(g, radius, margin=3.0, stride_in=1, stride_out=1):
    n = g.n[: g.dim]
    grid = np.stack(np.meshgrid(*[np.arange(a) for a in n], indexing="ij"), -1).reshape(-1, g.dim)
    pos = np.asarray(g.origin[: g.dim]) + g.h * grid
    d = np.linalg.norm(pos - g.center[None], axis=1)
    ins = np.where(d < radius - margin * g.h)[0][::stride_in]
    out = np.where(d > radius + margin * g.h)[0][::stride_out]
    return grid[ins], pos[ins] - g.center, grid[out]


def test_volume_laplace3d_gauss_and_harmonic(orc):
    g = I.sphere3d(32, 0.35)
    p = orc.problem(g, orc.LAPLACE3D)
    gi, rel, go = _targets(g, 0.35, stride_in=7, stride_out=41)
    assert len(gi) > 50 and len(go) > 50
    ones, zeros = np.ones(g.m), np.zeros(g.m)
    assert np.abs(orc.volume(p, zeros, ones, gi) - 1.0).max() < 1e-2
    assert np.abs(orc.volume(p, zeros, ones, go)).max() < 5e-3
    u, q = I.harmonic_3d_xyz(g)
    scale = np.abs(u).max()
    ex = rel[:, 0] * rel[:, 1] * rel[:, 2]
    assert np.abs(orc.volume(p, q, u, gi) - ex).max() / scale < 3e-3
    assert np.abs(orc.volume(p, q, u, go)).max() / scale < 1e-3
    # each layer alone is far from the field: both signs matter
    assert np.abs(orc.volume(p, q, zeros, gi) - ex).max() / scale > 0.05
    assert np.abs(orc.volume(p, zeros, u, gi) - ex).max() / scale > 0.05


def test_volume_laplace2d_gauss_and_harmonic(orc):
    g = I.circle2d(64, 0.4)
    p = orc.problem(g, orc.LAPLACE2D)
    gi, rel, go = _targets(g, 0.4, stride_in=5, stride_out=5)
    ones, zeros = np.ones(g.m), np.zeros(g.m)
    assert np.abs(orc.volume(p, zeros, ones, gi) - 1.0).max() < 2e-2
    assert np.abs(orc.volume(p, zeros, ones, go)).max() < 2e-2
    u, q = I.harmonic_2d_x2y2(g)
    scale = np.abs(u).max()
    ex = rel[:, 0] ** 2 - rel[:, 1] ** 2
    assert np.abs(orc.volume(p, q, u, gi) - ex).max() / scale < 2e-2
    assert np.abs(orc.volume(p, q, u, go)).max() / scale < 2e-2
    assert np.abs(orc.volume(p, q, np.zeros(g.m), gi) - ex).max() / scale > 0.1


def test_volume_navier_rigid_and_linear(orc):
    nu, mu = 0.3, 1.0
    lam = 2 * mu * nu / (1 - 2 * nu)
    g = I.sphere3d(16, 0.35)
    p = orc.problem(g, orc.NAVIER3D, nu, mu)
    gi, rel, go = _targets(g, 0.35, stride_in=3, stride_out=17)
    m = g.m
    for k in range(3):
        u = np.zeros((3, m))
        u[k] = 1.0
        e = np.zeros((3, len(gi)))
        e[k] = 1.0
        assert np.abs(orc.volume(p, np.zeros((3, m)), u, gi) - e).max() < 3e-2
        assert np.abs(orc.volume(p, np.zeros((3, m)), u, go)).max() < 1e-2
    E = np.random.default_rng(11).normal(size=(3, 3))
    Es = 0.5 * (E + E.T)
    u = (g.rel() @ E.T).T
    sig = lam * np.trace(Es) * np.eye(3) + 2 * mu * Es
    t = (g.normals @ sig.T).T
    scale = np.abs(u).max()
    assert np.abs(orc.volume(p, t, u, gi) - (rel @ E.T).T).max() / scale < 1e-2
    assert np.abs(orc.volume(p, t, u, go)).max() / scale < 1e-2


@pytest.mark.parametrize("kernel", ["laplace2d", "laplace3d", "navier"])
def test_volume_at_nodes_is_the_operator_without_self_terms(orc, kernel):
    if kernel == "laplace2d":
        g, kk, nc = I.circle2d(32, 0.4), orc.LAPLACE2D, 1
    elif kernel == "laplace3d":
        g, kk, nc = I.sphere3d(16, 0.35), orc.LAPLACE3D, 1
    else:
        g, kk, nc = I.sphere3d(12, 0.35), orc.NAVIER3D, 3
    p = orc.problem(g, kk)
    rng = np.random.default_rng(5)
    q = rng.uniform(-1, 1, (nc, g.m))
    u = rng.uniform(-1, 1, (nc, g.m))
    gidx = orc.snap(p)
    v = np.reshape(orc.volume(p, q, u, gidx), (nc, g.m))
    # c = 0: r = D[u] - S[q] with the exact self term of the single layer
    r = np.reshape(orc.apply(p, q, u, cmode=orc.C_USER, cuser=np.zeros((g.m, nc * nc))), (nc, g.m))
    k0 = orc.grid_k0(kk, g.h, p.nu, p.mu)
    for j in range(g.m):
        w = g.weights[j]
        if kk == orc.LAPLACE2D:
            d = np.array([[k0[0, 0] * w - orc.self_laplace2d(w)]])
        elif kk == orc.LAPLACE3D:
            d = np.array([[k0[0, 0] * w - orc.self_laplace3d(w)]])
        else:
            d = k0 * w - orc.self_kelvin(w, g.normals[j], p.nu, p.mu)
        want = -r[:, j] + d @ q[:, j]
        assert np.abs(v[:, j] - want).max() <= 1e-12 * (1 + np.abs(r[:, j]).max())
