"""Pins of the premise and the oracle of the paper's CG solve (end of Sec. 4):
the Dirichlet single-layer matrix S = G W becomes symmetric positive definite
after the scaling W^1/2 S W^-1/2 (3D; 2D for boundaries of logarithmic
capacity below 1), and CG on it reaches the textbook LU solution of the
Dirichlet system."""

import numpy as np
import pytest

from paper_1809_00845_amd import inputs as I


def _geoms(orc):
    return [
        ("circle", I.circle2d(32, 0.4), orc.LAPLACE2D),
        ("square", I.square2d(32, 25), orc.LAPLACE2D),
        ("sphere", I.sphere3d(12, 0.35), orc.LAPLACE3D),
        ("cube", I.cube3d(16, 10), orc.LAPLACE3D),
    ]


def test_symmetrised_single_layer_is_spd(orc):
    for name, g, kernel in _geoms(orc):
        p = orc.problem(g, kernel)
        S, _, _ = orc.assemble(p)
        sw = np.sqrt(g.weights)
        A = sw[:, None] * S / sw[None, :]
        assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max(), name
        ev = np.linalg.eigvalsh(0.5 * (A + A.T))
        assert ev.min() > 0, (name, ev.min())
        # S itself is not symmetric when the weights differ
        if np.ptp(g.weights) > 1e-3 * g.weights.max():
            assert np.abs(S - S.T).max() > 1e-6 * np.abs(S).max(), name


def test_2d_capacity_above_one_loses_definiteness(orc):
    # the same circle scaled by 4 (radius 1.6 > 1, capacity 1.6): S gains a
    # negative eigenvalue, so CG does not apply there
    g = I.circle2d(32, 0.4)
    big = type(g)(g.dim, g.n, 4 * g.h, g.origin, 4 * np.asarray(g.nodes), g.normals, 4 * g.weights, 4 * g.center)
    p = orc.problem(big, orc.LAPLACE2D)
    S, _, _ = orc.assemble(p)
    sw = np.sqrt(big.weights)
    A = sw[:, None] * S / sw[None, :]
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() < 0


@pytest.mark.parametrize("precond", [False, True])
def test_cg_reaches_the_lu_solution(orc, precond):
    for name, g, kernel in _geoms(orc):
        p = orc.problem(g, kernel)
        u, _ = (I.harmonic_2d_x2y2 if kernel == orc.LAPLACE2D else I.harmonic_3d_xyz)(g)
        q_lu = orc.solve_lu(p, np.zeros(g.m, dtype=np.uint8), u)
        q, it = orc.dirichlet_cg(p, u, tol=1e-12, precond=precond)
        assert np.linalg.norm(q - q_lu) <= 1e-9 * np.linalg.norm(q_lu), name
        assert 0 < it < g.m, name
        # started from the solution, no iteration is needed
        _, it0 = orc.dirichlet_cg(p, u, tol=1e-8, precond=precond, x0=q_lu)
        assert it0 == 0, name
