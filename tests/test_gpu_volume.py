"""GPU parity of the grid evaluation (bemfft_eval_grid): S[q] - D[u] at every
point of the grid box, against the oracle's direct sum at the same points.

Bar (normwise, scale = sum of the terms' magnitudes at each point, from the
oracle): 1e-12 in FP64; 2e-5 in FP32, as for the boundary operator (the
same transforms and products, plus one more inverse stage).
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_1809_00845_amd import binding as B  # noqa: E402
from paper_1809_00845_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = {B.FP64: 1e-12, B.FP32: 2e-5}
ORC_KIND = {B.LAPLACE2D: O.LAPLACE2D, B.LAPLACE3D: O.LAPLACE3D, B.NAVIER3D: O.NAVIER3D}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.load()
    return torch.device("cuda:0")


def _t(a, dev):
    return torch.tensor(np.ascontiguousarray(a), device=dev)


def _box_points(info, dim):
    """Grid indices (x, y[, z]) of the evaluated box, in the output's order."""
    n0, n1 = info["n"][0], info["n"][1]
    if dim == 2:
        y, x = np.meshgrid(np.arange(n1), np.arange(n0), indexing="ij")
        return np.stack([x.ravel(), y.ravel()], -1)
    z0, nz = info["z_lo"], info["z_count"]
    z, y, x = np.meshgrid(np.arange(z0, z0 + nz), np.arange(n1), np.arange(n0), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], -1)


def _volume_parity(dev, g, kernel, precision, seed=0, sample=None, nu=0.3, mu=1.0):
    nc = 3 if kernel == B.NAVIER3D else 1
    m = len(g.weights)
    rng = np.random.default_rng(seed)
    q = rng.uniform(-1, 1, (nc, m))
    u = rng.uniform(-1, 1, (nc, m))
    plan = B.Plan(g, kernel, precision=precision, nu=nu, mu=mu)
    info = plan.info()
    out = plan.eval_grid(_t(q, dev), _t(u, dev))
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(nc, -1)
    pts = _box_points(info, g.dim)
    assert got.shape[1] == len(pts)
    idx = np.arange(len(pts)) if sample is None else np.unique(
        np.r_[rng.choice(len(pts), sample, replace=False), 0, len(pts) - 1])
    p = O.problem(g, ORC_KIND[kernel], nu, mu)
    ref, sc = O.volume(p, q if nc > 1 else q[0], u if nc > 1 else u[0], pts[idx], with_scale=True)
    ref = np.reshape(ref, (nc, -1))
    err = np.abs(got[:, idx] - ref).max() / np.max(sc)
    plan.close()
    return err, info, got, pts


@pytest.mark.parametrize("precision", [B.FP64, B.FP32])
@pytest.mark.parametrize("case", ["sphere24", "cube24", "circle64", "navier16"])
def test_eval_grid_whole_box_vs_oracle(dev, case, precision):
    if case == "sphere24":  # P = 64 > 2n: the x and y cuts at n < P/2
        g, kernel = I.sphere3d(24, 0.35), B.LAPLACE3D
    elif case == "cube24":  # box faces in grid planes: the long-row transforms
        g, kernel = I.cube3d(24, 15), B.LAPLACE3D
    elif case == "circle64":
        g, kernel = I.circle2d(64, 0.4), B.LAPLACE2D
    else:
        g, kernel = I.sphere3d(16, 0.35), B.NAVIER3D
    err, info, _, _ = _volume_parity(dev, g, kernel, precision)
    assert err < TOL[precision], (case, err)


def test_eval_grid_2d_padded_1024_sampled(dev):
    # the 500-per-side square on its 500^2 grid (P = 1024)
    g = I.square2d(500, 500)
    err, info, _, _ = _volume_parity(dev, g, B.LAPLACE2D, B.FP64, seed=6, sample=300)
    assert info["pad"][0] == 1024 and err < TOL[B.FP64]


def test_eval_grid_odd_row_count(dev):
    # 2D, ny odd: the last pencil of the x pass carries one row
    g = I.circle2d(45, 0.4)
    err, info, got, _ = _volume_parity(dev, g, B.LAPLACE2D, B.FP64, seed=3)
    assert info["n"][1] % 2 == 1 and err < TOL[B.FP64]


@pytest.mark.parametrize("precision", [B.FP64, B.FP32])
def test_eval_grid_full_size_cube_sampled(dev, precision):
    # the 128^3 cube of the throughput measurement: 58,808 nodes, P = 256
    g = I.cube3d(128, 100)
    err, info, _, _ = _volume_parity(dev, g, B.LAPLACE3D, precision, seed=4, sample=150)
    assert info["pad"][0] == 256 and err < TOL[precision]


def test_eval_grid_navier_star_sampled(dev):
    # the 192^3 Navier star (P = 384, 3 outputs), FP32
    spec = I.draw_stars(1, 1)[0]
    g = I.star3d(192, spec)
    err, info, _, _ = _volume_parity(dev, g, B.NAVIER3D, B.FP32, seed=5, sample=40)
    assert info["pad"][0] == 384 and err < TOL[B.FP32]


def test_eval_grid_interior_field_at_full_size(dev):
    """Property at any size: u = 1, q = 0 gives 1 inside and 0 outside
    (Gauss); harmonic data give the harmonic function inside.  128^3 sphere,
    every box point at least 6 cells from the boundary.  The bounds are the
    discretisation error of the snapped boundary, which the oracle shows at
    the same points (Gauss: 3.7e-3 inside, 5.2e-3 outside at 6-8 cells;
    1.5e-2 at 3-4 cells)."""
    g = I.sphere3d(128, 0.35)
    plan = B.Plan(g, B.LAPLACE3D, precision=B.FP32)
    info = plan.info()
    pts = _box_points(info, 3)
    pos = np.asarray(g.origin) + g.h * pts
    d = np.linalg.norm(pos - g.center[None], axis=1)
    ins, outs = d < 0.35 - 6 * g.h, d > 0.35 + 6 * g.h
    ones = torch.ones(g.m, dtype=torch.float64, device=dev)
    v = plan.eval_grid(torch.zeros_like(ones), ones).cpu().numpy().reshape(-1)
    assert np.abs(v[ins] - 1).max() < 1e-2 and np.abs(v[outs]).max() < 1e-2
    u, q = I.harmonic_3d_xyz(g)
    v = plan.eval_grid(_t(q, dev), _t(u, dev)).cpu().numpy().reshape(-1)
    rel = pos - g.center
    ex = rel[:, 0] * rel[:, 1] * rel[:, 2]
    scale = np.abs(u).max()
    assert np.abs(v[ins] - ex[ins]).max() / scale < 1e-3 and np.abs(v[outs]).max() / scale < 1e-3
    plan.close()


def test_eval_grid_after_solve_reproduces_dirichlet_data(dev):
    """Solve for q from Dirichlet data, then evaluate inside: the field equals
    the harmonic function the data came from (the step after the solve)."""
    g = I.sphere3d(64, 0.35)
    u, _ = I.harmonic_3d_xyz(g)
    plan = B.Plan(g, B.LAPLACE3D, precision=B.FP64)
    bc = torch.zeros(g.m, dtype=torch.uint8, device=dev)
    ut = _t(u, dev)
    q, res = plan.solve(bc, ut, tol=1e-8)
    assert res["status"] == 0
    v = plan.eval_grid(q, ut).cpu().numpy().reshape(-1)
    pts = _box_points(plan.info(), 3)
    pos = np.asarray(g.origin) + g.h * pts
    d = np.linalg.norm(pos - g.center[None], axis=1)
    ins = d < 0.35 - 4 * g.h
    rel = pos - g.center
    ex = rel[:, 0] * rel[:, 1] * rel[:, 2]
    assert np.abs(v[ins] - ex[ins]).max() / np.abs(u).max() < 1e-2
    plan.close()


def test_eval_grid_rejects_null(dev):
    g = I.sphere3d(16, 0.35)
    plan = B.Plan(g, B.LAPLACE3D)
    st = B.load().bemfft_eval_grid(plan.handle, None, None, None, None)
    assert st == B.EINVAL
    plan.close()
