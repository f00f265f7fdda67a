"""Cell-mean kernels (plan option cell_quad, the constant elements of Sec. 4 /
Fig. 5 taken literally): the HIP path against the oracle run with the same
rule, for every kernel family, every working precision, the grid
evaluation, a solve and the full-size cube.

The GPU derives its Gauss-Legendre points by Newton's method on the host; the
oracle takes numpy's leggauss.  Bars are those of the point-sampled operator:
1e-12 in FP64, 2e-5 in FP32 (normwise against the oracle's term scale), 2e-3
in the 16-bit form.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_1809_00845_amd import binding as B  # noqa: E402
from paper_1809_00845_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = {B.FP64: 1e-12, B.FP32: 2e-5, B.BF16_MFMA: 2e-3}
ORC = {B.LAPLACE2D: O.LAPLACE2D, B.LAPLACE3D: O.LAPLACE3D, B.NAVIER3D: O.NAVIER3D, B.HALFSPACE: O.HALFSPACE}
NU, MU = 0.3, 1.0


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.load()
    return torch.device("cuda:0")


def _t(a, dev):
    return torch.tensor(np.ascontiguousarray(a), device=dev)


def _case(name):
    if name == "sphere24":
        return I.sphere3d(24, 0.35), B.LAPLACE3D, 4
    if name == "cube24":
        return I.cube3d(24, 15), B.LAPLACE3D, 2
    if name == "circle64":
        return I.circle2d(64, 0.4), B.LAPLACE2D, 4
    if name == "navier16":
        return I.sphere3d(16, 0.35), B.NAVIER3D, 3
    return I.halfspace_patch(64, 0.35), B.HALFSPACE, 4


def _apply(dev, g, kernel, precision, quad, q, u):
    nc = q.shape[0]
    plan = B.Plan(g, kernel, precision=precision, nu=NU, mu=MU, cell_quad=quad)
    r = plan.apply(_t(q, dev), _t(u, dev))
    torch.cuda.synchronize()
    out = r.cpu().numpy().reshape(nc, -1)
    info = plan.info()
    plan.close()
    return out, info


def _inputs(g, kernel, seed):
    nc = 3 if kernel in (B.NAVIER3D, B.HALFSPACE) else 1
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, (nc, g.m)), rng.uniform(-1, 1, (nc, g.m))


def _oracle(g, kernel, quad, q, u, targets=None):
    p = O.problem(g, ORC[kernel], NU, MU, cell_quad=quad)
    nc = q.shape[0]
    ref, sc = O.apply(p, q if nc > 1 else q[0], u if nc > 1 else u[0], with_scale=True, targets=targets)
    return np.reshape(ref, (nc, -1)), np.max(sc)


@pytest.mark.parametrize("precision", [B.FP64, B.FP32])
@pytest.mark.parametrize("case", ["sphere24", "cube24", "circle64", "navier16", "halfspace64"])
def test_cell_mean_apply_vs_oracle(dev, case, precision):
    g, kernel, quad = _case(case)
    q, u = _inputs(g, kernel, 0)
    r, info = _apply(dev, g, kernel, precision, quad, q, u)
    ref, sc = _oracle(g, kernel, quad, q, u)
    err = np.abs(r - ref).max() / sc
    assert err < TOL[precision], (case, err)
    assert info["spectrum_parity_residual"] < 1e-14
    if precision == B.FP64:
        # the option changes the operator by far more than the bar
        ref0, _ = _oracle(g, kernel, 0, q, u)
        assert np.abs(ref0 - ref).max() / sc > 1e-6


@pytest.mark.parametrize("quad", [2, 5, 8])
def test_cell_mean_rules_of_every_size(dev, quad):
    g = I.sphere3d(16, 0.35)
    q, u = _inputs(g, B.LAPLACE3D, quad)
    r, _ = _apply(dev, g, B.LAPLACE3D, B.FP64, quad, q, u)
    ref, sc = _oracle(g, B.LAPLACE3D, quad, q, u)
    assert np.abs(r - ref).max() / sc < TOL[B.FP64]


def test_one_point_rule_equals_point_sampling(dev):
    g = I.sphere3d(16, 0.35)
    q, u = _inputs(g, B.LAPLACE3D, 1)
    r1, _ = _apply(dev, g, B.LAPLACE3D, B.FP64, 1, q, u)
    r0, _ = _apply(dev, g, B.LAPLACE3D, B.FP64, 0, q, u)
    np.testing.assert_array_equal(r1, r0)


def test_cell_mean_bf16(dev):
    g = I.sphere3d(32, 0.35)
    q, u = _inputs(g, B.LAPLACE3D, 2)
    r, _ = _apply(dev, g, B.LAPLACE3D, B.BF16_MFMA, 4, q, u)
    ref, sc = _oracle(g, B.LAPLACE3D, 4, q, u)
    assert np.abs(r - ref).max() / sc < TOL[B.BF16_MFMA]


def test_cell_mean_grid_field(dev):
    g = I.sphere3d(24, 0.35)
    q, u = _inputs(g, B.LAPLACE3D, 3)
    plan = B.Plan(g, B.LAPLACE3D, precision=B.FP64, cell_quad=4)
    info = plan.info()
    got = plan.eval_grid(_t(q, dev), _t(u, dev)).cpu().numpy().reshape(-1)
    plan.close()
    n0, n1 = info["n"][0], info["n"][1]
    z0, nz = info["z_lo"], info["z_count"]
    z, y, x = np.meshgrid(np.arange(z0, z0 + nz), np.arange(n1), np.arange(n0), indexing="ij")
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], -1)
    idx = np.unique(np.r_[np.random.default_rng(5).choice(len(pts), 400, replace=False), 0, len(pts) - 1])
    p = O.problem(g, O.LAPLACE3D, cell_quad=4)
    ref, sc = O.volume(p, q[0], u[0], pts[idx], with_scale=True)
    assert np.abs(got[idx] - ref).max() / np.max(sc) < TOL[B.FP64]


def test_cell_mean_mixed_solve_vs_lu(dev):
    g = I.sphere3d(24, 0.35)
    u, qv = I.harmonic_3d_xyz(g)
    bc = I.mixed_bc_upper(g)
    known = np.where(bc == 0, u, qv)
    plan = B.Plan(g, B.LAPLACE3D, precision=B.FP64, cell_quad=4)
    x, info = plan.solve(_t(bc, dev), _t(known, dev), tol=1e-10)
    plan.close()
    assert info["status"] == 0 and info["true_relres"] <= 1e-10
    xl = O.solve_lu(O.problem(g, O.LAPLACE3D, cell_quad=4), bc, known)
    assert np.linalg.norm(x.cpu().numpy() - xl) / np.linalg.norm(xl) < 1e-6


def test_cell_mean_full_size_cube_sampled(dev):
    # the 128^3 cube (58,808 nodes, P = 256), first 120 targets
    g = I.cube3d(128, 100)
    q, u = _inputs(g, B.LAPLACE3D, 4)
    r, info = _apply(dev, g, B.LAPLACE3D, B.FP32, 4, q, u)
    ref, sc = _oracle(g, B.LAPLACE3D, 4, q, u, targets=(0, 120))
    assert info["pad"][0] == 256
    assert np.abs(r[:, :120] - ref).max() / sc < TOL[B.FP32]
