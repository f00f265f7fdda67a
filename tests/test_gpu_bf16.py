"""The 16-bit form (BEMFFT_BF16_MFMA): BF16 storage of the transformed
fields, the inverse z results and the kernel spectra, z transforms as dense
DFT matrix products on the matrix cores with FP32 accumulation.  Parity with
the FP64 oracle at a stated bound, on every compiled z length and at full
size, and FP64-refined solves that reach FP64 accuracy.

Bar (normwise against the oracle's term scale, as the FP32 bar): BF16 keeps
8 significant bits, unit round-off u = 2^-9 ~ 2e-3.  A value is rounded
where it is stored (Y, Z, spectra), as each stage's matrix operand (two
stages forward, two inverse) and in the DFT matrices themselves; the
roundings are independent and each transform sum is bounded by the term
magnitudes, so the error stays a fraction of u of the term scale.  Measured
1.3e-4 to 4.3e-4 on every case below; BAR = 2e-3 (one unit round-off)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_1809_00845_amd import binding as B  # noqa: E402
from paper_1809_00845_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu

BAR = 2e-3
KINDS = {B.LAPLACE3D: O.LAPLACE3D, B.NAVIER3D: O.NAVIER3D}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.load()
    return torch.device("cuda:0")


def _t(a, dev):
    return torch.tensor(np.ascontiguousarray(a), device=dev)


def _err(dev, g, kernel, targets=None, seed=0, precision=None):
    nc = 3 if kernel == B.NAVIER3D else 1
    m = len(g.weights)
    rng = np.random.default_rng(seed)
    q = rng.uniform(-1, 1, (nc, m))
    u = rng.uniform(-1, 1, (nc, m))
    plan = B.Plan(g, kernel, precision=B.BF16_MFMA if precision is None else precision)
    r = plan.apply(_t(q, dev), _t(u, dev))
    torch.cuda.synchronize()
    r = r.cpu().numpy().reshape(nc, m)
    info = plan.info()
    plan.close()
    p = O.problem(g, KINDS[kernel])
    ref, sc = O.apply(p, q if nc > 1 else q[0], u if nc > 1 else u[0], with_scale=True, targets=targets)
    ref = np.reshape(ref, (nc, -1))
    t0, t1 = targets or (0, m)
    return np.abs(r[:, t0:t1] - ref).max() / np.max(sc), info


@pytest.mark.parametrize("n", [16, 32, 48, 64, 96, 128, 160, 192, 256])
def test_bf16_every_z_length(dev, n):
    """Sphere on n^3 padded to 2n: z lengths 32 ... 512 (one, two or eight
    pencils per 16 x 16 tile, or two tiles per pencil)."""
    g = I.sphere3d(n, 0.35)
    tg = (g.m // 3, min(g.m, g.m // 3 + 300))
    err, info = _err(dev, g, B.LAPLACE3D, targets=tg)
    print(f"bf16 sphere n={n} P={2 * n}: {err:.2e}")
    assert info["precision"] == B.BF16_MFMA and info["pad"][2] == 2 * n
    assert err < BAR, (n, err)


def test_bf16_long_rows_and_ragged_grid(dev):
    """Face planes whose rows take the row FFT; and unequal axes (40 x 24 x
    20 padded 96 x 64 x 64) with a shape that touches a few planes only."""
    err, _ = _err(dev, I.cube3d(48, 30).permuted(3), B.LAPLACE3D)
    print(f"bf16 cube48: {err:.2e}")
    assert err < BAR
    rng = np.random.default_rng(5)
    gi = np.stack([rng.integers(3, 37, 300), rng.integers(2, 22, 300), rng.integers(8, 13, 300)], 1)

    class G:
        pass

    g = G()
    g.dim, g.n, g.h, g.origin = 3, (40, 24, 20), 1.0 / 40, (0.0, 0.0, 0.0)
    g.nodes = gi * g.h
    nv = rng.normal(size=(300, 3))
    g.normals = nv / np.linalg.norm(nv, axis=1, keepdims=True)
    g.weights = rng.uniform(0.2, 1.5, 300) * g.h ** 2
    err, info = _err(dev, g, B.LAPLACE3D)
    print(f"bf16 ragged: {err:.2e}")
    assert info["pad"] == [96, 64, 64] and err < BAR


@pytest.mark.parametrize("n", [16, 24])
def test_bf16_navier_sphere(dev, n):
    err, info = _err(dev, I.sphere3d(n, 0.35), B.NAVIER3D)
    print(f"bf16 navier sphere n={n}: {err:.2e}")
    assert info["nspectra"] == 24 and err < BAR


def test_bf16_config2_cube_full_size(dev):
    g = I.cube3d(128, 100)
    for tg in ((0, 400), (29000, 29400)):
        err, info = _err(dev, g, B.LAPLACE3D, targets=tg)
        print(f"bf16 cube128 {tg}: {err:.2e}")
        assert info["pad"] == [256, 256, 256] and err < BAR


def test_bf16_config3_navier_star_full_size(dev):
    """The 192^3 star padded to 384^3 (two column tiles per z pencil)."""
    g = I.star3d(192, I.draw_stars(1, 1)[0])
    err, info = _err(dev, g, B.NAVIER3D, targets=(2000, 2120))
    print(f"bf16 navier star192: {err:.2e}")
    assert info["pad"] == [384, 384, 384] and err < BAR
    # the spectra are stored in 16 bits, kz rows padded to 200 values
    assert info["spectra_bytes"] == 24 * 193 * 193 * 200 * 2


def test_bf16_refined_solves_reach_fp64(dev):
    """FP64 residuals, BF16-transform corrections: the mixed sphere problem
    and a Navier mixed problem reach 1e-10 in the FP64 residual and the
    oracle's LU solution."""
    g = I.sphere3d(32, 0.35)
    u, q = I.harmonic_3d_xyz(g)
    bc = I.mixed_bc_upper(g)
    known = np.where(bc == 0, u, q)
    plan = B.Plan(g, B.LAPLACE3D, precision=B.BF16_MFMA, keep_fp64=True)
    x, info = plan.solve(_t(bc, dev), _t(known, dev), tol=1e-10, refine=1, inner_tol=1e-2)
    print("bf16 refined sphere:", info)
    assert info["status"] == 0 and info["true_relres"] <= 1e-10
    xl = O.solve_lu(O.problem(g, O.LAPLACE3D), bc, known)
    assert np.linalg.norm(x.cpu().numpy() - xl) / np.linalg.norm(xl) < 1e-6
    plan.close()
    g = I.sphere3d(16, 0.35)
    rng = np.random.default_rng(4)
    bcn = np.stack([(g.rel()[:, 2] < 0).astype(np.uint8)] * 3)
    kn = rng.uniform(-1, 1, (3, g.m))
    pn = B.Plan(g, B.NAVIER3D, precision=B.BF16_MFMA, keep_fp64=True)
    xn, info = pn.solve(_t(bcn, dev), _t(kn, dev), tol=1e-10, refine=1, inner_tol=1e-2)
    print("bf16 refined navier:", info)
    assert info["status"] == 0 and info["true_relres"] <= 1e-10
    xl = O.solve_lu(O.problem(g, O.NAVIER3D, 0.3, 1.0), bcn, kn).reshape(-1)
    assert np.linalg.norm(xn.cpu().numpy().reshape(-1) - xl) / np.linalg.norm(xl) < 1e-6
    pn.close()


def test_bf16_grid_field(dev):
    """The field over the grid box through the 16-bit passes, at every point
    of a small sphere's box, against the oracle's representation formula."""
    g = I.sphere3d(24, 0.35)
    rng = np.random.default_rng(3)
    q = rng.uniform(-1, 1, g.m)
    u = rng.uniform(-1, 1, g.m)
    plan = B.Plan(g, B.LAPLACE3D, precision=B.BF16_MFMA)
    out = plan.eval_grid(_t(q, dev), _t(u, dev))
    torch.cuda.synchronize()
    inf = plan.info()
    plan.close()
    z0, nz = inf["z_lo"], inf["z_count"]
    zz, yy, xx = np.meshgrid(np.arange(z0, z0 + nz), np.arange(24), np.arange(24), indexing="ij")
    pts = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1)
    ref, sc = O.volume(O.problem(g, O.LAPLACE3D), q, u, pts, with_scale=True)
    err = np.abs(out.cpu().numpy().ravel() - ref).max() / sc.max()
    print(f"bf16 grid field: {err:.2e}")
    assert err < BAR


def test_bf16_deterministic_and_rejections(dev):
    g = I.sphere3d(32, 0.35)
    rng = np.random.default_rng(2)
    q = _t(rng.uniform(-1, 1, g.m), dev)
    u = _t(rng.uniform(-1, 1, g.m), dev)
    plan = B.Plan(g, B.LAPLACE3D, precision=B.BF16_MFMA)
    r1 = plan.apply(q, u).clone()
    r2 = plan.apply(q, u)
    torch.cuda.synchronize()
    assert torch.equal(r1, r2)
    with pytest.raises(B.BemfftError) as ei:
        B.Batch([plan], nrhs=1)
    assert ei.value.status == B.EINVAL
    plan.close()
    c = I.circle2d(32, 0.3)
    with pytest.raises(B.BemfftError) as ei:
        B.Plan(c, B.LAPLACE2D, precision=B.BF16_MFMA)
    assert ei.value.status == B.EINVAL
