"""The allocation-free solve entry point (bemfft_solve_noalloc) against
bemfft_solve, through the C ABI: same options, same answer, on two calls in
a row (the second with a smaller problem, so the fixed workspace holds the
first call's leftovers), plus an FP32 refined solve and the size limit."""

import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_1809_00845_amd import binding as B  # noqa: E402
from paper_1809_00845_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.load()
    return torch.device("cuda:0")


def _t(a, dev):
    return torch.tensor(np.ascontiguousarray(a), device=dev)


def _mixed(g):
    uh, qh = I.harmonic_3d_xyz(g)
    bc = I.mixed_bc_upper(g)
    return bc, np.where(bc == 0, uh, qh)


def _free_bytes():
    hip = ctypes.CDLL("libamdhip64.so")
    free, total = ctypes.c_size_t(), ctypes.c_size_t()
    assert hip.hipMemGetInfo(ctypes.byref(free), ctypes.byref(total)) == 0
    return free.value


def _both(plan, bc, known, dev, **kw):
    n = plan.ncomp * plan.m
    xa = torch.zeros(n, dtype=torch.float64, device=dev)
    xb = torch.zeros(n, dtype=torch.float64, device=dev)
    ia = B.bemfft_solve(plan.handle, _t(bc, dev), _t(known, dev), xa, n=n, **kw)
    ib = B.bemfft_solve_noalloc(plan.handle, _t(bc, dev), _t(known, dev), xb, n=n, **kw)
    torch.cuda.synchronize()
    return xa.cpu().numpy(), ia, xb.cpu().numpy(), ib


def test_noalloc_solve_matches_solve_twice_then_smaller(dev):
    # first call: 48^3 sphere (5,242 unknowns), restart 100
    g1 = I.sphere3d(48, 0.35)
    bc1, k1 = _mixed(g1)
    p1 = B.Plan(g1, B.LAPLACE3D, precision=B.FP64)
    xa, ia, xb, ib = _both(p1, bc1, k1, dev, tol=1e-10)
    assert ia["status"] == 0 and ib["status"] == 0
    assert ib["iters"] == ia["iters"] and ib["true_relres"] <= 1e-10
    assert np.array_equal(xa, xb)  # same kernels, same order: bit for bit
    xl = O.solve_lu(O.problem(g1, O.LAPLACE3D), bc1, k1)
    assert np.linalg.norm(xb - xl) / np.linalg.norm(xl) < 1e-7
    # second call, smaller problem (the workspace still holds the first one's data)
    g2 = I.sphere3d(16, 0.35)
    bc2, k2 = _mixed(g2)
    p2 = B.Plan(g2, B.LAPLACE3D, precision=B.FP64)
    xa, ia, xb, ib = _both(p2, bc2, k2, dev, tol=1e-10, restart=20)
    assert ib["status"] == 0 and ib["iters"] == ia["iters"]
    assert np.array_equal(xa, xb)
    xl = O.solve_lu(O.problem(g2, O.LAPLACE3D), bc2, k2)
    assert np.linalg.norm(xb - xl) / np.linalg.norm(xl) < 1e-7
    p1.close()
    p2.close()


def test_noalloc_refined_fp32_navier_and_initial_guess(dev):
    g = I.sphere3d(16, 0.35)
    rng = np.random.default_rng(4)
    bc = np.stack([(g.rel()[:, 2] < 0).astype(np.uint8)] * 3)
    known = rng.uniform(-1, 1, (3, g.m))
    p32 = B.Plan(g, B.NAVIER3D, precision=B.FP32, keep_fp64=True)
    xa, ia, xb, ib = _both(p32, bc, known, dev, tol=1e-9, refine=1, inner_tol=1e-3)
    assert ib["status"] == 0 and ib["true_relres"] <= 1e-9 and ib["outer"] == ia["outer"]
    assert np.array_equal(xa, xb)
    xl = O.solve_lu(O.problem(g, O.NAVIER3D, 0.3, 1.0), bc, known).reshape(-1)
    assert np.linalg.norm(xb - xl) / np.linalg.norm(xl) < 1e-6
    p32.close()


def test_noalloc_allocates_nothing_and_checks_its_limit(dev):
    g = I.sphere3d(64, 0.35)
    bc, known = _mixed(g)
    plan = B.Plan(g, B.LAPLACE3D, precision=B.FP64)  # the plan allocates; the solve must not
    n = plan.m
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    bct, kt = _t(bc, dev), _t(known, dev)
    torch.cuda.synchronize()
    before = _free_bytes()
    info = B.bemfft_solve_noalloc(plan.handle, bct, kt, x, n=n, tol=1e-8)
    torch.cuda.synchronize()
    after = _free_bytes()
    assert info["status"] == 0 and info["true_relres"] <= 1e-8
    # bemfft_solve would take (restart + 10) * n doubles here (8.6 MB)
    assert before - after < (1 << 20), (before, after)
    plan.close()
    # a basis that does not fit: EINVAL before any device work (a Navier plan
    # with 15.7k unknowns; restart 400 would need 6.4M doubles of 4.19M)
    gn = I.sphere3d(48, 0.35)
    pn = B.Plan(gn, B.NAVIER3D, precision=B.FP32)
    nn = 3 * gn.m
    assert (400 + 10) * nn + 132096 > B.NOALLOC_SCRATCH_BYTES // 8
    xn = torch.zeros(nn, dtype=torch.float64, device=dev)
    bcn = _t(np.zeros(nn, dtype=np.uint8), dev)
    kn = _t(np.ones(nn), dev)
    with pytest.raises(B.BemfftError) as ei:
        B.bemfft_solve_noalloc(pn.handle, bcn, kn, xn, n=nn, restart=400)
    assert ei.value.status == B.EINVAL and "largest restart" in B.last_error()
    pn.close()
