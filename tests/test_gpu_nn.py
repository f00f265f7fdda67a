"""GPU parity of the learned-start network (bemfft_net_*) against the CPU
FP64 reference in oracle/nn_oracle.py, and the gain of the trained guess.

Bars (FP32 storage and arithmetic on the GPU): input channels 1e-6 of each
channel's largest value (one FP32 rounding per node value); forward output
1e-5 of max |y| (FP32 sums of <= 16*27 products per layer over 4 layers);
gradients 2e-4 of max |g| per entry (FP32 sums over up to G^3 voxels, in
chunks) and 2e-5 normwise.
"""

import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from oracle import nn_oracle as NN  # noqa: E402
from paper_1809_00845_amd import binding as B  # noqa: E402
from paper_1809_00845_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu
DIL = (1, 2, 4, 8)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.load()
    return torch.device("cuda:0")


def _rand_params(net, seed, scale=0.2):
    rng = np.random.default_rng(seed)
    p = (scale * rng.standard_normal(net.nparam)).astype(np.float32)
    net.set_params(p)
    return p.astype(np.float64)


def _sparse_input(G, seed, frac=0.15, cin=6):
    rng = np.random.default_rng(seed)
    x = np.zeros((cin, G ** 3), dtype=np.float32)
    k = max(1, int(frac * G ** 3))
    vox = rng.choice(G ** 3, size=k, replace=False)
    x[:, vox] = rng.standard_normal((cin, k)).astype(np.float32)
    return x


def test_net_params_roundtrip(dev):
    net = B.Net(8, DIL, seed=3)
    assert net.nparam == sum(co * ci * 27 + co for ci, co in NN.layer_shapes(4))
    p = net.params()
    # He-normal init: zero biases, spread of the first layer sqrt(2 / (6*27))
    lp = NN.unpack(p.astype(np.float64), 4)
    assert all(np.all(b == 0) for _, b in lp)
    assert abs(lp[0][0].std() - math.sqrt(2 / (6 * 27))) < 0.1 * math.sqrt(2 / (6 * 27))
    q = np.arange(net.nparam, dtype=np.float32)
    net.set_params(q)
    assert np.array_equal(net.params(), q)
    net.close()


def test_net_input_channels(dev):
    G = 24
    g = I.sphere3d(G, 0.35)
    rng = np.random.default_rng(0)
    u = rng.uniform(-1, 1, g.m)
    s = 1.0 / math.sqrt(np.mean(u * u))
    plan = B.Plan(g, B.LAPLACE3D, precision=B.FP64)
    net = B.Net(G, DIL)
    x = torch.empty((6, G ** 3), dtype=torch.float32, device=dev)
    net.input(plan, None, torch.tensor(u, device=dev), s, x)
    torch.cuda.synchronize()
    p = O.problem(g, O.LAPLACE3D)
    b = -O.apply(p, np.zeros(g.m), u)
    ref = NN.channels(O.snap(p), G, g.h, g.weights, g.normals, u, b, None, s).reshape(6, -1)
    got = x.cpu().numpy()
    for c in range(6):
        assert np.abs(got[c] - ref[c]).max() <= 1e-6 * np.abs(ref[c]).max(), c
    net.close()
    plan.close()


@pytest.mark.parametrize("G", [9, 23])
def test_net_forward_matches_oracle(dev, G):
    net = B.Net(G, DIL, seed=1)
    p = _rand_params(net, G)
    x = _sparse_input(G, G)
    y = torch.empty(G ** 3, dtype=torch.float32, device=dev)
    net.forward(torch.tensor(x, device=dev), y)
    torch.cuda.synchronize()
    ref = NN.forward(p, list(DIL), x.astype(np.float64).reshape(6, G, G, G))[0].ravel()
    got = y.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()
    net.close()


@pytest.mark.parametrize("G,dil", [(9, (1, 2, 4, 8)), (23, (1, 2, 4, 8)), (32, (1, 2, 4, 8)), (13, (3, 1))])
def test_net_infer_fp16_matches_oracle(dev, G, dil):
    """FP16 storage, FP32 accumulation on the matrix cores.  Bar: 1e-2 of
    max |y| -- FP16 rounding (2^-11) of the inputs of every layer, growing
    through <= 4 layers of sums of up to 432 products."""
    net = B.Net(G, dil, seed=1)
    p = _rand_params(net, 50 + G)
    x = _sparse_input(G, 60 + G)
    y = torch.empty(G ** 3, dtype=torch.float32, device=dev)
    net.infer(torch.tensor(x, device=dev), y)
    torch.cuda.synchronize()
    ref = NN.forward(p, list(dil), x.astype(np.float64).reshape(6, G, G, G))[0].ravel()
    got = y.cpu().numpy()
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 1e-2 * scale
    assert np.linalg.norm(got - ref) <= 3e-3 * np.linalg.norm(ref)
    net.close()


def test_net_full_size_sampled(dev):
    """The bench's network on its 96^3 grid (dilations 1, 2, 4, 8), FP32
    forward and FP16 inference, at sampled voxels (grid corners, faces and
    interior).  The receptive field is +-15 voxels (1 + 2 + 4 + 8), so the
    oracle evaluates each sampled voxel exactly on a 31^3 window of the grid
    that holds it: the window is centred on the voxel except where it would
    leave the grid, where it is shifted inwards so that its edge is the grid's
    edge (the network zero-pads every layer there, as the oracle does at the
    window's edge)."""
    G, dil, R = 96, (1, 2, 4, 8), 15
    W = 2 * R + 1
    net = B.Net(G, dil, seed=5)
    p = _rand_params(net, 31, scale=0.15)
    x = _sparse_input(G, 32, frac=0.02)
    xt = torch.tensor(x, device=dev)
    y32 = torch.empty(G ** 3, dtype=torch.float32, device=dev)
    y16 = torch.empty(G ** 3, dtype=torch.float32, device=dev)
    net.forward(xt, y32)
    net.infer(xt, y16)
    torch.cuda.synchronize()
    y32, y16 = y32.cpu().numpy(), y16.cpu().numpy()
    x4 = x.astype(np.float64).reshape(6, G, G, G)
    pts = [(0, 0, 0), (G - 1, G - 1, G - 1), (0, 47, 95), (48, 48, 48), (10, 90, 30), (95, 3, 60), (33, 66, 7)]
    refs, g32, g16 = [], [], []
    for c in pts:
        st = [min(max(ci - R, 0), G - W) for ci in c]
        crop = x4[:, st[0]:st[0] + W, st[1]:st[1] + W, st[2]:st[2] + W]
        yc = NN.forward(p, list(dil), crop)[0]
        refs.append(yc[c[0] - st[0], c[1] - st[1], c[2] - st[2]])
        v = (c[0] * G + c[1]) * G + c[2]
        g32.append(y32[v])
        g16.append(y16[v])
    refs, g32, g16 = map(np.asarray, (refs, g32, g16))
    scale = np.abs(refs).max()
    assert np.abs(g32 - refs).max() <= 1e-5 * scale
    assert np.abs(g16 - refs).max() <= 1e-2 * scale
    net.close()


@pytest.mark.parametrize("G,dil", [(10, (1, 2, 4, 8)), (23, (1, 2, 4, 8)), (12, (1, 3)), (17, (2, 1, 1))])
def test_net_gradients_match_oracle(dev, G, dil):
    net = B.Net(G, dil, seed=2)
    p = _rand_params(net, 100 + G)
    x = _sparse_input(G, 200 + G)
    rng = np.random.default_rng(G)
    nt = max(4, G ** 3 // 20)
    vox = rng.choice(G ** 3, size=nt, replace=False).astype(np.int32)
    tgt = rng.standard_normal(nt).astype(np.float32)
    wt = (rng.uniform(0.5, 1.5, nt) / nt).astype(np.float32)
    L, g = net.gradients(torch.tensor(x, device=dev), torch.tensor(vox, device=dev), torch.tensor(tgt, device=dev),
                         torch.tensor(wt, device=dev))
    Lr, gr = NN.loss_and_grad(p, list(dil), x.astype(np.float64).reshape(6, G, G, G), vox, tgt.astype(np.float64),
                              wt.astype(np.float64))
    assert abs(L - Lr) <= 1e-5 * abs(Lr)
    assert np.abs(g - gr).max() <= 2e-4 * np.abs(gr).max()
    assert np.linalg.norm(g - gr) <= 2e-5 * np.linalg.norm(gr)
    # run to run: the same bits (fixed-order reductions, one target per voxel)
    _, g2 = net.gradients(torch.tensor(x, device=dev), torch.tensor(vox, device=dev), torch.tensor(tgt, device=dev),
                          torch.tensor(wt, device=dev))
    assert np.array_equal(g, g2)
    net.close()


def test_net_gradients_full_size_sampled(dev):
    """Gradients on the bench's 96^3 grid (dilations 1, 2, 4, 8) for a loss
    on eight target voxels (corners, faces, interior).  A target's output
    depends only on inputs within 15 voxels of it, and so does every
    activation on its gradient paths, so the oracle computes each target's
    gradient exactly on the 31^3 window that holds it (shifted inwards at
    the grid's edge, where the network zero-pads as the oracle does at the
    window's edge); their sum must equal the GPU's full-grid gradient, whose
    sums run over every voxel of the grid.  Bars as for the small grids."""
    G, dil, R = 96, (1, 2, 4, 8), 15
    W = 2 * R + 1
    net = B.Net(G, dil, seed=6)
    p = _rand_params(net, 41, scale=0.15)
    x = _sparse_input(G, 42, frac=0.02)
    pts = [(0, 0, 0), (G - 1, G - 1, G - 1), (0, 47, 95), (48, 48, 48), (10, 90, 30), (95, 3, 60), (33, 66, 7),
           (70, 20, 85)]
    vox = np.array([(c[0] * G + c[1]) * G + c[2] for c in pts], dtype=np.int32)
    rng = np.random.default_rng(43)
    tgt = rng.standard_normal(len(pts)).astype(np.float32)
    wt = rng.uniform(0.5, 1.5, len(pts)).astype(np.float32)
    L, g = net.gradients(torch.tensor(x, device=dev), torch.tensor(vox, device=dev), torch.tensor(tgt, device=dev),
                         torch.tensor(wt, device=dev))
    net.close()
    x4 = x.astype(np.float64).reshape(6, G, G, G)
    Lr, gr = 0.0, np.zeros_like(p)
    for i, c in enumerate(pts):
        st = [min(max(ci - R, 0), G - W) for ci in c]
        crop = x4[:, st[0]:st[0] + W, st[1]:st[1] + W, st[2]:st[2] + W]
        lv = ((c[0] - st[0]) * W + (c[1] - st[1])) * W + (c[2] - st[2])
        Li, gi = NN.loss_and_grad(p, list(dil), crop, np.array([lv]), np.array([float(tgt[i])]),
                                  np.array([float(wt[i])]))
        Lr += Li
        gr += gi
    assert abs(L - Lr) <= 1e-5 * abs(Lr)
    assert np.abs(g - gr).max() <= 2e-4 * np.abs(gr).max()
    assert np.linalg.norm(g - gr) <= 2e-5 * np.linalg.norm(gr)


def test_net_adam_steps_match_oracle(dev):
    G = 11
    net = B.Net(G, DIL, seed=4)
    p = _rand_params(net, 7)
    x = _sparse_input(G, 8)
    rng = np.random.default_rng(9)
    nt = 60
    vox = rng.choice(G ** 3, size=nt, replace=False).astype(np.int32)
    tgt = rng.standard_normal(nt).astype(np.float32)
    wt = np.full(nt, 1.0 / nt, dtype=np.float32)
    args = [torch.tensor(a, device=dev) for a in (x, vox, tgt, wt)]
    lr = 1e-3
    m, v = np.zeros_like(p), np.zeros_like(p)
    x64 = x.astype(np.float64).reshape(6, G, G, G)
    for t in (1, 2, 3):
        Lr, gr = NN.loss_and_grad(p, list(DIL), x64, vox, tgt.astype(np.float64), wt.astype(np.float64))
        L = net.train_step(*args, lr)
        assert abs(L - Lr) <= 1e-5 * abs(Lr)
        p_next, m, v = NN.adam(p, gr, m, v, t, lr)
        got = net.params().astype(np.float64)
        # the step is ~lr sign(g) early on: compare where the gradient is well
        # above its FP32 error, bound the rest by the step size
        big = np.abs(gr) > 1e-2 * np.abs(gr).max()
        assert np.abs(got - p_next)[big].max() <= 2e-2 * lr
        assert np.abs(got - p).max() <= 1.0001 * lr * t
        p = got  # follow the GPU parameters
    net.close()


def test_solve_guess_fallback(dev):
    g = I.sphere3d(32, 0.35)
    rng = np.random.default_rng(1)
    u, _ = I.random_harmonic_3d(g, rng)
    plan = B.Plan(g, B.LAPLACE3D, precision=B.FP64)
    bc = torch.zeros(g.m, dtype=torch.uint8, device=dev)
    known = torch.tensor(u, device=dev)
    q0, i0 = plan.solve(bc, known, tol=1e-8)
    assert i0["status"] == 0 and i0["x0_used"] == 0
    # a guess worse than zero is dropped: the same iterations as plain GMRES
    bad = torch.tensor(1e3 * rng.standard_normal(g.m), device=dev)
    _, ib = plan.solve(bc, known, bad, tol=1e-8, use_x0=2)
    assert ib["x0_used"] == 0 and ib["x0_relres"] > 1.0 and ib["iters"] == i0["iters"]
    # the converged solution as the guess: kept, residual already small
    good = q0.clone()
    _, ig = plan.solve(bc, known, good, tol=1e-6, use_x0=2)
    assert ig["x0_used"] == 1 and ig["x0_relres"] < 1e-7 and ig["iters"] == 0
    assert ig["true_relres"] <= 1e-6
    plan.close()


@pytest.mark.slow
def test_learned_start_gain(dev):
    """Train on GPU-solved star problems (seed 3) and compare GMRES from the
    learned start against GMRES from zero on held-out problems.

    What the network gains: its guess removes most of the initial residual
    (median ||b - A x0|| / ||b|| well below 1/2), yet GMRES needs about as
    many iterations from it as from zero, because the residual it leaves
    lies in the slowly converging (high-frequency) part of the spectrum.
    The test pins both facts and that the fallback keeps the loss bounded."""
    from paper_1809_00845_amd import learned as LS

    G, ntr, nte = 32, 96, 24
    probs = LS.problem_set(G, ntr + nte, seed=3)
    net = B.Net(G, DIL, seed=0)
    train = LS.make_samples(net, probs[:ntr])
    test_s = LS.make_samples(net, probs[ntr:])
    e0 = LS.relative_error(net, test_s)
    LS.train(net, train, epochs=8, lr=2e-3, progress_s=0)
    e1 = LS.relative_error(net, test_s)
    rows = LS.evaluate(net, probs[ntr:])
    sm = LS.summary(rows)
    print("learned start (G=32):", sm, "rel err", e0, "->", e1)
    assert e1 < 0.5 * e0
    assert sm["all_converged"] and sm["relres_max"] <= 1e-6
    assert sm["guess_relres_median"] < 0.5
    assert sm["iters_learned_mean"] <= sm["iters_plain_mean"] + 1.0
    assert all(r["iters1"] <= r["iters0"] + 3 for r in rows)
    net.close()
