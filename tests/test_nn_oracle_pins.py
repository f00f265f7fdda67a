"""Pins of the CPU reference of the learned-start network (oracle/nn_oracle.py).

Each check ties the reference to something other than itself: a brute-force
loop, a library routine for the textbook special case (torch's conv3d and
autograd, torch.optim.Adam, all in FP64 on the CPU), central finite
differences, an adjoint identity, or a closed form.
"""

import numpy as np
import pytest
import torch

from oracle import nn_oracle as nn

DIL = [1, 2, 4]


def _params(rng, layers, cin=nn.CIN, width=16, scale=0.3):
    lp = [(scale * rng.standard_normal((co, ci, 27)), scale * rng.standard_normal(co))
          for ci, co in nn.layer_shapes(layers, cin, width)]
    return nn.pack(lp)


def test_conv_bruteforce():
    rng = np.random.default_rng(0)
    G, ci, co, d = 5, 2, 3, 2
    x = rng.standard_normal((ci, G, G, G))
    W = rng.standard_normal((co, ci, 27))
    b = rng.standard_normal(co)
    out = nn.conv(x, W, b, d)
    ref = np.zeros_like(out)
    for c in range(co):
        for z in range(G):
            for y in range(G):
                for xx in range(G):
                    s = b[c]
                    for k in range(ci):
                        for oz in (-1, 0, 1):
                            for oy in (-1, 0, 1):
                                for ox in (-1, 0, 1):
                                    zz, yy, x2 = z + d * oz, y + d * oy, xx + d * ox
                                    if 0 <= zz < G and 0 <= yy < G and 0 <= x2 < G:
                                        s += W[c, k, (oz + 1) * 9 + (oy + 1) * 3 + ox + 1] * x[k, zz, yy, x2]
                    ref[c, z, y, xx] = s
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("d", [1, 2, 4, 8])
def test_conv_matches_torch(d):
    rng = np.random.default_rng(d)
    G, ci, co = 12, 5, 16
    x = rng.standard_normal((ci, G, G, G))
    W = rng.standard_normal((co, ci, 27))
    b = rng.standard_normal(co)
    ref = torch.nn.functional.conv3d(torch.from_numpy(x)[None], torch.from_numpy(W.reshape(co, ci, 3, 3, 3)),
                                     torch.from_numpy(b), padding=d, dilation=d)[0].numpy()
    np.testing.assert_allclose(nn.conv(x, W, b, d), ref, rtol=0, atol=1e-11)


def test_conv_transpose_is_adjoint():
    rng = np.random.default_rng(1)
    G, ci, co, d = 9, 4, 3, 2
    x = rng.standard_normal((ci, G, G, G))
    g = rng.standard_normal((co, G, G, G))
    W = rng.standard_normal((co, ci, 27))
    lhs = np.sum(nn.conv(x, W, np.zeros(co), d) * g)
    rhs = np.sum(x * nn.conv_transpose_data(g, W, d))
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def _problem(rng, G=7, nt=40, cin=nn.CIN):
    x = np.zeros((cin, G, G, G))
    vox = rng.choice(G ** 3, size=nt, replace=False)
    for c in range(cin):
        x[c].flat[vox] = rng.standard_normal(nt)
    tgt = rng.standard_normal(nt)
    wt = rng.uniform(0.5, 1.5, nt) / nt
    return x, vox, tgt, wt


def test_gradient_finite_differences():
    rng = np.random.default_rng(2)
    x, vox, tgt, wt = _problem(rng)
    p = _params(rng, 3)
    L, g = nn.loss_and_grad(p, DIL, x, vox, tgt, wt)
    idx = rng.choice(len(p), size=30, replace=False)
    # the bias and the last layer are always touched
    idx = np.concatenate([idx, [len(p) - 1, len(p) - 2, 16 * nn.CIN * 27]])
    eps = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        fd = (nn.loss_and_grad(pp, DIL, x, vox, tgt, wt)[0] - nn.loss_and_grad(pm, DIL, x, vox, tgt, wt)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_gradient_matches_autograd():
    rng = np.random.default_rng(3)
    x, vox, tgt, wt = _problem(rng, G=8, nt=60)
    dil = [1, 2, 4, 8]
    p = _params(rng, 4)
    L, g = nn.loss_and_grad(p, dil, x, vox, tgt, wt)
    lp = nn.unpack(p, 4)
    ts = [(torch.tensor(W.reshape(W.shape[0], W.shape[1], 3, 3, 3), requires_grad=True),
           torch.tensor(b, requires_grad=True)) for W, b in lp]
    a = torch.from_numpy(x)[None]
    for l, ((W, b), d) in enumerate(zip(ts, dil)):
        a = torch.nn.functional.conv3d(a, W, b, padding=d, dilation=d)
        if l < 3:
            a = torch.relu(a)
    y = a.reshape(-1)
    e = y[torch.from_numpy(vox)] - torch.from_numpy(tgt)
    Lt = torch.sum(torch.from_numpy(wt) * e * e)
    Lt.backward()
    gt = np.concatenate([np.concatenate([W.grad.numpy().ravel(), b.grad.numpy()]) for W, b in ts])
    assert abs(L - Lt.item()) <= 1e-12 * abs(L)
    np.testing.assert_allclose(g, gt, rtol=1e-9, atol=1e-12 * np.abs(gt).max())


def test_shared_voxel_targets_add():
    # two targets on one voxel: the loss is the sum of both squared errors
    rng = np.random.default_rng(4)
    x, vox, tgt, wt = _problem(rng, G=6, nt=10)
    vox = vox.copy()
    vox[1] = vox[0]
    p = _params(rng, 2)
    y = nn.forward(p, [1, 2], x)[0].ravel()
    L, _ = nn.loss_and_grad(p, [1, 2], x, vox, tgt, wt)
    assert abs(L - np.sum(wt * (y[vox] - tgt) ** 2)) <= 1e-12 * L


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr = 1e-3
    p1, m, v = nn.adam(p, g, np.zeros(50), np.zeros(50), 1, lr)
    # bias-corrected first moment / sqrt(second) = g / |g| on the first step
    np.testing.assert_allclose(p1, p - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_adam_matches_torch():
    rng = np.random.default_rng(6)
    p = rng.standard_normal(20)
    A = rng.standard_normal((20, 20))
    lr = 1e-2
    tp = torch.tensor(p, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    m, v = np.zeros(20), np.zeros(20)
    for t in range(1, 8):
        g = A.T @ (A @ p) - 1.0
        p, m, v = nn.adam(p, g, m, v, t, lr)
        opt.zero_grad()
        tg = torch.from_numpy(A).T @ (torch.from_numpy(A) @ tp) - 1.0
        tp.grad = tg.detach()
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-12)


def test_channels_sums():
    from paper_1809_00845_amd import inputs
    import oracle

    g = inputs.sphere3d(24, 0.35)
    idx = oracle.snap(oracle.problem(g, oracle.LAPLACE3D))
    u = np.ones(g.m)
    b = np.full(g.m, 2.0)
    x = nn.channels(idx, 24, g.h, g.weights, g.normals, u, b, None, 1.0)
    a_sum = g.weights.sum() / g.h ** 2
    # total area in voxel units, and a closed surface has zero mean normal
    assert abs(x[0].sum() - a_sum) <= 1e-12 * a_sum
    for c in (1, 2, 3):
        assert abs(x[c].sum()) <= 1e-2 * a_sum
    # u = 1, s = 1: the data channel equals the area channel
    np.testing.assert_allclose(x[4], x[0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(x[5], 2.0 * x[0], rtol=0, atol=1e-12)
    # Neumann slots carry no Dirichlet data
    bc = np.ones(g.m, dtype=np.uint8)
    assert np.abs(nn.channels(idx, 24, g.h, g.weights, g.normals, u, b, bc, 1.0)[4]).max() == 0.0
