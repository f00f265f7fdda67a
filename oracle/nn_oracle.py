"""CPU FP64 reference of the learned-start network (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may use this module.  It shares no code with the GPU library.

The network is an addition to the paper's method (the paper solves from a
zero start): it maps a Dirichlet problem of Sec. 4 (u given on the boundary,
q sought) to a guess of q for the iterative solve.  Everything here is
written from the definitions, in numpy FP64:

* input channels on the n^3 grid, summed over the nodes of each voxel:
  a = w/h^2, a*n_x, a*n_y, a*n_z, a*s*u, a*s*b (u the Dirichlet data,
  s = 1/rms(u) over Dirichlet slots, b the right-hand side of the solve:
  minus the operator applied to the known values, eq. 4 with the unknowns
  set to zero);
* output y at the voxel of node j approximates s*h*q_j (a flux per voxel
  length, O(1) for smooth data), so the guess is q_j = y / (s h);
* layers: 3x3x3 cross-correlation with dilation d and zero padding,
  out[c, p] = b[c] + sum_{ci, o in {-1,0,1}^3} W[c, ci, o] x[ci, p + d o],
  ReLU after every layer but the last;
* loss L = sum_i wt_i (y[vox_i] - t_i)^2, gradients by the chain rule;
* Adam (Kingma & Ba 2015, Algorithm 1) with bias-corrected moments.

Parameters are one flat vector, per layer W[cout][cin][27] then b[cout];
tap index (oz+1)*9 + (oy+1)*3 + (ox+1).  Arrays are [channel][z][y][x].
"""

from __future__ import annotations

import numpy as np

OFFSETS = [(oz, oy, ox) for oz in (-1, 0, 1) for oy in (-1, 0, 1) for ox in (-1, 0, 1)]


CIN = 6


def layer_shapes(layers: int, cin: int = CIN, width: int = 16):
    """(cin, cout) of every layer: cin -> width -> ... -> width -> 1."""
    return [(cin if l == 0 else width, 1 if l == layers - 1 else width) for l in range(layers)]


def unpack(params, layers: int, cin: int = CIN, width: int = 16):
    """Split the flat parameter vector into [(W[cout, cin, 27], b[cout])]."""
    out, k = [], 0
    for ci, co in layer_shapes(layers, cin, width):
        W = np.asarray(params[k:k + co * ci * 27], dtype=np.float64).reshape(co, ci, 27)
        k += co * ci * 27
        b = np.asarray(params[k:k + co], dtype=np.float64)
        k += co
        out.append((W, b))
    if k != len(params):
        raise ValueError("parameter vector length does not match the layer shapes")
    return out


def pack(layer_params):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layer_params])


def channels(grid_index, G: int, h: float, weights, normals, u, b, bc, s: float):
    """Input channels [6, G, G, G] of a problem (nodes snapped to grid_index,
    [m, 3] as (ix, iy, iz)); bc = None means every slot is Dirichlet."""
    x = np.zeros((CIN, G, G, G))
    a = np.asarray(weights, dtype=np.float64) / (h * h)
    dir_ = np.ones(len(a), dtype=bool) if bc is None else (np.asarray(bc) == 0)
    uu = np.where(dir_, np.asarray(u, dtype=np.float64), 0.0)
    vals = [a, a * normals[:, 0], a * normals[:, 1], a * normals[:, 2], a * s * uu,
            a * s * np.asarray(b, dtype=np.float64)]
    ix, iy, iz = grid_index[:, 0], grid_index[:, 1], grid_index[:, 2]
    for c, v in enumerate(vals):
        np.add.at(x[c], (iz, iy, ix), v)
    return x


def shifted(x, oz, oy, ox):
    """y[..., z, y, x] = x[..., z+oz, y+oy, x+ox], zero outside the grid."""
    G = x.shape[-1]
    y = np.zeros_like(x)
    if max(abs(oz), abs(oy), abs(ox)) >= G:
        return y

    def rng(o):
        return (slice(max(0, -o), G - max(0, o)), slice(max(0, o), G - max(0, -o)))

    (dz, sz), (dy, sy), (dx, sx) = rng(oz), rng(oy), rng(ox)
    y[..., dz, dy, dx] = x[..., sz, sy, sx]
    return y


def conv(x, W, b, d: int):
    """Dilated 3x3x3 cross-correlation with zero padding: [cin,G,G,G] -> [cout,G,G,G]."""
    out = np.broadcast_to(b[:, None, None, None], (W.shape[0],) + x.shape[1:]).copy()
    for t, (oz, oy, ox) in enumerate(OFFSETS):
        xs = shifted(x, d * oz, d * oy, d * ox)
        out += np.tensordot(W[:, :, t], xs, axes=([1], [0]))
    return out


def conv_transpose_data(g, W, d: int):
    """dL/dx of conv given dL/dout = g: sum_c sum_o W[c, ci, o] g[c, p - d o]."""
    out = np.zeros((W.shape[1],) + g.shape[1:])
    for t, (oz, oy, ox) in enumerate(OFFSETS):
        gs = shifted(g, -d * oz, -d * oy, -d * ox)
        out += np.tensordot(W[:, :, t], gs, axes=([0], [0]))
    return out


def conv_weight_grad(g, x, d: int):
    """dL/dW[c, ci, o] = sum_p g[c, p] x[ci, p + d o]; dL/db[c] = sum_p g[c, p]."""
    gW = np.zeros((g.shape[0], x.shape[0], 27))
    for t, (oz, oy, ox) in enumerate(OFFSETS):
        xs = shifted(x, d * oz, d * oy, d * ox)
        gW[:, :, t] = np.tensordot(g, xs, axes=([1, 2, 3], [1, 2, 3]))
    return gW, g.sum(axis=(1, 2, 3))


def forward(params, dilations, x, cin: int = CIN, width: int = 16):
    """Returns (y [G,G,G], list of layer inputs, list of pre-activations)."""
    lp = unpack(params, len(dilations), cin, width)
    inputs, pres = [], []
    a = np.asarray(x, dtype=np.float64)
    for l, ((W, b), d) in enumerate(zip(lp, dilations)):
        inputs.append(a)
        z = conv(a, W, b, d)
        pres.append(z)
        a = np.maximum(z, 0.0) if l < len(dilations) - 1 else z
    return a[0], inputs, pres


def loss_and_grad(params, dilations, x, vox, tgt, wt, cin: int = CIN, width: int = 16):
    """L = sum_i wt_i (y.flat[vox_i] - tgt_i)^2 and dL/dparams (flat)."""
    lp = unpack(params, len(dilations), cin, width)
    y, inputs, pres = forward(params, dilations, x, cin, width)
    yf = y.ravel()
    e = yf[vox] - tgt
    L = float(np.sum(wt * e * e))
    gy = np.zeros_like(yf)
    np.add.at(gy, vox, 2.0 * wt * e)
    g = gy.reshape((1,) + y.shape)
    grads = [None] * len(lp)
    for l in range(len(lp) - 1, -1, -1):
        W, _ = lp[l]
        grads[l] = conv_weight_grad(g, inputs[l], dilations[l])
        if l > 0:
            g = conv_transpose_data(g, W, dilations[l]) * (pres[l - 1] > 0.0)
    return L, pack(grads)


def adam(params, grad, m, v, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (params, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v
