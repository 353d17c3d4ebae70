"""Float64 reference of the learned preconditioner's convolution network.

Not from the paper: the paper's preconditioner is the semi-implicit
Richardson scheme; the network here is trained to add a correction to it.
This module is the plain CPU definition the GPU kernels are checked
against (forward, input and weight gradients, loss, Adam), written with
numpy and obviously-correct index maps.

Network: 3x3 convolutions C_in -> 32 -> 32 -> 32 -> 32 -> 1, ReLU after
every layer but the last.  Weights w[l] have shape [C_out, C_in, 3, 3]
(w[co, ci, dy+1, dx+1]), biases b[l] shape [C_out].

Padding on the sphere (the same closure as the elliptic operator): longitude
is periodic; the row beyond a pole is the polar row seen across the pole,
i.e. shifted by NX/2 in longitude.  The gradient with respect to the input
is the exact adjoint of that gather (scatter-add through the same index
map), so pole rows receive the contributions of their across-pole copies.
"""
from __future__ import annotations

import numpy as np

WIDTH = 32
LAYERS = 5


def neighbour_index(ny, nx):
    """(rows, cols) of shape [3, 3, ny, nx]: the source pixel read by output
    pixel (j, i) for tap (dy, dx) in {-1, 0, 1}^2."""
    j = np.arange(ny)[:, None]
    i = np.arange(nx)[None, :]
    rows = np.empty((3, 3, ny, nx), dtype=np.int64)
    cols = np.empty((3, 3, ny, nx), dtype=np.int64)
    for a, dy in enumerate((-1, 0, 1)):
        for b, dx in enumerate((-1, 0, 1)):
            jj = j + dy + 0 * i
            ii = (i + dx) % nx + 0 * j
            south = jj < 0
            north = jj >= ny
            jj = np.where(south, 0, np.where(north, ny - 1, jj))
            ii = np.where(south | north, (ii + nx // 2) % nx, ii)
            rows[a, b] = jj
            cols[a, b] = ii
    return rows, cols


def conv3x3(x, w, b, idx=None):
    """x [C_in, ny, nx] -> [C_out, ny, nx]."""
    cin, ny, nx = x.shape
    rows, cols = neighbour_index(ny, nx) if idx is None else idx
    out = np.broadcast_to(b[:, None, None], (w.shape[0], ny, nx)).astype(np.float64).copy()
    for a in range(3):
        for c in range(3):
            patch = x[:, rows[a, c], cols[a, c]]          # [C_in, ny, nx]
            out += np.einsum("oi,ijk->ojk", w[:, :, a, c], patch)
    return out


def conv3x3_backward(x, w, dout, idx=None):
    """Gradients of sum(dout * conv3x3(x, w, b)) with respect to x, w, b."""
    cin, ny, nx = x.shape
    rows, cols = neighbour_index(ny, nx) if idx is None else idx
    dx = np.zeros_like(x, dtype=np.float64)
    dw = np.zeros_like(w, dtype=np.float64)
    for a in range(3):
        for c in range(3):
            patch = x[:, rows[a, c], cols[a, c]]
            dw[:, :, a, c] = np.einsum("ojk,ijk->oi", dout, patch)
            contrib = np.einsum("oi,ojk->ijk", w[:, :, a, c], dout)    # gradient at the source pixels
            for ci in range(cin):
                np.add.at(dx[ci], (rows[a, c], cols[a, c]), contrib[ci])
    db = dout.sum(axis=(1, 2))
    return dx, dw, db


def init_params(c_in, rng, width=WIDTH):
    """He-style initialisation; the last layer starts at zero (the network
    initially adds no correction)."""
    shapes = [(width, c_in)] + [(width, width)] * 3 + [(1, width)]
    params = []
    for n, (co, ci) in enumerate(shapes):
        std = np.sqrt(2.0 / (9 * ci))
        w = rng.standard_normal((co, ci, 3, 3)) * std
        if n == len(shapes) - 1:
            w *= 0.0
        params.append((w, np.zeros(co)))
    return params


def forward(params, x):
    """Returns the list of layer outputs (post-activation; the last is linear)."""
    idx = neighbour_index(x.shape[1], x.shape[2])
    acts = [x]
    h = x
    for n, (w, b) in enumerate(params):
        h = conv3x3(h, w, b, idx)
        if n < len(params) - 1:
            h = np.maximum(h, 0.0)
        acts.append(h)
    return acts


def backward(params, acts, dy):
    """Gradients of sum(dy * network(x)); returns [(dw, db)] per layer and dx."""
    idx = neighbour_index(acts[0].shape[1], acts[0].shape[2])
    grads = [None] * len(params)
    d = dy
    for n in range(len(params) - 1, -1, -1):
        w, _ = params[n]
        if n < len(params) - 1:
            d = d * (acts[n + 1] > 0.0)
        dx, dw, db = conv3x3_backward(acts[n], w, d, idx)
        grads[n] = (dw, db)
        d = dx
    return grads, d


def mse_loss(y, t):
    """mean((y - t)^2) and its gradient with respect to y."""
    diff = y - t
    n = diff.size
    return float(np.sum(diff * diff) / n), 2.0 * diff / n


def adam_step(param, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) with bias correction; returns new
    (param, m, v).  `step` counts from 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return param - lr * mhat / (np.sqrt(vhat) + eps), m, v
