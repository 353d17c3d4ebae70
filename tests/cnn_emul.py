"""The network of oracle/cnn.py evaluated with bfloat16 rounding at the points
where the GPU kernels round (weights, the network input, each hidden
activation, each back-propagated gradient); the arithmetic between those
points is the oracle's float64 arithmetic.  Test infrastructure only."""
from __future__ import annotations

import numpy as np
import torch

from oracle import cnn


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), through float32 as the
    kernels do, returned as float64."""
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32))
    return t.to(torch.bfloat16).to(torch.float64).numpy()


def flatten(params):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params]).astype(np.float32)


def unflatten(flat, c_in):
    shapes = [(cnn.WIDTH, c_in)] + [(cnn.WIDTH, cnn.WIDTH)] * 3 + [(1, cnn.WIDTH)]
    out, k = [], 0
    for co, ci in shapes:
        w = np.asarray(flat[k:k + co * ci * 9], dtype=np.float64).reshape(co, ci, 3, 3)
        k += co * ci * 9
        b = np.asarray(flat[k:k + co], dtype=np.float64)
        k += co
        out.append((w, b))
    assert k == len(flat)
    return out


def forward(params, x):
    """x [C_in, ny, nx] -> list of layer inputs (bf16-rounded) and the output."""
    idx = cnn.neighbour_index(x.shape[1], x.shape[2])
    acts = [bf16(x)]
    h = acts[0]
    for n, (w, b) in enumerate(params):
        h = cnn.conv3x3(h, bf16(w), np.asarray(b, dtype=np.float32).astype(np.float64), idx)
        if n < len(params) - 1:
            h = bf16(np.maximum(h, 0.0))
        acts.append(h)
    return acts


def backward(params, acts, dy):
    """Weight and bias gradients of sum(dy * network) [(dw, db)] per layer."""
    idx = cnn.neighbour_index(acts[0].shape[1], acts[0].shape[2])
    grads = [None] * len(params)
    d = bf16(dy)[None]
    for n in range(len(params) - 1, -1, -1):
        w, _ = params[n]
        dx, dw, db = cnn.conv3x3_backward(acts[n], bf16(w), d, idx)
        grads[n] = (dw, db)
        if n > 0:
            d = bf16(dx * (acts[n] > 0.0))
    return grads
