"""Pins of the float64 reference of the learned preconditioner's network.

The convolution is checked against a brute-force triple loop with the
sphere closure written out case by case, the gradients against central
finite differences, the padding adjoint against the dot-product identity,
and Adam against its closed form after one step."""
import numpy as np
import pytest

from oracle import cnn


def brute_conv(x, w, b):
    cin, ny, nx = x.shape
    out = np.zeros((w.shape[0], ny, nx))
    for co in range(w.shape[0]):
        for j in range(ny):
            for i in range(nx):
                s = b[co]
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        jj, ii = j + dy, (i + dx) % nx
                        if jj < 0:          # across the south pole
                            jj, ii = 0, (ii + nx // 2) % nx
                        elif jj >= ny:      # across the north pole
                            jj, ii = ny - 1, (ii + nx // 2) % nx
                        s += np.dot(w[co, :, dy + 1, dx + 1], x[:, jj, ii])
                out[co, j, i] = s
    return out


def test_conv_matches_brute_force():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 4, 8))
    w = rng.standard_normal((5, 3, 3, 3))
    b = rng.standard_normal(5)
    assert np.allclose(cnn.conv3x3(x, w, b), brute_conv(x, w, b), rtol=1e-12, atol=1e-12)


def test_padding_adjoint_identity():
    # <conv(x), y> with zero bias equals <x, conv^T(y)> computed by the backward pass
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 4, 8))
    y = rng.standard_normal((3, 4, 8))
    w = rng.standard_normal((3, 2, 3, 3))
    lhs = np.sum(cnn.conv3x3(x, w, np.zeros(3)) * y)
    dx, _, _ = cnn.conv3x3_backward(x, w, y)
    assert np.isclose(lhs, np.sum(x * dx), rtol=1e-12)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    params = cnn.init_params(2, rng, width=4)
    w_last, b_last = params[-1]
    params[-1] = (rng.standard_normal(w_last.shape) * 0.3, b_last)
    x = rng.standard_normal((2, 4, 8))
    t = rng.standard_normal((1, 4, 8))

    def loss(ps, xx):
        y = cnn.forward(ps, xx)[-1]
        return cnn.mse_loss(y, t)[0]

    acts = cnn.forward(params, x)
    _, dy = cnn.mse_loss(acts[-1], t)
    grads, dx = cnn.backward(params, acts, dy)
    h = 1e-6
    for n in (0, 2, 4):
        w, b = params[n]
        for _ in range(4):
            idx = tuple(rng.integers(s) for s in w.shape)
            wp, wm = w.copy(), w.copy()
            wp[idx] += h
            wm[idx] -= h
            pp = list(params); pp[n] = (wp, b)
            pm = list(params); pm[n] = (wm, b)
            fd = (loss(pp, x) - loss(pm, x)) / (2 * h)
            assert np.isclose(grads[n][0][idx], fd, rtol=1e-5, atol=1e-9), (n, idx)
        k = int(rng.integers(b.shape[0]))
        bp, bm = b.copy(), b.copy()
        bp[k] += h
        bm[k] -= h
        pp = list(params); pp[n] = (w, bp)
        pm = list(params); pm[n] = (w, bm)
        assert np.isclose(grads[n][1][k], (loss(pp, x) - loss(pm, x)) / (2 * h), rtol=1e-5, atol=1e-9)
    # input gradient, including pixels in the polar rows
    for idx in [(0, 0, 1), (1, 3, 6), (0, 2, 3)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        assert np.isclose(dx[idx], (loss(params, xp) - loss(params, xm)) / (2 * h), rtol=1e-5, atol=1e-9)


def test_adam_one_step_closed_form():
    # after one step with zero moments the update is lr * g / (|g| + eps')
    g = np.array([0.5, -2.0, 1e-3])
    p, m, v = cnn.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.1)
    assert np.allclose(p, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_last_layer_starts_at_zero():
    params = cnn.init_params(4, np.random.default_rng(3))
    x = np.random.default_rng(4).standard_normal((4, 8, 16))
    assert np.all(cnn.forward(params, x)[-1] == 0.0)
    assert [p[0].shape for p in params] == [(32, 4, 3, 3), (32, 32, 3, 3), (32, 32, 3, 3), (32, 32, 3, 3), (1, 32, 3, 3)]
