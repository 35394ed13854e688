"""Pins of the MLP-surrogate oracle (CPU): bfloat16 rounding cases, finite
differences of the float64 network, closed-form special cases, the loss
gradient and the Adam first-step property."""
import numpy as np
import pytest

from oracle import mlp


def test_bf16_rounding_cases():
    u = 2.0 ** -7  # bf16 spacing just above 1
    cases = [(1.0, 1.0), (1.0 + u, 1.0 + u),
             (1.0 + u / 2, 1.0),                    # tie -> even (mantissa 0)
             (1.0 + 1.5 * u, 1.0 + 2 * u),          # tie -> even (mantissa 2)
             (1.0 + u / 2 + 2.0 ** -20, 1.0 + u),   # just above the tie
             (1.0 + u / 2 - 2.0 ** -20, 1.0),       # just below the tie
             (-(1.0 + 1.5 * u), -(1.0 + 2 * u)),
             (3.0, 3.0), (0.0, 0.0), (2.0 ** -130, 2.0 ** -130)]
    for x, want in cases:
        assert mlp.bf16(np.array([x]))[0] == want, x
    # every bf16 value is a float32 whose low 16 bits are zero
    r = mlp.bf16(np.random.default_rng(0).normal(size=1000) * 100)
    assert np.all((r.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)
    # relative error at most half a bf16 ulp
    x = np.random.default_rng(1).uniform(0.5, 2.0, size=1000)
    assert np.max(np.abs(mlp.bf16(x) - x) / x) <= 2.0 ** -8 * (1 + 1e-6)


def test_normalize_and_embedding():
    lo, hi = np.array([0.0, 0.0, 8e9]), np.array([180.0, 360.0, 12e9])
    xn = mlp.normalize(np.array([[0.0, 0.0, 8e9], [180.0, 360.0, 12e9], [90.0, 180.0, 10e9]]), lo, hi)
    assert np.allclose(xn, [[-1, -1, -1], [1, 1, 1], [0, 0, 0]])
    B = np.random.default_rng(2).normal(size=(16, 3))
    g = mlp.embed(np.random.default_rng(3).uniform(-1, 1, size=(50, 3)), B)
    assert g.shape == (50, 32)
    assert np.allclose(g[:, :16] ** 2 + g[:, 16:] ** 2, 1.0)
    z = mlp.embed(np.ones((3, 3)), np.zeros((16, 3)))
    assert np.array_equal(z[:, :16], np.zeros((3, 16))) and np.array_equal(z[:, 16:], np.ones((3, 16)))


def _tiny(seed=0, n_ff=4, width=8, depth=2):
    dims = mlp.layer_dims(n_ff, width, depth)
    params = mlp.init_params(dims, seed)
    rng = np.random.default_rng(seed + 100)
    B = rng.normal(scale=0.7, size=(n_ff, 3))
    pts = np.stack([rng.uniform(0, 180, 13), rng.uniform(0, 360, 13), rng.uniform(8e9, 12e9, 13)], axis=1)
    lo, hi = np.array([0.0, 0.0, 8e9]), np.array([180.0, 360.0, 12e9])
    t = rng.normal(size=(13, 4))
    return dims, params, B, pts, lo, hi, t


def test_backward_matches_central_differences():
    dims, params, B, pts, lo, hi, t = _tiny()
    y, cache = mlp.forward(params, B, pts, lo, hi, mlp.ACT_SILU, rounding=False)
    g = mlp.flatten(mlp.backward(params, cache, y, t))
    v0 = mlp.flatten(params)
    fd = np.zeros_like(v0)
    h = 1e-6
    for i in range(len(v0)):
        vp, vm = v0.copy(), v0.copy()
        vp[i] += h
        vm[i] -= h
        yp, _ = mlp.forward(mlp.unflatten(vp, dims), B, pts, lo, hi, mlp.ACT_SILU, rounding=False)
        ym, _ = mlp.forward(mlp.unflatten(vm, dims), B, pts, lo, hi, mlp.ACT_SILU, rounding=False)
        fd[i] = (mlp.loss(yp, t) - mlp.loss(ym, t)) / (2 * h)
    rel = np.linalg.norm(g - fd) / np.linalg.norm(fd)
    assert rel <= 1e-6, rel


def test_activation_derivatives():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    for kind in (mlp.ACT_SILU, mlp.ACT_RELU):
        fd = (mlp.act(z + h, kind) - mlp.act(z - h, kind)) / (2 * h)
        ok = np.abs(z) > 1e-3  # away from the ReLU kink
        assert np.allclose(mlp.act_grad(z, kind)[ok], fd[ok], rtol=1e-6, atol=1e-8)
    assert mlp.act(np.array([0.0]), mlp.ACT_SILU)[0] == 0.0
    assert np.isclose(mlp.act(np.array([1.0]), mlp.ACT_SILU)[0], 1.0 / (1.0 + np.exp(-1.0)))


def test_special_cases_by_hand():
    dims, params, B, pts, lo, hi, t = _tiny(seed=5, n_ff=2, width=3, depth=1)
    # zero output weights: the output is the output bias for every point
    p0 = [(W.copy(), b.copy()) for W, b in params]
    p0[-1] = (np.zeros_like(p0[-1][0]), p0[-1][1])
    y, _ = mlp.forward(p0, B, pts, lo, hi)
    assert np.array_equal(y, np.broadcast_to(p0[-1][1], y.shape))
    # one hidden ReLU layer written out element by element (no rounding)
    (W1, b1), (W2, b2) = params
    y, _ = mlp.forward(params, B, pts, lo, hi, mlp.ACT_RELU, rounding=False)
    for i, p in enumerate(pts):
        xn = [2 * (p[c] - lo[c]) / (hi[c] - lo[c]) - 1 for c in range(3)]
        feats = []
        for f in range(2):
            a = 2 * np.pi * sum(B[f, c] * xn[c] for c in range(3))
            feats.append(np.sin(a))
        for f in range(2):
            a = 2 * np.pi * sum(B[f, c] * xn[c] for c in range(3))
            feats.append(np.cos(a))
        hid = [max(0.0, sum(W1[j, k] * feats[k] for k in range(4)) + b1[j]) for j in range(3)]
        out = [sum(W2[o, j] * hid[j] for j in range(3)) + b2[o] for o in range(4)]
        assert np.allclose(y[i], out, rtol=1e-12, atol=1e-12)


def test_loss_gradient_and_prediction_layout():
    rng = np.random.default_rng(7)
    y, t = rng.normal(size=(5, 4)), rng.normal(size=(5, 4))
    h = 1e-7
    g = 2 * (y - t) / 20
    for i in range(5):
        for j in range(4):
            yp, ym = y.copy(), y.copy()
            yp[i, j] += h
            ym[i, j] -= h
            assert np.isclose((mlp.loss(yp, t) - mlp.loss(ym, t)) / (2 * h), g[i, j], rtol=1e-5)
    tc = np.array([[1 + 2j, 3 - 4j]])
    assert np.array_equal(mlp.targets_real(tc, 2.0), [[0.5, 1.0, 1.5, -2.0]])


def test_adam_first_step_moves_by_lr_in_the_gradient_sign():
    rng = np.random.default_rng(9)
    w0, g = rng.normal(size=100), rng.normal(size=100)
    w1, m, v = mlp.adam_step(w0, g, np.zeros(100), np.zeros(100), 1, 1e-3)
    # bias correction makes the first step lr * g / (|g| + eps): lr in the sign of g
    assert np.allclose(w1, w0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(np.abs(w1 - w0), 1e-3, rtol=1e-4)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    # constant gradient: m/(1-b1^t) and v/(1-b2^t) stay g and g^2, so every step moves lr*sign(g)
    w = w0.copy()
    m = np.zeros(100)
    v = np.zeros(100)
    for k in range(1, 6):
        w, m, v = mlp.adam_step(w, g, m, v, k, 1e-3)
    assert np.allclose(w, w0 - 5e-3 * g / (np.abs(g) + 1e-8), atol=1e-12)


def test_rounded_network_is_close_to_the_exact_one():
    dims, params, B, pts, lo, hi, t = _tiny(seed=3, n_ff=8, width=16, depth=3)
    y1, c1 = mlp.forward(params, B, pts, lo, hi)
    y0, c0 = mlp.forward(params, B, pts, lo, hi, rounding=False)
    assert np.max(np.abs(y1 - y0)) / np.max(np.abs(y0)) < 3e-2
    g1 = mlp.flatten(mlp.backward(params, c1, y1, t))
    g0 = mlp.flatten(mlp.backward(params, c0, y0, t))
    assert np.dot(g1, g0) / np.linalg.norm(g1) / np.linalg.norm(g0) > 0.99
