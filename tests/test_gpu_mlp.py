"""The surrogate network on the GPU (bf16 matrix-core products, fp32
accumulation) against the float64 oracle fed the same bf16-rounded weights
and features: forward values, per-tensor gradients, one Adam step, training
and determinism."""
import sys

import numpy as np
import pytest

from oracle import mlp as om

pytestmark = pytest.mark.gpu

LO = np.array([0.0, 0.0, 8.0e9])
HI = np.array([180.0, 360.0, 12.0e9])


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    from paper_2604_09243_amd import Context
    return Context(0)


def points(n, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(0, 180, n), rng.uniform(0, 360, n), rng.uniform(8e9, 12e9, n)], axis=1)


def oracle_of(net, kind):
    info = net.info()
    dims = om.layer_dims(info["n_ff"], info["width"], info["depth"])
    return om.unflatten(net.params().astype(np.float64), dims), net.features().astype(np.float64), dims


def cos_rel(a, b):
    a, b = np.ravel(a), np.ravel(b)
    cos = np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b))
    rel = np.linalg.norm(a - b) / np.linalg.norm(b)
    return cos, rel


@pytest.mark.parametrize("act,width,depth,n_ff", [(0, 256, 4, 64), (1, 128, 2, 64), (0, 384, 3, 128)])
def test_forward_matches_oracle(torch, ctx, act, width, depth, n_ff):
    say("case forward", act, width, depth, n_ff)
    net = ctx.mlp(LO, HI, out_scale=0.37, n_ff=n_ff, width=width, depth=depth, act=act, ff_sigma=2.0, seed=11)
    info = net.info()
    assert info["n_params"] == sum(o * i + o for o, i in om.layer_dims(n_ff, width, depth))
    params, B, _ = oracle_of(net, act)
    for n, seed in ((1, 1), (63, 2), (1000, 3)):
        pts = points(n, seed)
        A = net.predict(pts).cpu().numpy()
        Ao = om.predict(params, B, pts, LO, HI, 0.37, act)
        cos, rel = cos_rel(np.concatenate([A.real, A.imag]), np.concatenate([Ao.real, Ao.imag]))
        assert cos >= 0.9999 and rel <= 1e-2, (n, cos, rel)
        assert np.max(np.abs(A - Ao)) <= 2e-2 * np.max(np.abs(Ao)), n
    # a large ragged call (several inference chunks) on sampled rows
    pts = points(300_001, 4)
    A = net.predict(pts).cpu().numpy()
    pick = np.random.default_rng(5).choice(len(pts), 2000, replace=False)
    Ao = om.predict(params, B, pts[pick], LO, HI, 0.37, act)
    cos, rel = cos_rel(np.concatenate([A[pick].real, A[pick].imag]), np.concatenate([Ao.real, Ao.imag]))
    assert cos >= 0.9999 and rel <= 1e-2, (cos, rel)
    say("forward cos", cos, "rel", rel)


@pytest.mark.parametrize("act", [0, 1])
def test_gradients_match_oracle_per_tensor(torch, ctx, act):
    say("case gradients", act)
    net = ctx.mlp(LO, HI, out_scale=0.5, act=act, ff_sigma=2.0, seed=21)
    params, B, dims = oracle_of(net, act)
    for n, seed in ((777, 6), (64, 7), (4096, 8)):
        pts = points(n, seed)
        rng = np.random.default_rng(seed + 50)
        t = (rng.normal(size=(n, 2)) + 1j * rng.normal(size=(n, 2))) * 0.5
        g, loss = net.gradients(pts, t)
        y, cache = om.forward(params, B, pts, LO, HI, act)
        tr = om.targets_real(t, 0.5)
        go = om.backward(params, cache, y, tr)
        assert abs(loss - om.loss(y, tr)) <= 1e-3 * om.loss(y, tr)
        off = 0
        worst = (1.0, 0.0)
        for (o, i), (gW, gb) in zip(dims, go):
            for ref, size in ((gW, o * i), (gb, o)):
                cos, rel = cos_rel(g[off:off + size], ref)
                assert cos >= 0.999 and rel <= 1e-2, (n, o, i, size, cos, rel)
                worst = (min(worst[0], cos), max(worst[1], rel))
                off += size
        assert off == len(g)
        say("n", n, "worst cos", worst[0], "worst rel", worst[1])
    # bitwise reproducible
    g2, _ = net.gradients(pts, t)
    assert np.array_equal(g, g2)


def test_one_adam_step_matches_oracle(torch, ctx):
    say("case adam step")
    net = ctx.mlp(LO, HI, out_scale=1.0, ff_sigma=2.0, seed=31)
    params, B, dims = oracle_of(net, 0)
    w0 = net.params().astype(np.float64)
    n = 512
    pts = points(n, 9)
    t = np.exp(1j * np.random.default_rng(10).uniform(0, 6.28, size=(n, 2)))
    y, cache = om.forward(params, B, pts, LO, HI)
    g = om.flatten(om.backward(params, cache, y, om.targets_real(t, 1.0)))
    w_or, _, _ = om.adam_step(w0, g, np.zeros_like(w0), np.zeros_like(w0), 1, 1e-3)
    net.train(pts, t, epochs=1, batch=n, lr=1e-3, lr_min=1e-3)
    w1 = net.params().astype(np.float64)
    d_gpu, d_or = w1 - w0, w_or - w0
    big = np.abs(g) > 1e-3 * np.max(np.abs(g))
    agree = np.mean(np.sign(d_gpu[big]) == np.sign(d_or[big]))
    assert agree >= 0.99, agree
    assert np.max(np.abs(d_gpu[big] - d_or[big])) <= 1e-4
    assert np.max(np.abs(d_gpu)) <= 1e-3 * (1 + 1e-5)
    assert net.info()["adam_steps"] == 1


def test_training_fits_a_smooth_field(torch, ctx):
    say("case training")
    net = ctx.mlp(LO, HI, out_scale=1.0, ff_sigma=1.0, seed=41)
    pts = points(8192, 12)
    xn = om.normalize(pts, LO, HI)
    # a smooth complex field of the normalised inputs
    ph = 2.0 * xn[:, 0] + 3.0 * xn[:, 1] - 1.5 * xn[:, 2]
    amp = 1.0 + 0.3 * np.cos(2.0 * xn[:, 1])
    t = np.stack([amp * np.exp(1j * ph), 0.5 * amp * np.exp(-1j * ph)], axis=1)
    hist = net.train(pts, t, epochs=40, batch=1024, lr=2e-3, lr_min=1e-4, seed=1)
    say("loss", hist[0], "->", hist[-1])
    assert hist[-1] < 0.02 * hist[0]
    test = points(2000, 13)
    xt = om.normalize(test, LO, HI)
    pht = 2.0 * xt[:, 0] + 3.0 * xt[:, 1] - 1.5 * xt[:, 2]
    ampt = 1.0 + 0.3 * np.cos(2.0 * xt[:, 1])
    tt = np.stack([ampt * np.exp(1j * pht), 0.5 * ampt * np.exp(-1j * pht)], axis=1)
    A = net.predict(test).cpu().numpy()
    rms = np.sqrt(np.mean(np.abs(A - tt) ** 2)) / np.sqrt(np.mean(np.abs(tt) ** 2))
    say("held-out relative rms", rms)
    assert rms < 0.1


def test_errors(torch, ctx):
    from paper_2604_09243_amd import sbr
    with pytest.raises(sbr.SbrError):
        ctx.mlp(LO, HI, n_ff=48)
    with pytest.raises(sbr.SbrError):
        ctx.mlp(LO, HI, width=200)
    with pytest.raises(sbr.SbrError):
        ctx.mlp(HI, LO)
    net = ctx.mlp(LO, HI)
    with pytest.raises(sbr.SbrError):
        net.set_params(np.zeros(10, np.float32))
