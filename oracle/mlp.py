"""Oracle of the Fourier-feature MLP surrogate: float64 forward, backward,
loss and Adam step of the exact network the GPU trains and evaluates.

TEST INFRASTRUCTURE ONLY (see the package header).  Plain numpy, written from
the definitions below; it shares nothing with the HIP kernels.

Network (input = one (theta_deg, phi_deg, f_hz) point):
  xn    = 2 (x - lo) / (hi - lo) - 1, per coordinate (lo, hi: the model's
          input ranges)
  gamma = [sin(2 pi B xn), cos(2 pi B xn)], B: [n_ff, 3] fixed (random
          Fourier features), so gamma has 2 n_ff entries
  h0    = bf16(gamma)
  z_l   = h_{l-1} bf16(W_l)^T + b_l,  h_l = bf16(act(z_l)),  l = 1..depth
  y     = h_depth bf16(W_out)^T + b_out  (4 outputs)
  A_HH  = s (y0 + j y1),  A_VV = s (y2 + j y3)   (s: the output scale)
act is SiLU, z / (1 + exp(-z)), or ReLU.  bf16(.) rounds to the nearest
bfloat16 (ties to even); the kernels round at exactly these points, and
with ``rounding=False`` the oracle is the plain float64 network (used for
the finite-difference pin).

Loss: mean over the M points and 4 outputs of (y - t / s)^2.
Backward (same rounding points as the kernels):
  dy      = 2 (y - t/s) / (4 M)
  dW_out  = dy^T h_depth,  db_out = sum_i dy,  dh_depth = dy bf16(W_out)
  for l = depth..1:
    dz = dh_l * act'(z_l);  dzb = bf16(dz)
    dW_l = dzb^T h_{l-1};  db_l = sum_i dz;  dh_{l-1} = dzb bf16(W_l)
Adam (Kingma and Ba, Algorithm 1): m = b1 m + (1 - b1) g,
v = b2 v + (1 - b2) g^2, w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Parity status: pinned by tests/test_oracle_mlp.py (finite differences of
the float64 network, bf16 rounding cases, closed-form special cases, the
Adam first-step property).
"""
import numpy as np

ACT_SILU, ACT_RELU = 0, 1


def bf16(x):
    """Round float64/float32 values to the nearest bfloat16 (ties to even),
    returned as float64.  Values are first rounded to float32, which is what
    the kernels hold before converting."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def layer_dims(n_ff=64, width=256, depth=4):
    """[(n_out, n_in)] of the hidden layers and the output layer."""
    dims = [(width, 2 * n_ff)] + [(width, width)] * (depth - 1) + [(4, width)]
    return dims


def init_params(dims, seed):
    """A seeded He-style initialisation (used only to make test inputs)."""
    rng = np.random.default_rng(seed)
    ps = []
    for n_out, n_in in dims:
        W = rng.normal(scale=np.sqrt(2.0 / n_in), size=(n_out, n_in)).astype(np.float32)
        b = rng.normal(scale=0.05, size=n_out).astype(np.float32)
        ps.append((W.astype(np.float64), b.astype(np.float64)))
    return ps


def flatten(params):
    """Parameter vector in the order W_1, b_1, ..., W_out, b_out (row-major)."""
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])


def unflatten(vec, dims):
    out, o = [], 0
    for n_out, n_in in dims:
        W = np.asarray(vec[o:o + n_out * n_in], dtype=np.float64).reshape(n_out, n_in)
        o += n_out * n_in
        b = np.asarray(vec[o:o + n_out], dtype=np.float64)
        o += n_out
        out.append((W, b))
    return out


def normalize(pts, lo, hi):
    pts = np.asarray(pts, dtype=np.float64)
    lo, hi = np.asarray(lo, dtype=np.float64), np.asarray(hi, dtype=np.float64)
    return 2.0 * (pts - lo) / (hi - lo) - 1.0


def embed(xn, B):
    """Random Fourier features of normalised inputs: [sin(2 pi B x), cos(2 pi B x)]."""
    arg = 2.0 * np.pi * (np.asarray(xn, dtype=np.float64) @ np.asarray(B, dtype=np.float64).T)
    return np.concatenate([np.sin(arg), np.cos(arg)], axis=1)


def act(z, kind):
    if kind == ACT_SILU:
        return z / (1.0 + np.exp(-z))
    return np.maximum(z, 0.0)


def act_grad(z, kind):
    if kind == ACT_SILU:
        s = 1.0 / (1.0 + np.exp(-z))
        return s * (1.0 + z * (1.0 - s))
    return (z > 0.0).astype(np.float64)


def forward(params, B, pts, lo, hi, kind=ACT_SILU, rounding=True):
    """Returns (y [M, 4], cache) for raw points pts [M, 3]."""
    R = bf16 if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    h = R(embed(normalize(pts, lo, hi), B))
    hs, zs = [h], []
    for W, b in params[:-1]:
        z = h @ R(W).T + b
        zs.append(z)
        h = R(act(z, kind))
        hs.append(h)
    W, b = params[-1]
    y = h @ R(W).T + b
    return y, dict(hs=hs, zs=zs, rounding=rounding, kind=kind)


def predict(params, B, pts, lo, hi, scale, kind=ACT_SILU, rounding=True):
    """Complex A [M, 2] (HH, VV)."""
    y, _ = forward(params, B, pts, lo, hi, kind, rounding)
    return scale * np.stack([y[:, 0] + 1j * y[:, 1], y[:, 2] + 1j * y[:, 3]], axis=1)


def targets_real(t_complex, scale):
    t = np.asarray(t_complex) / scale
    return np.stack([t[:, 0].real, t[:, 0].imag, t[:, 1].real, t[:, 1].imag], axis=1)


def loss(y, t):
    return float(np.mean((y - t) ** 2))


def backward(params, cache, y, t):
    """Gradients [(dW, db)] of the mean-squared loss for targets t [M, 4]."""
    R = bf16 if cache["rounding"] else (lambda v: np.asarray(v, dtype=np.float64))
    kind = cache["kind"]
    hs, zs = cache["hs"], cache["zs"]
    M = y.shape[0]
    dy = 2.0 * (y - t) / (4.0 * M)
    Wo, _ = params[-1]
    grads = [None] * len(params)
    grads[-1] = (dy.T @ hs[-1], dy.sum(axis=0))
    dh = dy @ R(Wo)
    for l in range(len(params) - 2, -1, -1):
        dz = dh * act_grad(zs[l], kind)
        dzb = R(dz)
        grads[l] = (dzb.T @ hs[l], dz.sum(axis=0))
        if l > 0:
            dh = dzb @ R(params[l][0])
    return grads


def adam_step(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update of float64 arrays; returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
