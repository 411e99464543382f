"""Reference MLP of the learned cache -- TEST INFRASTRUCTURE ONLY.

Plain numpy in binary64.  The network maps a vertex (normalised position q in
[0,1]^3, shading normal n in [-1,1]^3) to three log sample counts:
  features: sin / cos(2^k pi x) for k = 0..5 of each of the 6 inputs (72),
            zero-padded to 80;
  three hidden layers of 64 units with ReLU; a linear output of 3 units
  (padded to 16 in the parameter layout, padding fixed at zero).
The learned cache is not in the paper (its Sec. 6 asks for smoothly varying
counts); this follows the configuration of the learned-cache workload.

`forward(..., bf16=True)` reproduces the device arithmetic's roundings:
features, weights and hidden activations rounded to bfloat16 (round to
nearest even), biases and sums in binary64 here (binary32 on the device).
The backward pass is pinned by central finite differences on the unrounded
network (tests/test_mlp_ref.py).
"""
from __future__ import annotations

import numpy as np

N_IN, N_FEAT, N_FEAT_PAD, N_HID, N_OUT, N_OUT_PAD = 6, 72, 80, 64, 3, 16
SHAPES = [("W1", (N_HID, N_FEAT_PAD)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_HID, N_HID)), ("b3", (N_HID,)), ("W4", (N_OUT_PAD, N_HID)), ("b4", (N_OUT_PAD,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(flat):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(flat[o:o + n], np.float64).reshape(shp)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], np.float64).ravel() for name, _ in SHAPES])


def bf16(x):
    """binary32 -> bfloat16 (round to nearest even) -> binary64."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def encode(x):
    """x [N, 6] -> features [N, 80]: sin, cos of 2^k pi x_d, d-major."""
    x = np.asarray(x, np.float64)
    f = np.zeros((x.shape[0], N_FEAT_PAD))
    for d in range(N_IN):
        for k in range(6):
            a = np.pi * (2.0 ** k) * x[:, d]
            f[:, (d * 6 + k) * 2] = np.sin(a)
            f[:, (d * 6 + k) * 2 + 1] = np.cos(a)
    return f


def forward(flat, x, bf16_round=True):
    p = unpack(flat)
    r = bf16 if bf16_round else (lambda v: np.asarray(v, np.float64))
    h0 = r(encode(x))
    cache = [h0]
    h = h0
    for l in (1, 2, 3):
        z = h @ r(p[f"W{l}"]).T + p[f"b{l}"]
        h = r(np.maximum(z, 0.0))
        cache.append(h)
    y = h @ r(p["W4"]).T + p["b4"]
    return y[:, :N_OUT], cache


def loss_and_grad(flat, x, target, weight, bf16_round=True):
    """L = (1/N) sum_i sum_t w_it (y_it - y*_it)^2 and dL/dparams (binary64)."""
    p = unpack(flat)
    r = bf16 if bf16_round else (lambda v: np.asarray(v, np.float64))
    y, cache = forward(flat, x, bf16_round)
    n = x.shape[0]
    diff = y - target
    loss = float(np.sum(weight * diff * diff) / n)
    dy = np.zeros((n, N_OUT_PAD))
    dy[:, :N_OUT] = 2.0 * weight * diff / n
    g = {}
    dz = dy
    for l in (4, 3, 2, 1):
        hprev = cache[l - 1]
        g[f"W{l}"] = dz.T @ hprev
        g[f"b{l}"] = dz.sum(0)
        if l > 1:
            dh = dz @ r(p[f"W{l}"])
            dz = dh * (hprev > 0)
    return loss, pack(g)


def adam_step(flat, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.99, eps=1e-8):
    """One Adam update in binary32 (step counts from 1)."""
    f32 = np.float32
    g = np.asarray(grad, f32)
    m = (f32(b1) * np.asarray(m, f32) + f32(1 - b1) * g).astype(f32)
    v = (f32(b2) * np.asarray(v, f32) + f32(1 - b2) * g * g).astype(f32)
    mh = m / f32(1 - b1 ** step)
    vh = v / f32(1 - b2 ** step)
    w = (np.asarray(flat, f32) - f32(lr) * mh / (np.sqrt(vh) + f32(eps))).astype(f32)
    return w, m, v


def init_params(seed=1):
    """He-uniform weights, zero biases, zero output padding."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in SHAPES:
        if name.startswith("b"):
            p[name] = np.zeros(shp)
        else:
            bound = np.sqrt(6.0 / shp[1])
            p[name] = rng.uniform(-bound, bound, shp)
    p["W4"][N_OUT:] = 0.0
    p["W4"] *= 0.1
    return pack(p).astype(np.float32)
