"""FP64 reference of the warm-start 3D U-Net (forward and analytic backward).

TEST INFRASTRUCTURE ONLY.  The GPU library is checked against this; the
product path never imports it.  The paper has no learned component: this
network only proposes the starting point x_0 of the FISTA solve, whose
objective still decides the result.

Architecture (channels-last volumes [z][y][x][c]):
  level l = 0..L-1 has C_l = base * 2^l channels;
  encoder level l: two 3x3x3 convolutions (padding 1) each followed by ReLU,
    then 2x2x2 max pooling (except at the bottom level);
  decoder level l (from L-2 down to 0): 2x2x2 stride-2 transposed convolution
    C_{l+1} -> C_l (no activation), concatenation [up, skip] (up first), two
    3x3x3 convolutions + ReLU;
  head: 1x1x1 convolution C_0 -> 1 followed by ReLU (x_0 >= 0).
Every convolution has a bias.  Training loss: weighted mean squared error of
the head's pre-activation (before the ReLU, which applies at inference) to the
target.

Storage precision (optional): with store=bf16_round, every activation a
layer writes (convolution outputs after ReLU, up-convolution outputs) is
rounded to bfloat16 before the next layer reads it, so that the ReLU masks and
max-pooling choices are taken on the same stored values as in a network kept
in bfloat16; the arithmetic stays FP64 and the backward pass treats the
rounding as the identity.  The head output is not rounded.

Parameters are a dict of arrays:
  conv weights w[kz][ky][kx][cin][cout], bias b[cout];
  transposed-conv weights u[dz][dy][dx][cin][cout], bias b[cout];
  head weights h[cin], bias scalar.
"""
from __future__ import annotations

import numpy as np

__all__ = ["layer_specs", "init_params", "forward", "loss_and_grads", "conv3", "conv3_backward",
           "maxpool2", "maxpool2_backward", "upconv2", "upconv2_backward", "bf16_round"]


def bf16_round(a):
    """Nearest bfloat16 value (ties to even) of the float32 value of `a`.

    bfloat16 keeps the top 16 bits of an IEEE float32 (sign, 8 exponent bits,
    7 fraction bits); rounding adds half of the dropped range, plus one when the
    kept part is odd, before truncating.  Finite inputs only."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def layer_specs(levels: int, base: int):
    """Ordered (name, kind, cin, cout) of every parameterised layer."""
    ch = [base * (2 ** l) for l in range(levels)]
    specs = []
    cin = 1
    for l in range(levels):
        specs.append((f"enc{l}a", "conv", cin, ch[l]))
        specs.append((f"enc{l}b", "conv", ch[l], ch[l]))
        cin = ch[l]
    for l in range(levels - 2, -1, -1):
        specs.append((f"up{l}", "up", ch[l + 1], ch[l]))
        specs.append((f"dec{l}a", "conv", 2 * ch[l], ch[l]))
        specs.append((f"dec{l}b", "conv", ch[l], ch[l]))
    specs.append(("head", "head", ch[0], 1))
    return specs


def init_params(levels: int, base: int, rng: np.random.Generator):
    p = {}
    for name, kind, cin, cout in layer_specs(levels, base):
        if kind == "conv":
            p[name + ".w"] = rng.standard_normal((3, 3, 3, cin, cout)) * np.sqrt(2.0 / (27 * cin))
            p[name + ".b"] = 0.01 * rng.standard_normal(cout)
        elif kind == "up":
            p[name + ".w"] = rng.standard_normal((2, 2, 2, cin, cout)) * np.sqrt(1.0 / cin)
            p[name + ".b"] = 0.01 * rng.standard_normal(cout)
        else:
            p[name + ".w"] = rng.standard_normal(cin) * np.sqrt(1.0 / cin)
            p[name + ".b"] = np.array(0.01)
    return p


# ----------------------------------------------------------------------------
# Layers (definitions written out)
# ----------------------------------------------------------------------------
def conv3(x, w, b):
    """y[p, co] = b[co] + sum_{k, ci} w[k][ci][co] x[p + k - 1, ci], zero padding."""
    D, H, W, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    y = np.broadcast_to(b, (D, H, W, w.shape[-1])).copy()
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                y += xp[kz:kz + D, ky:ky + H, kx:kx + W, :] @ w[kz, ky, kx]
    return y


def conv3_backward(x, w, gy):
    """Gradients of conv3 w.r.t. x, w, b given dL/dy."""
    D, H, W, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                sl = xp[kz:kz + D, ky:ky + H, kx:kx + W, :]
                gw[kz, ky, kx] = np.einsum("zyxc,zyxo->co", sl, gy)
                gxp[kz:kz + D, ky:ky + H, kx:kx + W, :] += gy @ w[kz, ky, kx].T
    return gxp[1:-1, 1:-1, 1:-1, :], gw, gy.sum(axis=(0, 1, 2))


def maxpool2(x):
    """2x2x2 max pooling; returns (y, argmax index 0..7 as dz*4 + dy*2 + dx)."""
    D, H, W, C = x.shape
    blocks = x.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).transpose(0, 2, 4, 1, 3, 5, 6)
    flat = blocks.reshape(D // 2, H // 2, W // 2, 8, C)
    idx = flat.argmax(axis=3)
    y = np.take_along_axis(flat, idx[:, :, :, None, :], axis=3)[:, :, :, 0, :]
    return y, idx


def maxpool2_backward(gy, idx, shape):
    D, H, W, C = shape
    flat = np.zeros((D // 2, H // 2, W // 2, 8, C))
    np.put_along_axis(flat, idx[:, :, :, None, :], gy[:, :, :, None, :], axis=3)
    blocks = flat.reshape(D // 2, H // 2, W // 2, 2, 2, 2, C).transpose(0, 3, 1, 4, 2, 5, 6)
    return blocks.reshape(D, H, W, C)


def upconv2(x, u, b):
    """y[2q + d, co] = b[co] + sum_ci x[q, ci] u[d][ci][co]."""
    D, H, W, _ = x.shape
    co = u.shape[-1]
    y = np.empty((2 * D, 2 * H, 2 * W, co))
    for dz in range(2):
        for dy in range(2):
            for dx in range(2):
                y[dz::2, dy::2, dx::2, :] = x @ u[dz, dy, dx] + b
    return y


def upconv2_backward(x, u, gy):
    gx = np.zeros_like(x)
    gu = np.zeros_like(u)
    for dz in range(2):
        for dy in range(2):
            for dx in range(2):
                g = gy[dz::2, dy::2, dx::2, :]
                gx += g @ u[dz, dy, dx].T
                gu[dz, dy, dx] = np.einsum("zyxc,zyxo->co", x, g)
    return gx, gu, gy.sum(axis=(0, 1, 2))


def relu(a):
    return np.maximum(a, 0.0)


# ----------------------------------------------------------------------------
# Network
# ----------------------------------------------------------------------------
def forward(params, x, levels, base, keep=False, store=None):
    """x: [D][H][W] input; returns y [D][H][W] (and the activation cache).
    store: optional rounding applied to every stored activation (bf16_round)."""
    st = store if store is not None else (lambda a: a)
    cache = {}
    h = x[..., None].astype(np.float64)
    skips = []
    for l in range(levels):
        for s in ("a", "b"):
            a = conv3(h, params[f"enc{l}{s}.w"], params[f"enc{l}{s}.b"])
            cache[f"enc{l}{s}.in"] = h
            h = st(relu(a))
            cache[f"enc{l}{s}.out"] = h
        if l < levels - 1:
            skips.append(h)
            cache[f"pool{l}.in"] = h
            h, idx = maxpool2(h)
            cache[f"pool{l}.idx"] = idx
    for l in range(levels - 2, -1, -1):
        cache[f"up{l}.in"] = h
        up = st(upconv2(h, params[f"up{l}.w"], params[f"up{l}.b"]))
        h = np.concatenate([up, skips[l]], axis=-1)
        for s in ("a", "b"):
            a = conv3(h, params[f"dec{l}{s}.w"], params[f"dec{l}{s}.b"])
            cache[f"dec{l}{s}.in"] = h
            h = st(relu(a))
            cache[f"dec{l}{s}.out"] = h
    cache["head.in"] = h
    y = relu(h @ params["head.w"] + params["head.b"])
    cache["head.out"] = y
    return (y, cache) if keep else y


def loss_and_grads(params, x, target, levels, base, store=None, pos_weight=1.0):
    """Weighted MSE loss (1/n) sum w (z - t)^2 of the head's pre-activation z,
    w = pos_weight where t > 0 and 1 elsewhere, and its gradient for every
    parameter."""
    _, c = forward(params, x, levels, base, keep=True, store=store)
    z = c["head.in"] @ params["head.w"] + params["head.b"]
    n = z.size
    w = np.where(target > 0, pos_weight, 1.0)
    loss = float((w * (z - target) ** 2).sum() / n)
    gy = 2.0 * w * (z - target) / n
    return loss, _backward(params, c, gy, levels, base)


def _backward(params, c, gy, levels, base):
    ch = [base * (2 ** l) for l in range(levels)]
    g = {}
    g["head.w"] = np.einsum("zyxc,zyx->c", c["head.in"], gy)
    g["head.b"] = np.array(gy.sum())
    gh = gy[..., None] * params["head.w"]
    gskip = [None] * (levels - 1)
    # decoder from the finest level (the last one built) down to the coarsest
    for l in range(0, levels - 1):
        for s in ("b", "a"):
            name = f"dec{l}{s}"
            ga = gh * (c[name + ".out"] > 0)
            gh, g[name + ".w"], g[name + ".b"] = conv3_backward(c[name + ".in"], params[name + ".w"], ga)
        gup, gskip[l] = gh[..., :ch[l]], gh[..., ch[l]:]
        gh, g[f"up{l}.w"], g[f"up{l}.b"] = upconv2_backward(c[f"up{l}.in"], params[f"up{l}.w"], gup)
    # gh is now the gradient w.r.t. the bottom level's output
    for l in range(levels - 1, -1, -1):
        if l < levels - 1:
            gh = maxpool2_backward(gh, c[f"pool{l}.idx"], c[f"pool{l}.in"].shape) + gskip[l]
        for s in ("b", "a"):
            name = f"enc{l}{s}"
            ga = gh * (c[name + ".out"] > 0)
            gh, g[name + ".w"], g[name + ".b"] = conv3_backward(c[name + ".in"], params[name + ".w"], ga)
    return g
