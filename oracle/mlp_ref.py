"""CPU reference of the surrogate network and of two-stage unweighting.

TEST INFRASTRUCTURE ONLY (imported by ``tests/`` and the benchmark's CPU
baseline, never by the product path; shares no code with the HIP kernels).

Network (the learned part of the build; not in the paper): a multilayer
perceptron with ``depth`` hidden layers of width ``width`` and SiLU
activations, x -> y, trained by mean squared error with Adam.
    h_0 = x,  z_l = W_l h_{l-1} + b_l,  h_l = silu(z_l) (l = 1..depth),
    y = w_out . h_depth + b_out,  silu(z) = z sigmoid(z),
    silu'(z) = sigmoid(z) (1 + z (1 - sigmoid(z))).
Loss L = mean_m (y_m - t_m)^2.  Adam (Kingma, Ba 2015) with bias correction:
    m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
    theta <- theta - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Flat parameter layout shared with the GPU library (an interface, not code):
    [W_1 (width x n_in, row-major), b_1, W_2 (width x width), b_2, ...,
     W_depth, b_depth, w_out (width), b_out].

Two-stage unweighting (Danziger, Janssen, Schumann, Siegert, SciPost Phys. 12
(2022) 164): with surrogate weight s and exact weight w of a point,
    stage 1: accept with probability min(1, s / s_max)            (uniform u1)
    stage 2: accept with probability min(1, (w/s) / r_max)         (uniform u2)
    output weight max(1, s/s_max) * max(1, (w/s)/r_max),
so that E[accepted x weight] = w / (s_max r_max) for every point.
"""
from __future__ import annotations

import numpy as np


def n_params(n_in: int = 24, width: int = 256, depth: int = 4) -> int:
    return width * n_in + width + (depth - 1) * (width * width + width) + width + 1


def unpack(theta, n_in=24, width=256, depth=4):
    """Views (W_l, b_l) for l = 1..depth and (w_out, b_out) into the flat vector."""
    theta = np.asarray(theta)
    layers = []
    o = 0
    fan_in = n_in
    for _ in range(depth):
        W = theta[o:o + width * fan_in].reshape(width, fan_in)
        o += width * fan_in
        b = theta[o:o + width]
        o += width
        layers.append((W, b))
        fan_in = width
    w_out = theta[o:o + width]
    o += width
    b_out = theta[o:o + 1]
    o += 1
    assert o == theta.size
    return layers, w_out, b_out


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def silu(z):
    return z * sigmoid(z)


def silu_prime(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def forward(theta, x, n_in=24, width=256, depth=4, keep=False):
    layers, w_out, b_out = unpack(theta, n_in, width, depth)
    h = np.asarray(x, dtype=np.float64)
    zs, hs = [], [h]
    for W, b in layers:
        z = h @ W.T + b
        h = silu(z)
        zs.append(z)
        hs.append(h)
    y = h @ w_out + b_out[0]
    return (y, zs, hs) if keep else y


def loss_and_grad(theta, x, t, n_in=24, width=256, depth=4):
    """Mean squared error and its gradient with respect to the flat parameters."""
    y, zs, hs = forward(theta, x, n_in, width, depth, keep=True)
    m = len(t)
    r = y - t
    loss = float(np.mean(r * r))
    dy = 2.0 * r / m
    layers, w_out, _ = unpack(theta, n_in, width, depth)
    g_layers = [None] * depth
    g_wout = hs[-1].T @ dy
    g_bout = np.array([dy.sum()])
    dh = np.outer(dy, w_out)
    for l in range(depth - 1, -1, -1):
        dz = dh * silu_prime(zs[l])
        gW = dz.T @ hs[l]
        gb = dz.sum(axis=0)
        g_layers[l] = (gW, gb)
        if l > 0:
            dh = dz @ layers[l][0]
    parts = []
    for gW, gb in g_layers:
        parts += [gW.ravel(), gb]
    parts += [g_wout, g_bout]
    return loss, np.concatenate(parts)


def adam_step(theta, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(a):
    """Round float64 values to the nearest bfloat16 (ties to even), as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def two_stage(s, w, u1, u2, s_max, r_max):
    """Accept decisions and output weights of two-stage unweighting."""
    s = np.asarray(s, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    a1 = s / s_max
    acc1 = u1 < np.minimum(1.0, a1)
    r = np.where(s > 0, w / np.where(s > 0, s, 1.0), 0.0)
    a2 = r / r_max
    acc2 = acc1 & (u2 < np.minimum(1.0, a2))
    weight = np.maximum(1.0, a1) * np.maximum(1.0, a2)
    return acc1, acc2, np.where(acc2, weight, 0.0)
