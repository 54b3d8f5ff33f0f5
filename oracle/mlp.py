"""CPU oracle of the per-point warm-start MLP (test infrastructure).

A 5 -> 128 -> 128 -> 128 -> 4 perceptron with GELU (erf form) on the hidden
layers, evaluated in float64 with the same quantisation points as the HIP
kernels: bfloat16 (round to nearest even) copies of the weights, the inputs and
the hidden activations that feed each matrix product; the backward pass rounds
the pre-activation gradients of the two 128 x 128 layers to bfloat16 before
their products.  With ``quantize=False`` every rounding is skipped, which gives
the smooth float64 network that the finite-difference pins use.

Parameters are one flat float32 vector of 34,308 entries:
W1[128][5], b1[128], W2[128][128], b2[128], W3[128][128], b3[128], W4[4][128], b4[4].
The loss is the mean over points and the 4 outputs of (y - t)^2.
Adam (Kingma and Ba, 2015) updates float32 master weights.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SHAPES = [("W1", (128, 5)), ("b1", (128,)), ("W2", (128, 128)), ("b2", (128,)),
          ("W3", (128, 128)), ("b3", (128,)), ("W4", (4, 128)), ("b4", (4,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)
assert N_PARAMS == 34308


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = theta[o:o + k].reshape(shape)
        o += k
    return out


def pack(parts: dict) -> np.ndarray:
    return np.concatenate([np.asarray(parts[n], dtype=np.float64).reshape(-1) for n, _ in SHAPES])


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) via float32; returns float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if np.any(nan):
        out[nan] = np.nan
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(theta, X, quantize=True):
    """Returns (Y, cache).  X: [M][5] features."""
    q = bf16 if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    P = unpack(np.asarray(theta, dtype=np.float64))
    W = {k: q(P[k]) for k in ("W1", "W2", "W3", "W4")}
    x = q(X)
    z1 = x @ W["W1"].T + P["b1"]
    h1 = q(gelu(z1))
    z2 = h1 @ W["W2"].T + P["b2"]
    h2 = q(gelu(z2))
    z3 = h2 @ W["W3"].T + P["b3"]
    h3 = q(gelu(z3))
    y = h3 @ W["W4"].T + P["b4"]
    return y, dict(x=x, z1=z1, h1=h1, z2=z2, h2=h2, z3=z3, h3=h3, W=W)


def loss_and_grad(theta, X, T, quantize=True):
    """Loss and its gradient (flat, float64) with respect to the parameters."""
    q = bf16 if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    M = X.shape[0]
    y, c = forward(theta, X, quantize)
    r = y - T
    loss = float(np.mean(r * r))
    dy = 2.0 * r / (4.0 * M)
    W = c["W"]
    g = {}
    g["W4"] = dy.T @ c["h3"]
    g["b4"] = dy.sum(axis=0)
    dz3 = q((dy @ W["W4"]) * gelu_prime(c["z3"]))
    g["W3"] = dz3.T @ c["h2"]
    g["b3"] = dz3.sum(axis=0)
    dz2 = q((dz3 @ W["W3"]) * gelu_prime(c["z2"]))
    g["W2"] = dz2.T @ c["h1"]
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ W["W2"]) * gelu_prime(c["z1"])
    g["W1"] = dz1.T @ c["x"]
    g["b1"] = dz1.sum(axis=0)
    return loss, pack(g)


def adam(theta, m, v, grad, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in float32 (returns new theta, m, v)."""
    theta = np.asarray(theta, np.float32)
    g = np.asarray(grad, np.float32)
    m = (b1 * m + (1 - b1) * g).astype(np.float32)
    v = (b2 * v + (1 - b2) * g * g).astype(np.float32)
    mh = m / np.float32(1 - b1 ** step)
    vh = v / np.float32(1 - b2 ** step)
    theta = (theta - np.float32(lr) * mh / (np.sqrt(vh) + np.float32(eps))).astype(np.float32)
    return theta, m, v


def features(x, y, ptype, mach, aoa_deg):
    """Warm-start features [n][5] of the points of one cloud (float64).

    f0 = (x - 1/2) / (1 + r), f1 = y / (1 + r), r = |(x - 1/2, y)|;
    f2 = 2 d / (d + 0.1) - 1, d = distance to the nearest wall point (brute force);
    f3 = (M - 0.6) / 0.25; f4 = (aoa - 2) / 6 (degrees).
    """
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    wall = np.flatnonzero(np.asarray(ptype) == 0)
    if wall.size:
        d = np.empty(x.size)
        for i in range(x.size):
            d[i] = math.sqrt(float(np.min((x[i] - x[wall]) ** 2 + (y[i] - y[wall]) ** 2)))
    else:
        d = np.full(x.size, 1e3)
    ex = x - 0.5
    r = np.sqrt(ex * ex + y * y)
    F = np.empty((x.size, 5))
    F[:, 0] = ex / (1.0 + r)
    F[:, 1] = y / (1.0 + r)
    F[:, 2] = 2.0 * d / (d + 0.1) - 1.0
    F[:, 3] = (mach - 0.6) / 0.25
    F[:, 4] = (aoa_deg - 2.0) / 6.0
    return F


def targets(U, mach, aoa_deg, gamma=1.4):
    """Deviation of U ([4][n]) from the free stream: (rho - 1, u - u_inf, v - v_inf, gamma p - 1)."""
    a = math.radians(aoa_deg)
    rho = U[0]
    u, v = U[1] / rho, U[2] / rho
    p = (gamma - 1.0) * (U[3] - 0.5 * rho * (u * u + v * v))
    return np.stack([rho - 1.0, u - mach * math.cos(a), v - mach * math.sin(a), gamma * p - 1.0], 1)


def state_from_prediction(Y, ptype, tx, ty, mach, aoa_deg, gamma=1.4):
    """U ([4][n]) of a predicted deviation Y ([n][4]): outer points at the free
    stream, wall points with the velocity projected on the wall tangent."""
    a = math.radians(aoa_deg)
    ui, vi = mach * math.cos(a), mach * math.sin(a)
    Y = np.where((np.asarray(ptype) == 2)[:, None], 0.0, np.asarray(Y, np.float64))
    rho = 1.0 + Y[:, 0]
    u = ui + Y[:, 1]
    v = vi + Y[:, 2]
    p = (1.0 + Y[:, 3]) / gamma
    wall = np.asarray(ptype) == 0
    ut = u * tx + v * ty
    u = np.where(wall, ut * tx, u)
    v = np.where(wall, ut * ty, v)
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])
