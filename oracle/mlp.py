"""Multilayer perceptron for the learned warm start (oracle; test infrastructure only).

The network maps slab features to coarse initial factors: layers
x_{l+1} = GELU(W_l x_l + b_l) with a linear last layer, squared-error loss,
Adam updates.  Two arithmetic modes:

  * "f64":  everything in FP64 (the plain definition; pinned by finite
    differences below);
  * "bf16": the device's rounding points emulated: each layer's input and
    weights rounded to BF16 (round to nearest, ties to even) before the
    product, accumulation and everything else in FP64.  The device accumulates
    in FP32, so its results differ from this mode only by FP32 summation
    error.

GELU(z) = z Phi(z) with Phi the standard normal CDF (erf form), derivative
Phi(z) + z phi(z).  Adam with bias correction (beta1 = 0.9, beta2 = 0.999,
eps = 1e-8); the gradient of the BF16 weights is applied to FP32 master
weights (the device rounds the masters to FP32 after each step).
"""
import numpy as np
from scipy.special import erf


def bf16_round(x):
    """Round FP64/FP32 values to the nearest BF16 value (ties to even), via the
    FP32 bit pattern; returns float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    out[nan] = np.nan
    return out.reshape(np.shape(x))


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def init(widths, seed):
    """He-style initial weights (normal, std sqrt(2/in)), zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ws = [rng.standard_normal((o, i)) * np.sqrt(2.0 / i) for i, o in zip(widths[:-1], widths[1:])]
    bs = [np.zeros(o) for o in widths[1:]]
    return Ws, bs


def forward(Ws, bs, X, mode="f64"):
    """X: batch x in.  Returns (Y, cache) with cache = per layer (input used, z)."""
    cache = []
    a = np.asarray(X, dtype=np.float64)
    L = len(Ws)
    for l, (W, b) in enumerate(zip(Ws, bs)):
        xin = bf16_round(a) if mode == "bf16" else a
        Wq = bf16_round(W) if mode == "bf16" else W
        z = xin @ Wq.T + b
        cache.append((xin, z))
        a = gelu(z) if l < L - 1 else z
    return a, cache


def loss(Y, T):
    """Mean squared error over every entry, and dL/dY."""
    n = Y.size
    d = Y - T
    return float(np.sum(d * d) / n), 2.0 * d / n


def backward(Ws, bs, cache, dY, mode="f64"):
    """Gradients (dW, db) for every layer; the BF16 mode differentiates the
    rounded forward with the rounding treated as identity (the weights' and
    inputs' gradients flow through unchanged)."""
    L = len(Ws)
    dWs, dbs = [None] * L, [None] * L
    g = dY
    for l in reversed(range(L)):
        xin, z = cache[l]
        dz = g * gelu_grad(z) if l < L - 1 else g
        dWs[l] = dz.T @ xin
        dbs[l] = dz.sum(axis=0)
        Wq = bf16_round(Ws[l]) if mode == "bf16" else Ws[l]
        g = dz @ Wq
    return dWs, dbs


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [np.zeros_like(p) for p in params]
        self.v = [np.zeros_like(p) for p in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for p, g, m, v in zip(params, grads, self.m, self.v):
            m *= self.b1
            m += (1.0 - self.b1) * g
            v *= self.b2
            v += (1.0 - self.b2) * g * g
            p -= self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps)
        return params
