"""FP64 reference for the learned seeder (test infrastructure only).

An MLP maps an EE target (position scaled by the arm's reach, unit
quaternion with w >= 0: 7 inputs) to K joint-space seeds (7*K outputs):
hidden layers Linear + SiLU, linear output.  It is trained on (FK(q), q)
pairs with a min-over-seeds loss
    L = mean_b min_k || qhat_{b,k} - q_b ||^2   (argmin ties -> lowest k)
and Adam (Kingma & Ba 2015: beta1 0.9, beta2 0.999, eps 1e-8, bias
correction, no weight decay).

Two modes:
  * exact FP64 (finite-difference gradient checks);
  * BF16 emulation: the weights and each layer's input activations are
    rounded to bfloat16 (round to nearest even) exactly where the GPU
    kernels round them, products accumulated in FP64.
Only tests and the benchmark's CPU leg use this module.
"""
from __future__ import annotations

import numpy as np


def bf16(x):
    """Round float64/float32 values to bfloat16 (RNE), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounding = ((u >> 16) & 1) + 0x7FFF
    r = ((u + rounding) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if nan.any():
        out = np.where(nan, np.nan, out)
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, x, emulate_bf16=False):
    """params: list of (W [out,in], b [out]).  Returns (y, cache)."""
    h = np.asarray(x, dtype=np.float64)
    cache = []
    L = len(params)
    for i, (W, b) in enumerate(params):
        hin = bf16(h) if emulate_bf16 else h
        Wq = bf16(W) if emulate_bf16 else W
        z = hin @ Wq.T + b
        cache.append((hin, Wq, z))
        h = silu(z) if i < L - 1 else z
    return h, cache


def min_over_k_loss(y, q, K):
    """y [B, 7K], q [B, 7] -> (loss, argmin k [B], dL/dy [B, 7K])."""
    B, n = q.shape
    yh = y.reshape(B, K, n)
    d = ((yh - q[:, None, :]) ** 2).sum(-1)
    k = np.argmin(d, axis=1)             # first minimum on ties
    loss = d[np.arange(B), k].mean()
    g = np.zeros_like(yh)
    g[np.arange(B), k] = 2.0 * (yh[np.arange(B), k] - q) / B
    return loss, k, g.reshape(B, K * n)


def backward(params, cache, dy, emulate_bf16=False):
    """Gradients [(dW, db)] of the loss given dL/dy.

    With emulate_bf16 the upstream gradient of each hidden layer is rounded
    to bfloat16 before it multiplies the weights and the stored inputs
    (the GPU keeps it in BF16 for its matrix-core products)."""
    grads = [None] * len(params)
    g = np.asarray(dy, dtype=np.float64)
    for i in range(len(params) - 1, -1, -1):
        hin, Wq, z = cache[i]
        if i < len(params) - 1:
            g = g * silu_grad(z)
        gq = bf16(g) if emulate_bf16 else g
        grads[i] = (gq.T @ hin, g.sum(0))
        if i > 0:
            g = gq @ Wq
    return grads


class Adam:
    """Adam (Kingma & Ba 2015, Algorithm 1): per parameter array
        m_t = b1 m_{t-1} + (1 - b1) g_t,   v_t = b2 v_{t-1} + (1 - b2) g_t^2,
        theta_t = theta_{t-1} - lr (m_t / (1 - b1^t)) / (sqrt(v_t / (1 - b2^t)) + eps).
    The moments ``m[layer][0|1]`` / ``v[layer][0|1]`` (weights, bias) start at
    zero; ``t`` counts the steps taken."""

    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [[np.zeros(np.shape(W)), np.zeros(np.shape(b))] for W, b in params]
        self.v = [[np.zeros(np.shape(W)), np.zeros(np.shape(b))] for W, b in params]
        self.t = 0

    def step(self, params, grads):
        """New parameters [(W, b)] after one step with gradients [(dW, db)]."""
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        out = []
        for i, (layer, glayer) in enumerate(zip(params, grads)):
            new = []
            for j in range(2):
                g = np.asarray(glayer[j], dtype=np.float64)
                self.m[i][j] = self.b1 * self.m[i][j] + (1 - self.b1) * g
                self.v[i][j] = self.b2 * self.v[i][j] + (1 - self.b2) * g * g
                mhat = self.m[i][j] / c1
                vhat = self.v[i][j] / c2
                new.append(layer[j] - self.lr * mhat / (np.sqrt(vhat) + self.eps))
            out.append(tuple(new))
        return out


def encode_targets(p, quat, reach):
    """Network input: [p / reach, quaternion with w >= 0] -> [B, 7]."""
    p = np.asarray(p, dtype=np.float64)
    qt = np.asarray(quat, dtype=np.float64).copy()
    qt /= np.linalg.norm(qt, axis=1, keepdims=True)
    qt[qt[:, 0] < 0] *= -1.0
    return np.concatenate([p / reach, qt], axis=1)
