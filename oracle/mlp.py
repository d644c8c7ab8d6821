"""FP64 reference of the surrogate MLP (202 -> 64 -> 64 -> 6, GELU).

TEST INFRASTRUCTURE ONLY: the GPU library trains and runs the network with
its own BF16 MFMA kernels; this module recomputes the same quantities in
float64 with NumPy so that the tests can check the GPU forward pass,
gradients and Adam steps.  It is not part of the paper's method (the
surrogate is an extension beside it).

Conventions shared with the GPU side (and nothing else):
  parameters W1 [202, 64], b1 [64], W2 [64, 64], b2 [64], W3 [64, 6], b3 [6];
  y = W3^T gelu(W2^T gelu(W1^T x + b1) + b2) + b3 per row;
  gelu(x) = 0.5 x (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3)));
  loss = mean over rows and outputs of (y - t)^2;
  Adam: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
        p -= lr * (m / (1-b1^k)) / (sqrt(v / (1-b2^k)) + eps).
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 202, 64, 6
NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")
SHAPES = {"W1": (N_IN, N_HID), "b1": (N_HID,), "W2": (N_HID, N_HID), "b2": (N_HID,),
          "W3": (N_HID, N_OUT), "b3": (N_OUT,)}
_C = np.sqrt(2.0 / np.pi)


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(_C * (x + 0.044715 * x ** 3)))


def gelu_grad(x):
    u = _C * (x + 0.044715 * x ** 3)
    th = np.tanh(u)
    return 0.5 * (1.0 + th) + 0.5 * x * (1.0 - th ** 2) * _C * (1.0 + 3 * 0.044715 * x ** 2)


def _same(a):
    return a


def round_bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    Goes through float32 first, as a float32 value is what a kernel rounds."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(a))


def forward(p, X, q=_same):
    """q rounds the activations that feed the next product (identity by
    default; round_bf16 mimics a kernel that stores them in BF16)."""
    X = np.asarray(X, np.float64)
    Z1 = X @ p["W1"] + p["b1"]
    H1 = q(gelu(Z1))
    Z2 = H1 @ p["W2"] + p["b2"]
    H2 = q(gelu(Z2))
    Y = H2 @ p["W3"] + p["b3"]
    return Y, (X, Z1, H1, Z2, H2)


def loss_and_grads(p, X, T, q=_same):
    """Mean-square loss and its gradients.  With q = round_bf16 the operands
    of every product are rounded where a BF16 kernel rounds them (the
    activations, the output gradient and the pre-activation gradients);
    bias gradients sum the unrounded values."""
    Y, (X, Z1, H1, Z2, H2) = forward(p, X, q)
    T = np.asarray(T, np.float64)
    n = Y.size
    loss = float(np.sum((Y - T) ** 2) / n)
    dY = 2.0 * (Y - T) / n
    g = {"W3": H2.T @ q(dY), "b3": dY.sum(0)}
    dZ2 = (q(dY) @ p["W3"].T) * gelu_grad(Z2)
    g["W2"] = H1.T @ q(dZ2)
    g["b2"] = dZ2.sum(0)
    dZ1 = (q(dZ2) @ p["W2"].T) * gelu_grad(Z1)
    g["W1"] = X.T @ q(dZ1)
    g["b1"] = dZ1.sum(0)
    return loss, g


def adam_step(p, g, m, v, k, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (k = 1 for the first); returns new (p, m, v)."""
    out_p, out_m, out_v = {}, {}, {}
    for n in NAMES:
        out_m[n] = beta1 * m[n] + (1 - beta1) * g[n]
        out_v[n] = beta2 * v[n] + (1 - beta2) * g[n] ** 2
        mh = out_m[n] / (1 - beta1 ** k)
        vh = out_v[n] / (1 - beta2 ** k)
        out_p[n] = p[n] - lr * mh / (np.sqrt(vh) + eps)
    return out_p, out_m, out_v
