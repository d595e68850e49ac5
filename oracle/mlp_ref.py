"""Plain FP64 numpy reference of the surrogate network and its training loss.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/): used to check the HIP
forward, loss and backward kernels.  Written from the definitions: a
2-128-128-128-3 multilayer perceptron with SiLU activations,
silu(x) = x / (1 + exp(-x)), over the inside of the stellar disc, inputs
x = (2 sqrt(1 - z/(1-k)) - 1, (k - 0.155)/0.145), outputs compared with
  t0 = lambda_e/k^2, t1 = (alpha_1/k^2 - sqrt(1 - z^2))/k^2, t2 = eta_d/k^2,
alpha_1 = lambda_d + 2/3 Theta(k - z) (the three limb-darkening-factored
Mandel & Agol functions, Sect. 2.2.1), and the weighted squared error, mean
over rows and outputs of w(k) c_j (y_j - t_j)^2 with w(k) = (k/0.3)^8 + 1e-5
and c = (0.1, 1, 0.1).  Weights are row-major [out][in] as in the C ABI.
"""
from __future__ import annotations

import numpy as np

NAMES = ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4")
SHAPES = {"W1": (128, 2), "b1": (128,), "W2": (128, 128), "b2": (128,), "W3": (128, 128),
          "b3": (128,), "W4": (3, 128), "b4": (3,)}


def init_weights(seed=0):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) for every weight and bias."""
    rng = np.random.default_rng(seed)
    out = {}
    for n in NAMES:
        fan_in = SHAPES["W" + n[1]][1]
        out[n] = rng.uniform(-1, 1, SHAPES[n]) / np.sqrt(fan_in)
    return out


def features(zk):
    z, k = zk[:, 0], zk[:, 1]
    return np.stack([2 * np.sqrt(np.maximum(0.0, 1 - z / (1 - k))) - 1, (k - 0.155) / 0.145], 1)


def targets(zk, alpha):
    """The three training targets of rows (z, k) with functions alpha."""
    z, k = zk[:, 0], zk[:, 1]
    k2 = k * k
    return np.stack([alpha[:, 0] / k2, (alpha[:, 1] / k2 - np.sqrt(np.maximum(0.0, 1 - z * z))) / k2,
                     alpha[:, 2] / k2], 1)


def row_weights(zk):
    k = zk[:, 1]
    return ((k / 0.3) ** 8 + 1e-5)[:, None] * np.array([0.1, 1.0, 0.1])[None, :]


def silu(x):
    return x / (1 + np.exp(-x))


def forward(w, zk):
    """Returns y [n][3] and the pre-activations of the three hidden layers."""
    h = features(zk)
    pres = []
    for l in (1, 2, 3):
        p = h @ w[f"W{l}"].T + w[f"b{l}"]
        pres.append(p)
        h = silu(p)
    return h @ w["W4"].T + w["b4"], pres


def loss(w, zk, alpha):
    y, _ = forward(w, zk)
    return float(np.mean(row_weights(zk) * (y - targets(zk, alpha)) ** 2))


def grad(w, zk, alpha):
    """Analytic gradient of loss() by the chain rule, layer by layer."""
    y, pres = forward(w, zk)
    n = len(zk)
    dy = 2 * row_weights(zk) * (y - targets(zk, alpha)) / (3 * n)
    g = {}
    hs = [features(zk)] + [silu(p) for p in pres]
    g["W4"] = dy.T @ hs[3]
    g["b4"] = dy.sum(0)
    d = dy @ w["W4"]
    for l in (3, 2, 1):
        p = pres[l - 1]
        s = 1 / (1 + np.exp(-p))
        d = d * (s * (1 + p * (1 - s)))
        g[f"W{l}"] = d.T @ hs[l - 1]
        g[f"b{l}"] = d.sum(0)
        d = d @ w[f"W{l}"]
    return g
