"""Pins of the FP64 numpy network reference: its analytic gradient against
central finite differences, and its forward pass against a direct
per-row evaluation of the definition."""
import numpy as np

from oracle import mlp_ref as R


def _data(n=40, seed=3):
    rng = np.random.default_rng(seed)
    zk = np.stack([rng.uniform(0, 1.2, n), rng.uniform(0.01, 0.3, n)], 1)
    alpha = rng.uniform(0, 0.05, (n, 3))
    return zk, alpha


def test_gradient_matches_finite_differences():
    w = R.init_weights(1)
    zk, alpha = _data()
    g = R.grad(w, zk, alpha)
    rng = np.random.default_rng(7)
    for name in R.NAMES:
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in w[name].shape)
            h = 1e-6
            wp = {k: v.copy() for k, v in w.items()}
            wm = {k: v.copy() for k, v in w.items()}
            wp[name][idx] += h
            wm[name][idx] -= h
            fd = (R.loss(wp, zk, alpha) - R.loss(wm, zk, alpha)) / (2 * h)
            assert abs(fd - g[name][idx]) <= 1e-7 * max(1.0, abs(fd)) + 1e-10, (name, idx)


def test_forward_matches_rowwise_definition():
    w = R.init_weights(2)
    zk, _ = _data(5)
    y, _ = R.forward(w, zk)
    for i, (z, k) in enumerate(zk):
        h = np.array([2 * z / (1 + k) - 1, (k - 0.155) / 0.145])
        for l in (1, 2, 3):
            pre = np.array([sum(w[f"W{l}"][o, j] * h[j] for j in range(len(h))) + w[f"b{l}"][o]
                            for o in range(128)])
            h = pre / (1 + np.exp(-pre))
        out = w["W4"] @ h + w["b4"]
        assert np.allclose(out, y[i], rtol=1e-13, atol=1e-13)
