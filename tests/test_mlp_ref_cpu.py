"""Pins of the FP64 numpy network reference: its analytic gradient against
central finite differences, and its forward pass against a direct
per-row evaluation of the definition."""
import numpy as np

from oracle import mlp_ref as R


def _data(n=40, seed=3):
    rng = np.random.default_rng(seed)
    k = rng.uniform(0.01, 0.3, n)
    z = rng.uniform(0, 1, n) * (1 - k)
    zk = np.stack([z, k], 1)
    # functions of the size the network sees: targets of order one
    k2 = k * k
    alpha = np.stack([k2, k2 * (np.sqrt(1 - z * z) + k2 * rng.normal(0, 1, n)),
                      0.5 * k2 * (k2 + 2 * z * z)], 1) * (1 + 0.01 * rng.normal(0, 1, (n, 3)))
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
        h = np.array([2 * np.sqrt(1 - z / (1 - k)) - 1, (k - 0.155) / 0.145])
        for l in (1, 2, 3):
            pre = np.array([sum(w[f"W{l}"][o, j] * h[j] for j in range(len(h))) + w[f"b{l}"][o]
                            for o in range(128)])
            h = pre / (1 + np.exp(-pre))
        out = w["W4"] @ h + w["b4"]
        assert np.allclose(out, y[i], rtol=1e-13, atol=1e-13)


def test_targets_and_weights_written_out():
    """The loss of a network that outputs zero is the weighted mean square of
    the targets, each written out here from its definition for one row."""
    w = R.init_weights(4)
    for n in R.NAMES:
        w[n] = np.zeros_like(w[n])
    z, k = 0.37, 0.21
    a = np.array([[k * k, 0.8 * k * k, 0.5 * k * k * (k * k + 2 * z * z)]])
    t = [1.0, (0.8 - np.sqrt(1 - z * z)) / (k * k), 0.5 * (k * k + 2 * z * z)]
    wk = (k / 0.3) ** 8 + 1e-5
    expect = (0.1 * wk * t[0] ** 2 + wk * t[1] ** 2 + 0.1 * wk * t[2] ** 2) / 3
    assert abs(R.loss(w, np.array([[z, k]]), a) - expect) <= 1e-15
