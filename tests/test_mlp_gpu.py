"""Surrogate network on the GPU: exact targets, float forward/backward against
the FP64 numpy reference, the bf16-MFMA inference against the float forward
(which checks the MFMA operand layout), training, and the trust map's
guarantee that surrogate results stay within tolerance."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pt():
    import torch
    assert torch.cuda.is_available()
    from paper_1504_07433_amd import pthip
    return pthip


def say(*a):
    print(*a, flush=True)


def _params(pt, seed=0):
    import torch
    from oracle import mlp_ref as R
    w = R.init_weights(seed)
    return w, {n: torch.as_tensor(w[n], dtype=torch.float32, device="cuda").contiguous() for n in R.NAMES}


CKPT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1504_07433_amd", "data",
                    "surrogate.npz")


def _zk(n, seed=1):
    """(z, k) anywhere along a transit: z in [0, 1.35]."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(0, 1.35, n), rng.uniform(0.01, 0.3, n)], 1)


def _zk_disc(n, seed=1):
    """(z, k) inside the stellar disc, the network's domain."""
    rng = np.random.default_rng(seed)
    k = rng.uniform(0.01, 0.3, n)
    return np.stack([rng.uniform(0, 1, n) * (1 - k), k], 1)


def _alpha_like(zk, seed=0):
    """Functions of the size the network sees (targets of order one)."""
    rng = np.random.default_rng(seed)
    z, k = zk[:, 0], zk[:, 1]
    k2 = k * k
    return np.stack([k2, k2 * (np.sqrt(1 - z * z) + k2 * rng.normal(0, 1, len(z))),
                     0.5 * k2 * (k2 + 2 * z * z)], 1) * (1 + 0.01 * rng.normal(0, 1, (len(z), 3)))


def test_datagen_matches_oracle(pt):
    from oracle import oracle as O
    zk = _zk(3000)
    zk[:10, 0] = zk[:10, 1]                  # z = k exactly
    zk[10:20, 0] = 1 - zk[10:20, 1]          # z = 1 - k
    got = pt.mlp_datagen(zk).cpu().numpy()
    ref = O.surrogate_targets(zk)
    assert np.abs(got - ref).max() <= 1e-10


def test_forward_and_backward_match_reference(pt):
    import torch
    from oracle import mlp_ref as R
    w, P = _params(pt, 3)
    zk = _zk_disc(5000, 2).astype(np.float32).astype(np.float64)
    alpha = _alpha_like(zk)
    zk32 = torch.as_tensor(zk, dtype=torch.float32, device="cuda").contiguous()
    act = torch.empty((5000, 3, 128), dtype=torch.float32, device="cuda")
    y = pt.mlp_forward(P, zk32, act).cpu().numpy()
    zk_f = zk.astype(np.float32).astype(np.float64)
    yref, _ = R.forward(w, zk_f)
    assert np.abs(y - yref).max() <= 2e-5 * max(1.0, np.abs(yref).max())
    dout = torch.empty((5000, 3), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    a_dev = torch.as_tensor(alpha, device="cuda")
    pt.mlp_loss_grad(pt.mlp_forward(P, zk32, act), zk32, a_dev, dout, loss)
    assert loss.item() == pytest.approx(R.loss(w, zk_f, alpha), rel=1e-4)
    grads = {n: torch.zeros_like(t) for n, t in P.items()}
    pt.mlp_backward(P, zk32, act, dout, grads)
    gref = R.grad(w, zk_f, alpha)
    for n in R.NAMES:
        g = grads[n].cpu().numpy()
        scale = np.abs(gref[n]).max()
        assert np.abs(g - gref[n]).max() <= 1e-3 * scale + 1e-9, n


def test_adam_step_matches_definition(pt):
    import torch
    w, P = _params(pt, 4)
    grads = {n: torch.full_like(t, 0.5) for n, t in P.items()}
    m = {n: torch.zeros_like(t) for n, t in P.items()}
    v = {n: torch.zeros_like(t) for n, t in P.items()}
    before = {n: t.clone() for n, t in P.items()}
    pt.mlp_adam_step(P, grads, m, v, 1, 1e-2)
    for n in P:   # first step: w -= lr * g/|g| (bias-corrected moments)
        d = (before[n] - P[n]).cpu().numpy()
        assert np.allclose(d, 1e-2, rtol=1e-4)


@pytest.mark.parametrize("split,tol", [("1", 2e-4), ("0", 1e-2)])
def test_mfma_inference_matches_float_forward(pt, monkeypatch, split, tol):
    """The register-resident MFMA inference against the float training
    forward on random weights: with the hi/lo split (~16-bit operands) and
    with plain bf16 operands (8-bit mantissas, float accumulation).  Any
    mistake in the operand layout or the column order of the packed weights
    breaks the agreement by far more than either tolerance."""
    import torch
    monkeypatch.setenv("PT_MLP_SPLIT", split)
    w, P = _params(pt, 5)
    pt.surrogate_set(P)
    zk32 = torch.as_tensor(_zk_disc(4096, 6), dtype=torch.float32, device="cuda").contiguous()
    y_inf = pt.mlp_infer(zk32).cpu().numpy()
    y_fwd = pt.mlp_forward(P, zk32).cpu().numpy()
    err = np.abs(y_inf - y_fwd).max() / np.abs(y_fwd).max()
    say("mfma vs float forward, relative, split", split, err)
    assert err <= tol


def test_training_reduces_loss_and_error_map_holds(pt):
    """A short training run on the library's kernels lowers the loss; with the
    resulting network installed, the surrogate's three functions (network
    inside the disc where its error map allows, exact elsewhere) bound the
    flux error of every quadratic law with uniform-(q1, q2) coefficients by
    1e-5 at any (z, k) of a transit."""
    from oracle import oracle as O
    from paper_1504_07433_amd.surrogate import Surrogate
    s = Surrogate(seed=5)
    zk32, alpha = s.make_data(400_000, seed=5)
    hist = s.train(zk32, alpha, steps=600, batch=16384, log_every=100)
    say("loss history", hist)
    assert hist[-1][1] < 0.05 * hist[0][1]
    frac = s.install()
    say("trusted fraction", frac)
    assert 0.0 <= frac <= 1.0
    zk = np.concatenate([_zk(20000, 9), _zk_disc(20000, 10)])
    got = pt.surrogate_eval(zk).cpu().numpy()
    ref = O.surrogate_targets(zk.astype(np.float32).astype(np.float64))
    bound = 2 * np.abs(got[:, 0] - ref[:, 0]) + 4 * np.abs(got[:, 1] - ref[:, 1]) + 2 * np.abs(got[:, 2] - ref[:, 2])
    say("surrogate bound max", bound.max())
    assert bound.max() <= 1e-5


def _installed(pt):
    from paper_1504_07433_amd.surrogate import Surrogate
    s = Surrogate()
    s.load(CKPT)
    return s.install()


def test_committed_network_covers_the_disc(pt):
    """The committed network, installed: most error-map cells accept it for
    any quadratic law, and where they do its functions are within the flux
    tolerance of the exact ones (checked here on fresh points)."""
    from oracle import oracle as O
    frac = _installed(pt)
    say("committed network: cells accepted for any law", frac)
    assert frac >= 0.8
    zk = _zk_disc(50000, 11)
    got = pt.surrogate_eval(zk).cpu().numpy()
    ref = O.surrogate_targets(zk.astype(np.float32).astype(np.float64))
    assert 4 * np.abs(got[:, 1] - ref[:, 1]).max() <= 1e-5
    assert np.abs(got[:, [0, 2]] - ref[:, [0, 2]]).max() <= 1e-8


def test_batch_surrogate_parity_and_network_share(pt):
    """The committed network in the batch path on spectrophotometric light
    curves (the metric's workload, 64 bands, 1500 exposures) and on
    long-cadence ones (10 subsamples per exposure): every output within 1e-5
    of the oracle, and the network (counted on the device) takes at least
    half of the in-transit (point, band) pairs of the spectrophotometric
    batch."""
    from oracle import oracle as O
    from paper_1504_07433_amd import workloads as W
    _installed(pt)
    b = W.config3(n_vec=4, n_band=64, n_exp=1500)
    ref = O.lc_batch(b, model=0)
    db = pt.DeviceBatch(b)
    pt.surrogate_counters(reset=True)
    got = pt.lc_batch(db, "ma", prec="surrogate").cpu().numpy().astype(np.float64)
    net, exact = pt.surrogate_counters(reset=True)
    err = np.abs(got - ref).max()
    say("batch surrogate max|dF|", err, "network points", net, "exact in-transit points", exact)
    assert err <= 1e-5
    n_in = np.count_nonzero(ref < 1.0)
    assert abs(net + exact - n_in) <= 1e-3 * n_in
    assert net >= 0.5 * (net + exact)
    b2 = W.config2(n_vec=4, n_windows=2)
    got2 = pt.lc_batch(pt.DeviceBatch(b2), "ma", prec="surrogate").cpu().numpy().astype(np.float64)
    net2, exact2 = pt.surrogate_counters(reset=True)
    say("long-cadence: network points", net2, "exact", exact2)
    assert np.abs(got2 - O.lc_batch(b2, model=0)).max() <= 1e-5
    assert net2 > 0


def test_batch_surrogate_ragged_edge_cases(pt):
    """The two-pass surrogate path on a ragged batch: light curves with more
    subsamples than one LDS chunk (the per-band orbit branch, several listed
    subsamples per flux element), k above the network's range and above 1/2,
    a planet larger than the star, an empty light curve and one without
    bands, against the oracle; and NaN throughout for an invalid band and an
    invalid orbit."""
    from oracle import oracle as O
    from paper_1504_07433_amd import workloads as W
    _installed(pt)
    b = W.config4(n_lc=10, n_min=20, n_max=300, max_nss=3, max_bands=3)
    b["nss"][1] = 20
    b["nss"][2] = 37
    for i in range(len(b["t_start"])):          # times across the transit at t0 = 0
        s0, c = b["t_start"][i], b["t_count"][i]
        b["t"][s0:s0 + c] = np.linspace(-0.07, 0.07, c)
    b["k"][b["band_off"][3]] = 0.7
    b["k"][b["band_off"][4]] = 1.4
    b["t_count"][5] = 0
    b["band_off"][7:] -= (b["band_off"][7] - b["band_off"][6])
    b["band_off"][6] = b["band_off"][7]
    nb = np.diff(b["band_off"]).astype(np.int64)
    sizes = nb * b["t_count"]
    b["flux_off"] = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    b["n_flux"] = int(sizes.sum())
    b["k"] = b["k"][:b["band_off"][-1]].copy()
    b["u"] = b["u"][:b["band_off"][-1]].copy()
    ref = O.lc_batch(b, model=0)
    assert np.count_nonzero(ref < 1.0) > len(ref) // 4       # the transits are sampled
    pt.surrogate_counters(reset=True)
    got = pt.lc_batch(pt.DeviceBatch(b), "ma", prec="surrogate").cpu().numpy().astype(np.float64)
    net, exact = pt.surrogate_counters(reset=True)
    say("ragged surrogate: max|dF|", np.abs(got - ref).max(), "network", net, "exact", exact)
    assert np.abs(got - ref).max() <= 1e-5
    assert net > 0
    # an invalid band (k = NaN) and an invalid orbit (e = 1.5): NaN in every exposure
    b["k"][b["band_off"][0]] = np.nan
    b["e"][2] = 1.5
    got = pt.lc_batch(pt.DeviceBatch(b), "ma", prec="surrogate").cpu().numpy()
    blk0 = got[b["flux_off"][0]:b["flux_off"][0] + b["t_count"][0]]
    blk2 = got[b["flux_off"][2]:b["flux_off"][2] + nb[2] * b["t_count"][2]]
    assert np.all(np.isnan(blk0)) and np.all(np.isnan(blk2))
