"""Seeded synthetic inputs for the transit-model hot path.

This module only draws random numbers and lays them out; it holds none of the
model's arithmetic (no orbit, no flux), so that the HIP path and the FP64 CPU
oracle can both be fed from it without sharing any of the method.

Every workload is a plain dict of numpy arrays in the batch layout used by the
C ABI (structure of arrays, one entry per light curve or per passband):

  t          float64 [n_t]          exposure mid-times (days), a pool
  t_start    int64   [n_lc]         first time of light curve i in ``t``
  t_count    int64   [n_lc]         number of exposures of light curve i
  t0, P, aR, b, e, w, t_exp
             float64 [n_lc]         conjunction time, period, a/R*, impact
                                    parameter, eccentricity, argument of
                                    periastron (rad), exposure time (days)
  nss        int32   [n_lc]         subsamples per exposure (>= 1)
  band_off   int32   [n_lc+1]       passbands of light curve i are
                                    band_off[i] .. band_off[i+1]-1
  k          float64 [n_band]       radius ratio per passband
  u          float64 [n_band, 2]    quadratic limb darkening (u1, u2)
  flux_off   int64   [n_lc]         output block of light curve i starts here;
                                    the block is [n_band_i][t_count_i]

The shapes follow the paper's workloads: Kepler long-cadence data with
supersampling (Sect. 1 footnote and Sect. 3.2), spectrophotometric multi-band
light curves (Sect. 1), and about a third of the points in transit (Sect. 4).
No public data set is used; everything is drawn from a seeded generator.
"""
from __future__ import annotations

import numpy as np

P_DAYS = 3.0                    # orbital period used by the batch workloads
LONG_CADENCE_EXPOSURE = 29.4 / (24 * 60)   # Kepler long cadence, days
WINDOW_HALF = 0.08              # days around each transit centre
WINDOW_POINTS = 2000


def kipping_q_to_u(q1: np.ndarray, q2: np.ndarray):
    """Quadratic coefficients from the uniform (q1, q2) sampling of
    Kipping (2013, MNRAS 435, 2152): u1 = 2 sqrt(q1) q2, u2 = sqrt(q1)(1-2 q2).
    This is an input prior, not part of the transit model."""
    sq = np.sqrt(q1)
    return 2.0 * sq * q2, sq * (1.0 - 2.0 * q2)


def _empty_batch(n_lc):
    return dict(
        t0=np.zeros(n_lc), P=np.zeros(n_lc), aR=np.zeros(n_lc), b=np.zeros(n_lc),
        e=np.zeros(n_lc), w=np.zeros(n_lc), t_exp=np.zeros(n_lc),
        nss=np.ones(n_lc, np.int32))


def _finish(batch, t, t_start, t_count, nb_per_lc, k, u, name):
    n_lc = len(t_start)
    band_off = np.zeros(n_lc + 1, np.int32)
    band_off[1:] = np.cumsum(nb_per_lc)
    sizes = np.asarray(nb_per_lc, np.int64) * np.asarray(t_count, np.int64)
    flux_off = np.zeros(n_lc, np.int64)
    flux_off[1:] = np.cumsum(sizes)[:-1]
    batch.update(
        name=name, t=np.ascontiguousarray(t, np.float64),
        t_start=np.asarray(t_start, np.int64), t_count=np.asarray(t_count, np.int64),
        band_off=band_off, k=np.ascontiguousarray(k, np.float64),
        u=np.ascontiguousarray(np.asarray(u, np.float64).reshape(-1, 2)),
        flux_off=flux_off, n_flux=int(sizes.sum()))
    for key in ("t0", "P", "aR", "b", "e", "w", "t_exp"):
        batch[key] = np.ascontiguousarray(batch[key], np.float64)
    batch["nss"] = np.ascontiguousarray(batch["nss"], np.int32)
    return batch


def n_points(batch) -> int:
    """Model points = sum over light curves of bands x exposures x subsamples."""
    nb = np.diff(batch["band_off"]).astype(np.int64)
    return int((nb * batch["t_count"] * batch["nss"].astype(np.int64)).sum())


def windows_times(n_windows: int, period: float = P_DAYS) -> np.ndarray:
    """Exposure times in windows of +-0.08 d around n*P, 2000 evenly spaced
    points per window."""
    base = np.linspace(-WINDOW_HALF, WINDOW_HALF, WINDOW_POINTS)
    return (np.arange(n_windows)[:, None] * period + base[None, :]).ravel()


def config1(seed: int = 1):
    """A single light curve: circular orbit, P=3 d, t0=0, a/R*=10, b=0.3,
    k=0.1, u=(0.4, 0.2), 1000 evenly spaced times in [-0.2, 0.2] d, one band,
    no supersampling; each parameter jittered by U(-1e-4, 1e-4)."""
    rng = np.random.default_rng(seed)
    j = lambda: rng.uniform(-1e-4, 1e-4)
    b = _empty_batch(1)
    b["t0"][0] = 0.0 + j(); b["P"][0] = 3.0 + j(); b["aR"][0] = 10.0 + j()
    b["b"][0] = 0.3 + j()
    k = np.array([0.1 + j()])
    u = np.array([[0.4 + j(), 0.2 + j()]])
    t = np.linspace(-0.2, 0.2, 1000)
    return _finish(b, t, [0], [1000], [1], k, u, "single-lc-1000")


def _random_orbits(rng, n):
    """Eccentric orbits of the long-cadence batch: k~U(.05,.2), b~U(0,.9),
    a/R*~U(5,30), e~U(0,.3), w~U(0,2pi), (u1,u2) from uniform (q1,q2)."""
    k = rng.uniform(0.05, 0.2, n)
    bb = rng.uniform(0.0, 0.9, n)
    aR = rng.uniform(5.0, 30.0, n)
    e = rng.uniform(0.0, 0.3, n)
    w = rng.uniform(0.0, 2 * np.pi, n)
    q1 = rng.uniform(0, 1, n); q2 = rng.uniform(0, 1, n)
    u1, u2 = kipping_q_to_u(q1, q2)
    return k, bb, aR, e, w, u1, u2


def config2(seed: int = 2, n_vec: int = 256, n_windows: int = 100,
            nss: int = 10):
    """Long-cadence batch: 256 eccentric parameter vectors sharing 200k
    exposure times (100 transit windows x 2000 points), 29.4 min exposures
    supersampled x10, one band each."""
    rng = np.random.default_rng(seed)
    k, bb, aR, e, w, u1, u2 = _random_orbits(rng, n_vec)
    b = _empty_batch(n_vec)
    b["t0"][:] = 0.0; b["P"][:] = P_DAYS; b["aR"][:] = aR; b["b"][:] = bb
    b["e"][:] = e; b["w"][:] = w; b["t_exp"][:] = LONG_CADENCE_EXPOSURE
    b["nss"][:] = nss
    t = windows_times(n_windows)
    n_t = len(t)
    return _finish(b, t, np.zeros(n_vec, np.int64), np.full(n_vec, n_t),
                   np.ones(n_vec, np.int64), k, np.stack([u1, u2], 1),
                   f"long-cadence-{n_vec}x{n_t}x{nss}")


def config3(seed: int = 3, n_vec: int = 1024, n_band: int = 64,
            n_exp: int = 1500):
    """Spectrophotometric batch: 1024 circular-orbit vectors x 64 passbands
    (per band k~U(.09,.11), u1~U(.1,.6), u2~U(0,.3)), a/R*~U(9,11),
    b~U(.2,.4), t0~U(-.01,.01) d, 1500 exposures evenly over +-2 h, no
    supersampling."""
    rng = np.random.default_rng(seed)
    b = _empty_batch(n_vec)
    b["t0"][:] = rng.uniform(-0.01, 0.01, n_vec)
    b["P"][:] = P_DAYS
    b["aR"][:] = rng.uniform(9.0, 11.0, n_vec)
    b["b"][:] = rng.uniform(0.2, 0.4, n_vec)
    k = rng.uniform(0.09, 0.11, n_vec * n_band)
    u = np.stack([rng.uniform(0.1, 0.6, n_vec * n_band),
                  rng.uniform(0.0, 0.3, n_vec * n_band)], 1)
    t = np.linspace(-2.0 / 24, 2.0 / 24, n_exp)
    return _finish(b, t, np.zeros(n_vec, np.int64), np.full(n_vec, n_exp),
                   np.full(n_vec, n_band), k, u,
                   f"spectrophotometric-{n_vec}x{n_band}x{n_exp}")


def config4(seed: int = 4, n_lc: int = 4096, n_min: int = 500,
            n_max: int = 100_000, max_nss: int = 15, max_bands: int = 16):
    """Uneven batch: 4096 light curves, lengths log-uniform in [500, 1e5],
    supersampling U{1..15}, passbands U{1..16}, eccentric orbits as in the
    long-cadence batch, per-band k = k_lc * U(0.95, 1.05).  Every light curve
    has its own block of times (2000-point windows around n*P)."""
    rng = np.random.default_rng(seed)
    lens = np.exp(rng.uniform(np.log(n_min), np.log(n_max), n_lc)).astype(np.int64)
    nss = rng.integers(1, max_nss + 1, n_lc)
    nb = rng.integers(1, max_bands + 1, n_lc)
    k_lc, bb, aR, e, w, _, _ = _random_orbits(rng, n_lc)
    b = _empty_batch(n_lc)
    b["t0"][:] = 0.0; b["P"][:] = P_DAYS; b["aR"][:] = aR; b["b"][:] = bb
    b["e"][:] = e; b["w"][:] = w; b["t_exp"][:] = LONG_CADENCE_EXPOSURE
    b["nss"][:] = nss
    n_band = int(nb.sum())
    k = np.repeat(k_lc, nb) * rng.uniform(0.95, 1.05, n_band)
    q1 = rng.uniform(0, 1, n_band); q2 = rng.uniform(0, 1, n_band)
    u1, u2 = kipping_q_to_u(q1, q2)
    pattern = windows_times(int(np.ceil(n_max / WINDOW_POINTS)))
    t_start = np.zeros(n_lc, np.int64)
    t_start[1:] = np.cumsum(lens)[:-1]
    t = np.concatenate([pattern[:n] for n in lens])
    return _finish(b, t, t_start, lens, nb, k, np.stack([u1, u2], 1),
                   f"uneven-{n_lc}lc")


def config5_training(seed: int = 5, n: int = 10_000_000,
                     k_range=(0.01, 0.3), band: float = 1e-3,
                     contact_frac: float = 0.2, contact_width: float = 0.1):
    """(z, k) training pairs for the surrogate, which serves the inside of the
    stellar disc: k ~ U(.01, .3), s = z/(1 - k - band) ~ U(0, 1), plus an extra
    ``contact_frac`` of samples with s = 1 - ``contact_width`` U^2 (denser
    towards the inner contact z = 1 - k).  z is rounded to float (the network's
    input type) so that targets are exact at the inputs the network sees.
    Returns an [m, 2] float64 array of (z, k)."""
    rng = np.random.default_rng(seed)
    m = int(round(contact_frac * n))
    k = rng.uniform(*k_range, n + m)
    s = rng.uniform(0.0, 1.0, n + m)
    s[n:] = 1.0 - contact_width * rng.uniform(0.0, 1.0, m) ** 2
    z = (s * (1.0 - k - band)).astype(np.float32).astype(np.float64)
    k = k.astype(np.float32).astype(np.float64)
    zk = np.stack([np.minimum(z, np.nextafter(1.0 - k - band, 0.0)), k], 1)
    return zk[rng.permutation(n + m)]


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4}


def subset(batch, lcs):
    """A batch holding only the light curves ``lcs`` (for sampled checks).
    Times are re-packed so the result is self-contained."""
    lcs = np.asarray(lcs, np.int64)
    out = {key: batch[key][lcs] for key in
           ("t0", "P", "aR", "b", "e", "w", "t_exp", "nss")}
    ts, ks, us, nbs, counts = [], [], [], [], []
    for i in lcs:
        s, c = batch["t_start"][i], batch["t_count"][i]
        ts.append(batch["t"][s:s + c]); counts.append(c)
        b0, b1 = batch["band_off"][i], batch["band_off"][i + 1]
        ks.append(batch["k"][b0:b1]); us.append(batch["u"][b0:b1]); nbs.append(b1 - b0)
    t_start = np.zeros(len(lcs), np.int64)
    t_start[1:] = np.cumsum(counts)[:-1]
    return _finish(out, np.concatenate(ts), t_start, counts, nbs,
                   np.concatenate(ks), np.concatenate(us), batch["name"] + "-subset")
