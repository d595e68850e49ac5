"""Helpers to check large batches against the oracle on sampled outputs."""
import numpy as np


def single_exposure_subset(batch, pairs):
    """A batch whose light curve j is light curve pairs[j][0] of ``batch``
    restricted to its exposure pairs[j][1] (all of its bands).  Returns the
    batch and, for each output of it, the index of the same output in the
    full batch's flux array."""
    lcs = np.array([p[0] for p in pairs], np.int64)
    idx = np.array([p[1] for p in pairs], np.int64)
    out = {key: np.ascontiguousarray(batch[key][lcs]) for key in
           ("t0", "P", "aR", "b", "e", "w", "t_exp", "nss")}
    t = batch["t"][batch["t_start"][lcs] + idx]
    nb = (batch["band_off"][lcs + 1] - batch["band_off"][lcs]).astype(np.int64)
    band_off = np.zeros(len(lcs) + 1, np.int32)
    band_off[1:] = np.cumsum(nb)
    ks = np.concatenate([batch["k"][batch["band_off"][l]:batch["band_off"][l + 1]] for l in lcs])
    us = np.concatenate([batch["u"][batch["band_off"][l]:batch["band_off"][l + 1]] for l in lcs])
    flux_off = np.zeros(len(lcs), np.int64)
    flux_off[1:] = np.cumsum(nb)[:-1]
    out.update(t=np.ascontiguousarray(t), t_start=np.arange(len(lcs), dtype=np.int64),
               t_count=np.ones(len(lcs), np.int64), band_off=band_off, k=ks, u=us,
               flux_off=flux_off, n_flux=int(nb.sum()), name="sample")
    full_idx = np.concatenate([batch["flux_off"][l] + np.arange(n) * batch["t_count"][l] + i
                               for l, i, n in zip(lcs, idx, nb)])
    return out, full_idx


def random_pairs(batch, n, seed=0, in_transit_bias=None):
    """n random (light curve, exposure) pairs, light curves weighted by their
    number of exposures x bands."""
    rng = np.random.default_rng(seed)
    nb = np.diff(batch["band_off"]).astype(np.int64)
    w = (batch["t_count"] * (nb > 0)).astype(np.float64)
    lcs = rng.choice(len(w), size=n, p=w / w.sum())
    idx = (rng.random(n) * batch["t_count"][lcs]).astype(np.int64)
    return list(zip(lcs, idx))
