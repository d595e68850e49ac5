"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances (max |dF| against the oracle):
  PT_PREC_FP64: 1e-8 everywhere; 1e-11 more than 1e-5 away from z = k and
                z = 1 - k (closer, both sides evaluate closed forms whose
                terms cancel: as |z-k|^-1 near z = k, and as z^-1/2 near
                z = 1 - k = 0 when k = 1; inside 1e-9 of z = k both snap).
  PT_PREC_FP32: 1e-6.
Gimenez is compared at the same number of Jacobi terms (the truncated series
is the definition being checked).
"""
import numpy as np
import pytest

from tests.sampling import random_pairs, single_exposure_subset

pytestmark = pytest.mark.gpu

TOL64, TOL64_FAR, TOL32 = 1e-8, 1e-11, 1e-6
LDS = np.array([[0.0, 0.0], [0.4, 0.2], [0.6, 0.3], [0.1, 0.55], [1.0, -0.2]])


@pytest.fixture(scope="module")
def pt():
    import torch
    assert torch.cuda.is_available()
    from paper_1504_07433_amd import pthip
    return pthip


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    return oracle


def say(*a):
    print(*a, flush=True)


def z_grid(k):
    base = np.linspace(0, 1 + k + 0.05, 3001)
    offs = np.concatenate([np.logspace(-13, -1, 49), -np.logspace(-13, -1, 49), [0.0]])
    pts = [base]
    for c in (k, 1 - k, 1 + k, 0.0):
        pts.append(c + offs)
    z = np.concatenate(pts)
    return z[z >= 0]


def oracle_flux(O, z, k, u):
    al = O.ma_alpha_many(z, k)
    out = []
    for u1, u2 in u:
        c = u1 + 2 * u2
        out.append(1 - ((1 - c) * al[:, 0] + c * al[:, 1] + u2 * al[:, 2]) / (1 - u1 / 3 - u2 / 6))
    return np.array(out)


KS = [0.005, 0.01, 0.05, 0.1, 0.2, 0.3, 0.45, 0.5, 0.6, 0.9, 1.0, 1.3]


@pytest.mark.parametrize("k", KS)
def test_ma_quad_fp64_and_fp32(pt, O, k):
    say("ma_quad k =", k)
    z = z_grid(k)
    ref = oracle_flux(O, z, k, LDS)
    g64 = pt.ma_quad(z, k, LDS, "fp64").cpu().numpy()
    d = np.abs(g64 - ref)
    far = (np.abs(z - k) > 1e-5) & (np.abs(z - (1 - k)) > 1e-5)
    assert d.max() <= TOL64, (d.max(), z[np.argmax(d.max(0))])
    assert d[:, far].max() <= TOL64_FAR, d[:, far].max()
    g32 = pt.ma_quad(z, k, LDS, "fp32").cpu().numpy()
    # the float path evaluates at z rounded to float: compare there ...
    zf = z.astype(np.float32).astype(np.float64)
    ref32 = oracle_flux(O, zf, k, LDS)
    d32 = np.abs(g32 - ref32)
    assert d32.max() <= TOL32, (d32.max(), zf[np.argmax(d32.max(0))])
    # ... and at the caller's double z, where the rounding of z to float is
    # charged to the float path too (its share: |F(z) - F(float(z))|)
    dz = np.abs(g32 - ref)
    say("ma_quad fp32 k", k, "at float z", d32.max(), "at double z", dz.max(),
        "z rounding share", np.abs(ref - ref32).max())
    assert dz.max() <= TOL32, (dz.max(), z[np.argmax(dz.max(0))])


def test_ma_quad_special_values(pt):
    z = np.array([-0.5, -1e-12, 1.1, 1.2, 5.0, np.nan])
    f = pt.ma_quad(z, 0.1, LDS, "fp64").cpu().numpy()
    assert np.all(f[:, :5] == 1.0)
    assert np.all(np.isnan(f[:, 5]))
    f32 = pt.ma_quad(z, 0.1, LDS, "fp32").cpu().numpy()
    assert np.all(f32[:, :5] == 1.0) and np.all(np.isnan(f32[:, 5]))
    # star fully covered
    assert np.abs(pt.ma_quad(np.array([0.0, 0.2]), 1.5, LDS, "fp64").cpu().numpy()).max() < 1e-15


@pytest.mark.parametrize("npol", [1, 20, 50, 200, 512])
@pytest.mark.parametrize("nldc", [1, 2, 4])
def test_gimenez(pt, O, npol, nldc):
    rng = np.random.default_rng(npol * 10 + nldc)
    for k in (0.02, 0.1, 0.3):
        say("gimenez k npol nldc", k, npol, nldc)
        z = np.concatenate([np.linspace(0, 1 + k + 0.02, 301), [k, 1 - k, 1 + k, -0.3]])
        u = rng.uniform(-0.2, 0.5, (3, nldc))
        ref = np.array([O.gimenez_flux(z, k, uu, npol) for uu in u])
        g64 = pt.gimenez(z, k, u, npol, "fp64").cpu().numpy()
        assert np.abs(g64 - ref).max() <= 1e-12
        zf = z.astype(np.float32).astype(np.float64)
        ref32 = np.array([O.gimenez_flux(zf, k, uu, npol) for uu in u])
        g32 = pt.gimenez(z, k, u, npol, "fp32").cpu().numpy()
        assert np.abs(g32 - ref32).max() <= TOL32


def test_orbit(pt, O):
    from paper_1504_07433_amd import workloads as W
    b = W.config2(n_vec=32, n_windows=3)
    t = np.concatenate([b["t"][::7], np.linspace(-4, 4, 801)])
    for i in range(32):
        prm = (b["t0"][i], b["P"][i], b["aR"][i], b["b"][i], b["e"][i], b["w"][i])
        ref = O.orbit_z(t, *prm)
        z64 = pt.orbit_z(t, *prm, prec="fp64").cpu().numpy()
        assert np.abs(z64 - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max())
        z32 = pt.orbit_z(t, *prm, prec="fp32").cpu().numpy()
        # in front of the star and near transit, where the flux depends on z;
        # behind the star (z < 0) the flux is 1 whatever |z|
        near = (ref > 0) & (ref < 2)
        assert np.abs(z32 - ref)[near].max() <= 2e-6
        assert (np.abs(z32 - ref) / np.maximum(1, np.abs(ref))).max() <= 2e-5


def _run(pt, b, model, prec, npol=50, u=None):
    db = pt.DeviceBatch(b, u=u)
    return pt.lc_batch(db, model, npol=npol, prec=prec).cpu().numpy().astype(np.float64)


def _gim_u(b):
    return np.stack([b["u"][:, 0] + 2 * b["u"][:, 1], -b["u"][:, 1]], 1)


def test_batch_single_lc(pt, O):
    from paper_1504_07433_amd import workloads as W
    b = W.config1()
    ref = O.lc_batch(b, model=0)
    assert np.abs(_run(pt, b, "ma", "fp64") - ref).max() <= TOL64
    assert np.abs(_run(pt, b, "ma", "fp32") - ref).max() <= TOL32
    ug = _gim_u(b)
    refg = O.lc_batch(b, model=1, npol=50, u=ug)
    assert np.abs(_run(pt, b, "gimenez", "fp64", u=ug) - refg).max() <= 1e-12
    assert np.abs(_run(pt, b, "gimenez", "fp32", u=ug) - refg).max() <= TOL32


def test_batch_long_cadence_small(pt, O):
    from paper_1504_07433_amd import workloads as W
    b = W.config2(n_vec=8, n_windows=2)
    ref = O.lc_batch(b, model=0)
    g32 = _run(pt, b, "ma", "fp32")
    g64 = _run(pt, b, "ma", "fp64")
    say("long-cadence small: fp32", np.abs(g32 - ref).max(), "fp64", np.abs(g64 - ref).max())
    assert np.abs(g32 - ref).max() <= TOL32
    assert np.abs(g64 - ref).max() <= TOL64
    assert (ref < 1).mean() > 0.2                       # really in transit


def test_batch_spectrophotometric_small(pt, O):
    from paper_1504_07433_amd import workloads as W
    b = W.config3(n_vec=6, n_band=64, n_exp=1500)
    ref = O.lc_batch(b, model=0)
    assert np.abs(_run(pt, b, "ma", "fp32") - ref).max() <= TOL32
    assert np.abs(_run(pt, b, "ma", "fp64") - ref).max() <= TOL64
    bs = W.config3(n_vec=2, n_band=64, n_exp=1500)
    ug = _gim_u(bs)
    refg = O.lc_batch(bs, model=1, npol=50, u=ug)
    assert np.abs(_run(pt, bs, "gimenez", "fp32", u=ug) - refg).max() <= TOL32
    assert np.abs(_run(pt, bs, "gimenez", "fp64", u=ug) - refg).max() <= 1e-12


@pytest.mark.parametrize("npol,nldc", [(1, 1), (5, 3), (60, 4), (61, 2), (100, 4), (512, 2)])
def test_batch_gimenez_orders_and_laws(pt, O, npol, nldc):
    """The batch's folded Chebyshev rows at small and large npol (rows of more
    than one wavefront of coefficients, one to many Clenshaw blocks, a fold
    row of exactly 64 coefficients at npol = 60 and one past it at 61) and
    general laws of 1..4 coefficients, FP32 and FP64, against the oracle."""
    from paper_1504_07433_amd import workloads as W
    b = W.config3(n_vec=3, n_band=6, n_exp=300)
    rng = np.random.default_rng(npol + 10 * nldc)
    ug = rng.uniform(-0.2, 0.6, (len(b["k"]), nldc)) / nldc
    say("gimenez batch npol", npol, "nldc", nldc)
    ref = O.lc_batch(b, model=1, npol=npol, u=ug)
    assert np.abs(_run(pt, b, "gimenez", "fp32", npol=npol, u=ug) - ref).max() <= TOL32
    assert np.abs(_run(pt, b, "gimenez", "fp64", npol=npol, u=ug) - ref).max() <= 1e-12


def test_batch_uneven_small(pt, O):
    from paper_1504_07433_amd import workloads as W
    b = W.config4(n_lc=48, n_min=50, n_max=3000)
    ref = O.lc_batch(b, model=0)
    g32 = _run(pt, b, "ma", "fp32")
    say("uneven small: fp32", np.abs(g32 - ref).max())
    assert np.abs(g32 - ref).max() <= TOL32
    assert np.abs(_run(pt, b, "ma", "fp64") - ref).max() <= TOL64
    ug = _gim_u(b)
    sub = W.subset(b, np.arange(12))
    refg = O.lc_batch(sub, model=1, npol=30, u=_gim_u(sub))
    assert np.abs(_run(pt, sub, "gimenez", "fp32", npol=30, u=_gim_u(sub)) - refg).max() <= TOL32


def test_batch_edge_cases(pt, O):
    from paper_1504_07433_amd import workloads as W
    b = W.config4(n_lc=10, n_min=20, n_max=300, max_nss=3, max_bands=3)
    b["nss"][1] = 20                         # more subsamples than one LDS chunk
    b["nss"][2] = 37
    for i in range(len(b["t_start"])):          # times across the transit at t0 = 0
        s0, c = b["t_start"][i], b["t_count"][i]
        b["t"][s0:s0 + c] = np.linspace(-0.07, 0.07, c)
    b["k"][b["band_off"][3]] = 0.7           # k > 1/2: exact path in the float kernel
    b["k"][b["band_off"][4]] = 1.4           # planet larger than the star
    # an empty light curve and one without bands
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
    for prec, tol in (("fp32", TOL32), ("fp64", TOL64)):
        g = _run(pt, b, "ma", prec)
        assert np.abs(g - ref).max() <= tol, prec
    # the same ragged batch through the Gimenez kernels
    ug = _gim_u(b)
    refg = O.lc_batch(b, model=1, npol=20, u=ug)
    for prec, tol in (("fp32", TOL32), ("fp64", TOL64)):
        g = _run(pt, b, "gimenez", prec, npol=20, u=ug)
        assert np.abs(g - refg).max() <= tol, ("gimenez", prec)


def _wide_batch(seed=11):
    """Light curves with many bands (16, 17, 33, 64, 70) beside narrow ones,
    ragged exposure counts around one wave (1, 63, 64, 65, ...), 1, 2, 3, 5 and
    19 subsamples, times across the transit (the first and the last light
    curve with whole waves outside the in-transit window): the tail of the
    tile list splits the wide light curves' tiles into runs of bands."""
    from paper_1504_07433_amd import workloads as W
    rng = np.random.default_rng(seed)
    nb = np.array([64, 70, 17, 16, 15, 33, 1, 40, 64], np.int64)
    cnt = np.array([130, 65, 63, 1, 200, 97, 64, 300, 190], np.int64)
    nss = np.array([1, 1, 3, 1, 2, 19, 1, 5, 1], np.int32)
    n = len(nb)
    b = W._empty_batch(n)
    b["t0"][:] = rng.uniform(-0.01, 0.01, n)
    b["P"][:] = 3.0
    b["aR"][:] = rng.uniform(8.0, 12.0, n)
    b["b"][:] = rng.uniform(0.1, 0.6, n)
    b["e"][:] = np.where(np.arange(n) % 3 == 0, 0.0, rng.uniform(0.0, 0.3, n))
    b["w"][:] = rng.uniform(0, 2 * np.pi, n)
    b["t_exp"][:] = 0.004
    b["nss"][:] = nss
    span = np.where((np.arange(n) == 0) | (np.arange(n) == n - 1), 0.25, 0.09)   # whole waves out of window
    t = np.concatenate([np.linspace(-h, h, c) for h, c in zip(span, cnt)])
    t_start = np.concatenate([[0], np.cumsum(cnt)[:-1]])
    k = rng.uniform(0.05, 0.15, int(nb.sum()))
    u = np.stack([rng.uniform(0.1, 0.6, len(k)), rng.uniform(0.0, 0.3, len(k))], 1)
    return W._finish(b, t, t_start, cnt, nb, k, u, "wide")


def test_band_split_tiles_match_oracle(pt, O):
    """Tiles split into runs of bands (and whole tiles of the narrow light
    curves) against the oracle element by element, float and FP64; then one
    invalid band in each of two wide light curves: NaN in that band only,
    including its exposures outside the in-transit window, where a wave with
    every band valid stores 1 without reading the band constants."""
    b = _wide_batch()
    ref = O.lc_batch(b, model=0)
    assert np.count_nonzero(ref < 1.0) > len(ref) // 4
    for prec, tol in (("fp32", TOL32), ("fp64", TOL64)):
        g = _run(pt, b, "ma", prec)
        assert np.abs(g - ref).max() <= tol, prec
    ug = _gim_u(b)
    refg = O.lc_batch(b, model=1, npol=20, u=ug)
    g = _run(pt, b, "gimenez", "fp32", npol=20, u=ug)
    assert np.abs(g - refg).max() <= TOL32
    bad = [int(b["band_off"][0]) + 5, int(b["band_off"][8]) + 63]   # band 5 of the first, the last of the last
    b["k"][bad[0]] = -0.1
    b["u"][bad[1], 0] = np.nan
    for prec in ("fp32", "fp64"):
        g = _run(pt, b, "ma", prec)
        for lc, band in ((0, 5), (8, 63)):
            o, c = int(b["flux_off"][lc]), int(b["t_count"][lc])
            blk = g[o:o + (b["band_off"][lc + 1] - b["band_off"][lc]) * c].reshape(-1, c)
            assert np.all(np.isnan(blk[band])), (prec, lc)
            rest = np.delete(blk, band, axis=0)
            r_ref = np.delete(ref[o:o + blk.size].reshape(-1, c), band, axis=0)
            assert np.abs(rest - r_ref).max() <= (TOL32 if prec == "fp32" else TOL64), (prec, lc)
            assert np.any(r_ref == 1.0)                 # the light curve has out-of-window exposures


def test_batch_extreme_shapes(pt, O):
    """A light curve with 40,000 bands (more than a tile may be split over:
    its tiles stay whole), one with 200 subsamples (13 LDS chunks, the orbit
    per band), and one of a single exposure and band, against the oracle."""
    from paper_1504_07433_amd import workloads as W
    rng = np.random.default_rng(21)
    nb = np.array([40000, 3, 1], np.int64)
    cnt = np.array([7, 50, 1], np.int64)
    b = W._empty_batch(3)
    b["t0"][:] = [0.0, 0.005, -0.003]
    b["P"][:] = 3.0
    b["aR"][:] = [10.0, 8.0, 12.0]
    b["b"][:] = [0.3, 0.5, 0.1]
    b["e"][:] = [0.0, 0.2, 0.1]
    b["w"][:] = [0.0, 1.0, 4.0]
    b["t_exp"][:] = [0.001, 0.02, 0.01]
    b["nss"][:] = [1, 200, 1]
    t = np.concatenate([np.linspace(-0.06, 0.06, 7), np.linspace(-0.08, 0.08, 50), [0.0]])
    k = rng.uniform(0.05, 0.15, int(nb.sum()))
    u = np.stack([rng.uniform(0.1, 0.6, len(k)), rng.uniform(0.0, 0.3, len(k))], 1)
    b = W._finish(b, t, [0, 7, 57], cnt, nb, k, u, "extreme")
    ref = O.lc_batch(b, model=0)
    assert np.count_nonzero(ref < 1.0) > len(ref) // 4
    for prec, tol in (("fp32", TOL32), ("fp64", TOL64)):
        g = _run(pt, b, "ma", prec)
        assert np.abs(g - ref).max() <= tol, prec


def _contact_batch(O, seed, e_max, nss, t_exp):
    """Light curves sampled densely around their first and last contacts
    (located on the oracle's z), eccentric orbits up to e_max, two bands per
    light curve with different k: checks that the per-orbit in-transit window
    keeps every point the model needs."""
    from paper_1504_07433_amd import workloads as W
    rng = np.random.default_rng(seed)
    n = 24
    b = W._empty_batch(n)
    ts, t_start, t_count, ks, us = [], [], [], [], []
    off = 0
    for i in range(n):
        while True:
            e, w, aR, bb = rng.uniform(0, e_max), rng.uniform(0, 2 * np.pi), rng.uniform(2.5, 30), rng.uniform(0, 1.15)
            if bb / aR * (1 + e * np.sin(w)) / (1 - e * e) < 0.99:
                break
        P, t0 = 3.0, rng.uniform(-0.01, 0.01)
        k0 = rng.uniform(0.02, 0.3)
        b["t0"][i], b["P"][i], b["aR"][i], b["b"][i], b["e"][i], b["w"][i] = t0, P, aR, bb, e, w
        b["t_exp"][i], b["nss"][i] = t_exp, nss
        grid = t0 + P * np.linspace(-0.5, 0.5, 100001)
        z = O.orbit_z(grid, t0, P, aR, bb, e, w)
        kk = k0 * rng.uniform(0.95, 1.05, 2)
        inside = (z >= 0) & (z < 1 + kk.max())
        edges = np.flatnonzero(np.diff(inside.astype(np.int8)))
        t = [t0 + np.linspace(-0.05, 0.05, 101)]
        for j in edges:
            t.append(grid[j] + np.linspace(-0.003, 0.003, 301))
        t = np.sort(np.concatenate(t))
        ts.append(t); t_start.append(off); t_count.append(len(t)); off += len(t)
        ks.extend(kk)
        us.extend(np.stack(W.kipping_q_to_u(rng.uniform(0, 1, 2), rng.uniform(0, 1, 2)), 1))
    return W._finish(b, np.concatenate(ts), t_start, t_count, [2] * n, np.array(ks), np.array(us),
                     "contacts")


@pytest.mark.parametrize("nss,t_exp", [(1, 0.0), (7, 0.0204)])
def test_batch_circular_contacts(pt, O, nss, t_exp):
    """Circular orbits (their in-transit window in closed form), impact
    parameters up to 1.15, times dense around every contact."""
    b = _contact_batch(O, 31 + nss, 0.0, nss, t_exp)
    assert np.all(b["e"] == 0.0)
    ref = O.lc_batch(b, model=0)
    for prec, tol in (("fp64", TOL64), ("fp32", TOL32)):
        got = _run(pt, b, "ma", prec)
        say("circular contacts", prec, "max|dF|", np.abs(got - ref).max())
        assert np.abs(got - ref).max() <= tol, prec


@pytest.mark.parametrize("nss,t_exp", [(1, 0.0), (7, 0.0204)])
def test_batch_eccentric_contacts(pt, O, nss, t_exp):
    b = _contact_batch(O, 11 + nss, 0.85, nss, t_exp)
    ref = O.lc_batch(b, model=0)
    got = _run(pt, b, "ma", "fp64")
    say("contacts fp64 max|dF|", np.abs(got - ref).max())
    assert np.abs(got - ref).max() <= TOL64
    # the float orbit's z error grows like (a/R*) sqrt((1+e)/(1-e)) ulp(dM):
    # the float bar applies up to e = 0.6
    b = _contact_batch(O, 21 + nss, 0.6, nss, t_exp)
    ref = O.lc_batch(b, model=0)
    got = _run(pt, b, "ma", "fp32")
    say("contacts fp32 max|dF|", np.abs(got - ref).max())
    assert np.abs(got - ref).max() <= TOL32


# quadratic laws at the edges of the physical region (u1 >= 0, u1 + u2 <= 1,
# u1 + 2 u2 >= 0) and a typical one: the weight of lambda_d runs from 0
# (u = (2, -1)) to 2.4 (u = (0, 1)), the largest it takes
EXTREME_LAWS = [(0.4, 0.2), (0.0, 0.0), (1.0, 0.0), (0.0, 1.0), (2.0, -1.0), (0.9, -0.3)]


@pytest.mark.parametrize("nss,t_exp", [(1, 0.0), (7, 0.0204)])
def test_batch_extreme_laws_dense_contacts(pt, O, nss, t_exp):
    """The float path's loss with the weights folded into per-band
    coefficients, for laws at the edges of the physical region, on orbits
    with times dense around every contact (one subsample: the one-subsample
    kernel; seven: the general kernel)."""
    b = _contact_batch(O, 41 + nss, 0.6, nss, t_exp)
    nb = len(b["k"])
    b["u"] = np.array([EXTREME_LAWS[j % len(EXTREME_LAWS)] for j in range(nb)], np.float64)
    ref = O.lc_batch(b, model=0)
    for prec, tol in (("fp64", TOL64), ("fp32", TOL32)):
        got = _run(pt, b, "ma", prec)
        say("extreme laws", prec, "nss", nss, "max|dF|", np.abs(got - ref).max())
        assert np.abs(got - ref).max() <= tol, prec


def test_batch_nonphysical_parameters_give_nan(pt):
    from paper_1504_07433_amd import workloads as W
    b = W.config2(n_vec=4, n_windows=1)
    b["e"][1] = 1.2
    b["aR"][2] = -3.0
    b["k"][3] = np.nan                         # an invalid band: NaN in every exposure
    for prec in ("fp32", "fp64"):
        g = _run(pt, b, "ma", prec)
        blk = lambda i: g[b["flux_off"][i]:b["flux_off"][i] + b["t_count"][i]]
        assert np.all(np.isnan(blk(1))) and np.all(np.isnan(blk(2))) and np.all(np.isnan(blk(3))), prec
        assert np.all(np.isfinite(blk(0))), prec
    # limb-darkening coefficients with non-finite weights: an invalid band too
    b2 = W.config2(n_vec=3, n_windows=1)
    b2["u"][1, 0] = np.nan
    for prec in ("fp32", "fp64"):
        g2 = _run(pt, b2, "ma", prec)
        s1 = slice(b2["flux_off"][1], b2["flux_off"][1] + b2["t_count"][1])
        assert np.all(np.isnan(g2[s1])), prec
        assert np.all(np.isfinite(g2[:b2["flux_off"][1]])) and np.all(np.isfinite(g2[s1.stop:])), prec
    b["k"][3] = -0.1
    g = _run(pt, b, "ma", "fp32")
    assert np.all(np.isnan(g[b["flux_off"][3]:b["flux_off"][3] + b["t_count"][3]]))
    # the model variants too: NaN throughout for an invalid orbit or band,
    # whatever the variant's own handling of z
    b["k"][3] = np.nan
    ks = b["k"][np.isfinite(b["k"])]
    pt.ma_table_set(float(ks.min()), float(ks.max()), 16, 256)
    pt.gimenez_zgrid_set(64, 64)
    for model, prec in (("ma_interp", "fp32"), ("ma_khat", "fp32"), ("gimenez", "fp32"), ("gimenez", "fp64"),
                        ("gimenez_zinterp", "fp32")):
        g = _run(pt, b, model, prec, npol=20)
        blk = lambda i: g[b["flux_off"][i]:b["flux_off"][i] + b["t_count"][i]]
        assert np.all(np.isnan(blk(1))) and np.all(np.isnan(blk(2))) and np.all(np.isnan(blk(3))), model
        assert np.all(np.isfinite(blk(0))), model


def test_batch_deterministic_and_graph_matches_eager(pt, monkeypatch):
    from paper_1504_07433_amd import workloads as W
    b = W.config4(n_lc=32, n_min=100, n_max=4000)
    db = pt.DeviceBatch(b)
    first = pt.lc_batch(db, "ma", prec="fp32").cpu().numpy()
    for _ in range(4):                                  # graph replays
        assert np.array_equal(pt.lc_batch(db, "ma", prec="fp32").cpu().numpy(), first)
    monkeypatch.setenv("PT_NO_GRAPH", "1")
    assert np.array_equal(pt.lc_batch(db, "ma", prec="fp32").cpu().numpy(), first)


def test_batch_two_streams_same_shape(pt, O):
    """Two batches of one shape but different parameter values, enqueued on
    two streams without synchronisation between them: each stream has its own
    plan scratch (queue counters, orbit and band constants), so both results
    match the oracle."""
    import torch
    from paper_1504_07433_amd import workloads as W
    b1 = W.config4(seed=21, n_lc=16, n_min=200, n_max=3000)
    b2 = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in b1.items()}
    rng = np.random.default_rng(3)
    b2["aR"] = b2["aR"] * rng.uniform(0.9, 1.1, len(b2["aR"]))
    b2["k"] = b2["k"] * rng.uniform(0.8, 1.2, len(b2["k"]))
    b2["w"] = rng.uniform(0, 2 * np.pi, len(b2["w"]))
    ref1, ref2 = O.lc_batch(b1, model=0), O.lc_batch(b2, model=0)
    d1, d2 = pt.DeviceBatch(b1), pt.DeviceBatch(b2)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    outs = []
    for rep in range(3):
        with torch.cuda.stream(s1):
            g1 = pt.lc_batch(d1, "ma", prec="fp32")
        with torch.cuda.stream(s2):
            g2 = pt.lc_batch(d2, "ma", prec="fp32")
        outs.append((g1, g2))
    torch.cuda.synchronize()
    for g1, g2 in outs:
        assert np.abs(g1.cpu().numpy() - ref1).max() <= TOL32
        assert np.abs(g2.cpu().numpy() - ref2).max() <= TOL32


def test_autotune_keeps_results(pt, tmp_path):
    """The tuner times the default shape first and keeps a shape no slower
    than it; the tuned shape changes no result, and a cache file written by
    pt_tune_save gives a fresh library state the same shape."""
    from paper_1504_07433_amd import workloads as W
    b = W.config4(n_lc=40, n_min=100, n_max=5000)
    db = pt.DeviceBatch(b)
    before = pt.lc_batch(db, "ma", prec="fp32").cpu().numpy()
    rep = pt.autotune(db, "ma", prec="fp32")
    cands = rep["candidates"]
    assert cands[0].get("default") and len(cands) >= 5
    assert 0 < rep["best"]["ms"] <= rep["default_ms"] == cands[0]["ms"]
    te, wg = pt.launch_shape(db, "ma", prec="fp32")
    assert te == rep["best"]["tile_exposures"] and wg == rep["best"]["workgroups"]
    after = pt.lc_batch(db, "ma", prec="fp32").cpu().numpy()
    assert np.array_equal(before, after)
    path = str(tmp_path / "tune.jsonl")
    pt.tune_save(path)
    pt.release()
    assert pt.tune_load(path) >= 1
    again = pt.lc_batch(db, "ma", prec="fp32").cpu().numpy()
    assert pt.launch_shape(db, "ma", prec="fp32") == (te, wg)
    assert np.array_equal(before, again)


# --- full sizes, in the benchmark's launch configuration, on sampled outputs ----

def _bench_shapes(pt):
    """The tuned launch shapes bench.py loads, so that the full-size checks
    run the launch configuration the benchmark times."""
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_1504_07433_amd", "data", "tune_cache.jsonl")
    assert pt.tune_load(path) >= 1


def _sampled_check(pt, O, b, model, prec, tol, n_samples, npol=50, u=None, seed=0):
    _bench_shapes(pt)
    db = pt.DeviceBatch(b, u=u)
    import torch
    g = pt.lc_batch(db, model, npol=npol, prec=prec)
    say(b["name"], model, prec, "launch shape (tile exposures, workgroups)",
        pt.launch_shape(db, model, npol=npol, prec=prec))
    pairs = random_pairs(b, n_samples, seed=seed)
    sb, idx = single_exposure_subset(b, pairs)
    if u is not None:
        sb["u"] = np.concatenate([u[b["band_off"][l]:b["band_off"][l + 1]] for l, _ in pairs])
    got = g[torch.as_tensor(idx, device=g.device)].cpu().numpy().astype(np.float64)
    ref = O.lc_batch(sb, model=0 if model == "ma" else 1, npol=npol, u=None if u is None else sb["u"])
    err = np.abs(got - ref).max()
    say(b["name"], model, prec, "sampled max|dF|", err, "in transit", (ref < 1).mean())
    assert err <= tol
    return g


def test_full_long_cadence_sampled(pt, O):
    from paper_1504_07433_amd import workloads as W
    b = W.config2()
    _sampled_check(pt, O, b, "ma", "fp32", TOL32, 3000)
    _sampled_check(pt, O, b, "ma", "fp64", TOL64, 1500, seed=1)


def test_full_spectrophotometric_sampled(pt, O):
    from paper_1504_07433_amd import workloads as W
    b = W.config3()
    _sampled_check(pt, O, b, "ma", "fp32", TOL32, 400)
    _sampled_check(pt, O, b, "gimenez", "fp32", TOL32, 150, u=_gim_u(b), seed=2)
    # the FP64 kernels of the one-subsample shape
    _sampled_check(pt, O, b, "ma", "fp64", TOL64, 300, seed=3)
    _sampled_check(pt, O, b, "gimenez", "fp64", 1e-12, 100, u=_gim_u(b), seed=4)


def test_full_uneven_sampled(pt, O):
    from paper_1504_07433_amd import workloads as W
    b = W.config4()
    _sampled_check(pt, O, b, "ma", "fp32", TOL32, 1500)
    _sampled_check(pt, O, b, "ma", "fp64", TOL64, 500, seed=1)


# --- fused likelihood -------------------------------------------------------------------

@pytest.mark.skip(reason="fused likelihood switched off: its first GPU run stopped responding "
                         "(killed after 180 s of silence) and no cause has been shown yet")
@pytest.mark.parametrize("prec,ftol", [("fp32", TOL32), ("fp64", TOL64)])
def test_loglike_matches_oracle(pt, O, prec, ftol):
    import torch
    from paper_1504_07433_amd import workloads as W
    b = W.config4(n_lc=24, n_min=100, n_max=2000)
    b["nss"][3] = 19                            # the per-band orbit branch too
    F = O.lc_batch(b, model=0)
    rng = np.random.default_rng(0)
    sigma = rng.uniform(5e-4, 2e-3, len(b["t_start"]))
    nb = np.diff(b["band_off"]).astype(np.int64)
    sig_pt = np.repeat(sigma, nb * b["t_count"])
    obs = F + rng.normal(0, 1, len(F)) * sig_pt
    dtype = np.float32 if prec == "fp32" else np.float64
    obs = obs.astype(dtype)
    ref = O.loglike(b, obs.astype(np.float64), sigma, flux=F)
    db = pt.DeviceBatch(b)
    got = pt.lc_loglike(db, torch.as_tensor(obs, device="cuda"), sigma, prec=prec).cpu().numpy()
    # each model value may differ by ftol: |d log L| <= sum |r| ftol/sigma + N (ftol/sigma)^2
    for i in range(len(ref)):
        sl = slice(b["flux_off"][i], b["flux_off"][i] + nb[i] * b["t_count"][i])
        r = (obs[sl].astype(np.float64) - F[sl]) / sigma[i]
        bound = np.abs(r).sum() * ftol / sigma[i] + len(r) * (ftol / sigma[i]) ** 2 + 1e-9 * abs(ref[i])
        assert abs(got[i] - ref[i]) <= bound, (i, got[i], ref[i], bound)
    # deterministic
    again = pt.lc_loglike(db, torch.as_tensor(obs, device="cuda"), sigma, prec=prec).cpu().numpy()
    assert np.array_equal(got, again)


# --- paper variants: interpolated Mandel-Agol and the khat approximation -----------------

def test_interpolated_model_matches_oracle(pt, O):
    from paper_1504_07433_amd import workloads as W
    k_lo, k_hi, nk, nz = 0.09, 0.11, 16, 64
    pt.ma_table_set(k_lo, k_hi, nk, nz)
    tab = O.ma_table(k_lo, k_hi, nk, nz)
    b = W.config3(n_vec=3, n_band=8, n_exp=300)
    b["k"][0] = 0.2                            # outside the table: exact path
    ref = O.lc_batch_ma_variant(b, "interp", tab, k_lo, k_hi)
    got = _run(pt, b, "ma_interp", "fp32")
    assert np.abs(got - ref).max() <= TOL32


def test_interpolated_rows_every_chunk_length(pt, O):
    """Per-band table rows are read by code unrolled for the exact number of
    subsamples in a chunk (1..16; more than 16 run in chunks of 16 and a
    remainder): light curves with 1..20 subsamples against the oracle's
    tabulated variant."""
    from paper_1504_07433_amd import workloads as W
    b = W.config4(seed=7, n_lc=20, n_min=1500, n_max=2000)
    b["nss"][:] = np.arange(1, 21, dtype=np.int32)
    k_lo, k_hi, nk, nz = float(b["k"].min()), float(b["k"].max()), 64, 512
    pt.ma_table_set(k_lo, k_hi, nk, nz)
    tab = O.ma_table(k_lo, k_hi, nk, nz)
    say("chunk lengths: bands", len(b["k"]), "points", W.n_points(b))
    ref = O.lc_batch_ma_variant(b, "interp", tab, k_lo, k_hi)
    got = _run(pt, b, "ma_interp", "fp32")
    assert np.abs(got - ref).max() <= TOL32
    assert np.count_nonzero(ref < 1.0) > len(ref) // 10     # the transits are sampled


def test_interpolated_model_many_bands_matches_oracle(pt, O):
    """65536 passbands x 2048 z nodes exceed the size kept for per-band rows,
    so the kernel interpolates the shared (k, z) table directly."""
    from paper_1504_07433_amd import workloads as W
    k_lo, k_hi, nk, nz = 0.09, 0.11, 16, 2048
    pt.ma_table_set(k_lo, k_hi, nk, nz)
    tab = O.ma_table(k_lo, k_hi, nk, nz)
    b = W.config3(n_vec=1024, n_band=64, n_exp=12)
    b["k"][5] = 0.2                            # outside the table: exact path
    ref = O.lc_batch_ma_variant(b, "interp", tab, k_lo, k_hi)
    got = _run(pt, b, "ma_interp", "fp32")
    assert np.abs(got - ref).max() <= TOL32


def test_interpolated_model_meets_flux_gate(pt, O):
    """With 256 x 2048 nodes over the batch's k range the tabulated model
    stays within 1e-5 of the exact flux (measured on the oracle: ~1e-6), also
    around every contact of eccentric orbits."""
    from paper_1504_07433_amd import workloads as W
    for b in (W.config2(n_vec=16, n_windows=2), _contact_batch(O, 31, 0.5, 5, 0.0204)):
        k_lo, k_hi = float(b["k"].min()), float(b["k"].max())
        pt.ma_table_set(k_lo, k_hi, 256, 2048)
        got = _run(pt, b, "ma_interp", "fp32")
        err = np.abs(got - O.lc_batch(b, model=0)).max()
        say("interpolated model vs exact flux: max|dF|", err)
        assert err <= 1e-5


def test_khat_model_matches_oracle(pt, O):
    from paper_1504_07433_amd import workloads as W
    b = W.config3(n_vec=3, n_band=8, n_exp=300)
    ref = O.lc_batch_ma_variant(b, "khat")
    got = _run(pt, b, "ma_khat", "fp32")
    assert np.abs(got - ref).max() <= TOL32
    exact = O.lc_batch(b, model=0)
    say("khat approximation vs per-band k: max|dF|", np.abs(ref - exact).max())


def test_gimenez_zinterp_matches_oracle(pt, O):
    from paper_1504_07433_amd import workloads as W
    pt.gimenez_zgrid_set(50, 50)
    b = W.config3(n_vec=2, n_band=6, n_exp=300)
    ug = _gim_u(b)
    ref = O.lc_batch_gimenez_zinterp(b, 30, 50, 50, ug)
    got = _run(pt, b, "gimenez_zinterp", "fp32", npol=30, u=ug)
    assert np.abs(got - ref).max() <= TOL32
