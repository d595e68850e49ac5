"""ctypes wrapper of the FP64 CPU oracle (oracle.c) plus the small pieces that
are easiest to state in numpy.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the package smoke check
and by the benchmark's CPU-baseline leg.  The product path (the HIP library
and its Python binding) never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "oracle.c")

_dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i64 = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_i32 = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc -O2 (no fast-math) and OpenMP."""
    if force or not os.path.exists(LIB_PATH) or \
            os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-o", LIB_PATH + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=HERE)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        d = C.c_double
        for name, nargs in (("or_rf", 3), ("or_rd", 3), ("or_rj", 4), ("or_ellk", 1),
                            ("or_elle", 1), ("or_ellpi", 2)):
            f = getattr(L, name); f.restype = d; f.argtypes = [d] * nargs
        L.or_ma_alpha.restype = C.c_int
        L.or_ma_alpha.argtypes = [d, d, _dp]
        L.or_ma_flux.restype = d
        L.or_ma_flux.argtypes = [d, d, d, d]
        L.or_gimenez_alpha.restype = None
        L.or_gimenez_alpha.argtypes = [d, d, C.c_int, C.c_int, _dp]
        L.or_gimenez_flux.restype = d
        L.or_gimenez_flux.argtypes = [d, d, _dp, C.c_int, C.c_int]
        L.or_orbit_z.restype = d
        L.or_orbit_z.argtypes = [d] * 7
        L.or_last_newton_iters.restype = C.c_int
        L.or_num_threads.restype = C.c_int
        L.or_num_threads.argtypes = [C.c_int32]
        L.or_lc_batch.restype = C.c_int
        L.or_lc_batch.argtypes = [C.c_int32, _dp, _i64, _i64, _dp, _dp, _dp, _dp, _dp, _dp,
                                  _dp, _i32, _i32, _dp, _dp, C.c_int32, _i64, C.c_int32,
                                  C.c_int32, _dp, C.c_int32]
        _lib = L
    return _lib


# -- scalar / elementwise helpers ----------------------------------------------------

def ellk(m): return lib().or_ellk(float(m))
def elle(m): return lib().or_elle(float(m))
def ellpi(n, m): return lib().or_ellpi(float(n), float(m))
def rf(x, y, z): return lib().or_rf(float(x), float(y), float(z))
def rd(x, y, z): return lib().or_rd(float(x), float(y), float(z))
def rj(x, y, z, p): return lib().or_rj(float(x), float(y), float(z), float(p))


def ma_alpha(z, k):
    """(lambda_e, lambda_d + 2/3 Theta(k-z), eta_d) and the case number."""
    out = np.zeros(3)
    cs = lib().or_ma_alpha(float(z), float(k), out)
    return out, cs


def ma_alpha_many(z, k):
    z = np.broadcast_to(np.asarray(z, np.float64), np.broadcast(z, k).shape).ravel()
    k = np.broadcast_to(np.asarray(k, np.float64), z.shape).ravel()
    res = np.empty((z.size, 3))
    out = np.zeros(3)
    L = lib()
    for i in range(z.size):
        L.or_ma_alpha(z[i], k[i], out)
        res[i] = out
    return res


def ma_flux(z, k, u1, u2):
    z = np.atleast_1d(np.asarray(z, np.float64))
    L = lib()
    return np.array([L.or_ma_flux(zz, float(k), float(u1), float(u2)) for zz in z])


def gimenez_alpha(z, k, nldc, npol):
    out = np.zeros(nldc + 1)
    lib().or_gimenez_alpha(float(z), float(k), int(nldc), int(npol), out)
    return out


def gimenez_flux(z, k, u, npol):
    u = np.ascontiguousarray(u, np.float64)
    z = np.atleast_1d(np.asarray(z, np.float64))
    L = lib()
    return np.array([L.or_gimenez_flux(zz, float(k), u, len(u), int(npol)) for zz in z])


def orbit_z(t, t0, P, aR, b, e, w):
    t = np.atleast_1d(np.asarray(t, np.float64))
    L = lib()
    return np.array([L.or_orbit_z(tt, t0, P, aR, b, e, w) for tt in t])


def quadratic_to_general(u1, u2):
    """Quadratic (a, b) -> general-law (u_1, u_2) = (a + 2b, -b) (Sect. 2.1.2)."""
    return np.array([u1 + 2.0 * u2, -u2])


def lc_batch(batch, model: int = 0, npol: int = 50, u=None, nthreads: int = 0):
    """Supersampled ragged batch in FP64.  model 0: quadratic Mandel-Agol with
    batch['u'] = (u1, u2); model 1: Gimenez with general-law ``u`` (default:
    the quadratic coefficients transformed)."""
    if u is None:
        u = batch["u"] if model == 0 else np.stack(
            [batch["u"][:, 0] + 2 * batch["u"][:, 1], -batch["u"][:, 1]], 1)
    u = np.ascontiguousarray(u, np.float64)
    nldc = u.shape[1]
    flux = np.empty(batch["n_flux"])
    rc = lib().or_lc_batch(
        len(batch["t_start"]), batch["t"], batch["t_start"], batch["t_count"],
        batch["t0"], batch["P"], batch["aR"], batch["b"], batch["e"], batch["w"],
        batch["t_exp"], batch["nss"], batch["band_off"], batch["k"], u, nldc,
        batch["flux_off"], model, npol, flux, nthreads)
    if rc != 0:
        raise ValueError("oracle lc_batch: bad arguments")
    return flux


def num_threads(nthreads: int = 0) -> int:
    return lib().or_num_threads(nthreads)


def surrogate_targets(zk):
    """The three limb-darkening-factored Mandel-Agol functions
    (alpha_0, alpha_1, alpha_0 - alpha_2) = (lambda_e, lambda_d + 2/3 Theta,
    eta_d) at each (z, k) row; zero for z >= 1 + k."""
    zk = np.asarray(zk, np.float64)
    return ma_alpha_many(zk[:, 0], zk[:, 1])


def loglike(batch, obs, sigma, model: int = 0, npol: int = 50, u=None, flux=None):
    """Gaussian log-likelihood per light curve, written out from its
    definition: -1/2 sum ((obs - F)/sigma)^2 - N ln sigma - N/2 ln(2 pi)."""
    F = lc_batch(batch, model=model, npol=npol, u=u) if flux is None else flux
    out = np.empty(len(batch["t_start"]))
    for i in range(len(out)):
        nb = batch["band_off"][i + 1] - batch["band_off"][i]
        n = int(nb * batch["t_count"][i])
        sl = slice(batch["flux_off"][i], batch["flux_off"][i] + n)
        r = (np.asarray(obs[sl], np.float64) - F[sl]) / sigma[i]
        out[i] = -0.5 * np.sum(r * r) - n * np.log(sigma[i]) - 0.5 * n * np.log(2 * np.pi)
    return out


# -- model variants of the paper, written out from their definitions ----------------------

def ma_table(k_lo, k_hi, nk, nz):
    """The three Mandel-Agol functions on a uniform grid of nk radius ratios in
    [k_lo, k_hi] and nz distances in [0, 1 + k_hi] (Sect. 2.2.3)."""
    ks = np.linspace(k_lo, k_hi, nk)
    zs = np.linspace(0.0, 1.0 + k_hi, nz)
    tab = np.zeros((nk, nz, 3))
    for i, k in enumerate(ks):
        tab[i] = ma_alpha_many(zs, np.full(nz, k))
    return tab


def ma_interp_alpha(z, k, tab, k_lo, k_hi):
    """Bilinear interpolation of the table in (k, z); zero for z >= 1 + k or
    z < 0; exact values for k outside [k_lo, k_hi]."""
    nk, nz = tab.shape[:2]
    if z < 0 or z >= 1 + k:
        return np.zeros(3)
    if not (k_lo <= k <= k_hi):
        return ma_alpha(z, k)[0]
    fk = (k - k_lo) / (k_hi - k_lo) * (nk - 1)
    fz = z / (1 + k_hi) * (nz - 1)
    ik = min(nk - 2, max(0, int(fk)))
    iz = min(nz - 2, max(0, int(fz)))
    wk, wz = fk - ik, fz - iz
    return ((1 - wk) * (1 - wz) * tab[ik, iz] + (1 - wk) * wz * tab[ik, iz + 1]
            + wk * (1 - wz) * tab[ik + 1, iz] + wk * wz * tab[ik + 1, iz + 1])


def lc_batch_ma_variant(batch, variant, table=None, k_lo=None, k_hi=None):
    """Supersampled quadratic Mandel-Agol batch with the three functions taken
    (a) from the bilinear table ("interp", Sect. 2.2.3), or (b) at the light
    curve's mean radius ratio khat with the depth of band i multiplied by
    k_i^2 / khat^2 ("khat", Sect. 3.5).  Small batches only (Python loops)."""
    flux = np.empty(batch["n_flux"])
    for lc in range(len(batch["t_start"])):
        s0, cnt, n = batch["t_start"][lc], batch["t_count"][lc], int(batch["nss"][lc])
        b0, b1 = batch["band_off"][lc], batch["band_off"][lc + 1]
        if b1 == b0 or cnt == 0:
            continue
        prm = tuple(batch[key][lc] for key in ("t0", "P", "aR", "b", "e", "w"))
        t = batch["t"][s0:s0 + cnt]
        ts = (t[:, None] + batch["t_exp"][lc] * ((np.arange(n) + 0.5) / n - 0.5)[None, :]).ravel()
        z = orbit_z(ts, *prm)
        khat = batch["k"][b0:b1].mean()
        if variant == "khat":
            al_hat = ma_alpha_many(np.where(z < 0, 2.0 + khat, z), np.full(len(z), khat))
        for j, bnd in enumerate(range(b0, b1)):
            k = batch["k"][bnd]
            u1, u2 = batch["u"][bnd]
            c = u1 + 2 * u2
            w = np.array([1 - c, c, u2]) / (1 - u1 / 3 - u2 / 6)
            if variant == "interp":
                al = np.array([ma_interp_alpha(zz, k, table, k_lo, k_hi) for zz in z])
                loss = al @ w
            else:
                loss = (al_hat @ w) * (k * k / (khat * khat))
            off = batch["flux_off"][lc] + j * cnt
            flux[off:off + cnt] = 1 - loss.reshape(cnt, n).mean(1)
    return flux


def gimenez_zgrid(k, n_in, n_limb):
    """Nodes of the Gimenez z-space interpolation (Sect. 3.3): n_in points in
    [0, 1-k] and n_limb points in [1-k, 1+k] (the shared node 1-k counted in
    both)."""
    return (np.linspace(0.0, 1.0 - k, n_in), np.linspace(1.0 - k, 1.0 + k, n_limb))


def gimenez_zinterp_flux(z, k, u, npol, n_in, n_limb):
    """Flux linearly interpolated in z between the tabulated Gimenez model
    values at the nodes; 1 outside 0 <= z < 1 + k."""
    zi, zl = gimenez_zgrid(k, n_in, n_limb)
    fi = gimenez_flux(zi, k, u, npol)
    fl = gimenez_flux(zl, k, u, npol)
    z = np.atleast_1d(np.asarray(z, np.float64))
    out = np.ones_like(z)
    inside = (z >= 0) & (z <= 1 - k)
    limb = (z > 1 - k) & (z < 1 + k)
    out[inside] = np.interp(z[inside], zi, fi)
    out[limb] = np.interp(z[limb], zl, fl)
    return out


def lc_batch_gimenez_zinterp(batch, npol, n_in, n_limb, u):
    """Supersampled Gimenez batch with the flux interpolated in z between the
    per-band nodes (Sect. 3.3).  Small batches only (Python loops)."""
    flux = np.empty(batch["n_flux"])
    for lc in range(len(batch["t_start"])):
        s0, cnt, n = batch["t_start"][lc], batch["t_count"][lc], int(batch["nss"][lc])
        b0, b1 = batch["band_off"][lc], batch["band_off"][lc + 1]
        if b1 == b0 or cnt == 0:
            continue
        prm = tuple(batch[key][lc] for key in ("t0", "P", "aR", "b", "e", "w"))
        t = batch["t"][s0:s0 + cnt]
        ts = (t[:, None] + batch["t_exp"][lc] * ((np.arange(n) + 0.5) / n - 0.5)[None, :]).ravel()
        z = orbit_z(ts, *prm)
        for j, bnd in enumerate(range(b0, b1)):
            f = gimenez_zinterp_flux(z, batch["k"][bnd], u[bnd], npol, n_in, n_limb)
            off = batch["flux_off"][lc] + j * cnt
            flux[off:off + cnt] = f.reshape(cnt, n).mean(1)
    return flux
