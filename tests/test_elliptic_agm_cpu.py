"""The Mandel & Agol elliptic combination pref * (C_K K(m) + C_E E(m) + C_P Pi(n, m))
behind lambda_1 and lambda_2 (Sect. 2.2.1), as the library evaluates it: one
Bulirsch cel for the third-kind integral, with K and E taken from the same
arithmetic-geometric mean through Legendre's sum (DLMF 19.8.5-19.8.6).  Built
for the host, it is checked against Carlson's symmetric integrals evaluated in
40-digit arithmetic (mpmath), which share nothing with it: K = R_F(0, kc^2, 1),
E = R_F(0, kc^2, 1) - (m/3) R_D(0, kc^2, 1) (DLMF 19.25.1) and cel(kc, p, a, b) =
a R_F(0, kc^2, 1) + (b - p a)/3 R_J(0, kc^2, 1, p); the last identity is itself
checked against quadrature of cel's defining integral.  The extended precision
matters near z = k, where p grows like 1/(z-k)^2 and the identity's two terms
cancel."""
import ctypes
import os
import subprocess

import mpmath
import numpy as np
import pytest
from scipy import integrate, special

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    so = tmp_path_factory.mktemp("ell") / "libell.so"
    subprocess.run(["g++", "-O2", "-shared", "-fPIC", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
                    "-x", "c++", os.path.join(HERE, "elliptic_host.cpp"), "-o", str(so)], check=True)
    L = ctypes.CDLL(str(so))
    dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    L.ell_terms64.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, dp]
    L.ell_terms64.restype = None
    L.ell_agm64.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, dp]
    L.ell_agm64.restype = None
    return L


def cel_carlson(kc, p, a, b):
    x = kc * kc
    return a * special.elliprf(0.0, x, 1.0) + (b - p * a) / 3.0 * special.elliprj(0.0, x, 1.0, p)


def cel_quad(kc, p, a, b):
    f = lambda t: ((a * np.cos(t) ** 2 + b * np.sin(t) ** 2)
                   / ((np.cos(t) ** 2 + p * np.sin(t) ** 2) * np.sqrt(np.cos(t) ** 2 + kc * kc * np.sin(t) ** 2)))
    return integrate.quad(f, 0.0, np.pi / 2, epsabs=1e-14, epsrel=1e-13, limit=400)[0]


def test_cel_identity_against_quadrature():
    rng = np.random.default_rng(11)
    for _ in range(40):
        kc, p = rng.uniform(0.05, 1.0), np.exp(rng.uniform(-3, 3))
        a, b = rng.uniform(-3, 3, 2)
        q = cel_quad(kc, p, a, b)
        assert abs(cel_carlson(kc, p, a, b) - q) <= 1e-11 * max(1.0, abs(q)), (kc, p, a, b)


def _points(seed, n=2500):
    rng = np.random.default_rng(seed)
    k = rng.uniform(0.01, 0.5, n)
    z = (1.0 + k) * rng.uniform(0.0, 1.0, n)
    limb_rows = rng.uniform(0.0, 1.0, n) < 0.3
    z[limb_rows] = 1.0 - k[limb_rows] + 2.0 * k[limb_rows] * rng.uniform(0.0, 1.0, limb_rows.sum())
    # near the contacts z = k and z = 1 - k (the exact case table takes over within 1e-6)
    near = rng.uniform(0.0, 1.0, n) < 0.2
    off = 10.0 ** rng.uniform(-6, -2, near.sum()) * rng.choice([-1.0, 1.0], near.sum())
    z[near] = np.where(rng.uniform(0.0, 1.0, near.sum()) < 0.5, k[near], 1.0 - k[near]) + off
    keep = (z > 1e-6) & (z < 1.0 + k - 1e-9) & (np.abs(z - k) > 1e-6) & (np.abs(z - (1.0 - k)) > 1e-6)
    return np.ascontiguousarray(z[keep]), np.ascontiguousarray(k[keep])


def _reference(lib, z, k):
    out = np.empty(len(z))
    t = np.empty(7)
    with mpmath.workdps(40):
        for i in range(len(z)):
            lib.ell_terms64(z[i], k[i], int(z[i] > 1.0 - k[i]), t)
            kc, ck, ce, sp, cp, bt2, pref = (mpmath.mpf(float(v)) for v in t)
            x, p = kc * kc, sp * sp
            rf = mpmath.elliprf(0, x, 1)
            ee = rf - (1 - x) / 3 * mpmath.elliprd(0, x, 1)
            cel = cp * rf + (bt2 * sp - p * cp) / 3 * mpmath.elliprj(0, x, 1, p)
            out[i] = float(pref * (ck * rf + ce * ee + cel))
    return out


@pytest.fixture(scope="module")
def sample(lib):
    z, k = _points(5)
    return z, k, _reference(lib, z, k)


# fast = 1: the float path's seeds (float here, ~5e-8 on gfx950) with the
# square roots unrefined.  lambda_d enters the flux with weight c/N =
# (u1 + 2 u2) / (1 - u1/3 - u2/6) <= 2.4 over the physical quadratic laws, so
# 2e-7 here keeps the float path's flux within 4.8e-7 of the model (its
# tolerance is 1e-6).
@pytest.mark.parametrize("fast,tol", [(0, 1e-13), (1, 2e-7)])
def test_combination_against_carlson(lib, sample, fast, tol):
    z, k, ref = sample
    got = np.empty(len(z))
    lib.ell_agm64(len(z), z, k, fast, got)
    err = np.abs(got - ref)
    i = int(np.argmax(err))
    assert err[i] <= tol, (z[i], k[i], got[i], ref[i])
