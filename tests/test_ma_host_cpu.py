"""The library's Mandel & Agol functions (Sect. 2.2.1: lambda_e, lambda_d with
the 2/3 step inside the planet's disc, eta_d), built for the host from the
same header the kernels use, against the oracle: the double case table over
every case of the table (contacts, z = 0, z = k, z = 1 - k, k = 1/2, k > 1/2,
a covered star), and the float path's mixed-precision bulk form where the
kernels use it (k <= 1/2, more than 1e-6 from z = k and z = 1 - k)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
KS = [0.005, 0.05, 0.1, 0.3, 0.45, 0.5, 0.6, 0.9, 1.0, 1.3]


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    so = tmp_path_factory.mktemp("ma") / "libma.so"
    subprocess.run(["g++", "-O2", "-shared", "-fPIC", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
                    "-x", "c++", os.path.join(HERE, "ma_host.cpp"), "-o", str(so)], check=True)
    L = ctypes.CDLL(str(so))
    dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    L.ma_alpha64.argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_int, dp]
    L.ma_alpha64.restype = None
    L.ma_loss64.argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
    L.ma_loss64.restype = None
    return L


def _alpha(lib, z, k, exact):
    z = np.ascontiguousarray(z, np.float64)
    out = np.empty((len(z), 3))
    lib.ma_alpha64(len(z), z, k, exact, out)
    return out


def _grid(k):
    base = np.linspace(0.0, 1.0 + k + 0.05, 1201)
    offs = np.concatenate([np.logspace(-13, -1, 25), -np.logspace(-13, -1, 25), [0.0]])
    z = np.concatenate([base] + [c + offs for c in (k, 1.0 - k, 1.0 + k, 0.0)])
    return z[z >= 0.0]


@pytest.mark.parametrize("k", KS)
def test_case_table_double(lib, oracle, k):
    z = _grid(k)
    got, ref = _alpha(lib, z, k, 1), oracle.ma_alpha_many(z, k)
    d = np.abs(got - ref).max(1)
    far = (np.abs(z - k) > 1e-5) & (np.abs(z - (1.0 - k)) > 1e-5)
    assert d.max() <= 1e-8, (d.max(), z[np.argmax(d)])
    assert d[far].max() <= 1e-11, (d[far].max(), z[far][np.argmax(d[far])])


@pytest.mark.parametrize("k", [k for k in KS if k <= 0.5])
def test_mixed_bulk_form(lib, oracle, k):
    kf = float(np.float32(k))
    z = _grid(kf).astype(np.float32).astype(np.float64)
    z = z[(z < 1.0 + kf) & (np.abs(z - kf) >= 1e-6) & (np.abs(z - (1.0 - kf)) >= 1e-6)]
    got = _alpha(lib, z, kf, 0)
    ref = oracle.ma_alpha_many(z, kf)
    d = np.abs(got - ref).max(1)
    # the float rounding of the three results, and the unrefined square-root
    # seeds in lambda_d's elliptic combination; with flux weights <= 2.4 over
    # the physical quadratic laws 2e-7 keeps the flux within 4.8e-7
    assert d.max() <= 2e-7, (d.max(), z[np.argmax(d)])


# (u1, u2): a typical law, a uniform source, the linear law's extreme, a
# negative u2, and the largest weight of lambda_d over the physical laws
@pytest.mark.parametrize("u1,u2", [(0.4, 0.2), (0.0, 0.0), (1.0, 0.0), (0.9, -0.3), (0.0, 1.0)])
@pytest.mark.parametrize("k", [k for k in KS if k <= 0.5])
def test_folded_loss(lib, oracle, k, u1, u2):
    """The float path's loss with the weights folded into per-band
    coefficients equals w0 lambda_e + w1 lambda_d + w2 eta_d of the oracle's
    functions, weights (1 - c)/N, c/N, u2/N with c = u1 + 2 u2 and
    N = 1 - u1/3 - u2/6, to the float path's own accuracy."""
    kf = float(np.float32(k))
    z = _grid(kf).astype(np.float32).astype(np.float64)
    z = z[(z < 1.0 + kf) & (np.abs(z - kf) >= 1e-6) & (np.abs(z - (1.0 - kf)) >= 1e-6)]
    n = 1.0 - u1 / 3.0 - u2 / 6.0
    c = u1 + 2.0 * u2
    w = np.array([(1.0 - c) / n, c / n, u2 / n])
    got = np.empty(len(z))
    lib.ma_loss64(len(z), np.ascontiguousarray(z), kf, w[0], w[1], w[2], got)
    ref = oracle.ma_alpha_many(z, kf) @ w
    d = np.abs(got - ref)
    # within the float path's flux tolerance (1e-6) by a factor of two
    assert d.max() <= 5e-7, (d.max(), z[np.argmax(d)])

