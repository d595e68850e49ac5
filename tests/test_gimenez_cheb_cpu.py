"""The float path evaluates the Gimenez sums sum_j T_j P_j^(0,nu+1)(x)
(Sect. 2.1) in Chebyshev form: the per-band Jacobi coefficients are converted
with the Chebyshev coefficients of the Jacobi polynomials, then summed by
Clenshaw's Chebyshev recurrence.  Built here for the host in double, that
construction must give the oracle's alpha_n (same truncation npol)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    so = tmp_path_factory.mktemp("gimcheb") / "libgimcheb.so"
    subprocess.run(["g++", "-O2", "-shared", "-fPIC", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
                    "-x", "c++", os.path.join(HERE, "gimenez_cheb_host.cpp"), "-o", str(so)], check=True)
    L = ctypes.CDLL(str(so))
    dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    L.gim_cheb_alpha64.argtypes = [dp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, dp]
    L.gim_cheb_alpha64.restype = ctypes.c_int
    L.gim_fold_loss64.argtypes = [dp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, dp, dp]
    L.gim_fold_loss64.restype = ctypes.c_int
    return L


@pytest.mark.parametrize("npol", [1, 2, 5, 20, 50, 200])
def test_chebyshev_form_matches_oracle(lib, oracle, npol):
    nldc = 4
    for k in (0.03, 0.1, 0.3, 0.7):
        z = np.ascontiguousarray(np.linspace(0.0, 1.0 + k, 157)[:-1])
        got = np.zeros((len(z), nldc + 1))
        assert lib.gim_cheb_alpha64(z, len(z), k, nldc, npol, got) == 0
        ref = np.array([oracle.gimenez_alpha(zz, k, nldc, npol) for zz in z])
        scale = np.abs(ref).max()
        assert np.abs(got - ref).max() <= 1e-11 * max(scale, 1e-3), (npol, k, np.abs(got - ref).max(), scale)


@pytest.mark.parametrize("npol,nldc", [(1, 1), (5, 2), (20, 4), (50, 2), (50, 3), (200, 4)])
def test_folded_form_matches_oracle(lib, oracle, npol, nldc):
    """The batch's float path folds a band's limb-darkening weights and the
    factors (1 - c^2)^(nu+1) into two Chebyshev series E, O: the band's loss
    sum_n w_n alpha_n = E(x) + sqrt(1 - c^2) O(x)."""
    rng = np.random.default_rng(npol + nldc)
    for k in (0.03, 0.1, 0.3, 0.7):
        w = np.ascontiguousarray(rng.uniform(-1, 1, nldc + 1))
        z = np.ascontiguousarray(np.linspace(0.0, 1.0 + k, 157)[:-1])
        got = np.zeros(len(z))
        assert lib.gim_fold_loss64(z, len(z), k, nldc, npol, w, got) == 0
        ref = np.array([np.dot(w, oracle.gimenez_alpha(zz, k, nldc, npol)) for zz in z])
        scale = np.abs(ref).max()
        assert np.abs(got - ref).max() <= 1e-11 * max(scale, 1e-3), (npol, nldc, k, np.abs(got - ref).max(), scale)
