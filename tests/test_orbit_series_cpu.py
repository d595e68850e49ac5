"""The float path takes the subsamples' sky positions from power series
about each exposure's centre (one Kepler solve per exposure instead of one
per subsample, Sect. 3.2's supersampling).  Built here for the host in
double, the series must stay within the Cauchy bound that selects it, against
the oracle's z (one solve per subsample), and the selection must accept the
long-cadence workload."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    so = tmp_path_factory.mktemp("series") / "libseries.so"
    subprocess.run(["g++", "-O2", "-shared", "-fPIC", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
                    "-x", "c++", os.path.join(HERE, "orbit_series_host.cpp"), "-o", str(so)], check=True)
    L = ctypes.CDLL(str(so))
    dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    L.series_z64.argtypes = [ctypes.c_int, dp] + [ctypes.c_double] * 7 + [ctypes.c_int, ctypes.c_int, dp, dp]
    L.series_z64.restype = ctypes.c_int
    return L


def _series(lib, tc, t0, P, aR, b, e, w, texp, nss, order=6):
    z = np.zeros(len(tc) * nss)
    bound = np.zeros(1)
    assert lib.series_z64(len(tc), np.ascontiguousarray(tc), t0, P, aR, b, e, w, texp, nss, order, z,
                          bound) == 0
    return z, bound[0]


def _subsample_times(tc, texp, nss):
    return (tc[:, None] + ((np.arange(nss) + 0.5) / nss - 0.5)[None, :] * texp).reshape(-1)


@pytest.mark.parametrize("order", [4, 5, 6])
def test_series_within_its_bound(lib, oracle, order):
    """Random orbits (e up to 0.9, a/R* 2-40, P 0.5-30 d, exposures up to
    0.15 d, 4-16 subsamples), each order the kernels use: wherever the bound
    is finite, the series' z is within it (plus double rounding) at every
    subsample near conjunction."""
    rng = np.random.default_rng(11)
    checked = tight = 0
    for _ in range(150):
        aR = rng.uniform(2, 40); b = rng.uniform(0, 1.1); w = rng.uniform(0, 2 * np.pi)
        e = rng.choice([0.0, rng.uniform(0, 0.3), rng.uniform(0, 0.9)])
        P = rng.uniform(0.5, 30); texp = rng.uniform(0, 0.15); nss = int(rng.integers(4, 17))
        tc = np.linspace(-0.05, 0.05, 21) * P
        z, bound = _series(lib, tc, 0.0, P, aR, b, e, w, texp, nss, order)
        if bound >= 1e299:
            continue
        ref = oracle.orbit_z(_subsample_times(tc, texp, nss), 0.0, P, aR, b, e, w)
        err = np.abs(z - ref).max()
        assert err <= bound + 1e-11 * (1 + aR), (aR, b, e, w, P, texp, nss, err, bound)
        checked += 1
        tight += bound <= 3e-8
    assert checked >= 100 and tight >= 40


def test_series_selected_for_long_cadence(lib, oracle):
    """The long-cadence batch's orbits (e <= 0.3, a/R* 5-30, P = 3 d, 29.4 min
    exposures, 10 subsamples) all pass the 3e-8 selection at order 5, and the
    order-5 series stays within that bound of the oracle's z there."""
    from paper_1504_07433_amd import workloads as W
    bt = W.config2(n_vec=256, n_windows=1)
    tc = np.linspace(-0.15, 0.15, 61)
    for i in range(0, 256, 8):
        args = (bt["t0"][i], bt["P"][i], bt["aR"][i], bt["b"][i], bt["e"][i], bt["w"][i])
        z, bound = _series(lib, tc, *args, bt["t_exp"][i], int(bt["nss"][i]), 5)
        assert bound <= 3e-8
        ref = oracle.orbit_z(_subsample_times(tc, bt["t_exp"][i], int(bt["nss"][i])), *args)
        assert np.abs(z - ref).max() <= bound + 1e-11 * (1 + bt["aR"][i])


def test_series_bound_rejects_branch_point(lib):
    """An exposure wider than the distance to Kepler's branch point (e = 0.9,
    rho_e = 0.031 in mean anomaly) gets no finite bound."""
    z, bound = _series(lib, np.array([0.0]), 0.0, 3.0, 10.0, 0.3, 0.9, 1.0, 0.05, 8)
    assert bound >= 1e299
