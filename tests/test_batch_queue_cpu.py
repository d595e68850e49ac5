"""The persistent batch kernel's work list, built for the host: the tile plan
(longest tiles first, per-light-curve tile lists for the likelihood's
reduction) and the tile queue's pop protocol, run by every wave of a
persistent grid in random interleavings with the same next_tile the kernel
runs.  Each tile must be taken exactly once, every wave must stop after its
own tiles plus one dry pop per sub-queue, and the per-light-curve sums of the
per-tile partials must equal the direct sums."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    so = tmp_path_factory.mktemp("queue") / "libqueue.so"
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I/opt/rocm/include",
                    "-D__HIP_PLATFORM_AMD__", "-x", "c++", os.path.join(HERE, "batch_queue_host.cpp"),
                    "-o", str(so)], check=True)
    L = ctypes.CDLL(str(so))
    p64 = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
    p32 = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    L.queue_check.argtypes = [ctypes.c_int32, p64, p32, p32, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              ctypes.c_uint, p64]
    L.queue_check.restype = ctypes.c_int
    return L


def _check(lib, b, tile_e, workgroups, seed):
    stats = np.zeros(3, np.int64)
    rc = lib.queue_check(len(b["t_count"]), np.ascontiguousarray(b["t_count"], np.int64),
                         np.ascontiguousarray(b["nss"], np.int32), np.ascontiguousarray(b["band_off"], np.int32),
                         tile_e, workgroups, 4, seed, stats)
    assert rc == 0, f"check {rc} failed (tile {tile_e}, {workgroups} workgroups, seed {seed})"
    return stats


@pytest.mark.parametrize("tile_e", [64, 256, 1024])
def test_queue_takes_every_tile_once(lib, tile_e):
    """The likelihood test's batch (24 uneven light curves, one with 19
    subsamples) and a larger uneven batch, with as many workgroups as the GPU
    runs (1536) and with fewer than there are sub-queues."""
    from paper_1504_07433_amd import workloads as W
    small = W.config4(n_lc=24, n_min=100, n_max=2000)
    small["nss"][3] = 19
    large = W.config4(n_lc=400, n_min=500, n_max=20000)
    for b in (small, large):
        for wg in (1536, 5, 1):
            for seed in (1, 2):
                st = _check(lib, b, tile_e, wg, seed)
                assert st[1] <= st[0] + 4 * wg * 8


def test_empty_and_bandless_light_curves(lib):
    """Light curves with no exposures or no bands get no tile; a batch with no
    tile at all lets every wave stop after one dry pop per sub-queue."""
    b = {"t_count": np.array([0, 300, 50, 0], np.int64), "nss": np.array([1, 3, 2, 1], np.int32),
         "band_off": np.array([0, 2, 2, 5, 5], np.int32)}
    st = _check(lib, b, 64, 16, 3)
    assert st[0] == 1 and st[2] <= 8 + 1   # only light curve 2 has both bands and exposures
    none = {"t_count": np.array([0, 10], np.int64), "nss": np.array([1, 1], np.int32),
            "band_off": np.array([0, 1, 1], np.int32)}
    st = _check(lib, none, 64, 16, 4)
    assert st[0] == 0 and st[2] == 8
