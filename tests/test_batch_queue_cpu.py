"""The persistent batch kernel's work list, built for the host: the tile plan
(longest tiles first, the last ones split into runs of bands, per-light-curve
tile lists for the likelihood's reduction) and the tile queue's pop protocol, run by every wave of a
persistent grid in random interleavings with the same next_tile the kernel
runs.  Every (exposure, band) element must lie in exactly one tile, each tile
must be taken exactly once, every wave must stop after its own tiles plus one
dry pop per sub-queue, and the per-light-curve sums of the per-tile partials
must equal the direct sums."""
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
    L.queue_check.argtypes = [ctypes.c_int32, p64, p32, p32, ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                              ctypes.c_int, ctypes.c_uint, p64]
    L.queue_check.restype = ctypes.c_int
    return L


def _check(lib, b, tile_e, workgroups, seed, tail=0):
    stats = np.zeros(4, np.int64)
    rc = lib.queue_check(len(b["t_count"]), np.ascontiguousarray(b["t_count"], np.int64),
                         np.ascontiguousarray(b["nss"], np.int32), np.ascontiguousarray(b["band_off"], np.int32),
                         tile_e, tail, workgroups, 4, seed, stats)
    assert rc == 0, f"check {rc} failed (tile {tile_e}, tail {tail}, {workgroups} workgroups, seed {seed})"
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


@pytest.mark.parametrize("tile_e", [64, 512])
@pytest.mark.parametrize("tail", [1, 37, 600, 10 ** 9])
def test_split_tail_covers_every_element_once(lib, tile_e, tail):
    """The last `tail` tiles of light curves with 16 bands or more split into
    runs of at least 8 bands: every (exposure, band) element in exactly one
    tile, the pieces after the whole tiles, each part longest first, and the
    queue still hands out every tile once.  Batches: the uneven one (1-16 bands per light curve), a
    spectrophotometric-shaped one (64 bands, ragged lengths, 70 and 17
    bands), and a tail longer than the tile list."""
    from paper_1504_07433_amd import workloads as W
    uneven = W.config4(n_lc=60, n_min=100, n_max=3000)
    nb = np.array([64, 64, 70, 17, 15, 1, 64], np.int64)
    spectro = {"t_count": np.array([1500, 1437, 65, 200, 300, 129, 0], np.int64),
               "nss": np.array([1, 1, 3, 1, 2, 1, 1], np.int32),
               "band_off": np.concatenate([[0], np.cumsum(nb)]).astype(np.int32)}
    for b in (uneven, spectro):
        whole = _check(lib, b, tile_e, 16, 5)[0]
        st = _check(lib, b, tile_e, 16, 5, tail=tail)
        assert st[0] >= whole and st[3] >= min(tail, whole)
        _check(lib, b, tile_e, 1536, 6, tail=tail)


def test_split_pieces_of_a_wide_light_curve(lib):
    """One light curve of 64 bands and 130 exposures, tile 128, every tile in
    the tail: tiles of 128 and 2 exposures, each in four runs of 16 bands (8
    pieces); with 12 bands (fewer than 16) nothing is split."""
    b = {"t_count": np.array([130], np.int64), "nss": np.array([1], np.int32),
         "band_off": np.array([0, 64], np.int32)}
    st = _check(lib, b, 128, 4, 1, tail=100)
    assert st[0] == 8 and st[3] == 8
    b["band_off"] = np.array([0, 12], np.int32)
    st = _check(lib, b, 128, 4, 1, tail=100)
    assert st[0] == 2 and st[3] == 2
