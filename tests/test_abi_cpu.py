"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol include/pthip.h declares, and rejects bad arguments on the host
before any launch (so nothing here touches a device)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def pt():
    from paper_1504_07433_amd import pthip
    return pthip


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "pthip.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pt_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(pt):
    lib = C.CDLL(pt.LIB_PATH)
    names = declared_symbols()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(pt.SYMBOLS) == names


def test_version(pt):
    assert pt.version().startswith("pthip")


def _batch_struct(pt, **over):
    from paper_1504_07433_amd import workloads as W
    b = W.config1()
    h = {k: np.ascontiguousarray(b[k]) for k in ("t_start", "t_count", "nss", "band_off", "flux_off")}
    h.update({k: v for k, v in over.items() if k in h})
    s = pt.PtBatch()
    s.n_lc, s.nldc, s.n_t, s.n_flux = 1, over.get("nldc", 2), len(b["t"]), over.get("n_flux", b["n_flux"])
    keep = []
    for k, v in h.items():
        v = np.ascontiguousarray(v)
        keep.append(v)
        setattr(s, k, C.c_void_p(v.ctypes.data))
    fake = C.c_void_p(0x1000)   # never dereferenced: validation fails first
    for k in ("t", "t0", "P", "aR", "b", "e", "w", "t_exp", "k", "u"):
        setattr(s, k, fake)
    return s, keep


@pytest.mark.parametrize("over,msg", [
    (dict(nss=np.array([0], np.int32)), "nss"),
    (dict(t_count=np.array([-1], np.int64)), "t_count"),
    (dict(t_start=np.array([5], np.int64)), "outside the pool"),
    (dict(n_flux=10), "outside n_flux"),
    (dict(band_off=np.array([1, 0], np.int32)), "band_off"),
    (dict(nldc=3), "nldc"),
])
def test_batch_validation(pt, over, msg):
    s, keep = _batch_struct(pt, **over)
    st = pt.lib.pt_lc_batch(C.byref(s), 0, 50, 1, C.c_void_p(0x2000), None)
    assert st == pt.PT_ERR_ARG
    assert msg in pt.lib.pt_last_error().decode()


def test_batch_validation_gimenez_npol(pt):
    s, keep = _batch_struct(pt, nldc=2)
    assert pt.lib.pt_lc_batch(C.byref(s), 1, 0, 1, C.c_void_p(0x2000), None) == pt.PT_ERR_ARG
    assert "npol" in pt.lib.pt_last_error().decode()
    assert pt.lib.pt_lc_batch(C.byref(s), 1, 513, 1, C.c_void_p(0x2000), None) == pt.PT_ERR_ARG


def test_overlapping_blocks_rejected(pt):
    from paper_1504_07433_amd import workloads as W
    b = W.config2(n_vec=3, n_windows=1)
    s = pt.PtBatch()
    arrs = dict(t_start=b["t_start"], t_count=b["t_count"], nss=b["nss"], band_off=b["band_off"],
                flux_off=np.array([0, 10, 4000], np.int64))
    keep = [np.ascontiguousarray(v) for v in arrs.values()]
    s.n_lc, s.nldc, s.n_t, s.n_flux = 3, 2, len(b["t"]), 10 ** 6
    for (k, _), v in zip(arrs.items(), keep):
        setattr(s, k, C.c_void_p(v.ctypes.data))
    for k in ("t", "t0", "P", "aR", "b", "e", "w", "t_exp", "k", "u"):
        setattr(s, k, C.c_void_p(0x1000))
    assert pt.lib.pt_lc_batch(C.byref(s), 0, 50, 1, C.c_void_p(0x2000), None) == pt.PT_ERR_ARG
    assert "overlap" in pt.lib.pt_last_error().decode()


@pytest.mark.parametrize("args,msg", [
    ((-1, 0.0, 3.0, 10.0, 0.3, 0.0, 0.0), "n ="),
    ((10, 0.0, -3.0, 10.0, 0.3, 0.0, 0.0), "period"),
    ((10, 0.0, 3.0, 0.0, 0.3, 0.0, 0.0), "aR"),
    ((10, 0.0, 3.0, 10.0, 0.3, 1.0, 0.0), "eccentricity"),
    ((10, 0.0, 3.0, 10.0, -0.1, 0.1, 0.0), "impact"),
    ((10, 0.0, 3.0, 2.0, 3.0, 0.0, 0.0), "cos i"),
])
def test_orbit_validation(pt, args, msg):
    n = args[0]
    st = pt.lib.pt_orbit_z(C.c_void_p(0x1000), n, *args[1:], 0, C.c_void_p(0x2000), None)
    assert st == pt.PT_ERR_ARG
    assert msg in pt.lib.pt_last_error().decode()


def test_model_validation(pt):
    L = pt.lib
    p = C.c_void_p(0x1000)
    assert L.pt_ma_quad(p, 10, 0.0, p, 1, 0, p, None) == pt.PT_ERR_ARG      # k <= 0
    assert L.pt_ma_quad(p, 10, 0.1, p, 0, 0, p, None) == pt.PT_ERR_ARG      # nb < 1
    assert L.pt_ma_quad(p, 10, 0.1, p, 1, 2, p, None) == pt.PT_ERR_ARG      # surrogate prec here
    assert L.pt_gimenez(p, 10, 0.1, p, 5, 1, 50, 0, p, None) == pt.PT_ERR_ARG   # nldc
    assert L.pt_gimenez(p, 10, 0.1, p, 2, 1, 0, 0, p, None) == pt.PT_ERR_ARG    # npol
    assert L.pt_gimenez(p, 10, 0.1, None, 2, 1, 50, 0, p, None) == pt.PT_ERR_ARG  # NULL u


def test_fault_injection_reports_hip_error(pt, monkeypatch):
    monkeypatch.setenv("PT_FAULT_INJECT", "hip")
    st = pt.lib.pt_orbit_z(C.c_void_p(0x1000), 10, 0.0, 3.0, 10.0, 0.3, 0.0, 0.0, 0,
                           C.c_void_p(0x2000), None)
    assert st == pt.PT_ERR_HIP
    assert "fault injected" in pt.lib.pt_last_error().decode()


def test_empty_batch_is_ok_without_device(pt):
    s = pt.PtBatch()
    s.n_lc, s.nldc = 0, 2
    assert pt.lib.pt_lc_batch(C.byref(s), 0, 50, 1, None, None) == pt.PT_OK


def test_noalloc_host_checks(pt):
    """pt_lc_batch_noalloc validates like pt_lc_batch, covers the quadratic
    Mandel-Agol model in FP32/FP64 only, and rejects a batch whose scratch
    exceeds its static array before any HIP call."""
    L = pt.lib
    s, keep = _batch_struct(pt)
    assert L.pt_lc_batch_noalloc(C.byref(s), 1, 1, C.c_void_p(0x2000), None) == pt.PT_ERR_UNSUPPORTED
    assert L.pt_lc_batch_noalloc(C.byref(s), 0, 2, C.c_void_p(0x2000), None) == pt.PT_ERR_UNSUPPORTED
    assert L.pt_lc_batch_noalloc(C.byref(s), 0, 1, None, None) == pt.PT_ERR_ARG
    assert "flux is NULL" in L.pt_last_error().decode()
    s, keep = _batch_struct(pt, nss=np.array([0], np.int32))
    assert L.pt_lc_batch_noalloc(C.byref(s), 0, 1, C.c_void_p(0x2000), None) == pt.PT_ERR_ARG
    assert "nss" in L.pt_last_error().decode()
    # 200,000 passbands need ~21 MB of band constants: over the 16 MiB array
    nb = 200_000
    s, keep = _batch_struct(pt, band_off=np.array([0, nb], np.int32), n_flux=nb * 1000)
    st = L.pt_lc_batch_noalloc(C.byref(s), 0, 1, C.c_void_p(0x2000), None)
    assert st == pt.PT_ERR_ARG
    msg = L.pt_last_error().decode()
    assert "too large for pt_lc_batch_noalloc" in msg and str(16 << 20) in msg


def test_noalloc_empty_batch_is_ok_without_device(pt):
    s = pt.PtBatch()
    s.n_lc, s.nldc = 0, 2
    assert pt.lib.pt_lc_batch_noalloc(C.byref(s), 0, 1, None, None) == pt.PT_OK


def test_tune_cache_round_trip_and_errors(pt, tmp_path):
    """The tuned-shape file: lines are read back as written, a malformed line
    is refused with its line number, and a missing file is an error."""
    good = tmp_path / "tune.jsonl"
    good.write_text(
        '{"key": "gfx950|m0 p0 q1 n2 l2 t10 f20|00:8;", "tile_exposures": 512, "workgroups": 1536, '
        '"cu": 256, "ms": 1.5, "default_ms": 1.6}\n'
        '{"key": "gfx950|m1 p50 q0 n3 l2 t10 f20|01:8;", "tile_exposures": 64, "workgroups": 256, '
        '"cu": 256, "ms": 0.25, "default_ms": 0.25}\n')
    assert pt.tune_load(str(good)) == 2
    out = tmp_path / "out.jsonl"
    pt.tune_save(str(out))
    lines = out.read_text().splitlines()
    keys = {ln.split('"key": "')[1].split('"')[0]: ln for ln in lines}
    assert "gfx950|m0 p0 q1 n2 l2 t10 f20|00:8;" in keys
    assert '"tile_exposures": 64, "workgroups": 256' in keys["gfx950|m1 p50 q0 n3 l2 t10 f20|01:8;"]
    bad = tmp_path / "bad.jsonl"
    bad.write_text(good.read_text().splitlines()[0] + "\n" + '{"key": "x", "tile_exposures": 0}\n')
    with pytest.raises(pt.PthipError, match="bad.jsonl:2"):
        pt.tune_load(str(bad))
    with pytest.raises(pt.PthipError, match="cannot read"):
        pt.tune_load(str(tmp_path / "missing.jsonl"))
    pt.release()
