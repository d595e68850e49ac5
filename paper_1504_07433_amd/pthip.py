"""Python binding of libpthip.so (the C ABI in include/pthip.h).

Argument marshalling only: every step of the model runs in the library's HIP
kernels.  Torch tensors provide device memory and the current stream.  If the
library is not built, importing this module raises ImportError; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpthip.so")

PT_OK, PT_ERR_ARG, PT_ERR_HIP, PT_ERR_NOMEM, PT_ERR_UNSUPPORTED = 0, 1, 2, 3, 4
PREC = {"fp64": 0, "fp32": 1, "surrogate": 2}
MODEL = {"ma": 0, "gimenez": 1, "ma_interp": 2, "ma_khat": 3, "gimenez_zinterp": 4}


class PthipError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"pthip status {status}: {msg}")
        self.status = status


class PtBatch(C.Structure):
    _fields_ = [
        ("n_lc", C.c_int32), ("nldc", C.c_int32), ("n_t", C.c_int64), ("n_flux", C.c_int64),
        ("t_start", C.c_void_p), ("t_count", C.c_void_p), ("nss", C.c_void_p),
        ("band_off", C.c_void_p), ("flux_off", C.c_void_p),
        ("t", C.c_void_p), ("t0", C.c_void_p), ("P", C.c_void_p), ("aR", C.c_void_p),
        ("b", C.c_void_p), ("e", C.c_void_p), ("w", C.c_void_p), ("t_exp", C.c_void_p),
        ("k", C.c_void_p), ("u", C.c_void_p),
    ]


class PtMlp(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4")]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built (python -m paper_1504_07433_amd.build)")
    L = C.CDLL(LIB_PATH)
    st = C.c_int
    vp, i64, i32, d, f = C.c_void_p, C.c_int64, C.c_int32, C.c_double, C.c_float
    sig = {
        "pt_version": (C.c_char_p, []),
        "pt_last_error": (C.c_char_p, []),
        "pt_release": (None, []),
        "pt_device_cu_count": (C.c_int, []),
        "pt_orbit_z": (st, [vp, i64, d, d, d, d, d, d, C.c_int, vp, vp]),
        "pt_ma_quad": (st, [vp, i64, d, vp, i32, C.c_int, vp, vp]),
        "pt_gimenez": (st, [vp, i64, d, vp, i32, i32, i32, C.c_int, vp, vp]),
        "pt_lc_batch": (st, [C.POINTER(PtBatch), C.c_int, i32, C.c_int, vp, vp]),
        "pt_ma_table_set": (st, [d, d, i32, i32, vp]),
        "pt_gimenez_zgrid_set": (st, [i32, i32]),
        "pt_lc_loglike": (st, [C.POINTER(PtBatch), C.c_int, i32, C.c_int, vp, vp, vp, vp]),
        "pt_autotune": (st, [C.POINTER(PtBatch), C.c_int, i32, C.c_int, vp, vp, C.c_char_p, C.c_size_t]),
        "pt_batch_launch_shape": (st, [C.POINTER(PtBatch), C.c_int, i32, C.c_int,
                                       C.POINTER(i32), C.POINTER(i32)]),
        "pt_lc_batch_noalloc": (st, [C.POINTER(PtBatch), C.c_int, C.c_int, vp, vp]),
        "pt_tune_save": (st, [C.c_char_p]),
        "pt_tune_load": (st, [C.c_char_p, C.POINTER(i32)]),
        "pt_mlp_datagen": (st, [vp, i64, vp, vp]),
        "pt_mlp_forward": (st, [C.POINTER(PtMlp), vp, i64, vp, vp, vp]),
        "pt_mlp_backward": (st, [C.POINTER(PtMlp), vp, vp, vp, i64, C.POINTER(PtMlp), vp]),
        "pt_mlp_adam_step": (st, [C.POINTER(PtMlp), C.POINTER(PtMlp), C.POINTER(PtMlp),
                                  C.POINTER(PtMlp), i64, f, f, f, f, vp]),
        "pt_mlp_loss_grad": (st, [vp, vp, vp, i64, vp, vp, vp]),
        "pt_surrogate_set": (st, [C.POINTER(PtMlp), d, d, d, vp]),
        "pt_surrogate_trusted_fraction": (d, []),
        "pt_surrogate_eval": (st, [vp, i64, vp, vp]),
        "pt_surrogate_counters": (st, [C.POINTER(C.c_uint64), i32]),
        "pt_mlp_infer": (st, [vp, i64, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


lib = _load()
SYMBOLS = [
    "pt_version", "pt_last_error", "pt_release", "pt_device_cu_count", "pt_orbit_z", "pt_ma_quad",
    "pt_gimenez", "pt_ma_table_set", "pt_gimenez_zgrid_set", "pt_lc_batch", "pt_lc_batch_noalloc", "pt_lc_loglike", "pt_autotune", "pt_batch_launch_shape",
    "pt_tune_save", "pt_tune_load", "pt_mlp_datagen",
    "pt_mlp_forward", "pt_mlp_backward", "pt_mlp_loss_grad", "pt_mlp_adam_step", "pt_surrogate_set",
    "pt_surrogate_trusted_fraction", "pt_surrogate_eval", "pt_surrogate_counters", "pt_mlp_infer",
]


def _check(status: int):
    if status != PT_OK:
        raise PthipError(status, lib.pt_last_error().decode())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        if x.numel() and not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return C.c_void_p(x.data_ptr()) if x.numel() else None
    if isinstance(x, np.ndarray):
        return C.c_void_p(x.ctypes.data) if x.size else None
    raise TypeError(type(x))


def _dev64(x, device="cuda"):
    if isinstance(x, torch.Tensor):
        assert x.dtype == torch.float64 and x.is_cuda, "expected a cuda float64 tensor"
        return x.contiguous()
    return torch.as_tensor(np.ascontiguousarray(x, np.float64), device=device)


def version() -> str:
    return lib.pt_version().decode()


def release():
    lib.pt_release()


def orbit_z(t, t0, P, aR, b, e, w, prec="fp64", out=None):
    t = _dev64(t)
    out = torch.empty_like(t) if out is None else out
    _check(lib.pt_orbit_z(_ptr(t), t.numel(), t0, P, aR, b, e, w, PREC[prec], _ptr(out), _stream()))
    return out


def ma_quad(z, k, u, prec="fp64", out=None):
    """u: [nb, 2] quadratic (u1, u2); returns flux [nb, n]."""
    z = _dev64(z)
    u = _dev64(u).reshape(-1, 2)
    nb = u.shape[0]
    out = torch.empty((nb, z.numel()), dtype=torch.float64, device=z.device) if out is None else out
    _check(lib.pt_ma_quad(_ptr(z), z.numel(), float(k), _ptr(u), nb, PREC[prec], _ptr(out), _stream()))
    return out


def gimenez(z, k, u, npol=50, prec="fp64", out=None):
    """u: [nb, nldc] general-law coefficients; returns flux [nb, n]."""
    z = _dev64(z)
    u = _dev64(u)
    if u.dim() == 1:
        u = u.reshape(1, -1)
    nb, nldc = u.shape
    out = torch.empty((nb, z.numel()), dtype=torch.float64, device=z.device) if out is None else out
    _check(lib.pt_gimenez(_ptr(z), z.numel(), float(k), _ptr(u), nldc, nb, npol, PREC[prec],
                          _ptr(out), _stream()))
    return out


class DeviceBatch:
    """A workload dict (see workloads.py) with its values copied to the GPU
    and its shape arrays kept on the host, as the C ABI expects."""

    VALUE_KEYS = ("t", "t0", "P", "aR", "b", "e", "w", "t_exp", "k")

    def __init__(self, batch, u=None, device="cuda"):
        self.host = {k: np.ascontiguousarray(batch[k]) for k in
                     ("t_start", "t_count", "nss", "band_off", "flux_off")}
        self.host["t_start"] = self.host["t_start"].astype(np.int64)
        self.host["t_count"] = self.host["t_count"].astype(np.int64)
        self.host["nss"] = self.host["nss"].astype(np.int32)
        self.host["band_off"] = self.host["band_off"].astype(np.int32)
        self.host["flux_off"] = self.host["flux_off"].astype(np.int64)
        self.dev = {k: torch.as_tensor(np.ascontiguousarray(batch[k], np.float64), device=device)
                    for k in self.VALUE_KEYS}
        uu = batch["u"] if u is None else u
        self.dev["u"] = torch.as_tensor(np.ascontiguousarray(uu, np.float64), device=device)
        self.nldc = int(self.dev["u"].shape[1]) if self.dev["u"].dim() == 2 else 2
        self.n_lc = len(self.host["t_start"])
        self.n_flux = int(batch["n_flux"])
        self.n_t = int(len(batch["t"]))

    def struct(self) -> PtBatch:
        h, d = self.host, self.dev
        s = PtBatch()
        s.n_lc, s.nldc, s.n_t, s.n_flux = self.n_lc, self.nldc, self.n_t, self.n_flux
        for k in ("t_start", "t_count", "nss", "band_off", "flux_off"):
            setattr(s, k, _ptr(h[k]))
        for k in self.VALUE_KEYS + ("u",):
            setattr(s, k, _ptr(d[k]))
        return s


def lc_batch(batch: DeviceBatch, model="ma", npol=50, prec="fp32", out=None):
    dtype = torch.float64 if prec == "fp64" else torch.float32
    if out is None:
        out = torch.empty(batch.n_flux, dtype=dtype, device=batch.dev["t"].device)
    s = batch.struct()
    _check(lib.pt_lc_batch(C.byref(s), MODEL[model], npol, PREC[prec], _ptr(out), _stream()))
    return out


def lc_batch_noalloc(batch: DeviceBatch, prec="fp32", out=None):
    """pt_lc_batch_noalloc: quadratic Mandel-Agol, no device allocation by the library."""
    dtype = torch.float64 if prec == "fp64" else torch.float32
    if out is None:
        out = torch.empty(batch.n_flux, dtype=dtype, device=batch.dev["t"].device)
    s = batch.struct()
    _check(lib.pt_lc_batch_noalloc(C.byref(s), MODEL["ma"], PREC[prec], _ptr(out), _stream()))
    return out


def ma_table_set(k_lo, k_hi, nk=128, nz=256):
    _check(lib.pt_ma_table_set(k_lo, k_hi, nk, nz, _stream()))


def gimenez_zgrid_set(n_in=50, n_limb=50):
    _check(lib.pt_gimenez_zgrid_set(n_in, n_limb))


def lc_loglike(batch: DeviceBatch, obs, sigma, model="ma", npol=50, prec="fp32", out=None):
    """Per-light-curve Gaussian log-likelihood of obs (pt_lc_batch layout)."""
    dtype = torch.float64 if prec == "fp64" else torch.float32
    assert obs.dtype == dtype and obs.is_cuda
    sigma = _dev64(sigma)
    if out is None:
        out = torch.empty(batch.n_lc, dtype=torch.float64, device=obs.device)
    s = batch.struct()
    _check(lib.pt_lc_loglike(C.byref(s), MODEL[model], npol, PREC[prec], _ptr(obs), _ptr(sigma), _ptr(out),
                             _stream()))
    return out


def autotune(batch: DeviceBatch, model="ma", npol=50, prec="fp32", out=None):
    dtype = torch.float64 if prec == "fp64" else torch.float32
    if out is None:
        out = torch.empty(batch.n_flux, dtype=dtype, device=batch.dev["t"].device)
    s = batch.struct()
    buf = C.create_string_buffer(1 << 16)
    _check(lib.pt_autotune(C.byref(s), MODEL[model], npol, PREC[prec], _ptr(out), _stream(), buf,
                           len(buf)))
    return json.loads(buf.value.decode())


def tune_save(path):
    """Writes every tuned launch shape to a JSON-lines file."""
    _check(lib.pt_tune_save(os.fsencode(path)))


def tune_load(path) -> int:
    """Merges a tuned-shape file into the library's cache; returns the number
    of entries read."""
    n = C.c_int32(0)
    _check(lib.pt_tune_load(os.fsencode(path), C.byref(n)))
    return n.value


def launch_shape(batch: DeviceBatch, model="ma", npol=50, prec="fp32"):
    s = batch.struct()
    te, wg = C.c_int32(), C.c_int32()
    _check(lib.pt_batch_launch_shape(C.byref(s), MODEL[model], npol, PREC[prec], C.byref(te), C.byref(wg)))
    return te.value, wg.value


# -- surrogate -------------------------------------------------------------------------

MLP_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4")
MLP_SHAPES = {"W1": (128, 2), "b1": (128,), "W2": (128, 128), "b2": (128,), "W3": (128, 128),
              "b3": (128,), "W4": (3, 128), "b4": (3,)}


def mlp_struct(params) -> PtMlp:
    """params: dict name -> contiguous float32 cuda tensor."""
    s = PtMlp()
    for n in MLP_NAMES:
        t = params[n]
        assert t.dtype == torch.float32 and t.is_cuda and t.is_contiguous() and tuple(t.shape) == MLP_SHAPES[n]
        setattr(s, n, _ptr(t))
    return s


def mlp_datagen(zk):
    zk = _dev64(zk).reshape(-1, 2)
    out = torch.empty((zk.shape[0], 3), dtype=torch.float64, device=zk.device)
    _check(lib.pt_mlp_datagen(_ptr(zk), zk.shape[0], _ptr(out), _stream()))
    return out


def mlp_forward(params, zk32, act=None):
    n = zk32.shape[0]
    out = torch.empty((n, 3), dtype=torch.float32, device=zk32.device)
    s = mlp_struct(params)
    _check(lib.pt_mlp_forward(C.byref(s), _ptr(zk32), n, _ptr(out), _ptr(act), _stream()))
    return out


def mlp_backward(params, zk32, act, dout, grads):
    s, g = mlp_struct(params), mlp_struct(grads)
    _check(lib.pt_mlp_backward(C.byref(s), _ptr(zk32), _ptr(act), _ptr(dout), zk32.shape[0], C.byref(g),
                               _stream()))


def mlp_loss_grad(out, zk32, alpha, dout, loss):
    _check(lib.pt_mlp_loss_grad(_ptr(out), _ptr(zk32), _ptr(alpha), out.shape[0], _ptr(dout), _ptr(loss),
                                _stream()))


def mlp_adam_step(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    sp, sg, sm, sv = (mlp_struct(x) for x in (params, grads, m, v))
    _check(lib.pt_mlp_adam_step(C.byref(sp), C.byref(sg), C.byref(sm), C.byref(sv), int(step), lr, beta1,
                                beta2, eps, _stream()))


def surrogate_set(params, fallback_band=1e-3, k_lo=0.01, k_hi=0.3):
    s = mlp_struct(params)
    _check(lib.pt_surrogate_set(C.byref(s), fallback_band, k_lo, k_hi, _stream()))
    return lib.pt_surrogate_trusted_fraction()


def surrogate_eval(zk):
    zk = _dev64(zk).reshape(-1, 2)
    out = torch.empty((zk.shape[0], 3), dtype=torch.float64, device=zk.device)
    _check(lib.pt_surrogate_eval(_ptr(zk), zk.shape[0], _ptr(out), _stream()))
    return out


def surrogate_counters(reset=False):
    """(points taken from the network, in-transit points evaluated exactly) by
    the surrogate batch path since installation or the last reset; waits for
    the device."""
    torch.cuda.synchronize()
    out = (C.c_uint64 * 2)()
    _check(lib.pt_surrogate_counters(out, 1 if reset else 0))
    return int(out[0]), int(out[1])


def mlp_infer(zk32):
    out = torch.empty((zk32.shape[0], 3), dtype=torch.float32, device=zk32.device)
    _check(lib.pt_mlp_infer(_ptr(zk32), zk32.shape[0], _ptr(out), _stream()))
    return out
