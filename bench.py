#!/usr/bin/env python3
"""Throughput of the transit-model hot path on one MI355X.

The metric is model points per second (parameter vector x passband x
exposure x subsample) at max |dF| <= 1e-5 against FP64, learned surrogate
against the plain model, on the spectrophotometric batch that the learned
surrogate is evaluated on: 1024 circular-orbit parameter vectors x 64
passbands (per-band k, u1, u2) x 1500 exposures, quadratic Mandel-Agol,
9.83e7 points per step, inputs resident in HBM.  On that batch the plain
float path, the plain FP64 path and the learned surrogate are timed on the
same inputs, and every output of the float and surrogate paths is compared
with the FP64 path's.  `value` is the faster of the plain float path and the
surrogate path among those within 1e-5 (config.path names it); a step is one
pt_lc_batch call of that path.

Side legs (under "paths"): the paper's tabulated model (Sect. 2.2.3) and the
Gimenez model on the same batch, the long-cadence batch (256 eccentric
vectors x 200,000 exposures x 10 subsamples) and the uneven batch (4096
light curves, one persistent launch), each with a roofline of its own.  Launch
shapes come from the tuned-shape cache written by pt_autotune when it has an
entry for a batch shape (--autotune re-tunes every leg and rewrites it).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
TUNE_CACHE = os.path.join(ROOT, "paper_1504_07433_amd", "data", "tune_cache.jsonl")
SURROGATE_CKPT = os.path.join(ROOT, "paper_1504_07433_amd", "data", "surrogate.npz")

# Algorithmic work per unit of the float path, in flops (FMA = 2, every other
# arithmetic instruction and each reciprocal / square root = 1), counted with
# the hardware flop counters on launches in which every lane does the same
# unit of work (bench.py --mode units; summary and command in
# profiles/unit_probes_flops.txt):
F_ORBIT_ECC = 86.0        # orbit of one in-transit point, e > 0: Kepler, z (float part)
F_ORBIT_CIRC = 40.0       # the same for e = 0
# The Mandel-Agol work per (point, band) is the batch kernel's own: the
# difference between the two-band and one-band probes (batch-in-2band and
# batch-in, batch-limb-2band and batch-limb).
F_MA_INSIDE = 135.0       # Mandel-Agol functions + limb darkening, z < 1 - k
F_MA_LIMB = 198.0         # the same, 1 - k < z < 1 + k
# Every point also pays the subsample offset of the mean anomaly and the
# accumulation (5 flops) and, per exposure, the FP64 phase and the flux (8);
# each further band of a point out of transit its accumulation and flux (2).
F_POINT, F_EXPOSURE, F_BAND_OUT = 5.0, 8.0, 2.0
# Light curves with 4..16 subsamples take the orbit from the per-exposure
# position series.  Their units are measured inside the batch kernel (probes
# batch-series-4 / -16 / -limb-16, one band, flops per point = A + B / nss):
# per in-transit point inside the disc or on the limb (series evaluation,
# Mandel-Agol, limb darkening, accumulation) and per exposure with an
# in-transit point (phase, one Kepler solve, series coefficients, flux).  The
# probes run at series order 4; order-5 light curves spend ~4 flops more per
# point and ~20 more per exposure, which the model does not charge.
F_SER_INSIDE = 146.0
F_SER_LIMB = 208.0
F_SER_EXPOSURE = 218.0
SERIES_NSS = (4, 16)
# MI355X published peaks.  The FP32 vector peak counts packed FP32 FMAs (two
# per lane per cycle); this build compiles with packed FP32 disabled, so the
# FP32 instructions it issues run at most at the non-packed rate, which is
# also the FP64 vector peak: 256 CU x 64 FMA lanes x 2 flops x 2.4 GHz.
PEAK_FP32 = 157.3e12
PEAK_NONPACKED = 78.6e12
PEAK_BF16_MFMA = 2.5e15
PEAK_VALU_ISSUE = 256 * 4 * 2.4e9 / 4   # wave64 VALU instructions per second
HBM_PEAK = 8.0e12
# MFMA work of one network evaluation per point: two 128 x 128 layers on
# v_mfma_f32_16x16x32_bf16 (the 2 -> 128 and 128 -> 3 layers run on the VALU),
# 2 x 128 x 128 x 2 flops; three bf16 products each with the hi/lo split (one
# with PT_MLP_SPLIT=0).
F_NET_MFMA = 2 * 128 * 128 * 2
NET_PRODUCTS = 1 if os.environ.get("PT_MLP_SPLIT") == "0" else 3
# Hardware counters of k_lc_batch<fp32, MA> per workload (profiles/
# k_lc_batch_fp32_ma_<workload>_counters.txt): wave64 VALU instructions per
# launch, FETCH_SIZE and WRITE_SIZE in KiB per launch.  HBM bytes = FETCH_SIZE
# x FETCH_SCALE + WRITE_SIZE x WRITE_SCALE, the factors being what the same
# counters read for an elementwise kernel that reads and writes 1 GiB
# (FETCH_SIZE 524309.7 KiB for 1 GiB read, WRITE_SIZE 1048576 KiB written).
COUNTERS = {
    "spectrophotometric": {"valu_insts": 1.56781e8, "fetch_kib": 95989.4, "write_kib": 456081.0},
    "long-cadence": {"valu_insts": 7.40083e8, "fetch_kib": 10963.7, "write_kib": 204913.0},
    "uneven": {"valu_insts": 6.17812e9, "fetch_kib": 410279.0, "write_kib": 2860780.0},
}
FETCH_SCALE, WRITE_SCALE = 1048576 / 524309.7, 1.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-side", action="store_true", help="skip the side legs")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the launch shape of every leg first and write the tuned-shape cache")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="tuned-shape cache read at start (and written by --autotune)")
    ap.add_argument("--mode", choices=("full", "kernel", "units"), default="full",
                    help="kernel: only the timed launches of one leg (for profilers); units: "
                         "divergence-free launches of each unit of work, for counting operations per unit")
    ap.add_argument("--kernel-model", choices=("ma", "ma_interp", "gimenez"), default="ma",
                    help="model timed by --mode kernel (ma_interp: tables over the batch's k range; "
                         "gimenez: npol = 50)")
    ap.add_argument("--kernel-prec", choices=("fp32", "fp64", "surrogate"), default="fp32",
                    help="precision timed by --mode kernel")
    ap.add_argument("--kernel-workload", choices=("spectrophotometric", "long-cadence", "uneven"),
                    default="spectrophotometric", help="workload timed by --mode kernel")
    return ap.parse_args()


def unit_probes():
    """Launches in which every lane takes the same path, so that hardware
    operation counters divided by the number of points give the operations
    per unit of work.  2^24 points each, two launches each:
      orbit-ecc   float orbit, e = 0.2, all points near conjunction (pt_orbit_z)
      orbit-circ  the same orbit with e = 0
      ma-inside   float Mandel-Agol, k = 0.1, z in (0, 1-k) (pt_ma_quad, 1 band)
      ma-limb     the same, z in (1-k, 1+k)
      gim-inside  float Gimenez, npol = 50, two coefficients, z in (0, 1-k)
      batch-cut   batch kernel, one light curve whose window holds no point
      batch-in    batch kernel, e = 0.2, every point inside the disc
      batch-limb  the same with b = 1, every point on the limb
      batch-in-2band, batch-limb-2band
                  the same with two bands (2^23 points, each in both bands):
                  the difference to the one-band launch is the Mandel-Agol
                  work per (point, band) of the batch kernel
      batch-series-4, batch-series-16
                  the same with 4 / 16 subsamples per exposure (0.01 d), the
                  orbit from the per-exposure position series
      batch-series-limb-16
                  the same with b = 1, every subsample on the limb
    and one elementwise kernel that reads 1 GiB and writes 1 GiB (the
    reference for the HBM byte counters)."""
    import torch
    from paper_1504_07433_amd import pthip, workloads as W
    n = 1 << 24

    def one_lc(b_imp, e, span, nss=1, t_exp=0.0, bands=1):
        ne = n // nss // bands
        b = W.config1()
        b["t"] = np.linspace(-span, span, ne)
        b["t_count"] = np.array([ne], np.int64)
        b["nss"] = np.array([nss], np.int32)
        b["t_exp"] = np.array([t_exp])
        b["b"] = np.array([b_imp]); b["e"] = np.array([e]); b["w"] = np.array([1.0])
        b["aR"] = np.array([10.0]); b["P"] = np.array([3.0]); b["t0"] = np.array([0.0])
        b["k"] = np.full(bands, 0.1); b["u"] = np.tile([[0.4, 0.2]], (bands, 1)); b["n_flux"] = ne * bands
        b["band_off"] = np.array([0, bands], np.int32)
        return b

    def report(name, out):
        torch.cuda.synchronize()
        fh = out.float().cpu().numpy().ravel()
        print(json.dumps({"probe": name, "points": n, "mean": float(fh.mean())}), flush=True)

    t = torch.linspace(-0.04, 0.04, n, dtype=torch.float64, device="cuda")
    for name, e in (("orbit-ecc", 0.2), ("orbit-circ", 0.0)):
        for _ in range(2):
            z = pthip.orbit_z(t, 0.0, 3.0, 10.0, 0.3, e, 1.0, prec="fp32")
        report(name, z)
    u = np.array([[0.4, 0.2]])
    for name, lo, hi in (("ma-inside", 0.005, 0.85), ("ma-limb", 0.905, 1.095)):
        zz = torch.linspace(lo, hi, n, dtype=torch.float64, device="cuda")
        for _ in range(2):
            f = pthip.ma_quad(zz, 0.1, u, prec="fp32")
        report(name, f)
    zz = torch.linspace(0.005, 0.85, n, dtype=torch.float64, device="cuda")
    for _ in range(2):
        f = pthip.gimenez(zz, 0.1, np.array([[0.8, -0.2]]), npol=50, prec="fp32")
    report("gim-inside", f)
    del zz, f, t, z
    for name, b in (("batch-cut", one_lc(1.5, 0.0, 0.04)), ("batch-in", one_lc(0.3, 0.2, 0.03)),
                    ("batch-in-2band", one_lc(0.3, 0.2, 0.03, bands=2)),
                    ("batch-limb", one_lc(1.0, 0.2, 0.01)), ("batch-limb-2band", one_lc(1.0, 0.2, 0.01, bands=2)),
                    ("batch-series-4", one_lc(0.3, 0.2, 0.025, 4, 0.01)),
                    ("batch-series-16", one_lc(0.3, 0.2, 0.025, 16, 0.01)),
                    ("batch-series-limb-16", one_lc(1.0, 0.2, 0.01, 16, 0.01))):
        db = pthip.DeviceBatch(b)
        for _ in range(2):
            f = pthip.lc_batch(db, "ma", prec="fp32")
        report(name, f)
        del db, f
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    torch.mul(x, 2.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "read+write 1 GiB"}), flush=True)


def timed(fn, steps, warmup):
    """Wall time and HIP-event time (torch's current stream, the stream the
    library launches on) of `steps` calls after `warmup` untimed ones."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, ev0.elapsed_time(ev1) / 1e3


def count_units(pt, batch):
    """Units of work of one launch, from z on the GPU (pt_orbit_z in FP64 per
    light curve over its subsample times): all orbit points, orbit points in
    transit for some band (eccentric and circular orbits apart), in-transit
    (band, point) pairs inside the disc and on the limb, out-of-transit
    (band, point) pairs; the same for light curves whose orbit comes from the
    per-exposure series (4..16 subsamples), plus their exposures holding an
    in-transit point."""
    import torch
    c = dict.fromkeys(("orbit_points", "orbit_points_ecc", "orbit_points_in_transit_ecc", "orbit_points_in_transit_circ",
                       "inside_points", "limb_points", "band_points_out", "series_points_in_transit",
                       "series_exposures_in_transit", "series_inside_points", "series_limb_points"), 0)
    for i in range(len(batch["t_start"])):
        b0, b1 = int(batch["band_off"][i]), int(batch["band_off"][i + 1])
        if b1 == b0:
            continue
        s, cnt, n = batch["t_start"][i], batch["t_count"][i], int(batch["nss"][i])
        t = torch.as_tensor(batch["t"][s:s + cnt], device="cuda")
        off = torch.as_tensor((np.arange(n) + 0.5) / n - 0.5, device="cuda") * float(batch["t_exp"][i])
        ts = (t[:, None] + off[None, :]).reshape(-1).contiguous()
        z = pt.orbit_z(ts, batch["t0"][i], batch["P"][i], batch["aR"][i], batch["b"][i],
                       batch["e"][i], batch["w"][i], prec="fp64")
        ks = torch.as_tensor(batch["k"][b0:b1], device="cuda")
        front = z >= 0
        tr = front & (z < 1 + ks.max())
        n_tr = int(tr.sum().item())
        ins = int((front[None, :] & (z[None, :] <= 1 - ks[:, None])).sum().item())
        lim = int((front[None, :] & (z[None, :] > 1 - ks[:, None]) & (z[None, :] < 1 + ks[:, None])).sum().item())
        c["orbit_points"] += ts.numel()
        if batch["e"][i] > 0:
            c["orbit_points_ecc"] += ts.numel()
        c["orbit_points_in_transit_ecc" if batch["e"][i] > 0 else "orbit_points_in_transit_circ"] += n_tr
        c["inside_points"] += ins
        c["limb_points"] += lim
        c["band_points_out"] += ts.numel() * (b1 - b0) - ins - lim
        if SERIES_NSS[0] <= n <= SERIES_NSS[1]:
            c["series_points_in_transit"] += n_tr
            c["series_exposures_in_transit"] += int(tr.reshape(-1, n).any(dim=1).sum().item())
            c["series_inside_points"] += ins
            c["series_limb_points"] += lim
    return c


def unit_flops(u, n_exposures):
    """Algorithmic flops of one launch of the float Mandel-Agol path from its
    units of work (count_units) and the per-unit figures above."""
    ser_in = u["series_points_in_transit"]
    orbit_in = u["orbit_points_in_transit_ecc"] + u["orbit_points_in_transit_circ"]
    ecc_share = u["orbit_points_in_transit_ecc"] / max(1, orbit_in)
    return ((u["orbit_points"] - ser_in) * F_POINT
            + (n_exposures - u["series_exposures_in_transit"]) * F_EXPOSURE
            + (orbit_in - ser_in) * (ecc_share * F_ORBIT_ECC + (1 - ecc_share) * F_ORBIT_CIRC)
            + (u["inside_points"] - u["series_inside_points"]) * F_MA_INSIDE
            + (u["limb_points"] - u["series_limb_points"]) * F_MA_LIMB
            + max(0, u["band_points_out"] - (u["orbit_points"] - orbit_in)) * F_BAND_OUT
            + u["series_inside_points"] * F_SER_INSIDE + u["series_limb_points"] * F_SER_LIMB
            + u["series_exposures_in_transit"] * F_SER_EXPOSURE)


# The survey's per-unit estimates of the same work (before counting): an
# orbit point 80 flops + 8 transcendentals with e > 0, 20 + 2 with e = 0; a
# Mandel-Agol (point, band) in transit 250 + 20; one out of transit 5.
S_ORBIT_ECC, S_ORBIT_CIRC, S_MA, S_OUT = 88.0, 22.0, 270.0, 5.0


def survey_flops(u):
    """Flops of one launch from the same units at the survey's estimates."""
    return (u["orbit_points_ecc"] * S_ORBIT_ECC + (u["orbit_points"] - u["orbit_points_ecc"]) * S_ORBIT_CIRC
            + (u["inside_points"] + u["limb_points"]) * S_MA + u["band_points_out"] * S_OUT)


def alu_roofline(pt, batch, workload, kernel_s):
    """Roofline object of k_lc_batch<fp32, MA> on a workload: algorithmic
    flops per launch / the launch's event-timed duration against the
    published FP32 vector peak (and the non-packed ceiling this build runs
    under); HBM bytes from the counter runs where they exist."""
    u = count_units(pt, batch)
    flops = unit_flops(u, int(batch["t_count"].sum()))
    achieved = flops / kernel_s
    hbm = batch["t"].nbytes + batch["n_flux"] * 4 + len(batch["t_start"]) * 8 * 8 + len(batch["k"]) * 3 * 8
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32, "traffic": None,
            "peak_nonpacked": PEAK_NONPACKED / 1e12, "frac_nonpacked": achieved / PEAK_NONPACKED,
            "kernel": "k_lc_batch<fp32, MA> (+ the window kernel)", "kernel_ms": kernel_s * 1e3,
            "algorithmic_flops_per_launch": flops, **u,
            "hbm_bytes_algorithmic": hbm, "hbm_frac": hbm / kernel_s / HBM_PEAK}
    # the same launch priced at the survey's per-unit estimates, for comparison
    sf = survey_flops(u)
    roof["survey_units"] = {"flops_per_launch": sf, "achieved": sf / kernel_s / 1e12,
                            "frac": sf / kernel_s / PEAK_FP32, "frac_nonpacked": sf / kernel_s / PEAK_NONPACKED}
    cnt = COUNTERS.get(workload)
    if cnt:
        roof["traffic"] = (cnt["fetch_kib"] * FETCH_SCALE + cnt["write_kib"] * WRITE_SCALE) * 1024.0
        roof["valu_issue_frac"] = cnt["valu_insts"] / kernel_s / PEAK_VALU_ISSUE
    return roof


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(batch, seconds=2.0, reps=5):
    """The oracle (C, -O2, OpenMP over (light curve, band)) on the first light
    curves of the headline batch, at all host threads and at one thread: the
    median of `reps` runs each, sample sizes set so that one run takes about
    `seconds` (one thread: half that)."""
    from oracle import oracle as O
    from paper_1504_07433_amd import workloads as W
    nthreads = O.num_threads(0)
    n_lc = len(batch["t_start"])

    def run(m, threads):
        sub = W.subset(batch, np.arange(m))
        t0 = time.perf_counter()
        O.lc_batch(sub, model=0, nthreads=threads)
        return time.perf_counter() - t0, W.n_points(sub), sub

    dt1, _, _ = run(1, nthreads)
    m_all = int(np.clip(round(seconds / max(dt1, 1e-4)), 1, n_lc))
    dt1s, _, _ = run(1, 1)
    m_one = int(np.clip(round(0.5 * seconds / max(dt1s, 1e-4)), 1, n_lc))
    res = {}
    for label, m, threads in (("all", m_all, nthreads), ("one", m_one, 1)):
        times = []
        for _ in range(reps):
            dt, pts, sub = run(m, threads)
            times.append(dt)
        items = int(np.diff(sub["band_off"]).sum())
        res[label] = (pts / float(np.median(times)), m, pts, items, float(np.median(times)))
    return {"value": res["all"][0], "unit": "points/s", "cores": nthreads, "kind": "oracle",
            "value_1thread": res["one"][0], "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "sample": f"first {res['all'][1]} light curves of {batch['name']} ({res['all'][2]:.3g} points, "
                      f"{res['all'][3]} (light curve, band) items, median of {reps} runs of {res['all'][4]:.2f} s "
                      f"at {nthreads} threads); 1 thread: first {res['one'][1]} light curves "
                      f"({res['one'][2]:.3g} points, median {res['one'][4]:.2f} s); FP64 quadratic Mandel-Agol"}


def max_dev(a, ref):
    """max |a - ref| over every output, on the GPU (NaN counts as a failure)."""
    d = (a.double() - ref).abs()
    if bool(d.isnan().any()):
        return float("nan")
    return float(d.max().item())


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the transit-model path runs on one GPU only; --gpus must be 1 "
                                   f"(got {args.gpus})"}))
        sys.exit(2)
    import torch
    from paper_1504_07433_amd import pthip, workloads as W
    torch.cuda.set_device(0)
    if args.mode == "units":
        unit_probes()
        return
    tuned = pthip.tune_load(args.tune_cache) if os.path.exists(args.tune_cache) and not args.autotune else 0
    sur = None
    if os.path.exists(SURROGATE_CKPT):
        from paper_1504_07433_amd.surrogate import Surrogate
        sur = Surrogate()
        sur.load(SURROGATE_CKPT)

    def prepare(fn, db, model, prec, out, npol=50):
        """Tunes the leg first under --autotune."""
        if args.autotune:
            rep = pthip.autotune(db, model, npol=npol, prec=prec, out=out)
            print(json.dumps({"autotune": model, "prec": prec, "best": rep["best"],
                              "default_ms": rep["default_ms"]}), file=sys.stderr, flush=True)
        return fn

    if args.mode == "kernel":
        # one leg, launches only (for profilers)
        kb = {"long-cadence": W.config2, "spectrophotometric": W.config3, "uneven": W.config4}[args.kernel_workload]()
        u = None
        if args.kernel_model == "gimenez":
            u = np.stack([kb["u"][:, 0] + 2 * kb["u"][:, 1], -kb["u"][:, 1]], 1)
        kdb = pthip.DeviceBatch(kb, u=u)
        kflux = torch.empty(kb["n_flux"], dtype=torch.float64 if args.kernel_prec == "fp64" else torch.float32,
                            device="cuda")
        if args.kernel_model == "ma_interp":
            pthip.ma_table_set(float(kb["k"].min()), float(kb["k"].max()), 256 if len(kb["k"]) <= 4096 else 16, 2048)
        if args.kernel_prec == "surrogate":
            sur.install()
        step = lambda: pthip.lc_batch(kdb, args.kernel_model, npol=50, prec=args.kernel_prec, out=kflux)
        wall, gpu_s = timed(step, args.steps, args.warmup)
        print(json.dumps({"mode": "kernel", "model": args.kernel_model, "prec": args.kernel_prec,
                          "workload": kb["name"], "ms_per_step": gpu_s / args.steps * 1e3,
                          "points_per_s": W.n_points(kb) * args.steps / gpu_s,
                          "launch_shape": pthip.launch_shape(kdb, args.kernel_model, npol=50,
                                                             prec=args.kernel_prec)}), flush=True)
        return

    # ---- headline: the spectrophotometric batch, plain float / FP64 / surrogate on the same inputs ----
    b3 = W.config3()
    d3 = pthip.DeviceBatch(b3)
    p3 = W.n_points(b3)
    f32 = torch.empty(b3["n_flux"], dtype=torch.float32, device="cuda")
    f64 = torch.empty(b3["n_flux"], dtype=torch.float64, device="cuda")
    fsu = torch.empty(b3["n_flux"], dtype=torch.float32, device="cuda")
    s64 = max(2, args.steps // 5)
    step32 = prepare(lambda: pthip.lc_batch(d3, "ma", prec="fp32", out=f32), d3, "ma", "fp32", f32)
    wall32, gpu32 = timed(step32, args.steps, args.warmup)
    step64 = prepare(lambda: pthip.lc_batch(d3, "ma", prec="fp64", out=f64), d3, "ma", "fp64", f64)
    wall64, gpu64 = timed(step64, s64, max(2, args.warmup // 4))
    legs = {
        "plain_fp32": {"points_per_s": p3 * args.steps / gpu32, "ms_per_step": gpu32 / args.steps * 1e3,
                       "wall_ms_per_step": wall32 / args.steps * 1e3, "steps": args.steps,
                       "max_abs_dF_vs_fp64_all_points": max_dev(f32, f64),
                       "launch_shape": pthip.launch_shape(d3, "ma", prec="fp32")},
        "plain_fp64": {"points_per_s": p3 * s64 / gpu64, "ms_per_step": gpu64 / s64 * 1e3,
                       "wall_ms_per_step": wall64 / s64 * 1e3, "steps": s64,
                       "launch_shape": pthip.launch_shape(d3, "ma", prec="fp64")},
    }
    if sur is not None:
        trusted = sur.install()
        stepsu = prepare(lambda: pthip.lc_batch(d3, "ma", prec="surrogate", out=fsu), d3, "ma", "surrogate", fsu)
        stepsu()
        pthip.surrogate_counters(reset=True)
        stepsu()
        torch.cuda.synchronize()
        net_pts, exact_pts = pthip.surrogate_counters(reset=True)
        wallsu, gpusu = timed(stepsu, s64, 2)
        ms_su = gpusu / s64
        legs["learned_surrogate"] = {
            "points_per_s": p3 * s64 / gpusu, "ms_per_step": ms_su * 1e3, "wall_ms_per_step": wallsu / s64 * 1e3,
            "steps": s64, "max_abs_dF_vs_fp64_all_points": max_dev(fsu, f64),
            "trust_map_fraction": trusted,
            "points_by_network": net_pts, "points_in_transit_exact": exact_pts,
            "network_share_of_in_transit_points": net_pts / max(1, net_pts + exact_pts),
            "mfma_roofline": {"bound": "mfma", "unit": "TFLOP/s", "peak": PEAK_BF16_MFMA / 1e12,
                              "algorithmic_flops_per_launch": net_pts * F_NET_MFMA,
                              "achieved": net_pts * F_NET_MFMA / ms_su / 1e12,
                              "frac": net_pts * F_NET_MFMA / ms_su / PEAK_BF16_MFMA,
                              "issued_mfma_flops_per_launch": net_pts * F_NET_MFMA * NET_PRODUCTS},
            "launch_shape": pthip.launch_shape(d3, "ma", prec="surrogate")}
        legs["surrogate_over_plain_fp32"] = legs["learned_surrogate"]["points_per_s"] / legs["plain_fp32"]["points_per_s"]
        legs["surrogate_over_plain_fp64"] = legs["learned_surrogate"]["points_per_s"] / legs["plain_fp64"]["points_per_s"]
    legs["plain_fp32_over_plain_fp64"] = legs["plain_fp32"]["points_per_s"] / legs["plain_fp64"]["points_per_s"]
    gate = 1e-5
    best = "plain_fp32"
    if sur is not None and legs["learned_surrogate"]["max_abs_dF_vs_fp64_all_points"] <= gate and \
            legs["learned_surrogate"]["points_per_s"] > legs["plain_fp32"]["points_per_s"]:
        best = "learned_surrogate"
    if not legs[best]["max_abs_dF_vs_fp64_all_points"] <= gate:
        print(json.dumps({"error": f"{best} exceeds max|dF| {gate} against the FP64 path", "legs": legs}))
        sys.exit(1)
    if best == "plain_fp32":
        value, ms, kernel_s = legs[best]["points_per_s"], gpu32 / args.steps * 1e3, gpu32 / args.steps
        roof = alu_roofline(pthip, b3, "spectrophotometric", kernel_s)
        dtype = "f32+f64"
    else:
        value, ms = legs[best]["points_per_s"], legs[best]["ms_per_step"]
        roof = dict(legs[best]["mfma_roofline"])
        roof["traffic"] = None
        dtype = "bf16+f32+f64"
    line = {
        "metric": "model points/sec (incl. supersamples) at max|dF|<=1e-5 vs FP64, surrogate vs plain",
        "value": value, "unit": "points/s", "n_gpus": 1, "steps": args.steps if best == "plain_fp32" else s64,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": b3["name"], "light_curves": 1024, "bands": 64, "exposures": 1500, "subsamples": 1,
                   "model": "quadratic Mandel-Agol", "path": best, "points_per_step": p3,
                   "surrogate_checkpoint": os.path.relpath(SURROGATE_CKPT, ROOT) if sur is not None else None,
                   "tuned_shapes_loaded": tuned},
        "roofline": roof,
        "legs": legs,
    }

    if not args.no_side:
        paths = {}
        # the paper's tabulated model (Sect. 2.2.3) on the same batch: shared (k, z) table
        pthip.ma_table_set(0.09, 0.11, 16, 2048)
        fi = torch.empty_like(f32)
        wi, gi = timed(prepare(lambda: pthip.lc_batch(d3, "ma_interp", prec="fp32", out=fi), d3, "ma_interp",
                               "fp32", fi), args.steps, args.warmup)
        paths["spectrophotometric_ma_interp_fp32"] = {
            "table": {"k_lo": 0.09, "k_hi": 0.11, "nk": 16, "nz": 2048},
            "points_per_s": p3 * args.steps / gi, "ms_per_step": gi / args.steps * 1e3,
            "max_abs_dF_vs_fp64_all_points": max_dev(fi, f64)}
        del fi
        ug = np.stack([b3["u"][:, 0] + 2 * b3["u"][:, 1], -b3["u"][:, 1]], 1)
        d3g = pthip.DeviceBatch(b3, u=ug)
        fg = torch.empty_like(f32)
        fg64 = torch.empty_like(f64)
        wg_, gg = timed(prepare(lambda: pthip.lc_batch(d3g, "gimenez", npol=50, prec="fp32", out=fg), d3g,
                                "gimenez", "fp32", fg), 20, 5)
        pthip.lc_batch(d3g, "gimenez", npol=50, prec="fp64", out=fg64)
        paths["spectrophotometric_gimenez50_fp32"] = {
            "points_per_s": p3 * 20 / gg, "ms_per_step": gg / 20 * 1e3,
            "max_abs_dF_vs_fp64_gimenez_all_points": max_dev(fg, fg64)}
        del d3g, fg, fg64
        # long-cadence batch: float path with its roofline, FP64, tabulated
        b2 = W.config2()
        d2 = pthip.DeviceBatch(b2)
        p2 = W.n_points(b2)
        g32 = torch.empty(b2["n_flux"], dtype=torch.float32, device="cuda")
        g64 = torch.empty(b2["n_flux"], dtype=torch.float64, device="cuda")
        w2, k2 = timed(prepare(lambda: pthip.lc_batch(d2, "ma", prec="fp32", out=g32), d2, "ma", "fp32", g32),
                       args.steps, args.warmup)
        w2d, k2d = timed(prepare(lambda: pthip.lc_batch(d2, "ma", prec="fp64", out=g64), d2, "ma", "fp64", g64),
                         s64, 5)
        k_lo, k_hi = float(b2["k"].min()), float(b2["k"].max())
        pthip.ma_table_set(k_lo, k_hi, 256, 2048)
        g2i = torch.empty_like(g32)
        w2i, k2i = timed(prepare(lambda: pthip.lc_batch(d2, "ma_interp", prec="fp32", out=g2i), d2, "ma_interp",
                                 "fp32", g2i), args.steps, args.warmup)
        paths["long_cadence"] = {
            "workload": b2["name"], "points": p2,
            "fp32": {"points_per_s": p2 * args.steps / k2, "ms_per_step": k2 / args.steps * 1e3,
                     "max_abs_dF_vs_fp64_all_points": max_dev(g32, g64),
                     "launch_shape": pthip.launch_shape(d2, "ma", prec="fp32"),
                     "roofline": alu_roofline(pthip, b2, "long-cadence", k2 / args.steps)},
            "fp64": {"points_per_s": p2 * s64 / k2d, "ms_per_step": k2d / s64 * 1e3},
            "ma_interp_fp32": {"table": {"k_lo": k_lo, "k_hi": k_hi, "nk": 256, "nz": 2048},
                               "points_per_s": p2 * args.steps / k2i, "ms_per_step": k2i / args.steps * 1e3,
                               "max_abs_dF_vs_fp64_all_points": max_dev(g2i, g64)}}
        paths["long_cadence"]["fp32_over_fp64"] = k2d / s64 / (k2 / args.steps)
        paths["long_cadence"]["interp_over_fp64"] = k2d / s64 / (k2i / args.steps)
        del d2, g32, g64, g2i
        # uneven batch in one persistent launch: float path with its roofline
        b4 = W.config4()
        d4 = pthip.DeviceBatch(b4)
        p4 = W.n_points(b4)
        f4 = torch.empty(b4["n_flux"], dtype=torch.float32, device="cuda")
        w4, k4 = timed(prepare(lambda: pthip.lc_batch(d4, "ma", prec="fp32", out=f4), d4, "ma", "fp32", f4), 10, 3)
        paths["uneven"] = {"workload": b4["name"], "points": p4, "points_per_s": p4 * 10 / k4,
                           "ms_per_step": k4 / 10 * 1e3, "launch_shape": pthip.launch_shape(d4, "ma", prec="fp32"),
                           "roofline": alu_roofline(pthip, b4, "uneven", k4 / 10)}
        del f4
        f464 = torch.empty(b4["n_flux"], dtype=torch.float64, device="cuda")
        pthip.lc_batch(d4, "ma", prec="fp64", out=f464)
        f4 = pthip.lc_batch(d4, "ma", prec="fp32")
        paths["uneven"]["max_abs_dF_vs_fp64_all_points"] = max_dev(f4, f464)
        del d4, f4, f464
        line["paths"] = paths
    if args.autotune:
        pthip.tune_save(args.tune_cache)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(b3)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
