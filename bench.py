#!/usr/bin/env python3
"""Throughput of the transit-model hot path on one MI355X.

A step is one pt_lc_batch call over the long-cadence batch: 256 eccentric
parameter vectors x 200,000 exposure times (100 transits) x 10 subsamples of
a 29.4-minute exposure, quadratic Mandel-Agol in the float path (orbit ->
z -> overlap functions -> limb darkening -> subsample mean), i.e. 5.12e8
model points per step with the inputs resident in HBM.

Prints one JSON line (see the keys below).  The FP64 path, the Gimenez model
on the spectrophotometric batch and (when installed) the surrogate are
timed on the side and reported under "paths".
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

# Algorithmic work per unit of the float path, in flops (FMA = 2, every other
# arithmetic instruction and each reciprocal / square root = 1), counted with
# the hardware flop counters on launches in which every lane does the same
# unit of work (bench.py --mode units; summary and command in
# profiles/unit_probes_flops.txt):
F_ORBIT_ECC = 86.0        # orbit of one in-transit point, e > 0: Kepler, z (float part)
F_MA_INSIDE = 214.6       # Mandel-Agol functions + limb darkening, z < 1 - k
F_MA_LIMB = 307.0         # the same, 1 - k < z < 1 + k
# Every point also pays the subsample offset of the mean anomaly and the
# accumulation (5 flops) and, per exposure, the FP64 phase and the flux (8).
F_POINT, F_EXPOSURE = 5.0, 8.0
# Light curves with 4..16 subsamples take the orbit from the per-exposure
# position series.  Their units are measured inside the batch kernel (probes
# batch-series-4 / -16 / -limb-16, one band, flops per point = A + B / nss):
# per in-transit point inside the disc or on the limb (series evaluation,
# Mandel-Agol, limb darkening, accumulation) and per exposure with an
# in-transit point (phase, one Kepler solve, series coefficients, flux).  The
# probes run at series order 4; order-5 light curves spend ~4 flops more per
# point and ~20 more per exposure, which the model does not charge.
F_SER_INSIDE = 176.0
F_SER_LIMB = 262.0
F_SER_EXPOSURE = 228.0
SERIES_NSS = (4, 16)
PEAK_ALU = 78.6e12        # 256 CU x 64 FMA lanes x 2 flops x 2.4 GHz (FP32 non-packed = FP64)
PEAK_VALU_ISSUE = 256 * 4 * 2.4e9 / 4   # wave64 VALU instructions per second
HBM_PEAK = 8.0e12
# From the counter runs of k_lc_batch<fp32, MA> on this workload
# (profiles/k_lc_batch_fp32_ma_long_cadence_counters.txt): wave64 VALU
# instructions per launch, and HBM bytes per launch from FETCH_SIZE and
# WRITE_SIZE (KiB) scaled by what the counters read for an elementwise kernel
# that reads and writes 1 GiB (FETCH_SIZE reads 524319 KiB for 1 GiB read,
# WRITE_SIZE 1048580 KiB for 1 GiB written).
VALU_INSTS_PER_LAUNCH = 8.71723e8
FETCH_KIB, WRITE_KIB = 10920.7, 204912.0
FETCH_SCALE, WRITE_SCALE = 1048576 / 524319, 1.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-side", action="store_true", help="skip the side paths")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--autotune", action="store_true", help="autotune the launch shape first")
    ap.add_argument("--mode", choices=("full", "kernel", "units"), default="full",
                    help="kernel: only the timed batch launches (for profilers); units: divergence-free "
                         "launches of each unit of work, for counting operations per unit")
    ap.add_argument("--kernel-model", choices=("ma", "ma_interp", "gimenez"), default="ma",
                    help="model timed by --mode kernel (ma_interp: tables over the batch's k range, "
                         "256 x 2048 nodes; gimenez: npol = 50)")
    ap.add_argument("--kernel-workload", choices=("long-cadence", "spectrophotometric", "uneven"),
                    default="long-cadence", help="workload timed by --mode kernel")
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

    def one_lc(b_imp, e, span, nss=1, t_exp=0.0):
        ne = n // nss
        b = W.config1()
        b["t"] = np.linspace(-span, span, ne)
        b["t_count"] = np.array([ne], np.int64)
        b["nss"] = np.array([nss], np.int32)
        b["t_exp"] = np.array([t_exp])
        b["b"] = np.array([b_imp]); b["e"] = np.array([e]); b["w"] = np.array([1.0])
        b["aR"] = np.array([10.0]); b["P"] = np.array([3.0]); b["t0"] = np.array([0.0])
        b["k"] = np.array([0.1]); b["u"] = np.array([[0.4, 0.2]]); b["n_flux"] = ne
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
    transit for some band, and in-transit (band, point) pairs inside the disc
    and on the limb; the same for light curves whose orbit comes from the
    per-exposure series (4..16 subsamples), plus their exposures holding an
    in-transit point."""
    import torch
    n_orbit = n_orbit_in = n_inside = n_limb = n_series_in = n_series_exp = n_ser_inside = n_ser_limb = 0
    for i in range(len(batch["t_start"])):
        s, c, n = batch["t_start"][i], batch["t_count"][i], int(batch["nss"][i])
        t = torch.as_tensor(batch["t"][s:s + c], device="cuda")
        off = torch.as_tensor((np.arange(n) + 0.5) / n - 0.5, device="cuda") * float(batch["t_exp"][i])
        ts = (t[:, None] + off[None, :]).reshape(-1).contiguous()
        z = pt.orbit_z(ts, batch["t0"][i], batch["P"][i], batch["aR"][i], batch["b"][i],
                       batch["e"][i], batch["w"][i], prec="fp64")
        n_orbit += ts.numel()
        ks = batch["k"][batch["band_off"][i]:batch["band_off"][i + 1]]
        tr = (z >= 0) & (z < 1 + float(ks.max()))
        n_tr = int(tr.sum().item())
        n_orbit_in += n_tr
        series = SERIES_NSS[0] <= n <= SERIES_NSS[1]
        if series:
            n_series_in += n_tr
            n_series_exp += int(tr.reshape(-1, n).any(dim=1).sum().item())
        for k in ks:
            k = float(k)
            ni = int(((z >= 0) & (z <= 1 - k)).sum().item())
            nl = int(((z > 1 - k) & (z < 1 + k)).sum().item())
            n_inside += ni
            n_limb += nl
            if series:
                n_ser_inside += ni
                n_ser_limb += nl
    return {"orbit_points": n_orbit, "orbit_points_in_transit": n_orbit_in,
            "inside_points": n_inside, "limb_points": n_limb,
            "series_points_in_transit": n_series_in, "series_exposures_in_transit": n_series_exp,
            "series_inside_points": n_ser_inside, "series_limb_points": n_ser_limb}


def cpu_baseline(batch, seconds):
    from oracle import oracle as O
    from paper_1504_07433_amd import workloads as W
    nthreads = O.num_threads(0)
    one = W.subset(batch, [0])
    t0 = time.perf_counter()
    O.lc_batch(one, model=0)
    dt1 = time.perf_counter() - t0
    m = int(np.clip(np.floor(seconds / max(dt1, 1e-3)), 1, len(batch["t_start"])))
    sub = W.subset(batch, np.arange(m))
    t0 = time.perf_counter()
    O.lc_batch(sub, model=0)
    dt = time.perf_counter() - t0
    pts = W.n_points(sub)
    return {"value": pts / dt, "unit": "points/s", "cores": nthreads, "kind": "oracle",
            "sample": f"first {m} of {len(batch['t_start'])} light curves of the same batch "
                      f"({pts:.3g} points, {dt:.1f} s, FP64 quadratic Mandel-Agol)"}


def sampled_error(pt, O, batch, flux, n=2000, model=0, npol=50, u=None, seed=0):
    import torch
    from tests.sampling import random_pairs, single_exposure_subset
    pairs = random_pairs(batch, n, seed=seed)
    sb, idx = single_exposure_subset(batch, pairs)
    if u is not None:
        sb["u"] = np.concatenate([u[batch["band_off"][l]:batch["band_off"][l + 1]] for l, _ in pairs])
    got = flux[torch.as_tensor(idx, device=flux.device)].cpu().numpy().astype(np.float64)
    ref = O.lc_batch(sb, model=model, npol=npol, u=None if u is None else sb["u"])
    return float(np.abs(got - ref).max())


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

    if args.mode == "kernel" and (args.kernel_model != "ma" or args.kernel_workload != "long-cadence"):
        # one model on one workload, launches only (for profilers)
        kb = {"long-cadence": W.config2, "spectrophotometric": W.config3, "uneven": W.config4}[args.kernel_workload]()
        u = None
        if args.kernel_model == "gimenez":
            u = np.stack([kb["u"][:, 0] + 2 * kb["u"][:, 1], -kb["u"][:, 1]], 1)
        kdb = pthip.DeviceBatch(kb, u=u)
        kflux = torch.empty(kb["n_flux"], dtype=torch.float32, device="cuda")
        if args.kernel_model == "ma_interp":
            pthip.ma_table_set(float(kb["k"].min()), float(kb["k"].max()), 256, 2048)
        step = lambda: pthip.lc_batch(kdb, args.kernel_model, npol=50, prec="fp32", out=kflux)
        wall, _ = timed(step, args.steps, args.warmup)
        print(json.dumps({"mode": "kernel", "model": args.kernel_model, "workload": kb["name"],
                          "ms_per_step": wall / args.steps * 1e3,
                          "points_per_s": W.n_points(kb) * args.steps / wall}), flush=True)
        return
    batch = W.config2()
    db = pthip.DeviceBatch(batch)
    points = W.n_points(batch)
    flux = torch.empty(batch["n_flux"], dtype=torch.float32, device="cuda")
    if args.autotune:
        rep = pthip.autotune(db, "ma", prec="fp32", out=flux)
        print(json.dumps({"autotune": rep}), file=sys.stderr, flush=True)
    step = lambda: pthip.lc_batch(db, "ma", prec="fp32", out=flux)
    wall, gpu_s = timed(step, args.steps, args.warmup)
    ms = wall / args.steps * 1e3
    value = points * args.steps / wall
    kernel_s = gpu_s / args.steps
    tile_e, wg = pthip.launch_shape(db, "ma", prec="fp32")
    if args.mode == "kernel":
        print(json.dumps({"mode": "kernel", "ms_per_step": ms, "points_per_s": value}), flush=True)
        return

    u = count_units(pthip, batch)
    n_in = u["inside_points"] + u["limb_points"]
    n_exposures = int(batch["t_count"].sum())
    flops = ((u["orbit_points"] - u["series_points_in_transit"]) * F_POINT
             + (n_exposures - u["series_exposures_in_transit"]) * F_EXPOSURE
             + (u["orbit_points_in_transit"] - u["series_points_in_transit"]) * F_ORBIT_ECC
             + (u["inside_points"] - u["series_inside_points"]) * F_MA_INSIDE
             + (u["limb_points"] - u["series_limb_points"]) * F_MA_LIMB
             + u["series_inside_points"] * F_SER_INSIDE + u["series_limb_points"] * F_SER_LIMB
             + u["series_exposures_in_transit"] * F_SER_EXPOSURE)
    achieved = flops / kernel_s
    hbm = (batch["t"].nbytes + batch["n_flux"] * 4 + 256 * 8 * 8)
    traffic = None
    if FETCH_KIB is not None and WRITE_KIB is not None:
        traffic = (FETCH_KIB * FETCH_SCALE + WRITE_KIB * WRITE_SCALE) * 1024.0
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_ALU / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK_ALU, "traffic": traffic,
            "kernel": "k_lc_batch<fp32, MA> (+ two small setup kernels)", "kernel_ms": kernel_s * 1e3,
            "algorithmic_flops_per_launch": flops, **u,
            "hbm_bytes_algorithmic": hbm, "hbm_frac": hbm / kernel_s / HBM_PEAK}
    if VALU_INSTS_PER_LAUNCH is not None:
        roof["valu_issue_frac"] = VALU_INSTS_PER_LAUNCH / kernel_s / PEAK_VALU_ISSUE
    line = {
        "metric": "model points/sec (incl. supersamples) at max|dF|<=1e-5 vs FP64, surrogate vs plain",
        "value": value, "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": batch["name"], "light_curves": 256, "exposures": int(batch["t_count"][0]),
                   "subsamples": 10, "bands": 1, "model": "quadratic Mandel-Agol", "precision": "fp32 path",
                   "points_per_step": points, "tile_exposures": tile_e, "workgroups": wg},
        "roofline": roof,
    }
    from oracle import oracle as O
    line["max_abs_dF_sampled"] = sampled_error(pthip, O, batch, flux)
    line["in_transit_fraction"] = n_in / points

    if not args.no_side:
        paths = {}
        flux64 = torch.empty(batch["n_flux"], dtype=torch.float64, device="cuda")
        s64 = max(2, args.steps // 5)
        w64, _ = timed(lambda: pthip.lc_batch(db, "ma", prec="fp64", out=flux64), s64, 5)
        paths["ma_fp64_same_workload"] = {"points_per_s": points * s64 / w64, "ms_per_step": w64 / s64 * 1e3,
                                          "max_abs_dF_sampled": sampled_error(pthip, O, batch, flux64, 1000)}
        paths["fp32_over_fp64_speedup"] = paths["ma_fp64_same_workload"]["ms_per_step"] / ms
        # the paper's tabulated model (Sect. 2.2.3) on the same workload: tables over
        # the batch's k range, error measured against the exact oracle
        k_lo, k_hi = float(batch["k"].min()), float(batch["k"].max())
        pthip.ma_table_set(k_lo, k_hi, 256, 2048)
        wi, _ = timed(lambda: pthip.lc_batch(db, "ma_interp", prec="fp32", out=flux), args.steps, args.warmup)
        paths["ma_interp_fp32_same_workload"] = {
            "table": {"k_lo": k_lo, "k_hi": k_hi, "nk": 256, "nz": 2048},
            "points_per_s": points * args.steps / wi, "ms_per_step": wi / args.steps * 1e3,
            "max_abs_dF_sampled_vs_exact": sampled_error(pthip, O, batch, flux)}
        paths["interp_over_plain_fp64"] = paths["ma_interp_fp32_same_workload"]["points_per_s"] / \
            paths["ma_fp64_same_workload"]["points_per_s"]
        paths["interp_over_plain_fp32"] = ms / paths["ma_interp_fp32_same_workload"]["ms_per_step"]
        b4 = W.config4()
        d4 = pthip.DeviceBatch(b4)
        p4 = W.n_points(b4)
        f4 = torch.empty(b4["n_flux"], dtype=torch.float32, device="cuda")
        w4, _ = timed(lambda: pthip.lc_batch(d4, "ma", prec="fp32", out=f4), 10, 3)
        te4, wg4 = pthip.launch_shape(d4, "ma", prec="fp32")
        paths["ma_fp32_uneven"] = {"workload": b4["name"], "points": p4, "points_per_s": p4 * 10 / w4,
                                   "ms_per_step": w4 / 10 * 1e3, "tile_exposures": te4, "workgroups": wg4,
                                   "max_abs_dF_sampled": sampled_error(pthip, O, b4, f4, 1000, seed=7)}
        del d4, f4
        b3 = W.config3()
        d3 = pthip.DeviceBatch(b3)
        ug = np.stack([b3["u"][:, 0] + 2 * b3["u"][:, 1], -b3["u"][:, 1]], 1)
        d3g = pthip.DeviceBatch(b3, u=ug)
        p3 = W.n_points(b3)
        f3 = torch.empty(b3["n_flux"], dtype=torch.float32, device="cuda")
        w3, _ = timed(lambda: pthip.lc_batch(d3, "ma", prec="fp32", out=f3), 20, 10)
        paths["ma_fp32_spectrophotometric"] = {"workload": b3["name"], "points_per_s": p3 * 20 / w3,
                                               "ms_per_step": w3 / 20 * 1e3}
        pthip.ma_table_set(0.09, 0.11, 16, 2048)
        w3i, _ = timed(lambda: pthip.lc_batch(d3, "ma_interp", prec="fp32", out=f3), 20, 10)
        paths["ma_interp_fp32_spectrophotometric"] = {
            "workload": b3["name"], "table": {"k_lo": 0.09, "k_hi": 0.11, "nk": 16, "nz": 2048},
            "points_per_s": p3 * 20 / w3i, "ms_per_step": w3i / 20 * 1e3,
            "max_abs_dF_sampled_vs_exact": sampled_error(pthip, O, b3, f3, 500, seed=3)}
        w3g, _ = timed(lambda: pthip.lc_batch(d3g, "gimenez", npol=50, prec="fp32", out=f3), 10, 3)
        paths["gimenez50_fp32_spectrophotometric"] = {
            "workload": b3["name"], "points_per_s": p3 * 10 / w3g, "ms_per_step": w3g / 10 * 1e3,
            "max_abs_dF_sampled": sampled_error(pthip, O, b3, f3, 200, model=1, u=ug)}
        ckpt = os.path.join(ROOT, "paper_1504_07433_amd", "data", "surrogate.npz")
        if os.path.exists(ckpt):
            from paper_1504_07433_amd.surrogate import Surrogate
            sur = Surrogate()
            sur.load(ckpt)
            frac = sur.install()
            f3s = torch.empty(b3["n_flux"], dtype=torch.float32, device="cuda")
            w3s, _ = timed(lambda: pthip.lc_batch(d3, "ma", prec="surrogate", out=f3s), 10, 3)
            paths["ma_surrogate_spectrophotometric"] = {
                "workload": b3["name"], "points_per_s": p3 * 10 / w3s, "ms_per_step": w3s / 10 * 1e3,
                "trusted_cell_fraction": frac,
                "max_abs_dF_sampled": sampled_error(pthip, O, b3, f3s, 300, seed=4)}
            paths["surrogate_over_plain_fp32"] = (w3 / 20) / (w3s / 10)
            paths["surrogate_over_plain_fp64_long_cadence_rate"] = (p3 * 10 / w3s) / paths["ma_fp64_same_workload"]["points_per_s"]
        line["paths"] = paths

    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(batch, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
