"""Trains the Mandel-Agol surrogate on the GPU and writes a checkpoint.

    python -m paper_1504_07433_amd.train_surrogate --steps 60000 --out surrogate.npz

Training data: 1e7 (z, k) pairs inside the stellar disc, k ~ U(0.01, 0.3),
z/(1-k-1e-3) ~ U(0, 1), plus 20 % denser towards the inner contact; targets
are the exact functions from the library's double-precision kernel.
Forward, loss, backward and Adam all run in libpthip.so; one cosine learning
rate schedule from --lr to 1e-6 over the run.  Prints one progress line per
2000 steps.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import torch

from . import pthip
from .surrogate import Surrogate

DEFAULT_CKPT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "surrogate.npz")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=10_000_000)
    ap.add_argument("--steps", type=int, default=60000)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--out", default=DEFAULT_CKPT)
    ap.add_argument("--resume", default=None)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    s = Surrogate(seed=args.seed)
    if args.resume:
        s.load(args.resume)
    t0 = time.perf_counter()
    zk32, alpha = s.make_data(args.samples, seed=args.seed)
    torch.cuda.synchronize()
    print(json.dumps({"phase": "data", "rows": int(zk32.shape[0]), "s": time.perf_counter() - t0}), flush=True)
    chunk = 2000
    done = 0
    while done < args.steps:
        n = min(chunk, args.steps - done)
        # one cosine schedule over the whole run, continued across chunks
        lr_hi = args.lr * 0.5 * (1 + torch.cos(torch.tensor(3.14159265 * done / args.steps)).item())
        lr_lo = args.lr * 0.5 * (1 + torch.cos(torch.tensor(3.14159265 * (done + n) / args.steps)).item())
        hist = s.train(zk32, alpha, steps=n, batch=args.batch, lr=max(lr_hi, 1e-6), lr_min=max(lr_lo, 1e-6),
                       log_every=n, seed=args.seed + done)
        done += n
        print(json.dumps({"phase": "train", "step": s.step, "loss": hist[-1][1],
                          "s": time.perf_counter() - t0}), flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    s.save(args.out)
    frac = s.install()
    print(json.dumps({"phase": "done", "steps": s.step, "trusted_fraction": frac, "checkpoint": args.out,
                      "s": time.perf_counter() - t0}), flush=True)


if __name__ == "__main__":
    main()
