"""Training driver of the learned surrogate of the Mandel & Agol functions.

The network maps (z, k) to the three limb-darkening-factored Mandel & Agol
functions.  Every arithmetic step runs in libpthip.so: exact targets
(pt_mlp_datagen), forward (pt_mlp_forward), loss and its gradient
(pt_mlp_loss_grad), backward (pt_mlp_backward) and Adam (pt_mlp_adam_step).
Python only sequences the calls and draws mini-batch indices.  After
training, pt_surrogate_set installs bf16 copies for the MFMA inference path
and lets the exact model build the trust map that decides where the network
may be used.  Checkpoints are .npz files (weights, Adam moments, step).
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import pthip, workloads as W


class Surrogate:
    def __init__(self, seed: int = 5, device: str = "cuda"):
        rng = np.random.default_rng(seed)
        self.device = device
        self.params = {}
        for n in pthip.MLP_NAMES:
            fan_in = pthip.MLP_SHAPES["W" + n[1]][1]
            v = rng.uniform(-1, 1, pthip.MLP_SHAPES[n]) / np.sqrt(fan_in)
            self.params[n] = torch.as_tensor(v, dtype=torch.float32, device=device).contiguous()
        self.grads = {n: torch.zeros_like(t) for n, t in self.params.items()}
        self.m = {n: torch.zeros_like(t) for n, t in self.params.items()}
        self.v = {n: torch.zeros_like(t) for n, t in self.params.items()}
        self.step = 0
        self.history = []

    # -- data -------------------------------------------------------------------------
    def make_data(self, n: int, seed: int = 5):
        """(z, k) pairs of the training recipe (inside the stellar disc, outside
        the fallback band of the inner contact) and the exact functions there."""
        zk = W.config5_training(seed=seed, n=n)
        zk64 = torch.as_tensor(zk, device=self.device)
        alpha = pthip.mlp_datagen(zk64)
        return zk64.float().contiguous(), alpha

    # -- training ---------------------------------------------------------------------
    def train(self, zk32, alpha, steps: int, batch: int = 65536, lr: float = 2e-3, lr_min: float = 1e-6,
              log_every: int = 500, seed: int = 0):
        g = torch.Generator(device=self.device)
        g.manual_seed(seed)
        n = zk32.shape[0]
        act = torch.empty((batch, 3, 128), dtype=torch.float32, device=self.device)
        dout = torch.empty((batch, 3), dtype=torch.float32, device=self.device)
        loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        t0 = time.perf_counter()
        for it in range(steps):
            idx = torch.randint(0, n, (batch,), device=self.device, generator=g)
            zb = zk32[idx].contiguous()
            ab = alpha[idx].contiguous()
            out = pthip.mlp_forward(self.params, zb, act)
            pthip.mlp_loss_grad(out, zb, ab, dout, loss)
            pthip.mlp_backward(self.params, zb, act, dout, self.grads)
            self.step += 1
            frac = it / max(1, steps - 1)
            lr_t = lr_min + 0.5 * (lr - lr_min) * (1 + np.cos(np.pi * frac))
            pthip.mlp_adam_step(self.params, self.grads, self.m, self.v, self.step, lr_t)
            if log_every and (it % log_every == 0 or it == steps - 1):
                self.history.append((self.step, float(loss.item()), time.perf_counter() - t0))
        torch.cuda.synchronize()
        return self.history

    def install(self, fallback_band: float = 1e-3, k_lo: float = 0.01, k_hi: float = 0.3) -> float:
        """Installs the network for PT_PREC_SURROGATE; returns the fraction of
        trust-map cells the exact model accepted."""
        return pthip.surrogate_set(self.params, fallback_band, k_lo, k_hi)

    # -- checkpoints ------------------------------------------------------------------
    def save(self, path: str):
        arr = {}
        for pre, d in (("w_", self.params), ("m_", self.m), ("v_", self.v)):
            for n, t in d.items():
                arr[pre + n] = t.cpu().numpy()
        arr["step"] = np.array(self.step)
        np.savez(path, **arr)

    def load(self, path: str):
        with np.load(path) as f:
            for pre, d in (("w_", self.params), ("m_", self.m), ("v_", self.v)):
                for n in d:
                    d[n].copy_(torch.as_tensor(f[pre + n], device=self.device))
            self.step = int(f["step"])
