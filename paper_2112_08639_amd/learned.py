"""Learned SCF start density (libdk calls only).

A per-grid-point network maps Gaussian descriptors of the atomic environment
to the density: descriptors d_k(x) (K widths, geometric between w_min and
w_max), standardised with training-set statistics, pass through
n_in -> hidden (x layers, SiLU) -> 1 (softplus) to y ~ rho / rho_bar
(rho_bar = N_e / volume); the start density is rho_0 = N_e y / int y.
Training: MSE on rho / rho_bar over random batches of (snapshot, point)
pairs, Adam.  The forward and backward passes, Adam and the descriptor
kernels all run in libdk; this module holds the buffers and the schedule.
Random draws (initial weights, batch indices) come from seeded host
generators and are passed in.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from . import _lib as L


@dataclass
class MlpConfig:
    n_w: int = 32
    w_min: float = 0.5
    w_max: float = 4.0
    hidden: int = 64
    layers: int = 3
    steps: int = 2000
    batch: int = 65536
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    seed_init: int = 5000
    seed_batch: int = 6000
    mode: int = L.DK_MLP_BF16

    def widths(self) -> np.ndarray:
        return self.w_min * (self.w_max / self.w_min) ** (np.arange(self.n_w) / (self.n_w - 1))

    def shape(self) -> L.MlpShape:
        return L.MlpShape(self.n_w, self.hidden, self.layers)


def init_params(cfg: MlpConfig) -> np.ndarray:
    """Uniform(-1/sqrt(n_in), 1/sqrt(n_in)) per layer (weights then biases), seeded."""
    rng = np.random.Generator(np.random.PCG64(cfg.seed_init))
    dims = [cfg.n_w] + [cfg.hidden] * cfg.layers + [1]
    parts = []
    for i in range(len(dims) - 1):
        bound = 1.0 / math.sqrt(dims[i])
        parts.append(rng.uniform(-bound, bound, dims[i + 1] * dims[i]))
        parts.append(rng.uniform(-bound, bound, dims[i + 1]))
    return np.concatenate(parts)


@dataclass
class TrainLog:
    losses: List[float] = field(default_factory=list)
    ms_per_step: float = 0.0


class LearnedStart:
    def __init__(self, h, n_grid: int, volume: float, n_e: float, cfg: Optional[MlpConfig] = None,
                 max_snapshots: int = 0, device: int = 0):
        self.h = h
        self.cfg = cfg or MlpConfig()
        self.n_grid = n_grid
        self.rho_bar = n_e / volume
        self.n_e = n_e
        self.dev = torch.device("cuda", device)
        c = self.cfg
        self.shape = c.shape()
        self.n_params = L.dk_mlp_param_count(self.shape)
        f32 = dict(dtype=torch.float32, device=self.dev)
        self.params = torch.as_tensor(init_params(c), **f32).contiguous()
        assert self.params.numel() == self.n_params
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.step_t = 0
        self.ws = torch.empty(L.dk_mlp_workspace_bytes(self.shape, c.batch) // 4 + 64, **f32)
        self.u = torch.empty(c.n_w * c.batch, **f32)
        self.t = torch.empty(c.batch, **f32)
        self.desc = torch.empty(max(max_snapshots, 1) * n_grid * c.n_w, **f32)
        self.rho = torch.empty(max(max_snapshots, 1) * n_grid, dtype=torch.float64, device=self.dev)
        self.count = 0
        self.mean = torch.zeros(c.n_w, dtype=torch.float64, device=self.dev)
        self.inv_std = torch.ones_like(self.mean)
        self.rng = np.random.Generator(np.random.PCG64(c.seed_batch))

    def descriptors(self, positions, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.n_grid * self.cfg.n_w, dtype=torch.float32, device=self.dev)
        L.dk_descriptors(self.h, positions, self.cfg.widths(), out)
        return out

    def add_snapshot(self, positions, rho: torch.Tensor) -> None:
        """Store one training pair: descriptors of `positions` and its converged density."""
        s = self.count
        ng, K = self.n_grid, self.cfg.n_w
        assert (s + 1) * ng * K <= self.desc.numel(), "snapshot capacity exceeded"
        self.descriptors(positions, self.desc[s * ng * K:(s + 1) * ng * K])
        self.rho[s * ng:(s + 1) * ng].copy_(rho)
        self.count += 1

    def fit(self, steps: Optional[int] = None, log_every: int = 0) -> TrainLog:
        c = self.cfg
        steps = c.steps if steps is None else steps
        n_pts = self.count * self.n_grid
        L.dk_descriptor_stats(self.h, self.desc, n_pts, c.n_w, self.mean, self.inv_std)
        idx = torch.empty(c.batch, dtype=torch.int64, device=self.dev)
        log = TrainLog()
        torch.cuda.synchronize(self.dev)
        import time
        t0 = time.perf_counter()
        for _ in range(steps):
            idx.copy_(torch.from_numpy(self.rng.integers(0, n_pts, c.batch, dtype=np.int64)))
            L.dk_mlp_gather(self.h, self.desc, self.rho, c.n_w, idx, c.batch, self.mean,
                            self.inv_std, 1.0 / self.rho_bar, self.u, self.t)
            loss = L.dk_mlp_loss_grad(self.h, self.shape, c.mode, self.params, self.u, self.t,
                                      c.batch, self.grad, self.ws)
            self.step_t += 1
            L.dk_adam_step(self.h, self.params, self.m, self.v, self.grad, self.step_t, c.lr,
                           c.beta1, c.beta2, c.eps)
            log.losses.append(loss)
            if log_every and self.step_t % log_every == 0:
                print(f"mlp step {self.step_t} loss {loss:.4e}", flush=True)
        torch.cuda.synchronize(self.dev)
        log.ms_per_step = (time.perf_counter() - t0) * 1e3 / max(steps, 1)
        return log

    def for_cell(self, h, n_grid: int, volume: float, n_e: float) -> "LearnedStart":
        """The trained network as a predictor on another cell of the same species and
        grid spacing (the descriptors are local): descriptors, grid and normalisation
        come from that cell's context `h`; weights and descriptor statistics are
        copied from this one."""
        other = LearnedStart(h, n_grid, volume, n_e, self.cfg, max_snapshots=0,
                             device=self.dev.index or 0)
        other.params.copy_(self.params)
        other.mean.copy_(self.mean)
        other.inv_std.copy_(self.inv_std)
        return other

    def predict(self, positions, rho_out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Start density (device FP64, N_grid) for the atoms at `positions`."""
        d = self.descriptors(positions)
        if rho_out is None:
            rho_out = torch.empty(self.n_grid, dtype=torch.float64, device=self.dev)
        L.dk_mlp_density(self.h, self.shape, self.cfg.mode, self.params, d, self.mean,
                         self.inv_std, self.n_e, rho_out, self.ws)
        return rho_out
