"""Sequencing of the libdk calls for one density evaluation.

Orchestration only: every array operation below is a libdk entry point (see
``_lib``); Python holds the device tensors and passes their pointers.  The
order is that of the density-kernel method (arXiv 2112.08639, Sec. 4):
orthonormalise and project the start block, then per filter pass take the
spectrum of H_s, filter, re-orthonormalise and project; finally the density
kernel with its Fermi level, the density, the energies and the forces.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L

PRECISIONS = {"fp64": L.DK_PREC_FP64, "mixed": L.DK_PREC_MIXED}


@dataclass(frozen=True)
class ProjectorModel:
    """Projector channels carried by every atom, (l, rc, gamma) each, and the
    relative truncation of the Gaussians; the tables are built on the device
    (dk_set_projector_model)."""
    channels: Sequence[Tuple[int, float, float]]
    cutoff_rel: float


class Context:
    """Owns a libdk context, its tables and its caller-side workspace tensor."""

    def __init__(self, problem, precision: str = "fp64", device: int = 0):
        L.load()
        self.precision = precision
        self.device = torch.device("cuda", device)
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        spec = problem.spec
        self.n_grid = problem.n_grid
        self.stream = torch.cuda.current_stream(self.device)
        nx, ny, nz = spec.shape
        lx, ly, lz = spec.cell
        self.h = L.dk_create(nx, ny, nz, lx, ly, lz, PRECISIONS[precision], device, self.stream)
        self.ws = None
        self.ws_key = None
        self.set_problem(problem)

    def set_problem(self, problem) -> None:
        self.problem = problem
        veff = torch.as_tensor(problem.veff, dtype=torch.float64, device=self.device).contiguous()
        L.dk_set_potential(self.h, veff)
        pr = problem.proj
        L.dk_set_projectors(self.h, pr["offsets"], pr["indices"], pr["values"], pr["gamma"],
                            pr["atom"], len(problem.positions))
        self.n_atoms = len(problem.positions)
        self.upper = L.dk_spectrum_upper_bound(self.h)

    def move_atoms(self, positions, projectors: ProjectorModel) -> None:
        """Projector tables for atoms at `positions` (host, n_atoms x 3), built on
        the device; the potential stays as set (a self-consistent loop replaces it)."""
        L.dk_set_projector_model(self.h, positions, projectors.channels, projectors.cutoff_rel)
        self.n_atoms = len(positions)
        self.upper = L.dk_spectrum_upper_bound(self.h)

    def ensure_workspace(self, n_s: int, n_pl: int) -> None:
        """Workspace for blocks of n_s columns and expansions up to degree n_pl.  The
        size also depends on the projector tables (the compact-support chunks of the
        integrals change when atoms move), so it is asked of libdk every time and the
        tensor grows, with 1/16 headroom, when the tables need more."""
        n_pl = n_pl if n_pl > 0 else L.DK_TAIL_MAX_DEGREE
        nbytes = L.dk_workspace_bytes(self.h, n_s, self.n_grid, n_pl)
        if self.ws is not None and self.ws.numel() * 8 >= nbytes:
            return
        if self.ws is not None:
            self.ws = None
            torch.cuda.empty_cache()
        self.ws = torch.empty((nbytes + nbytes // 16) // 8 + 64, dtype=torch.float64,
                              device=self.device)
        L.dk_set_workspace(self.h, self.ws)
        self.ws_key = (n_s, n_pl)

    def block(self, x0: np.ndarray) -> torch.Tensor:
        return torch.as_tensor(x0, device=self.device).to(self.dtype).contiguous()

    def close(self) -> None:
        if self.h is not None:
            L.dk_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Evaluation:
    X: torch.Tensor
    Hs: torch.Tensor
    Ds: torch.Tensor
    tau: torch.Tensor
    rho: torch.Tensor
    info: dict
    e_band: float
    e_ent: float
    free_energy: float
    forces: Optional[np.ndarray]
    bounds: list


def tau_length(n_pl: int) -> int:
    """Length of the trace buffer for degree n_pl (0: the tail rule's largest degree)."""
    return (n_pl if n_pl > 0 else L.DK_TAIL_MAX_DEGREE) + 1


def start(ctx: Context, X: torch.Tensor, Hs: torch.Tensor) -> None:
    L.dk_orthonormalize(ctx.h, X)
    L.dk_project(ctx.h, X, Hs)


def filter_pass(ctx: Context, X: torch.Tensor, Hs: torch.Tensor, degree: int, bounds=None):
    """bounds: (lam_min, lam_max) of Hs if already known (e.g. from the density kernel)."""
    lo, hi = bounds if bounds is not None else L.dk_spectral_bounds(ctx.h, Hs)[:2]
    L.dk_filter(ctx.h, X, degree, hi, ctx.upper, lo)
    L.dk_orthonormalize(ctx.h, X)
    L.dk_project(ctx.h, X, Hs)
    return (lo, hi, ctx.upper)


def kernel_and_density(ctx: Context, X, Hs, Ds, tau, rho, n_e, sigma, n_pl, gradv=None,
                       forces=True):
    info = L.dk_density_kernel(ctx.h, Hs, n_e, sigma, n_pl, Ds, tau)
    L.dk_density(ctx.h, X, Ds, rho)
    e_band, e_ent = L.dk_energy(ctx.h, tau, info.n_pl, info.mu, info.chi, info.xi, sigma)
    f = None
    if forces:
        f = L.dk_forces(ctx.h, X, Ds, rho, gradv, ctx.n_atoms)
    return info, e_band, e_ent, f


def evaluate(problem, precision: str = "fp64", passes: Optional[int] = None,
             degree: Optional[int] = None, n_pl: Optional[int] = None, forces: bool = True,
             device: int = 0, ctx: Optional[Context] = None, X0: Optional[np.ndarray] = None
             ) -> Evaluation:
    spec = problem.spec
    passes = spec.filter_passes if passes is None else passes
    degree = spec.filter_degree if degree is None else degree
    n_pl = spec.n_pl if n_pl is None else n_pl
    own = ctx is None
    ctx = Context(problem, precision, device) if own else ctx
    try:
        X = ctx.block(problem.x0 if X0 is None else X0)
        n_s = X.shape[0]
        ctx.ensure_workspace(n_s, n_pl)
        dev = ctx.device
        Hs = torch.zeros((n_s, n_s), dtype=torch.float64, device=dev)
        Ds = torch.zeros_like(Hs)
        tau = torch.zeros(tau_length(n_pl), dtype=torch.float64, device=dev)
        rho = torch.zeros(problem.n_grid, dtype=torch.float64, device=dev)
        start(ctx, X, Hs)
        bounds = [filter_pass(ctx, X, Hs, degree) for _ in range(passes)]
        gradv = None
        if forces:
            gradv = torch.as_tensor(problem.gradv, dtype=torch.float64, device=dev).contiguous()
        info, e_band, e_ent, f = kernel_and_density(ctx, X, Hs, Ds, tau, rho, problem.n_e,
                                                    spec.kT, n_pl, gradv, forces)
        return Evaluation(X, Hs, Ds, tau, rho, info.as_dict(), e_band, e_ent, e_band + e_ent,
                          f, bounds)
    finally:
        if own:
            ctx.close()
