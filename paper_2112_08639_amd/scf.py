"""Self-consistent loop around the density-kernel steps (libdk calls only).

One iteration (the paper runs the density-kernel evaluation inside SCF
iterations, Sec. 5):

  1. dk_scf_potential: V_c from -Lap_h V_c = 4 pi (rho_in + b) by CG (warm
     started from the previous V_c), V_eff = V_c + v_core + v_xc(rho_in), and the
     energy integrals; the context potential becomes V_eff;
  2. filter the block with H[V_eff]: `first_passes` passes from the
     orthonormalised start block in the first iteration, `later_passes` (1)
     afterwards; each pass takes its interval from the current H_s (for the
     first pass of a later iteration, the previous iteration's H_s, whose
     bounds the density kernel of that iteration has already found);
  3. density kernel, density, band and entropy energies;
  4. dk_pulay_mix: residual ||rho_out - rho_in|| / ||rho_out||; stop at `tol`,
     else rho_in <- the Pulay-mixed density.

Free energy (Harris-Foulkes form with rho_in):
  F = E_band + E_ent - int rho_in (V_c + v_xc) + E_xc[rho_in] + E_es[rho_in].
Forces at the last iteration: dk_local_forces (pseudocharge and core terms,
with V_c and rho_out) plus the nonlocal term of dk_forces.
"""

from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from . import _lib as L
from .pipeline import Context, filter_pass, kernel_and_density, start, tau_length


@dataclass
class LocalModel:
    z: float
    rc: float
    core_amp: float
    core_w2: float


@dataclass
class SCFRun:
    rho: torch.Tensor        # rho_out of the last iteration (device)
    rho_in: torch.Tensor
    vc: torch.Tensor
    X: torch.Tensor
    Ds: torch.Tensor
    mu: float
    e_band: float
    e_ent: float
    free_energy: float
    iterations: int
    converged: bool
    n_pl: int
    residuals: List[float] = field(default_factory=list)
    energies: List[float] = field(default_factory=list)
    iteration_ms: List[float] = field(default_factory=list)
    poisson_iters: List[int] = field(default_factory=list)
    forces: Optional[np.ndarray] = None
    stress: Optional[tuple] = None   # (kinetic, nonlocal, xc, electrostatic) 3x3 host arrays


def scf(problem, model: LocalModel, precision: str = "fp64", tol: float = 1e-6,
        max_iter: int = 60, first_passes: Optional[int] = None, degree: Optional[int] = None,
        n_pl: Optional[int] = None, history: int = 7, beta: float = 0.3,
        rho0: Optional[np.ndarray] = None, forces: bool = True, later_passes: int = 1,
        poisson_tol: float = 1e-10, poisson_max_iter: int = 20000,
        ctx: Optional[Context] = None, device: int = 0, callback=None,
        X_init: Optional[torch.Tensor] = None, mixing: str = "pulay", period: int = 2,
        k0: float = 1.0, kerker_tol: float = 1e-10, stress: bool = False,
        restart: bool = False, solver: str = "cg") -> SCFRun:
    """callback(iteration, residual, free_energy, ms), if given, runs after each iteration.
    X_init: start block on the device (e.g. the previous ionic step's orbitals), used in
    place; default: the problem's random start block.
    mixing: "pulay" (dk_pulay_mix) or "kerker" (dk_kerker_pulay_mix: Pulay on every
    period-th iteration, Kerker-preconditioned linear mixing otherwise, k0 in 1/bohr;
    restart: discard the stored pairs after every Pulay extrapolation).
    solver: "cg" or "aar", the linear solver of the Poisson and Kerker solves.
    stress: also the kinetic and nonlocal stress terms of the last iteration's orbitals
    and density kernel (dk_stress; needs device-built projector tables), and the
    exchange-correlation and electrostatic terms of its input density."""
    if mixing not in ("pulay", "kerker"):
        raise ValueError(f"scf: unknown mixing {mixing!r}")
    if solver not in ("cg", "aar"):
        raise ValueError(f"scf: unknown linear solver {solver!r}")
    spec = problem.spec
    first_passes = spec.filter_passes if first_passes is None else first_passes
    degree = spec.filter_degree if degree is None else degree
    n_pl = spec.n_pl if n_pl is None else n_pl
    own = ctx is None
    ctx = Context(problem, precision, device) if own else ctx
    try:
        h = ctx.h
        dev = ctx.device
        L.dk_set_linear_solver(h, L.DK_SOLVER_AAR if solver == "aar" else L.DK_SOLVER_CG)
        L.dk_set_atoms(h, problem.positions, model.z, model.rc, model.core_amp, model.core_w2)
        X = ctx.block(problem.x0) if X_init is None else X_init
        n_s = X.shape[0]
        ctx.ensure_workspace(n_s, n_pl)
        ng = problem.n_grid
        f64 = dict(dtype=torch.float64, device=dev)
        rho_in = torch.zeros(ng, **f64)
        if rho0 is None:
            L.dk_start_density(h, rho_in)
        else:
            rho_in.copy_(torch.as_tensor(rho0, **f64))
        rho_out = torch.zeros(ng, **f64)
        rho_next = torch.zeros(ng, **f64)
        vc = torch.zeros(ng, **f64)
        veff = torch.zeros(ng, **f64)
        nbytes = (L.dk_kerker_pulay_bytes(h, history) if mixing == "kerker"
                  else L.dk_pulay_bytes(h, history))
        state = torch.empty(nbytes // 8 + 1, **f64)
        Hs = torch.zeros((n_s, n_s), **f64)
        Ds = torch.zeros_like(Hs)
        tau = torch.zeros(tau_length(n_pl), **f64)
        residuals, energies, times, piters = [], [], [], []
        converged = False
        first = True
        it = 0
        info = None
        bounds = None  # of the H_s the last density kernel expanded
        e_band = e_ent = 0.0
        for it in range(1, max_iter + 1):
            torch.cuda.synchronize(dev)
            t0 = time.perf_counter()
            terms = L.dk_scf_potential(h, rho_in, vc, veff, poisson_tol, poisson_max_iter)
            ctx.upper = L.dk_spectrum_upper_bound(h)
            if first:
                start(ctx, X, Hs)
                passes = first_passes
                first = False
                bounds = None  # H_s of the start block
            else:
                passes = later_passes
            for k in range(passes):
                filter_pass(ctx, X, Hs, degree, bounds=bounds if k == 0 else None)
            if passes == 0:
                L.dk_project(h, X, Hs)
            info, e_band, e_ent, _ = kernel_and_density(ctx, X, Hs, Ds, tau, rho_out, problem.n_e,
                                                        spec.kT, n_pl, forces=False)
            bounds = (info.lam_min, info.lam_max)
            if mixing == "kerker":
                res = L.dk_kerker_pulay_mix(h, state, history, it - 1, period, beta, k0,
                                            kerker_tol, rho_in, rho_out, rho_next,
                                            restart=restart)
            else:
                res = L.dk_pulay_mix(h, state, history, it - 1, beta, rho_in, rho_out, rho_next)
            torch.cuda.synchronize(dev)
            times.append((time.perf_counter() - t0) * 1e3)
            F = L.dk_free_energy(h, terms, e_band, e_ent)
            residuals.append(res)
            energies.append(F)
            piters.append(terms.poisson_iters)
            if callback is not None:
                callback(it, res, F, times[-1])
            if res <= tol:
                converged = True
                break
            rho_in, rho_next = rho_next, rho_in
        f = None
        if forces:
            f = L.dk_local_forces(h, rho_out, vc, len(problem.positions))
            f = f + L.dk_forces(h, X, Ds, rho_out, None, ctx.n_atoms)
        st = None
        if stress:
            # orbital terms of the last orbitals and kernel; the exchange-correlation
            # term delta_ab (E_xc - int v_xc rho) / |Omega| of the last input density
            kin, nl = L.dk_stress(h, X, Ds)
            _, xc = L.dk_free_energy(h, terms, e_band, e_ent, xc_stress=True)
            st = (kin, nl, xc, L.dk_electrostatic_stress(h, rho_in, vc))
        return SCFRun(rho_out, rho_in, vc, X, Ds, info.mu, e_band, e_ent, energies[-1], it,
                      converged, info.n_pl, residuals, energies, times, piters, f, st)
    finally:
        if own:
            ctx.close()
