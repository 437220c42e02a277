"""Born-Oppenheimer molecular dynamics with density-kernel forces (libdk calls only).

Velocity Verlet in the NVE ensemble (the paper's application runs are quantum
molecular dynamics, Sec. 5): v += (dt/2) f/M, R += dt v, self-consistent
density and forces at the new positions, v += (dt/2) f/M.  Each ionic step
re-places the atoms' local fields (dk_set_atoms, inside the SCF) and the
projector tables (built on the device from a ProjectorModel, or by the
caller's `problem_at(positions)` on the host), and restarts the SCF from the
previous step's orbitals and density (or from a learned start density).  The conserved quantity is
E = F + (1/2) sum M v^2 with F the electronic free energy, whose
pseudocharge electrostatics include the ion-ion interaction.

With ensemble="nvk" the run is isokinetic (the Gaussian thermostat of the
paper's transport runs): the start velocities are rescaled to the kinetic
energy (3N - 3) T / 2 and each half kick is the exact isokinetic flow with the
forces held fixed (dk_isokinetic_kick), which keeps that kinetic energy.

Units: Hartree atomic units; 1 fs = 41.341374575751 a.u.; aluminium mass
26.9815385 u, 1 u = 1822.888486 electron masses.
"""

from __future__ import annotations

import dataclasses
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
import torch

from . import _lib as L
from .pipeline import Context, ProjectorModel
from .scf import LocalModel, scf

FS = 41.341374575751
AMU = 1822.888486
M_AL = 26.9815385 * AMU
EV = 1.0 / 27.211386245988


def maxwell_boltzmann(n_atoms: int, mass: float, temperature: float, seed: int) -> np.ndarray:
    """Seeded draw v = sqrt(T/M) N(0,1) per component, centre-of-mass velocity removed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = np.sqrt(temperature / mass) * rng.standard_normal((n_atoms, 3))
    return v - v.mean(axis=0)


def isokinetic_start(n_atoms: int, mass: float, temperature: float, seed: int) -> np.ndarray:
    """The Maxwell-Boltzmann draw rescaled to the kinetic energy (3N - 3) T / 2."""
    v = maxwell_boltzmann(n_atoms, mass, temperature, seed)
    k = 0.5 * mass * float(np.sum(v * v))
    return v * np.sqrt(0.5 * (3 * n_atoms - 3) * temperature / k)


@dataclass
class Trajectory:
    positions: List[np.ndarray] = field(default_factory=list)
    energies: List[float] = field(default_factory=list)       # F + kinetic, per step
    free_energies: List[float] = field(default_factory=list)
    kinetic: List[float] = field(default_factory=list)
    scf_iterations: List[int] = field(default_factory=list)
    scf_residuals: List[float] = field(default_factory=list)  # last SCF residual per step
    step_ms: List[float] = field(default_factory=list)
    forces: Optional[np.ndarray] = None
    stress: List[tuple] = field(default_factory=list)  # scf() stress terms per step, if asked
    velocities: List[np.ndarray] = field(default_factory=list)  # (n_atoms, 3) per step

    def total_stress(self) -> np.ndarray:
        """(steps+1, 3, 3): the sum of the stress terms of every step."""
        return np.stack([sum(np.asarray(t) for t in terms) for terms in self.stress])


def qmd(problem0, problem_at: Optional[Callable], model: LocalModel, precision: str = "mixed",
        steps: int = 20, dt_fs: float = 0.5, temperature: float = 10.0 * EV, mass: float = M_AL,
        v_seed: int = 7000, scf_tol: float = 1e-6, scf_max_iter: int = 40,
        later_passes: int = 1, first_passes: Optional[int] = None, step_passes: int = 1,
        start_density: Optional[Callable] = None, n_pl: Optional[int] = None,
        callback: Optional[Callable] = None, device: int = 0,
        projectors: Optional[ProjectorModel] = None,
        scf_callback: Optional[Callable] = None, ensemble: str = "nve",
        mixing: str = "pulay", stress: bool = False, restart: bool = False,
        solver: str = "cg") -> Trajectory:
    """projectors: build every step's projector tables on the device (and those
    of the first step too); otherwise problem_at(positions) -> problem for the
    moved atoms with host-built tables.
    start_density(positions) -> device FP64 density, if given, replaces the previous
    step's density as the SCF start of every ionic step.
    scf_callback(iteration, residual, free_energy, ms), if given, runs after every SCF
    iteration."""
    if projectors is None and problem_at is None:
        raise ValueError("qmd: give problem_at or projectors")
    if ensemble not in ("nve", "nvk"):
        raise ValueError(f"qmd: ensemble must be 'nve' or 'nvk', not {ensemble!r}")
    start_v = isokinetic_start if ensemble == "nvk" else maxwell_boltzmann

    def kick(v, f, tau):
        if ensemble == "nvk":
            L.dk_isokinetic_kick(ctx.h, v, f, tau, mass)
        else:
            L.dk_verlet_kick(ctx.h, v, f, tau, mass)
    cell = problem0.spec.a if problem0.spec.cubic else np.asarray(problem0.spec.cell)
    dt = dt_fs * FS
    n_atoms = len(problem0.positions)
    ctx = Context(problem0, precision, device)
    dev = ctx.device
    f64 = dict(dtype=torch.float64, device=dev)
    traj = Trajectory()
    try:
        x = torch.as_tensor(np.asarray(problem0.positions, dtype=np.float64).reshape(-1), **f64)
        v = torch.as_tensor(start_v(n_atoms, mass, temperature, v_seed).reshape(-1), **f64)
        if stress and projectors is None:
            raise ValueError("qmd: the stress needs device-built projector tables (projectors=)")
        kw = dict(tol=scf_tol, max_iter=scf_max_iter, later_passes=later_passes, n_pl=n_pl,
                  ctx=ctx, callback=scf_callback, mixing=mixing, stress=stress,
                  restart=restart, solver=solver)
        if projectors is not None:
            ctx.move_atoms(problem0.positions, projectors)
        rho0 = start_density(problem0.positions) if start_density else None
        run = scf(problem0, model, precision, first_passes=first_passes, rho0=rho0, **kw)
        f = torch.as_tensor(run.forces.reshape(-1), **f64)
        X = run.X
        rho_prev = run.rho.clone()
        ke = L.dk_kinetic_energy(ctx.h, v, mass)
        traj.positions.append(np.asarray(problem0.positions, dtype=np.float64).copy())
        traj.energies.append(run.free_energy + ke)
        traj.free_energies.append(run.free_energy)
        traj.kinetic.append(ke)
        traj.scf_iterations.append(run.iterations)
        traj.scf_residuals.append(run.residuals[-1])
        traj.step_ms.append(float(np.sum(run.iteration_ms)))
        traj.velocities.append(v.cpu().numpy().reshape(n_atoms, 3))
        if stress:
            traj.stress.append(run.stress)
        for step in range(1, steps + 1):
            torch.cuda.synchronize(dev)
            t0 = time.perf_counter()
            kick(v, f, 0.5 * dt)
            L.dk_verlet_drift(ctx.h, x, v, dt)
            pos = x.cpu().numpy().reshape(n_atoms, 3)
            if projectors is not None:
                inside = np.mod(pos, cell)
                ctx.move_atoms(inside, projectors)
                p = dataclasses.replace(problem0, positions=inside, _gradv=None)
            else:
                p = problem_at(pos)
                ctx.set_problem(p)
            rho0 = start_density(pos) if start_density else rho_prev
            run = scf(p, model, precision, first_passes=step_passes, rho0=rho0, X_init=X, **kw)
            f.copy_(torch.as_tensor(run.forces.reshape(-1), **f64))
            kick(v, f, 0.5 * dt)
            ke = L.dk_kinetic_energy(ctx.h, v, mass)
            rho_prev.copy_(run.rho)
            torch.cuda.synchronize(dev)
            traj.step_ms.append((time.perf_counter() - t0) * 1e3)
            traj.positions.append(pos.copy())
            traj.energies.append(run.free_energy + ke)
            traj.free_energies.append(run.free_energy)
            traj.kinetic.append(ke)
            traj.scf_iterations.append(run.iterations)
            traj.scf_residuals.append(run.residuals[-1])
            traj.velocities.append(v.cpu().numpy().reshape(n_atoms, 3))
            if stress:
                traj.stress.append(run.stress)
            if callback is not None:
                callback(step, traj)
        traj.forces = run.forces
        return traj
    finally:
        ctx.close()
