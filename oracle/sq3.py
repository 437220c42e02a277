"""Non-self-consistent density evaluation by the SQ3 steps (oracle).

Order of operations (Sec. 4): start from an orthonormalised block, then for
each filter pass take the spectrum of the current subspace Hamiltonian, filter,
re-orthonormalise and project; finally expand the density kernel, find the
Fermi level, and form the density, energies and forces.

Readings for what the paper leaves open:
  * filter interval: damp [a, b] with a = lambda_max(H_s) of the current
    subspace, b the closed-form upper bound of H, normalised at
    a0 = lambda_min(H_s); the first pass uses H_s of the orthonormalised
    start block;
  * projection H_s = h^3 Phi^T (H Phi), symmetrised as (H_s + H_s^T)/2;
  * band free energy of the fixed-potential problem F_b = E_band + E_ent.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

from .density import density, local_forces, nonlocal_forces
from .filter import chebyshev_filter
from .foe import DensityKernel, density_kernel
from .hamiltonian import Hamiltonian
from .orth import cholqr2


def project(H: Hamiltonian, Phi: np.ndarray) -> np.ndarray:
    Hs = H.h ** 3 * (Phi.T @ H.apply(Phi))
    return 0.5 * (Hs + Hs.T)


@dataclass
class SQ3Result:
    Phi: np.ndarray
    Hs: np.ndarray
    dk: DensityKernel
    rho: np.ndarray
    e_band: float
    e_ent: float
    free_energy: float
    forces: Optional[np.ndarray]
    forces_local: Optional[np.ndarray]
    forces_nonlocal: Optional[np.ndarray]
    bounds: list   # (a0, a, b) used by each filter pass


def filtered_subspace(problem, passes: int, degree: int, H: Optional[Hamiltonian] = None,
                      X0: Optional[np.ndarray] = None):
    H = Hamiltonian(problem) if H is None else H
    b = H.upper_bound()
    X = (problem.x0 if X0 is None else X0).T
    Phi = cholqr2(X, H.h)
    Hs = project(H, Phi)
    bounds = []
    for _ in range(passes):
        lam = np.linalg.eigvalsh(Hs)
        a0, a = float(lam[0]), float(lam[-1])
        bounds.append((a0, a, b))
        X = chebyshev_filter(H, Phi, degree, a, b, a0)
        Phi = cholqr2(X, H.h)
        Hs = project(H, Phi)
    return H, Phi, Hs, bounds


def run(problem, passes: Optional[int] = None, degree: Optional[int] = None,
        n_pl: Optional[int] = None, forces: bool = True,
        X0: Optional[np.ndarray] = None) -> SQ3Result:
    spec = problem.spec
    passes = spec.filter_passes if passes is None else passes
    degree = spec.filter_degree if degree is None else degree
    n_pl = spec.n_pl if n_pl is None else n_pl
    H, Phi, Hs, bounds = filtered_subspace(problem, passes, degree, X0=X0)
    dk = density_kernel(Hs, problem.n_e, spec.kT, n_pl)
    rho = density(Phi, dk.D)
    f = fl = fnl = None
    if forces:
        fl = local_forces(rho, problem.gradv, H.h)
        fnl = nonlocal_forces(H, Phi, dk.D, len(problem.positions))
        f = fl + fnl
    return SQ3Result(Phi, Hs, dk, rho, dk.e_band, dk.e_ent, dk.e_band + dk.e_ent,
                     f, fl, fnl, bounds)
