"""Self-consistent density by the SQ3 steps (oracle).

One SCF iteration (Sec. 5 runs the density-kernel evaluation inside a
standard SCF loop):

  1. effective potential from the input density rho_in:
       V_c = Poisson solution of -Lap_h V_c = 4 pi (rho_in + b)   (electrostatics),
       V_eff = V_c + V_core + v_xc(rho_in)                          (LDA, PW92);
  2. filter the auxiliary orbitals with H[V_eff]: the first iteration takes
     `first_passes` passes from the orthonormalised random start block, later
     iterations one pass each; the filter interval of a pass comes from the
     spectrum of the subspace Hamiltonian at hand (for the first pass of a
     later iteration: the previous iteration's H_s);
  3. orthonormalise, project, expand the density kernel (Fermi level, band
     and entropy energies), rho_out = 2 rowsum(Phi o Phi D_s);
  4. stop when ||rho_out - rho_in||_2 / ||rho_out||_2 <= tol, else
     rho_in <- Pulay mix (history 7, beta 0.3) and repeat; with
     mixing="kerker", Kerker-preconditioned periodic Pulay (period, k0).

Free energy (Harris-Foulkes form, evaluated with rho_in; it agrees with the
Mermin functional to second order in rho_out - rho_in):
  F = E_band + E_ent - int rho_in (V_c + v_xc) + E_xc[rho_in] + E_es[rho_in].
Forces at the last iteration: pseudocharge and core terms with V_c[rho_in] and
rho_out, plus the nonlocal term with the final Phi and D_s.

Start density (superposition of atomic densities): rho_0 = -b, the
pseudocharges' Gaussian electron clouds (integral N_e, zero net charge).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import electrostatics as es
from . import xc
from .density import density, nonlocal_forces
from .filter import chebyshev_filter
from .foe import density_kernel
from .hamiltonian import Hamiltonian
from .mixing import PeriodicPulay, Pulay
from .orth import cholqr2
from .sq3 import project


@dataclass
class LocalModel:
    z: float
    rc: float
    core_amp: float
    core_w2: float


@dataclass
class SCFResult:
    rho: np.ndarray          # rho_out of the last iteration
    rho_in: np.ndarray
    vc: np.ndarray
    veff: np.ndarray
    Phi: np.ndarray
    D: np.ndarray
    mu: float
    e_band: float
    e_ent: float
    free_energy: float
    iterations: int
    converged: bool
    residuals: List[float] = field(default_factory=list)
    energies: List[float] = field(default_factory=list)
    n_pl: int = 0
    forces: Optional[np.ndarray] = None


def effective_potential(problem, model: LocalModel, rho_in, b, vcore):
    n, a, h = problem.n, problem.spec.a, problem.h
    vc = es.poisson_fft(rho_in + b, n, a)
    eps, vxc = xc.lda(rho_in)
    veff = vc + vcore + vxc
    terms = {
        "e_xc": float(h ** 3 * np.sum(rho_in * eps)),
        "int_rho_vc": float(h ** 3 * np.sum(rho_in * vc)),
        "int_rho_vxc": float(h ** 3 * np.sum(rho_in * vxc)),
        "e_es": es.electrostatic_energy(rho_in, b, vc, h, es.self_energy(len(problem.positions),
                                                                        model.z, model.rc)),
    }
    return vc, vxc, veff, terms


def start_density(b: np.ndarray) -> np.ndarray:
    return -b


def scf(problem, model: LocalModel, tol: float = 1e-6, max_iter: int = 60,
        first_passes: Optional[int] = None, degree: Optional[int] = None,
        n_pl: Optional[int] = None, history: int = 7, beta: float = 0.3,
        rho0: Optional[np.ndarray] = None, forces: bool = True,
        later_passes: int = 1, X0: Optional[np.ndarray] = None, mixing: str = "pulay",
        period: int = 2, k0: float = 1.0, restart: bool = False) -> SCFResult:
    """later_passes: filter passes per iteration after the first (0 with N_s = N_grid
    gives the full-space SCF used as a pin).  X0: start block (N_grid x N_s), e.g. the
    orbitals of the previous ionic step; default the problem's random block."""
    spec = problem.spec
    n, a, h = problem.n, spec.a, problem.h
    first_passes = spec.filter_passes if first_passes is None else first_passes
    degree = spec.filter_degree if degree is None else degree
    n_pl = spec.n_pl if n_pl is None else n_pl
    pos = problem.positions
    b = es.pseudocharge(n, a, pos, model.z, model.rc)
    vcore = es.core_potential(n, a, pos, model.core_amp, model.core_w2)
    rho_in = start_density(b) if rho0 is None else np.asarray(rho0, dtype=np.float64).copy()
    if mixing == "kerker":
        mixer = PeriodicPulay(n, h, history, beta, period, k0, restart)
    elif mixing == "pulay":
        mixer = Pulay(history, beta)
    else:
        raise ValueError(f"scf: unknown mixing {mixing!r}")
    Phi = None
    Hs = None
    residuals, energies = [], []
    converged = False
    it = 0
    for it in range(1, max_iter + 1):
        vc, vxc, veff, terms = effective_potential(problem, model, rho_in, b, vcore)
        H = Hamiltonian(problem, veff)
        ub = H.upper_bound()
        if Phi is None:
            Phi = cholqr2((problem.x0.T if X0 is None else X0).copy(), h)
            Hs = project(H, Phi)
            passes = first_passes
        else:
            passes = later_passes
        for _ in range(passes):
            lam = np.linalg.eigvalsh(Hs)
            X = chebyshev_filter(H, Phi, degree, float(lam[-1]), ub, float(lam[0]))
            Phi = cholqr2(X, h)
            Hs = project(H, Phi)
        if passes == 0:
            Hs = project(H, Phi)
        dk = density_kernel(Hs, problem.n_e, spec.kT, n_pl)
        rho_out = density(Phi, dk.D)
        res = float(np.linalg.norm(rho_out - rho_in) / np.linalg.norm(rho_out))
        F = (dk.e_band + dk.e_ent - terms["int_rho_vc"] - terms["int_rho_vxc"]
             + terms["e_xc"] + terms["e_es"])
        residuals.append(res)
        energies.append(F)
        if res <= tol:
            converged = True
            break
        if it < max_iter:
            rho_in = mixer.mix(rho_in, rho_out)
    f = None
    if forces:
        m = model
        f = es.local_forces(n, a, pos, m.z, m.rc, m.core_amp, m.core_w2, rho_out, vc)
        f = f + nonlocal_forces(H, Phi, dk.D, len(pos))
    return SCFResult(rho_out, rho_in, vc, veff, Phi, dk.D, dk.mu, dk.e_band, dk.e_ent,
                     energies[-1], it, converged, residuals, energies, dk.n_pl, f)
