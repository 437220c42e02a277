"""Orbital terms of the Hellmann-Feynman stress tensor (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 3 rewrites the kinetic and nonlocal contributions to the stress in terms
of the auxiliary orbitals phi_i and the kernel-transformed orbitals
phi~_i = sum_j phi_j D_ji (Eqs. stressIRe and stressIIIRe); the full tensor
(Eq. Stress:NewForm) divides the sum of all contributions by the cell volume.
This module evaluates those two contributions, divided by |Omega|:

  kinetic   sigma^I_ab   = -2 sum_i int d_a phi_i  d_b phi~_i
  nonlocal  sigma^III_ab = -2 delta_ab sum_i sum_p gamma_p <chi_p, phi~_i><chi_p, phi_i>
                           -4 sum_i sum_p gamma_p <m^b_p, d_a phi~_i><chi_p, phi_i>

where d_a is the twelfth-order central first difference along axis a, every
integral is an h^3-weighted grid sum, and m^b_p is the first moment of the
periodically extended projector: the sum over images of
chi_p(x - R - L) (x - R - L)_b (the inner sum over J' of Eq. stressIIIRe).
The first nonlocal term is -delta_ab E_nl / |Omega|, E_nl = 2 tr(D Phi^T V_nl Phi)
the nonlocal energy.

The exchange-correlation term of Eq. Stress:NewForm,
  sigma^xc_ab = delta_ab (E_xc[rho] - int v_xc[rho] rho) / |Omega|,
is the strain derivative of E_xc for a density carried along by the strain
(rho -> rho / det F on the moved grid points), exactly also on the grid.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fd, xc
from .density import kernel_orbitals


def kinetic_stress(Phi: np.ndarray, D: np.ndarray, n: int, h: float) -> np.ndarray:
    """sigma^I (3 x 3, Ha/bohr^3) for orbitals Phi (N_grid, N_s) and kernel D."""
    Phit = kernel_orbitals(Phi, D)
    dphi = [fd.gradient(Phi, n, h, a) for a in range(3)]
    dphit = [fd.gradient(Phit, n, h, b) for b in range(3)]
    vol = (n * h) ** 3
    s = np.empty((3, 3))
    for a in range(3):
        for b in range(3):
            s[a, b] = -2.0 * h ** 3 * np.sum(dphi[a] * dphit[b])
    return s / vol


def nonlocal_stress(H, proj, Phi: np.ndarray, D: np.ndarray) -> np.ndarray:
    """sigma^III (3 x 3, Ha/bohr^3); H the oracle Hamiltonian of the problem
    whose projector tables (with their moments) are proj."""
    h3 = H.h ** 3
    vol = (H.n * H.h) ** 3
    Phit = kernel_orbitals(Phi, D)
    C = h3 * (H.chi.T @ Phi)          # <chi_p, phi_i>
    Ct = h3 * (H.chi.T @ Phit)        # <chi_p, phi~_i>
    gC = H.gamma[:, None] * C
    s = np.zeros((3, 3))
    e_nl = 2.0 * np.sum(Ct * gC)
    n_proj = len(H.gamma)
    cols = np.repeat(np.arange(n_proj), np.diff(proj["offsets"]))
    mom = [sp.csc_matrix((proj["moments"][b], (proj["indices"], cols)),
                         shape=(H.n_grid, n_proj)) for b in range(3)]
    for a in range(3):
        dphit = fd.gradient(Phit, H.n, H.h, a)
        for b in range(3):
            G = h3 * (mom[b].T @ dphit)  # <m^b_p, d_a phi~_i>
            s[a, b] = -4.0 * np.sum(G * gC)
    s -= e_nl * np.eye(3)
    return s / vol


def xc_stress(rho: np.ndarray, n: int, h: float) -> np.ndarray:
    """sigma^xc (3 x 3, Ha/bohr^3) of the LDA for the density rho on the n^3 grid."""
    eps, v = xc.lda(rho)
    e_xc = h ** 3 * float(np.sum(rho * eps))
    int_v_rho = h ** 3 * float(np.sum(v * rho))
    return (e_xc - int_v_rho) / (n * h) ** 3 * np.eye(3)
