"""Density and Hellmann-Feynman forces from the auxiliary orbitals (oracle).

Sec. 3 of the paper:
  * phi~_i = sum_j phi_j D_ji  (Eq. phi_tilde),
  * rho(x) = 2 sum_i phi~_i(x) phi_i(x)  (Eq. density:NewForm),
  * nonlocal force on atom I (Eq. force_nl:NewForm):
      f^nl_I = -4 sum_i sum_lm gamma_Il (int phi_i chi~_Ilm) (int grad phi~_i chi~_Ilm),
    with the gradient of phi~ taken by the twelfth-order central difference.
  * for the fixed-potential workloads the local force is the
    Hellmann-Feynman term int rho(x) grad v_I(x) dx, grad v_I being the
    gradient of atom I's local potential field (its only R dependence).
Integrals are grid sums times h^3.
"""

from __future__ import annotations

import numpy as np

from . import fd


def kernel_orbitals(Phi: np.ndarray, D: np.ndarray) -> np.ndarray:
    return Phi @ D


def density(Phi: np.ndarray, D: np.ndarray) -> np.ndarray:
    Phit = kernel_orbitals(Phi, D)
    return 2.0 * np.sum(Phit * Phi, axis=1)


def nonlocal_forces(H, Phi: np.ndarray, D: np.ndarray, n_atoms: int) -> np.ndarray:
    h3 = H.h ** 3
    Phit = kernel_orbitals(Phi, D)
    C = h3 * (H.chi.T @ Phi)                       # (N_proj, N_s)
    f = np.zeros((n_atoms, 3))
    for alpha in range(3):
        grad = fd.gradient(Phit, H.fd_n, H.fd_h, alpha)  # grad_alpha phi~_i
        Cg = h3 * (H.chi.T @ grad)
        per_proj = np.sum(C * Cg, axis=1)          # sum_i
        np.add.at(f[:, alpha], H.atom, -4.0 * H.gamma * per_proj)
    return f


def local_forces(rho: np.ndarray, gradv: np.ndarray, h: float) -> np.ndarray:
    """h^3 sum_x rho(x) grad v_I(x); gradv has shape (N_atoms, 3, N_grid)."""
    return h ** 3 * np.einsum("x,iax->ia", rho, gradv)
