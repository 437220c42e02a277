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

The electrostatic terms of Eq. Stress:NewForm for the pseudocharge model of
`electrostatics` (Gaussian charges b_I, core terms v_core,I, the continuum
self-energy, which does not depend on the strain):
  sigma^es_ab = ( (1/4 pi) int d_a V d_b V
                + sum_I int [sum_L d_a b_I(x - R - L) (x - R - L)_b] V
                + delta_ab (1/2) int (b - rho) V
                + sum_I int rho [sum_L d_a v_core,I(x - R - L) (x - R - L)_b] ) / |Omega|,
V the zero-mean solution of -Lap_h V = 4 pi (rho + b), d_a V by the
twelfth-order first difference, the Gaussians differentiated analytically.

The exchange-correlation term of Eq. Stress:NewForm,
  sigma^xc_ab = delta_ab (E_xc[rho] - int v_xc[rho] rho) / |Omega|,
is the strain derivative of E_xc for a density carried along by the strain
(rho -> rho / det F on the moved grid points), exactly also on the grid.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import electrostatics as es
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


def _moment_field(n: int, a: float, pos: np.ndarray, w2: float, ax: int, bx: int) -> np.ndarray:
    """sum over atoms and images of d_ax G(d) d_bx for G = prod_axes exp(-d^2/w2)."""
    x = np.arange(n) * (a / n)
    out = np.zeros(n ** 3)
    for p in pos:
        f = [es.periodic_gauss_1d(x, p[k], a, w2) for k in range(3)]
        # d_ax exp(-d^2/w2) = -2 d/w2 exp(...); times d_bx
        if ax == bx:
            f[ax] = -2.0 / w2 * es.periodic_gauss_1d(x, p[ax], a, w2, moment=2)
        else:
            f[ax] = -2.0 / w2 * es.periodic_gauss_1d(x, p[ax], a, w2, moment=1)
            f[bx] = es.periodic_gauss_1d(x, p[bx], a, w2, moment=1)
        out += (f[2][:, None, None] * f[1][None, :, None] * f[0][None, None, :]).reshape(-1)
    return out


def electrostatic_stress(n: int, a: float, pos: np.ndarray, z: float, rc: float, amp: float,
                         w2: float, rho: np.ndarray) -> np.ndarray:
    """sigma^es (3 x 3, Ha/bohr^3) for the density rho and atoms at pos."""
    h = a / n
    h3 = h ** 3
    b = es.pseudocharge(n, a, pos, z, rc)
    V = es.poisson_fft(rho + b, n, a)
    pref = -z * (np.pi * rc * rc) ** -1.5
    dV = [fd.gradient(V[:, None], n, h, ax)[:, 0] for ax in range(3)]
    s = np.zeros((3, 3))
    for ax in range(3):
        for bx in range(3):
            s[ax, bx] = (h3 * np.sum(dV[ax] * dV[bx]) / (4.0 * np.pi)
                         + h3 * pref * np.sum(_moment_field(n, a, pos, rc * rc, ax, bx) * V)
                         - h3 * amp * np.sum(_moment_field(n, a, pos, w2, ax, bx) * rho))
    s += 0.5 * h3 * float(np.sum((b - rho) * V)) * np.eye(3)
    return s / a ** 3
