"""LDA exchange-correlation of the unpolarised electron gas (oracle).

The paper's calculations use the local density approximation (Sec. 5); the
self-consistent workloads here take the Perdew-Wang 1992 parametrisation of
the correlation energy (Phys. Rev. B 45, 13244), written out from its
published form:

  r_s = (3 / (4 pi rho))^(1/3)
  eps_x(r_s) = -(3 / (4 pi)) (9 pi / 4)^(1/3) / r_s          (Slater exchange)
  eps_c(r_s) = -2 A (1 + alpha_1 r_s)
               * ln(1 + 1 / (2 A (beta_1 r_s^1/2 + beta_2 r_s + beta_3 r_s^3/2 + beta_4 r_s^2)))
  v_xc = d(rho eps_xc)/d rho = eps_xc - (r_s / 3) d eps_xc / d r_s

with the unpolarised parameters A = 0.031091, alpha_1 = 0.21370,
beta_1..4 = 7.5957, 3.5876, 1.6382, 0.49294 (Hartree units).  Densities at or
below RHO_FLOOR give eps_xc = v_xc = 0.

Pins (tests): v_xc against central differences of rho eps_xc; the high-density
limit eps_c ~ c0 ln r_s - c1 with c0 = (1 - ln 2)/pi^2 (the exact
random-phase coefficient, which A reproduces) and the c1 that beta_1 encodes;
the low-density limit eps_c ~ -(alpha_1/beta_4)/r_s; beta_2 = 2 A beta_1^2,
which removes the r_s^(1/2) term the exact high-density expansion lacks.
beta_3 has no closed-form pin: parity unpinned for it.
"""

from __future__ import annotations

import numpy as np

A = 0.031091
ALPHA1 = 0.21370
BETA = (7.5957, 3.5876, 1.6382, 0.49294)
RHO_FLOOR = 1e-20
CX = (3.0 / (4.0 * np.pi)) * (9.0 * np.pi / 4.0) ** (1.0 / 3.0)


def wigner_seitz_radius(rho):
    return (3.0 / (4.0 * np.pi * np.asarray(rho, dtype=np.float64))) ** (1.0 / 3.0)


def eps_x(rs):
    return -CX / rs


def eps_c(rs):
    b1, b2, b3, b4 = BETA
    q1 = 2.0 * A * (b1 * np.sqrt(rs) + b2 * rs + b3 * rs ** 1.5 + b4 * rs * rs)
    return -2.0 * A * (1.0 + ALPHA1 * rs) * np.log1p(1.0 / q1)


def deps_c_drs(rs):
    b1, b2, b3, b4 = BETA
    q0 = -2.0 * A * (1.0 + ALPHA1 * rs)
    q1 = 2.0 * A * (b1 * np.sqrt(rs) + b2 * rs + b3 * rs ** 1.5 + b4 * rs * rs)
    dq1 = A * (b1 / np.sqrt(rs) + 2.0 * b2 + 3.0 * b3 * np.sqrt(rs) + 4.0 * b4 * rs)
    return -2.0 * A * ALPHA1 * np.log1p(1.0 / q1) - q0 * dq1 / (q1 * q1 + q1)


def lda(rho):
    """(eps_xc, v_xc) per grid point for the density rho (bohr^-3)."""
    rho = np.asarray(rho, dtype=np.float64)
    live = rho > RHO_FLOOR
    rs = wigner_seitz_radius(np.where(live, rho, 1.0))
    ex = eps_x(rs)
    ec = eps_c(rs)
    vx = (4.0 / 3.0) * ex
    vc = ec - (rs / 3.0) * deps_c_drs(rs)
    eps = np.where(live, ex + ec, 0.0)
    v = np.where(live, vx + vc, 0.0)
    return eps, v


def energy(rho, h: float) -> float:
    """E_xc = h^3 sum rho eps_xc."""
    eps, _ = lda(rho)
    return float(h ** 3 * np.sum(np.asarray(rho) * eps))
