"""Green-Kubo transport coefficients from molecular-dynamics series (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 5 (high-temperature QMD) writes the self-diffusion coefficient and the
shear viscosity as time integrals of equilibrium autocorrelation functions:

  D(t)   = (1 / 3N) sum_i int_0^t <v_i(tau) . v_i(0)> dtau,
  eta(t) = (|Omega| / k_B T) int_0^t (1/5) sum_{m=1..5} <s_m(tau) s_m(0)> dtau,

with s_m the five independent components of the traceless (deviatoric) stress:
sigma_12, sigma_23, sigma_31, (sigma_11 - sigma_22)/2, (sigma_22 - sigma_33)/2.

Readings where the paper is silent:
  * the ensemble average <a(tau) b(0)> of a single run is the average over
    time origins: for a series of T samples at spacing dt, lag k uses the
    T - k origins t0 = 0 .. T-k-1;
  * a series of n_comp components is correlated component by component and
    averaged over the components: C(k) = sum_c sum_t0 s_c(t0+k) s_c(t0) /
    (n_comp (T - k)).  For the 3N velocity components this is the paper's
    VACF / 3, so D(t) = int_0^t C; for the five stress components it is the
    paper's SACF;
  * the time integral is the trapezoid rule on the sample spacing:
    I(0) = 0, I(k) = I(k-1) + dt (C(k-1) + C(k)) / 2;
  * the stress in the viscosity is the full microscopic stress of the cell:
    the Hellmann-Feynman stress of the electrons and ions minus the ions'
    momentum flux, sigma_ab - sum_I M v_Ia v_Ib / |Omega|.
"""

from __future__ import annotations

import numpy as np


def time_correlation(series: np.ndarray, max_lag: int) -> np.ndarray:
    """C(k), k = 0 .. max_lag - 1, of a (T, n_comp) series (see the readings)."""
    s = np.asarray(series, dtype=np.float64)
    if s.ndim == 1:
        s = s[:, None]
    T, n = s.shape
    if not 0 < max_lag <= T:
        raise ValueError("time_correlation: need 0 < max_lag <= T")
    out = np.empty(max_lag)
    for k in range(max_lag):
        out[k] = np.sum(s[k:] * s[:T - k]) / (n * (T - k))
    return out


def running_integral(c: np.ndarray, dt: float) -> np.ndarray:
    """Trapezoid running integral I(k) of samples c at spacing dt, I(0) = 0."""
    c = np.asarray(c, dtype=np.float64)
    out = np.zeros_like(c)
    for k in range(1, len(c)):
        out[k] = out[k - 1] + 0.5 * dt * (c[k - 1] + c[k])
    return out


def deviatoric_components(sigma: np.ndarray) -> np.ndarray:
    """(T, 3, 3) stresses -> (T, 5): sigma_12, sigma_23, sigma_31,
    (sigma_11 - sigma_22)/2, (sigma_22 - sigma_33)/2."""
    s = np.asarray(sigma, dtype=np.float64).reshape(-1, 3, 3)
    return np.stack([s[:, 0, 1], s[:, 1, 2], s[:, 2, 0],
                     0.5 * (s[:, 0, 0] - s[:, 1, 1]), 0.5 * (s[:, 1, 1] - s[:, 2, 2])], axis=1)


def ionic_momentum_flux(v: np.ndarray, mass: float, volume: float) -> np.ndarray:
    """sum_I M v_Ia v_Ib / |Omega| for velocities v (N, 3)."""
    v = np.asarray(v, dtype=np.float64).reshape(-1, 3)
    return mass * (v.T @ v) / volume


def self_diffusion(velocities: np.ndarray, dt: float, max_lag: int):
    """velocities (T, N, 3) -> (C(k) = VACF/3, D(t_k)) in bohr^2 per a.u. of time."""
    v = np.asarray(velocities, dtype=np.float64)
    c = time_correlation(v.reshape(v.shape[0], -1), max_lag)
    return c, running_integral(c, dt)


def viscosity(stress: np.ndarray, volume: float, kT: float, dt: float, max_lag: int):
    """stress (T, 3, 3) total microscopic stress -> (SACF(k), eta(t_k)) in
    Ha a.u.-time / bohr^3."""
    c = time_correlation(deviatoric_components(stress), max_lag)
    return c, (volume / kT) * running_integral(c, dt)
