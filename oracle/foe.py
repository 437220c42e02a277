"""Chebyshev Fermi-operator expansion of the density kernel (oracle).

Sec. 4 of the paper:
  * D_s = g(H_s, mu, sigma) with g the Fermi-Dirac function (Eq. DsHsRelation).
  * D_s ~ sum'_{j=0}^{n_pl} c_j(mu, sigma) T_j(Hhat), Hhat = (H_s - chi I)/xi,
    chi = (lambda_max + lambda_min)/2, xi = (lambda_max - lambda_min)/2; the
    prime halves the j = 0 term (Eq. ChebyshevExpansion).
  * c_j = (2/pi) int_{-1}^{1} g(xi t + chi) T_j(t) / sqrt(1 - t^2) dt
    (Eq. ChebyshevCoeff).
  * column n of D_s is sum'_j c_j t_n^j with t^0_n = e_n, t^1_n = Hhat e_n,
    t^{j+1}_n = 2 Hhat t^j_n - t^{j-1}_n (Eqs. DMCFinal, ThreeTermRecurrence).
  * mu solves 2 sum_n sum'_j c_j(mu) e_n^T t^j_n = N_e (Eq. FermiLevelCalc).
  * E_band = 2 sum_n sum'_j d_j e_n^T t^j_n and E_ent likewise with e_j, where
    d_j, e_j expand E g(E) and g log g + (1-g) log(1-g).  The entropy energy
    carries the factor sigma of the free-energy expression (Eq.
    FreeEnergy:NewForm); its expansion formula omits it, read here as
    E_ent = 2 sigma sum'_j e_j tau_j.

Readings (the paper states the integrals, not how to evaluate them):
  * integrals by K-node Gauss-Chebyshev quadrature, theta_k = pi (k + 1/2)/K,
    c_j = (2/K) sum_k f(xi cos theta_k + chi) cos(j theta_k),
    K = max(1024, 4 (n_pl + 1));
  * chi, xi from the exact extreme eigenvalues of H_s (if xi vanishes, xi = 1);
  * mu by bisection on [lambda_min - 40 sigma - 1, lambda_max + 40 sigma + 1]
    until the bracket is below 1e-14 max(1, |mu|) (at most 200 halvings);
    the midpoint of the last bracket is returned.
  * degree chosen by a tail rule when n_pl = 0 (the paper picks the degree per
    system for a target accuracy): try n = 32, 64, 128, 256; at each, solve
    for mu with the degree-n expansion and accept n once the coefficient tail
    sum_{n < j <= 4n} |c_j(mu)| (coefficients by the same quadrature with
    K = max(1024, 4(4n + 1)) nodes) is at most 1e-12.  No acceptable n up to
    256 is an error.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


class FermiLevelError(ValueError):
    pass


class DegreeError(ValueError):
    pass


TAIL_START, TAIL_CAP, TAIL_TOL = 32, 256, 1e-12


def fermi_dirac(E, mu: float, sigma: float):
    """g = (1 + exp(s))^{-1}, s = (E - mu)/sigma, with the exponent kept <= 0."""
    s = (np.asarray(E, dtype=np.float64) - mu) / sigma
    q = np.exp(-np.abs(s))
    return np.where(s > 0, q / (1.0 + q), 1.0 / (1.0 + q))


def _softplus(s):
    return np.maximum(s, 0.0) + np.log1p(np.exp(-np.abs(s)))


def entropy_density(E, mu: float, sigma: float):
    """g log g + (1 - g) log(1 - g), evaluated without cancellation."""
    s = (np.asarray(E, dtype=np.float64) - mu) / sigma
    g = fermi_dirac(E, mu, sigma)
    # log g = -softplus(s), log(1 - g) = -softplus(-s)
    return -(g * _softplus(s) + (1.0 - g) * _softplus(-s))


def n_nodes(n_pl: int) -> int:
    return max(1024, 4 * (n_pl + 1))


def quadrature_angles(K: int) -> np.ndarray:
    return np.pi * (np.arange(K) + 0.5) / K


def chebyshev_coefficients(fvals: np.ndarray, n_pl: int, theta: np.ndarray) -> np.ndarray:
    """c_j, j = 0..n_pl, from f sampled at the Gauss-Chebyshev nodes."""
    K = len(theta)
    j = np.arange(n_pl + 1)
    cosm = np.cos(np.outer(theta, j))  # (K, n_pl+1)
    return (2.0 / K) * (fvals @ cosm)


def prime_sum(coef: np.ndarray, tau: np.ndarray) -> float:
    """sum'_j coef_j tau_j  (first term halved)."""
    return float(np.dot(coef, tau) - 0.5 * coef[0] * tau[0])


def spectral_interval(Hs: np.ndarray):
    lam = np.linalg.eigvalsh(Hs)
    lo, hi = float(lam[0]), float(lam[-1])
    chi = 0.5 * (hi + lo)
    xi = 0.5 * (hi - lo)
    if xi <= 1e-12 * max(1.0, abs(chi)):
        xi = 1.0
    return lo, hi, chi, xi


def chebyshev_matrices(Hhat: np.ndarray, n_pl: int):
    """[T_0(Hhat), ..., T_n_pl(Hhat)] by the three-term recurrence, all columns at once."""
    ns = Hhat.shape[0]
    T = [np.eye(ns)]
    if n_pl >= 1:
        T.append(Hhat.copy())
    for _ in range(1, n_pl):
        T.append(2.0 * Hhat @ T[-1] - T[-2])
    return T


@dataclass
class DensityKernel:
    D: np.ndarray
    mu: float
    chi: float
    xi: float
    lam_min: float
    lam_max: float
    tau: np.ndarray
    c: np.ndarray
    d: np.ndarray
    e: np.ndarray
    e_band: float
    e_ent: float
    n_pl: int
    iterations: int


def electron_count(mu: float, tau, chi, xi, sigma, n_pl, theta) -> float:
    E = xi * np.cos(theta) + chi
    c = chebyshev_coefficients(fermi_dirac(E, mu, sigma), n_pl, theta)
    return 2.0 * prime_sum(c, tau)


def fermi_level(tau, chi, xi, lam_min, lam_max, sigma, n_e, n_pl, theta):
    lo = lam_min - 40.0 * sigma - 1.0
    hi = lam_max + 40.0 * sigma + 1.0
    f_lo = electron_count(lo, tau, chi, xi, sigma, n_pl, theta) - n_e
    f_hi = electron_count(hi, tau, chi, xi, sigma, n_pl, theta) - n_e
    if not (f_lo < 0.0 < f_hi):
        raise FermiLevelError(f"no sign change: N(lo)-N_e={f_lo}, N(hi)-N_e={f_hi}")
    it = 0
    while it < 200:
        mid = 0.5 * (lo + hi)
        if hi - lo <= 1e-14 * max(1.0, abs(mid)):
            break
        f_mid = electron_count(mid, tau, chi, xi, sigma, n_pl, theta) - n_e
        if f_mid < 0.0:
            lo = mid
        else:
            hi = mid
        it += 1
    return 0.5 * (lo + hi), it


def coefficient_tail(mu: float, chi: float, xi: float, sigma: float, n: int) -> float:
    """sum_{n < j <= 4n} |c_j(mu)| of the Fermi-Dirac expansion on [chi - xi, chi + xi]."""
    J = 4 * n
    theta = quadrature_angles(n_nodes(J))
    c = chebyshev_coefficients(fermi_dirac(xi * np.cos(theta) + chi, mu, sigma), J, theta)
    return float(np.abs(c[n + 1:]).sum())


def density_kernel(Hs: np.ndarray, n_e: float, sigma: float, n_pl: int) -> DensityKernel:
    """n_pl = 0 selects the degree by the tail rule (module docstring)."""
    ns = Hs.shape[0]
    if not (0.0 < n_e < 2.0 * ns):
        raise FermiLevelError("need 0 < N_e < 2 N_s")
    Hs = 0.5 * (Hs + Hs.T)
    lam_min, lam_max, chi, xi = spectral_interval(Hs)
    Hhat = (Hs - chi * np.eye(ns)) / xi
    tail_rule = n_pl == 0
    n_pl = TAIL_START if tail_rule else n_pl
    while True:
        T = chebyshev_matrices(Hhat, n_pl)
        tau = np.array([np.trace(t) for t in T])
        K = n_nodes(n_pl)
        theta = quadrature_angles(K)
        mu, iters = fermi_level(tau, chi, xi, lam_min, lam_max, sigma, n_e, n_pl, theta)
        if not tail_rule or coefficient_tail(mu, chi, xi, sigma, n_pl) <= TAIL_TOL:
            break
        if 2 * n_pl > TAIL_CAP:
            raise DegreeError(f"coefficient tail above {TAIL_TOL} at degree {n_pl}")
        n_pl *= 2
    E = xi * np.cos(theta) + chi
    c = chebyshev_coefficients(fermi_dirac(E, mu, sigma), n_pl, theta)
    d = chebyshev_coefficients(E * fermi_dirac(E, mu, sigma), n_pl, theta)
    e = chebyshev_coefficients(entropy_density(E, mu, sigma), n_pl, theta)
    D = 0.5 * c[0] * T[0]
    for j in range(1, n_pl + 1):
        D = D + c[j] * T[j]
    e_band = 2.0 * prime_sum(d, tau)
    e_ent = 2.0 * sigma * prime_sum(e, tau)
    return DensityKernel(D, mu, chi, xi, lam_min, lam_max, tau, c, d, e,
                         e_band, e_ent, n_pl, iters)
