"""Pins for the oracle's Fermi-operator expansion, Fermi level and energies.

References that do not use the expansion: the eigendecomposition of H_s
(numpy.linalg.eigh) gives g(H_s) exactly; scipy.optimize.brentq on
sum_i g(lambda_i; mu) = N_e/2 gives mu; the band and entropy energies have
closed forms in the eigenvalues; numpy.polynomial.chebyshev.chebinterpolate
gives interpolation coefficients at the same nodes.
"""

import numpy as np
import numpy.polynomial.chebyshev as npc
import pytest
from scipy.optimize import brentq

from oracle import foe


def _random_hs(ns, lo, hi, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((ns, ns)))
    lam = np.sort(rng.uniform(lo, hi, ns))
    return (Q * lam) @ Q.T, lam, Q


def test_fermi_dirac_and_entropy_closed_forms():
    E = np.linspace(-30, 30, 101)
    mu, s = 0.4, 1.7
    g = foe.fermi_dirac(E, mu, s)
    np.testing.assert_allclose(g, 1.0 / (1.0 + np.exp((E - mu) / s)), rtol=1e-14)
    ent = foe.entropy_density(E, mu, s)
    with np.errstate(divide="ignore", invalid="ignore"):
        ref = g * np.log(g) + (1 - g) * np.log1p(-g)
    ok = (g > 1e-300) & (g < 1 - 1e-15)
    np.testing.assert_allclose(ent[ok], ref[ok], rtol=1e-9, atol=1e-15)
    assert np.all(ent <= 0)


def test_coefficients_exact_for_chebyshev_polynomial():
    theta = foe.quadrature_angles(64)
    t = np.cos(theta)
    f = 3 * t ** 3 - 2 * t + 0.5           # = 0.75 T3 + 0.25 T1 ... written in monomials
    c = foe.chebyshev_coefficients(f, 6, theta)
    ref = npc.poly2cheb([0.5, -2.0, 0.0, 3.0])
    # with the halved first term: c0/2 = ref0
    np.testing.assert_allclose([c[0] / 2, c[1], c[2], c[3]], ref, atol=1e-14)
    np.testing.assert_allclose(c[4:], 0, atol=1e-14)


def test_coefficients_match_numpy_interpolation():
    K = 200
    theta = foe.quadrature_angles(K)
    chi, xi, mu, s = 1.0, 9.0, 2.5, 0.8
    c = foe.chebyshev_coefficients(foe.fermi_dirac(xi * np.cos(theta) + chi, mu, s), K - 1, theta)
    ref = npc.chebinterpolate(lambda t: foe.fermi_dirac(xi * t + chi, mu, s), K - 1)
    c_np = c.copy()
    c_np[0] /= 2
    np.testing.assert_allclose(c_np, ref, atol=5e-14)


@pytest.mark.parametrize("sigma,n_pl", [(1.0, 60), (0.3, 200)])
def test_density_kernel_vs_eigh(sigma, n_pl):
    ns = 40
    Hs, lam, Q = _random_hs(ns, -5.0, 6.0, seed=7)
    n_e = 31.0
    dk = foe.density_kernel(Hs, n_e, sigma, n_pl)
    # mu: brentq on the exact eigenvalue count
    mu_ref = brentq(lambda m: 2 * foe.fermi_dirac(lam, m, sigma).sum() - n_e, -50, 50, xtol=1e-15)
    g = foe.fermi_dirac(lam, mu_ref, sigma)
    D_ref = (Q * g) @ Q.T
    # tail bound of the truncated expansion at this mu
    theta = foe.quadrature_angles(4096)
    c_long = foe.chebyshev_coefficients(
        foe.fermi_dirac(dk.xi * np.cos(theta) + dk.chi, dk.mu, sigma), 2000, theta)
    tail = np.abs(c_long[n_pl + 1:]).sum()
    tol = 10 * tail + 1e-12
    assert abs(dk.mu - mu_ref) < max(tol, 1e-12) * 10
    np.testing.assert_allclose(dk.D, D_ref, atol=tol)
    assert abs(2 * np.trace(dk.D) - n_e) < 1e-10
    ev = np.linalg.eigvalsh(dk.D)
    assert ev.min() > -1e-10 and ev.max() < 1 + 1e-10
    e_band = 2 * np.sum(g * lam)
    e_ent = 2 * sigma * np.sum(foe.entropy_density(lam, mu_ref, sigma))
    assert abs(dk.e_band - e_band) < 1e-9 * max(1, abs(e_band)) + 100 * tail
    assert abs(dk.e_ent - e_ent) < 1e-9 * max(1, abs(e_ent)) + 100 * tail
    # band energy also equals 2 tr(D_s H_s)
    assert abs(dk.e_band - 2 * np.trace(dk.D @ Hs)) < 1e-9 * abs(e_band) + 100 * tail


def test_density_kernel_coarse_expansion_converges():
    # a too-low degree misses; the error falls as n_pl grows
    Hs, lam, Q = _random_hs(30, -3.0, 3.0, seed=8)
    sigma, n_e = 0.2, 20.0
    mu = brentq(lambda m: 2 * foe.fermi_dirac(lam, m, sigma).sum() - n_e, -50, 50, xtol=1e-15)
    D_ref = (Q * foe.fermi_dirac(lam, mu, sigma)) @ Q.T
    errs = [np.abs(foe.density_kernel(Hs, n_e, sigma, n).D - D_ref).max() for n in (10, 20, 40, 80)]
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 1e-8


def test_fermi_level_error_when_overfilled():
    Hs, _, _ = _random_hs(10, -1, 1, seed=9)
    with pytest.raises(foe.FermiLevelError):
        foe.density_kernel(Hs, 20.0, 0.5, 20)


@pytest.mark.parametrize("sigma,expect", [(2.0, 32), (1.0, 64), (0.5, 128), (0.3, 256)])
def test_tail_rule_degree(sigma, expect):
    # n_pl = 0: the first of 32, 64, ... whose coefficient tail at its own mu
    # is <= 1e-12; the result then equals the eigh definition to that tail
    ns = 40
    Hs, lam, Q = _random_hs(ns, -5.0, 6.0, seed=11)
    n_e = 31.0
    dk = foe.density_kernel(Hs, n_e, sigma, 0)
    assert dk.n_pl == expect
    assert foe.coefficient_tail(dk.mu, dk.chi, dk.xi, sigma, dk.n_pl) <= foe.TAIL_TOL
    if dk.n_pl > foe.TAIL_START:
        lower = foe.density_kernel(Hs, n_e, sigma, dk.n_pl // 2)
        assert foe.coefficient_tail(lower.mu, lower.chi, lower.xi, sigma, dk.n_pl // 2) > foe.TAIL_TOL
    mu_ref = brentq(lambda m: 2 * foe.fermi_dirac(lam, m, sigma).sum() - n_e, -50, 50, xtol=1e-15)
    D_ref = (Q * foe.fermi_dirac(lam, mu_ref, sigma)) @ Q.T
    np.testing.assert_allclose(dk.D, D_ref, atol=2e-11)
    assert abs(dk.mu - mu_ref) < 1e-10


def test_tail_rule_gives_up_beyond_cap():
    Hs, lam, Q = _random_hs(24, -5.0, 6.0, seed=12)
    with pytest.raises(foe.DegreeError):
        foe.density_kernel(Hs, 17.0, 0.01, 0)
