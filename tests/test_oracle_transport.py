"""Pins for the oracle's Green-Kubo functions (Sec. 5, high-temperature QMD).

* time correlation: closed forms for constant and linear series (lag offset and
  origin count), and an independent evaluation by zero-padded FFTs
  (Wiener-Khinchin) on random series;
* trapezoid integral: the geometric-series closed form on sampled exponentials,
  and convergence to the continuum integral tau as dt -> 0;
* deviatoric components: hand-evaluated values, zero for an isotropic stress;
* a stationary signal with a known autocorrelation: an average over many
  random-phase cosines has correlation cos(omega tau) / 2 up to sampling noise.
"""

import numpy as np
import pytest

from oracle import transport as tr


def test_constant_series():
    a = np.array([1.5, -2.0, 0.5])
    s = np.tile(a, (40, 1))
    c = tr.time_correlation(s, 25)
    np.testing.assert_allclose(c, np.mean(a * a), rtol=1e-15)


def test_linear_series_closed_form():
    # s(t) = a + b t (one component): sum_{t0=0}^{M-1} (a + b t0 + b k)(a + b t0), M = T - k
    a, b, T = 0.7, -0.13, 31
    s = (a + b * np.arange(T))[:, None]
    c = tr.time_correlation(s, T)
    for k in range(T):
        M = T - k
        S0, S1, S2 = M, M * (M - 1) / 2, (M - 1) * M * (2 * M - 1) / 6
        ref = (a * a * S0 + 2 * a * b * S1 + b * b * S2 + b * k * (a * S0 + b * S1)) / M
        assert abs(c[k] - ref) < 1e-12 * max(1.0, abs(ref))


def test_against_fft_correlation():
    rng = np.random.default_rng(3)
    T, n, K = 300, 7, 120
    s = rng.standard_normal((T, n))
    c = tr.time_correlation(s, K)
    f = np.fft.rfft(s, n=2 * T, axis=0)
    acf = np.fft.irfft(f * np.conj(f), n=2 * T, axis=0)[:K].sum(axis=1)
    ref = acf / (n * (T - np.arange(K)))
    np.testing.assert_allclose(c, ref, rtol=0, atol=1e-13)
    with pytest.raises(ValueError):
        tr.time_correlation(s, T + 1)


@pytest.mark.parametrize("dt", [0.3, 0.05])
def test_trapezoid_on_exponential(dt):
    tau, K = 2.0, 400
    q = np.exp(-dt / tau)
    c = q ** np.arange(K)
    got = tr.running_integral(c, dt)
    for k in (1, 17, K - 1):
        # dt [ (1 + q^k)/2 + sum_{j=1}^{k-1} q^j ]
        ref = dt * (0.5 * (1 + q ** k) + (q - q ** k) / (1 - q))
        assert abs(got[k] - ref) < 1e-13
    # continuum limit: int_0^inf e^{-t/tau} = tau, trapezoid error dt^2/(12 tau)
    assert abs(got[-1] - tau) < dt * dt / (12 * tau) * 1.05 + tau * q ** (K - 1)


def test_deviatoric_components():
    sig = np.array([[1.0, 2.0, 3.0], [2.0, 5.0, 7.0], [3.0, 7.0, 11.0]])
    s = tr.deviatoric_components(sig[None])[0]
    np.testing.assert_allclose(s, [2.0, 7.0, 3.0, -2.0, -3.0], rtol=1e-15)
    iso = 4.2 * np.eye(3)[None]
    np.testing.assert_allclose(tr.deviatoric_components(iso), 0.0, atol=1e-15)
    flux = tr.ionic_momentum_flux(np.array([[1.0, 2.0, 0.0], [0.0, 1.0, 3.0]]), 2.0, 4.0)
    np.testing.assert_allclose(flux, 0.5 * np.array([[1, 2, 0], [2, 5, 3], [0, 3, 9]]),
                               rtol=1e-15)


def test_random_phase_cosines_and_diffusion_integral():
    # v_c(t) = cos(omega t + phi_c) for many random phases: C(k) -> cos(omega k dt) / 2;
    # its integral sin(omega t) / (2 omega) is what self_diffusion returns
    rng = np.random.default_rng(8)
    T, n, dt, omega = 400, 3 * 400, 0.1, 0.7
    t = dt * np.arange(T)
    phi = rng.uniform(0, 2 * np.pi, n)
    v = np.cos(omega * t[:, None] + phi[None, :]).reshape(T, n // 3, 3)
    c, d = tr.self_diffusion(v, dt, 100)
    tau = dt * np.arange(100)
    assert np.abs(c - 0.5 * np.cos(omega * tau)).max() < 0.05
    assert np.abs(d - np.sin(omega * tau) / (2 * omega)).max() < 0.05
