"""Pins for the molecular-dynamics oracle: Verlet reversibility and energy
conservation with an exact-gradient force field (the pseudocharge
electrostatics and core term of a fixed electron density), and the
Maxwell-Boltzmann draw."""

import numpy as np
from scipy.integrate import solve_ivp

from oracle import electrostatics as es
from oracle import qmd


def _field(n=12, a=6.0):
    x = np.arange(n) * a / n
    rho = 0.2 + 0.05 * (np.cos(2 * np.pi * x / a)[None, None, :]
                        * np.sin(2 * np.pi * x / a)[:, None, None]).repeat(n, axis=1).reshape(-1)
    h = a / n

    def force(pos):
        b = es.pseudocharge(n, a, pos, 3.0, 0.8)
        src = rho - rho.mean() + b - b.mean()
        vc = es.poisson_fft(src, n, a)
        vcore = es.core_potential(n, a, pos, 1.5, 0.5)
        e = 0.5 * h ** 3 * np.sum(src * vc) + h ** 3 * np.sum(rho * vcore)
        return es.local_forces(n, a, pos, 3.0, 0.8, 1.5, 0.5, rho, vc), e

    return force


def test_maxwell_boltzmann_draw():
    v = qmd.maxwell_boltzmann(64, qmd.M_AL, 10 * qmd.EV, 7)
    assert np.abs(v.sum(axis=0)).max() < 1e-15
    t = 2 * qmd.kinetic_energy(v, qmd.M_AL) / (3 * 64)
    assert 0.7 < t / (10 * qmd.EV) < 1.3


def test_verlet_is_time_reversible_and_second_order():
    force = _field()
    x0 = np.array([[1.0, 2.0, 1.5], [4.1, 3.3, 4.4]])
    m = 2000.0
    v0 = np.array([[1e-3, -2e-3, 5e-4], [-1e-3, 2e-3, -5e-4]])
    f0, e0 = force(x0)
    x1, v1, f1, en = qmd.verlet(x0, v0, f0, m, 20.0, force, 20)
    assert np.abs(x1 - x0).max() > 0.5
    x2, v2, _, _ = qmd.verlet(x1, -v1, f1, m, 20.0, force, 20)
    assert np.abs(x2 - x0).max() < 1e-9
    assert np.abs(v2 + v0).max() < 1e-12
    # the energy error of velocity Verlet is second order in the step
    etot0 = e0 + qmd.kinetic_energy(v0, m)
    _, _, _, en_half = qmd.verlet(x0, v0, f0, m, 10.0, force, 40)
    err = max(abs(e - etot0) for e in en)
    err_half = max(abs(e - etot0) for e in en_half)
    assert 3.0 < err / err_half < 5.0


def test_isokinetic_kick_is_the_flow_of_its_equation():
    rng = np.random.default_rng(3)
    m = 50.0
    for scale in (1.0, 1e-3, 30.0):
        v0 = rng.standard_normal((5, 3))
        f = scale * rng.standard_normal((5, 3))
        tau = 0.7

        def rhs(_, u):
            g = f.ravel() / m
            return g - (g @ u) / (u @ u) * u

        ref = solve_ivp(rhs, (0.0, tau), v0.ravel(), method="DOP853", rtol=1e-13,
                        atol=1e-15).y[:, -1].reshape(5, 3)
        got = qmd.isokinetic_kick(v0, f, m, tau)
        assert np.abs(got - ref).max() < 1e-10 * np.abs(ref).max()
        assert abs(np.sum(got * got) / np.sum(v0 * v0) - 1.0) < 1e-14
    # no force: no change; force along v: speed kept, direction kept
    v0 = rng.standard_normal((4, 3))
    np.testing.assert_allclose(qmd.isokinetic_kick(v0, np.zeros((4, 3)), m, 1.0), v0, rtol=1e-15)
    np.testing.assert_allclose(qmd.isokinetic_kick(v0, 3.0 * v0, m, 1.0), v0, rtol=1e-14)


def test_isokinetic_verlet_keeps_kinetic_energy_and_is_reversible():
    force = _field()
    x0 = np.array([[1.0, 2.0, 1.5], [4.1, 3.3, 4.4], [2.5, 0.3, 5.1]])
    m = 2000.0
    v0 = qmd.isokinetic_start(3, m, 0.05, 11)
    assert abs(qmd.kinetic_energy(v0, m) - 0.5 * 6 * 0.05) < 1e-15
    assert np.abs(v0.sum(axis=0)).max() < 1e-15
    f0, _ = force(x0)
    x1, v1, f1, _ = qmd.isokinetic_verlet(x0, v0, f0, m, 20.0, force, 20)
    assert np.abs(x1 - x0).max() > 0.5
    assert abs(qmd.kinetic_energy(v1, m) / qmd.kinetic_energy(v0, m) - 1.0) < 1e-13
    x2, v2, _, _ = qmd.isokinetic_verlet(x1, -v1, f1, m, 20.0, force, 20)
    assert np.abs(x2 - x0).max() < 1e-9
    assert np.abs(v2 + v0).max() < 1e-12
