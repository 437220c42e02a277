"""Pins for the self-consistent-field support of the oracle.

* PW92: v_xc is the density derivative of rho eps_xc (central differences);
  Slater exchange in its second textbook form; the high- and low-density
  limits of the correlation energy (exact random-phase coefficient
  (1 - ln 2)/pi^2 and the constants the parametrisation encodes);
* Poisson: the FFT solution satisfies the pinned FD Laplacian to rounding;
* pseudocharges: discrete charge -Z per atom; their electrostatic energy
  equals the Ewald energy of point charges (itself independent of the
  splitting parameter) plus the Gaussian-background term, to the
  discretisation error;
* forces: pseudocharge and core forces are minus the position derivative of
  the electrostatic-plus-core energy (central differences);
* Pulay: a linear fixed-point problem in n unknowns is solved in n + 1 steps
  (n + 2 to rounding, the normal equations carrying a 1e-12 shift);
* SCF: in the full space (N_s = N_grid, no filtering) the SCF fixed point equals
  a brute-force SCF by dense diagonalisation, and the converged forces are
  minus the derivative of the converged free energy.
"""

import math

import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import electrostatics as es
from oracle import fd, foe, xc
from oracle.hamiltonian import Hamiltonian
from oracle.mixing import PeriodicPulay, Pulay, kerker
from oracle.scf import LocalModel, effective_potential, scf
from workloads import custom_spec, make_problem

MODEL = LocalModel(3.0, 0.8, 1.5, 0.5)


def test_pw92_potential_is_derivative_of_energy_density():
    rho = np.geomspace(1e-5, 10.0, 60)
    eps, v = xc.lda(rho)
    d = 1e-5 * rho
    ep, _ = xc.lda(rho + d)
    em, _ = xc.lda(rho - d)
    num = ((rho + d) * ep - (rho - d) * em) / (2 * d)
    np.testing.assert_allclose(v, num, rtol=1e-8)


def test_pw92_limits_and_exchange():
    rho = np.array([0.01, 0.3, 2.0])
    rs = xc.wigner_seitz_radius(rho)
    np.testing.assert_allclose(xc.eps_x(rs), -0.75 * (3 * rho / math.pi) ** (1 / 3), rtol=1e-14)
    # high density: eps_c = c0 ln rs - c1 + O(rs ln rs)
    c0 = (1 - math.log(2)) / math.pi ** 2
    r1, r2 = 1e-9, 1e-8
    slope = (xc.eps_c(r2) - xc.eps_c(r1)) / math.log(r2 / r1)
    assert abs(slope - c0) < 2e-5 * c0
    c1 = -(xc.eps_c(1e-10) - c0 * math.log(1e-10))
    assert abs(c1 - 0.046644) < 1e-5
    # low density: rs eps_c -> -alpha_1 / beta_4 = -0.43352
    assert abs(1e12 * xc.eps_c(1e12) + 0.43352) < 1e-5
    assert np.all(np.diff(xc.eps_c(np.geomspace(0.1, 50, 30))) > 0)  # eps_c < 0, rising to 0


def test_pw92_high_density_expansion_has_no_sqrt_rs_term():
    # The exact high-density expansion of the correlation energy goes
    # c0 ln rs - c1 + O(rs ln rs): no rs^(1/2) term.  In the PW92 form the
    # rs^(1/2) coefficient works out to 2A (beta_2/beta_1 - 2A beta_1), so the
    # expansion fixes beta_2 = 2A beta_1^2 (to the printed digits).
    # (c0 = A in this form; the slope test above pins A against (1 - ln 2)/pi^2)
    b1, b2 = xc.BETA[0], xc.BETA[1]
    assert abs(b2 - 2 * xc.A * b1 * b1) < 1e-4 * b2
    c1 = -2 * xc.A * math.log(2 * xc.A * b1)
    # the remainder after A ln rs - c1, over rs^(1/2), vanishes as rs -> 0
    # (a 1% error in beta_2 would leave about 3e-4 here)
    rems = [abs(xc.eps_c(rs) - (xc.A * math.log(rs) - c1)) / math.sqrt(rs)
            for rs in (1e-8, 1e-10, 1e-12)]
    assert rems[0] > rems[1] > rems[2] and rems[1] < 5e-6, rems


def test_pw92_floor():
    eps, v = xc.lda(np.array([0.0, -1e-12, 1e-21]))
    assert np.all(eps == 0) and np.all(v == 0)


def test_poisson_fft_solves_fd_system():
    n, a = 16, 6.0
    rng = np.random.default_rng(3)
    src = rng.standard_normal(n ** 3)
    v = es.poisson_fft(src, n, a)
    lap = fd.laplacian(v[:, None], n, a / n)[:, 0]
    np.testing.assert_allclose(-lap, 4 * np.pi * (src - src.mean()), atol=1e-11 * np.abs(src).max())
    assert abs(v.mean()) < 1e-14


def test_pseudocharge_electrostatics_matches_ewald():
    pos = np.array([[0.1, 0.2, 0.3], [3.9, 3.7, 0.2], [3.6, 0.3, 3.9], [0.4, 3.8, 3.5]])
    a, n, z, rc = 7.6, 36, 3.0, 0.8
    q = np.full(4, -z)
    ew = [es.ewald_energy(pos, q, a, eta) for eta in (0.6, 1.3)]
    assert abs(ew[0] - ew[1]) < 1e-12 * abs(ew[0])
    b = es.pseudocharge(n, a, pos, z, rc)
    h = a / n
    assert abs(h ** 3 * b.sum() + 4 * z) < 1e-12
    v = es.poisson_fft(b, n, a)
    Q = q.sum()
    e = (0.5 * h ** 3 * np.sum((b - b.mean()) * v) - es.self_energy(4, z, rc)
         - math.pi * Q * Q * rc * rc / a ** 3)
    assert abs(e - ew[0]) < 1e-7 * abs(ew[0])


def test_local_forces_are_energy_derivatives():
    n, a = 16, 6.0
    pos = np.array([[1.0, 2.0, 1.5], [4.1, 3.3, 4.4]])
    rng = np.random.default_rng(4)
    x = np.arange(n) * a / n
    rho = 0.1 + 0.02 * (np.sin(2 * np.pi * x / a)[None, None, :] *
                        np.cos(4 * np.pi * x / a)[:, None, None]).repeat(n, axis=1).reshape(-1)
    rho = rho + 0.001 * rng.standard_normal(n ** 3)
    h = a / n

    def energy(p):
        b = es.pseudocharge(n, a, p, 3.0, 0.8)
        src = rho - rho.mean() + b - b.mean()  # a neutral source
        vc = es.poisson_fft(src, n, a)
        vcore = es.core_potential(n, a, p, 1.5, 0.5)
        return 0.5 * h ** 3 * np.sum(src * vc) + h ** 3 * np.sum(rho * vcore), vc

    _, vc = energy(pos)
    f = es.local_forces(n, a, pos, 3.0, 0.8, 1.5, 0.5, rho, vc)
    d = 1e-4
    for i in range(2):
        for ax in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, ax] += d
            pm[i, ax] -= d
            num = -(energy(pp)[0] - energy(pm)[0]) / (2 * d)
            assert abs(f[i, ax] - num) < 1e-7 * max(1.0, abs(num))


def test_pulay_solves_linear_fixed_point_in_n_plus_one_steps():
    n = 5
    rng = np.random.default_rng(8)
    M = 0.5 * rng.standard_normal((n, n)) / math.sqrt(n)
    c = rng.standard_normal(n)
    exact = np.linalg.solve(np.eye(n) - M, c)
    mixer = Pulay(history=7, beta=0.3)
    x = np.zeros(n)
    first = mixer.mix(x, M @ x + c)
    np.testing.assert_allclose(first, 0.3 * c, atol=1e-15)  # first step: linear mixing
    x = first
    for _ in range(n):
        x = mixer.mix(x, M @ x + c)
    # n + 1 steps: exact up to the 1e-12 shift of the normal equations
    assert np.linalg.norm(x - exact) < 1e-6 * np.linalg.norm(exact)
    x = mixer.mix(x, M @ x + c)
    assert np.linalg.norm(x - exact) < 1e-13 * np.linalg.norm(exact)


def test_kerker_is_the_dense_operator():
    # P = (-L + k0^2)^{-1}(-L) with L the dense FD Laplacian of a 6^3 grid
    n, h, k0 = 6, 0.7, 0.8
    Lap = fd.laplacian(np.eye(n ** 3), n, h)
    P = np.linalg.solve(-Lap + k0 * k0 * np.eye(n ** 3), -Lap)
    F = np.random.default_rng(12).standard_normal(n ** 3)
    got = kerker(F, n, h, k0)
    np.testing.assert_allclose(got, P @ F, atol=1e-12 * np.abs(P @ F).max())
    assert abs(got.sum()) < 1e-11 * np.abs(F).sum()   # the mean is removed
    np.testing.assert_array_equal(kerker(F, n, h, 0.0), F)


def test_periodic_pulay_special_cases_and_convergence():
    n, h = 4, 0.9
    N = n ** 3
    rng = np.random.default_rng(13)
    # a contractive linear map whose fixed point has the mean of the start
    Q = np.linalg.qr(rng.standard_normal((N, N)))[0]
    M = Q @ np.diag(np.linspace(-0.6, 0.9, N)) @ Q.T
    c = rng.standard_normal(N)
    c -= c.mean()
    M -= M.mean(axis=0, keepdims=True)     # M x has zero mean for every x
    exact = np.linalg.solve(np.eye(N) - M, c)
    # period 1 without preconditioning is the Pulay step
    a, b = PeriodicPulay(n, h, history=5, beta=0.3, period=1, k0=0.0), Pulay(5, 0.3)
    x = y = np.zeros(N)
    for _ in range(8):
        x, y = a.mix(x, M @ x + c), b.mix(y, M @ y + c)
        np.testing.assert_allclose(x, y, atol=1e-14)
    # a period longer than the run is preconditioned linear mixing
    a = PeriodicPulay(n, h, history=5, beta=0.3, period=100, k0=1.1)
    x = np.zeros(N)
    for _ in range(5):
        want = x + 0.3 * kerker(M @ x + c - x, n, h, 1.1)
        x = a.mix(x, M @ x + c)
        np.testing.assert_allclose(x, want, atol=1e-14)
    # period 2 with the preconditioner converges, and faster than linear mixing
    def run(mixer, steps):
        x = np.zeros(N)
        for _ in range(steps):
            x = mixer.mix(x, M @ x + c)
        return np.linalg.norm(x - exact) / np.linalg.norm(exact)
    err_pp = run(PeriodicPulay(n, h, history=8, beta=0.3, period=2, k0=1.1), 40)
    err_lin = run(PeriodicPulay(n, h, history=8, beta=0.3, period=1000, k0=1.1), 40)
    assert err_pp < 1e-6 and err_pp < 1e-3 * err_lin


def _full_space_problem(pos=None, local_only=False):
    spec = custom_spec("scf_tiny", 95, 4.4, 1, 6, 216, 2.0, filter_degree=4,
                       filter_passes=0, n_pl=0, basis="sc", noise=False)
    p = make_problem(spec, positions=pos)
    if local_only:  # projectors off: the force is then exact for the discrete energy
        p.proj["gamma"] = np.zeros_like(p.proj["gamma"])
    return p


def _brute_scf(p, tol=1e-11):
    """Linear-mixing SCF with the exact Fermi-Dirac density matrix of the dense H."""
    n, a, h = p.n, p.spec.a, p.h
    b = es.pseudocharge(n, a, p.positions, MODEL.z, MODEL.rc)
    vcore = es.core_potential(n, a, p.positions, MODEL.core_amp, MODEL.core_w2)
    rho = -b
    for _ in range(400):
        _, _, veff, _ = effective_potential(p, MODEL, rho, b, vcore)
        lam, Q = np.linalg.eigh(Hamiltonian(p, veff).dense())
        mu = brentq(lambda m: 2 * foe.fermi_dirac(lam, m, p.spec.kT).sum() - p.n_e,
                    lam[0] - 60, lam[-1] + 60, xtol=1e-15)
        out = 2 * np.sum(Q * Q * foe.fermi_dirac(lam, mu, p.spec.kT)[None, :], axis=1) / h ** 3
        if np.linalg.norm(out - rho) <= tol * np.linalg.norm(out):
            return out
        rho = rho + 0.4 * (out - rho)
    raise AssertionError("brute-force SCF did not converge")


def test_full_space_scf_matches_brute_force():
    p = _full_space_problem()
    r = scf(p, MODEL, tol=1e-10, first_passes=0, later_passes=0, n_pl=0, forces=False)
    assert r.converged and r.iterations < 40
    ref = _brute_scf(p)
    np.testing.assert_allclose(r.rho, ref, atol=1e-8 * ref.max())
    assert abs(p.h ** 3 * r.rho.sum() - p.n_e) < 1e-10
    # Pulay needs far fewer iterations than the residual contraction of linear mixing
    assert r.residuals[-1] <= 1e-10


@pytest.mark.slow
def test_full_space_scf_forces_are_free_energy_derivatives():
    # local part only: the nonlocal force's finite-difference gradient of phi~
    # is pinned against free-energy differences on a finer grid elsewhere
    p = _full_space_problem(local_only=True)
    r = scf(p, MODEL, tol=1e-11, first_passes=0, later_passes=0, n_pl=0, forces=True)
    def central(ax, d):
        fs = []
        for sgn in (+1, -1):
            pos = p.positions.copy()
            pos[0, ax] += sgn * d
            q = _full_space_problem(pos, local_only=True)
            fs.append(scf(q, MODEL, tol=1e-11, first_passes=0, later_passes=0, n_pl=0, forces=False).free_energy)
        return -(fs[0] - fs[1]) / (2 * d)

    for ax in (0, 2):
        # Richardson extrapolation of central differences removes the O(d^2) term
        num = (4 * central(ax, 1e-3) - central(ax, 2e-3)) / 3
        assert abs(r.forces[0, ax] - num) < 2e-9, (ax, r.forces[0, ax], num)


# ------------------------------------------ restarted periodic Pulay, AAR --

def _linear_map(n, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    J = (Q * rng.uniform(-0.9, 0.6, n)) @ Q.T
    c = rng.standard_normal(n)
    return J, c, np.linalg.solve(np.eye(n) - J, c)


def test_restarted_periodic_pulay_finite_termination():
    # on a linear map G(x) = J x + c in n unknowns, a Pulay extrapolation over
    # n difference pairs lands on the fixed point (Anderson = GMRES on linear
    # problems).  With restarts and period n + 1 the first extrapolation (call
    # n + 1) has exactly the n pairs of calls 2..n+1 and must hit it.
    from oracle.mixing import PeriodicPulay
    n = 6
    J, c, xs = _linear_map(n, 4)
    # The normal equations' 1e-12 tr/m shift against the nearly colinear Krylov
    # pairs of the linear-mixing calls limits the landing to ~1e-5 here.
    mix = PeriodicPulay(1, 1.0, history=8, beta=0.3, period=n + 1, k0=0.0, restart=True)
    x = np.zeros(n)
    for call in range(1, n + 2):
        x = mix.mix(x, J @ x + c)
        if call < n + 1:
            assert np.linalg.norm(x - xs) > 1e-2 * np.linalg.norm(xs)
    assert np.linalg.norm(x - xs) < 1e-4 * np.linalg.norm(xs)
    # with n - 1 pairs (a Krylov space one short of R^n) the landing is worse
    mix2 = PeriodicPulay(1, 1.0, history=8, beta=0.3, period=n, k0=0.0, restart=True)
    y = np.zeros(n)
    for call in range(1, n + 1):
        y = mix2.mix(y, J @ y + c)
    assert np.linalg.norm(y - xs) > 3 * np.linalg.norm(x - xs)


def test_restart_discards_history():
    # after a restart the next extrapolation uses only the pairs gathered since:
    # period 2 with restarts uses one pair at call 2, two pairs at calls 4, 6, ...
    # (checked against an explicit one- and two-pair Anderson step)
    from oracle.mixing import PeriodicPulay, REG
    n = 5
    J, c, _ = _linear_map(n, 9)
    mix = PeriodicPulay(1, 1.0, history=7, beta=0.4, period=2, k0=0.0, restart=True)
    xs, fs = [], []
    x = np.random.default_rng(1).standard_normal(n)
    for call in range(1, 7):
        F = J @ x + c - x
        xs.append(x.copy())
        fs.append(F.copy())
        got = mix.mix(x, J @ x + c)
        if call % 2 == 0:
            first = 1 if call == 2 else call - 2
            dR = np.stack([xs[j] - xs[j - 1] for j in range(first, call)], axis=1)
            dF = np.stack([fs[j] - fs[j - 1] for j in range(first, call)], axis=1)
            A = dF.T @ dF
            A = A + REG * np.trace(A) / A.shape[0] * np.eye(A.shape[0])
            g = np.linalg.solve(A, dF.T @ F)
            ref = x - dR @ g + 0.4 * (F - dF @ g)
        else:
            ref = x + 0.4 * F
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-14)
        x = got
    with pytest.raises(ValueError):
        PeriodicPulay(1, 1.0, history=3, period=4, restart=True)


def test_aar_solves_spd_system():
    from oracle.linsolve import aar
    rng = np.random.default_rng(2)
    n = 40
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Q * rng.uniform(1.0, 20.0, n)) @ Q.T
    A = 0.5 * (A + A.T) + 25.0 * np.eye(n)  # diagonally weighted SPD
    b = rng.standard_normal(n)
    d = float(np.mean(np.diag(A)))
    x, it, rel = aar(lambda v: A @ v, b, np.zeros(n), d, 1e-12, 2000)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=0, atol=1e-10)
    assert rel <= 1e-12 and it > 0


def test_aar_poisson_matches_fft_solution():
    # the FD Poisson problem of the SCF: -Lap_h V = 4 pi (rho - mean), zero-mean
    # V; AAR with the Jacobi scaling against the exact FFT solution
    from oracle import electrostatics as es
    from oracle import fd
    from oracle.linsolve import aar
    n, a = 12, 6.0
    h = a / n
    rng = np.random.default_rng(6)
    src = rng.standard_normal(n ** 3)
    b = 4.0 * np.pi * (src - src.mean())
    w = fd.second_derivative_weights()
    diag = -3.0 * w[0] / (h * h)
    x, it, rel = aar(lambda v: -fd.laplacian(v[:, None], n, h)[:, 0], b, np.zeros(n ** 3), diag,
                     1e-11, 5000)
    x = x - x.mean()
    ref = es.poisson_fft(src, n, a)
    assert np.abs(x - ref).max() < 1e-9 * np.abs(ref).max()
