"""Pins for the oracle's Chebyshev filter and CholQR2.

Filter: on eigenvectors of H the filter must act as the scalar polynomial
T_m((t-c)/e) / T_m((a0-c)/e), evaluated independently with numpy's Chebyshev
series (numpy.polynomial.chebyshev) and applied through a dense
eigendecomposition.
CholQR2: compared with Householder QR (numpy.linalg.qr) with column signs
fixed, and checked for h^3 Phi^T Phi = I.
"""

import numpy as np
import numpy.polynomial.chebyshev as npc
import pytest

from oracle.filter import chebyshev_filter, filter_polynomial
from oracle.hamiltonian import Hamiltonian
from oracle.orth import NotPositiveDefinite, cholqr, cholqr2


def _cheb_ratio(t, m, a, b, a0):
    e, c = (b - a) / 2, (b + a) / 2
    coef = np.zeros(m + 1)
    coef[m] = 1.0
    return npc.chebval((t - c) / e, coef) / npc.chebval((a0 - c) / e, coef)


@pytest.mark.parametrize("m", [1, 2, 7, 20])
def test_filter_polynomial_scalar(m):
    a0, a, b = -1.3, 2.0, 40.0
    t = np.linspace(-1.3, 40.0, 57)
    np.testing.assert_allclose(filter_polynomial(t, m, a, b, a0),
                               _cheb_ratio(t, m, a, b, a0), rtol=1e-11, atol=1e-13)


def test_filter_on_eigenbasis(tiny_problem):
    H = Hamiltonian(tiny_problem)
    lam, Q = np.linalg.eigh(H.dense())
    rng = np.random.default_rng(3)
    X = rng.standard_normal((H.n_grid, 5))
    a0, a, b = lam[0], lam[40], H.upper_bound()
    m = 12
    Y = chebyshev_filter(H, X, m, a, b, a0)
    ref = Q @ (_cheb_ratio(lam, m, a, b, a0)[:, None] * (Q.T @ X))
    np.testing.assert_allclose(Y, ref, rtol=0, atol=1e-10 * np.abs(ref).max())


def test_filter_free_plane_wave():
    # constant potential, no projectors: a plane wave is an eigenvector
    from workloads import custom_spec, make_problem
    spec = custom_spec("flat", 91, 5.0, 1, 10, 4, 1.0, basis="sc", jitter="none", noise=False)
    p = make_problem(spec)
    H = Hamiltonian(p)
    H.veff = np.full(H.n_grid, -0.7)
    H.gamma[:] = 0.0
    from oracle import fd
    n, h = p.n, p.h
    idx = np.arange(n)
    k, j, i = np.meshgrid(idx, idx, idx, indexing="ij")
    th = 2 * np.pi * np.array([1, 2, 0]) / n
    wave = np.cos(th[0] * i + th[1] * j + th[2] * k).reshape(-1, 1)
    lam = fd.kinetic_symbol(th).sum() / (2 * h * h) - 0.7
    a0, a, b = -0.7, 5.0, H.upper_bound()
    Y = chebyshev_filter(H, wave, 9, a, b, a0)
    np.testing.assert_allclose(Y, _cheb_ratio(lam, 9, a, b, a0) * wave, atol=1e-10)


def test_cholqr2_matches_householder():
    rng = np.random.default_rng(4)
    h = 0.3
    X = rng.standard_normal((400, 30)) @ np.diag(np.logspace(0, 3, 30))
    Phi = cholqr2(X, h)
    Q, R = np.linalg.qr(X)
    Q = Q * np.sign(np.diag(R))[None, :]
    np.testing.assert_allclose(Phi, Q / h ** 1.5, atol=1e-11 / h ** 1.5)
    np.testing.assert_allclose(h ** 3 * Phi.T @ Phi, np.eye(30), atol=1e-14)


def test_cholqr_rejects_rank_deficient():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((100, 6))
    X[:, 3] = X[:, 1]
    with pytest.raises(NotPositiveDefinite):
        cholqr(X, 1.0)
