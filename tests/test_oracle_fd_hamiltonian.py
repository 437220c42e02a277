"""Pins for the oracle's finite differences and Hamiltonian.

The stencil weights are fixed by the moment conditions that define a
twelfth-order central difference (exactness on polynomials up to degree 13);
the discrete Laplacian by its action on plane waves; the Hamiltonian by its
symmetry and by the analytic spectrum of the free (kinetic-only) case.
"""

import numpy as np
import pytest

from oracle import fd
from oracle.hamiltonian import Hamiltonian


def test_second_derivative_moments():
    # sum_{|k|<=6} w_|k| k^(2m) = 2 [m == 1] for m = 0..6 fixes all 7 weights.
    w = fd.second_derivative_weights()
    for m in range(7):
        s = w[0] * (1.0 if m == 0 else 0.0) + 2.0 * sum(w[k] * k ** (2 * m) for k in range(1, 7))
        assert abs(s - (2.0 if m == 1 else 0.0)) < 1e-9 * max(1, 6 ** (2 * m)) * 1e-3


def test_first_derivative_moments():
    # sum_k a_k (k^(2m+1) - (-k)^(2m+1)) = [m == 0] for m = 0..5 fixes all 6 weights.
    a = fd.first_derivative_weights()
    for m in range(6):
        s = sum(a[k] * 2.0 * k ** (2 * m + 1) for k in range(1, 7))
        assert abs(s - (1.0 if m == 0 else 0.0)) < 1e-12 * 6 ** (2 * m + 1)


def test_known_weight_values():
    # the standard 12th-order central second-derivative coefficients
    w = fd.second_derivative_weights()
    ref = [-5369 / 1800, 12 / 7, -15 / 56, 10 / 189, -1 / 112, 2 / 1925, -1 / 16632]
    np.testing.assert_allclose(w, ref, rtol=1e-15, atol=0)


def test_symbol_is_twelfth_order():
    th = np.linspace(0.01, 0.3, 20)
    s = fd.kinetic_symbol(th)
    # s(theta) = theta^2 - C theta^14 + ..., C = 2 (6!)^2 / 14! for the 12th-order stencil
    C = 2 * 720 ** 2 / 87178291200
    assert np.all(np.abs(s - th ** 2) <= 1.1 * C * th ** 14 + 2e-15)
    big = th[-3:]
    ratio = (fd.kinetic_symbol(big) - big ** 2) / big ** 14
    np.testing.assert_allclose(ratio, -C, rtol=0.05)
    # at theta = pi the symbol is the maximum
    grid = np.linspace(0, np.pi, 2001)
    assert fd.kinetic_symbol(np.array([np.pi]))[0] >= fd.kinetic_symbol(grid).max() - 1e-12


@pytest.mark.parametrize("n", [8, 12])
def test_laplacian_on_plane_waves(n):
    h = 0.37
    idx = np.arange(n)
    k, j, i = np.meshgrid(idx, idx, idx, indexing="ij")
    rng = np.random.default_rng(0)
    for _ in range(4):
        mx, my, mz = rng.integers(-n // 2, n // 2, 3)
        th = 2 * np.pi * np.array([mx, my, mz]) / n
        wave = np.cos(th[0] * i + th[1] * j + th[2] * k + 0.3).reshape(-1, 1)
        lap = fd.laplacian(wave, n, h)
        lam = -fd.kinetic_symbol(th).sum() / h ** 2
        np.testing.assert_allclose(lap, lam * wave, atol=1e-11 * abs(lam) + 1e-12)


def test_gradient_on_plane_waves():
    n, h = 12, 0.5
    idx = np.arange(n)
    k, j, i = np.meshgrid(idx, idx, idx, indexing="ij")
    a = fd.first_derivative_weights()
    for direction, coord in enumerate((i, j, k)):
        th = 2 * np.pi * 2 / n
        wave = np.sin(th * coord).reshape(-1, 1)
        g = fd.gradient(wave, n, h, direction)
        factor = sum(2 * a[kk] * np.sin(kk * th) for kk in range(1, 7)) / h
        np.testing.assert_allclose(g, factor * np.cos(th * coord).reshape(-1, 1), atol=1e-12)
        # and the factor approximates the exact derivative th/h
        assert abs(factor - th / h) < 1e-4 * th / h


def test_hamiltonian_symmetric(tiny_problem):
    H = Hamiltonian(tiny_problem)
    rng = np.random.default_rng(1)
    u = rng.standard_normal(H.n_grid)
    v = rng.standard_normal(H.n_grid)
    lhs = u @ H.apply(v)
    rhs = H.apply(u) @ v
    assert abs(lhs - rhs) < 1e-13 * abs(lhs) * 100


def test_free_spectrum_matches_symbol(tiny_problem):
    # no potential, no projectors: eigenvalues are sum_axes s(theta_axis)/(2h^2)
    p = tiny_problem
    H = Hamiltonian(p)
    H.veff = np.zeros_like(H.veff)
    H.gamma = np.zeros_like(H.gamma)
    ev = np.linalg.eigvalsh(H.dense())
    th = 2 * np.pi * np.arange(p.n) / p.n
    s = fd.kinetic_symbol(th) / (2 * p.h ** 2)
    ref = np.sort((s[:, None, None] + s[None, :, None] + s[None, None, :]).ravel())
    np.testing.assert_allclose(ev, ref, atol=1e-11)


def test_upper_bound(tiny_problem):
    H = Hamiltonian(tiny_problem)
    ev = np.linalg.eigvalsh(H.dense())
    b = H.upper_bound()
    assert b >= ev[-1]
    assert b <= ev[-1] * 1.2


def test_projector_quadrature(tiny_problem):
    # h^3 chi^T chi: unit diagonal up to image overlap and sampling; the l=1
    # functions of one atom are mutually orthogonal by parity only on the
    # continuum, so just check the Gram matrix is positive definite and near 1.
    H = Hamiltonian(tiny_problem)
    G = H.h ** 3 * (H.chi.T @ H.chi).toarray()
    assert np.all(np.linalg.eigvalsh(G) > 0)
    assert np.allclose(np.diag(G), 1.0, atol=0.2)


# ------------------------------------------------------- orthorhombic grids --
# The same operators on an nx x ny x nz grid with spacings hx, hy, hz (flat
# index i + nx (j + ny k)).  Plane waves remain eigenvectors with the symbol
# summed per axis at that axis' spacing; the free spectrum is that sum over
# every wave vector of the grid.

def _noncubic_problem():
    from workloads import custom_spec, make_problem
    spec = custom_spec("ortho", 97, 4.0, 1, 8, 16, 1.0, basis="sc", noise=True,
                       dims=(8, 9, 10), lens=(3.6, 4.1, 4.9))
    return make_problem(spec, positions=np.array([[1.3, 2.2, 3.1]]))


def test_laplacian_on_plane_waves_orthorhombic():
    shape, spacing = (9, 12, 10), (0.31, 0.37, 0.43)
    nx, ny, nz = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    rng = np.random.default_rng(3)
    for _ in range(4):
        m = [rng.integers(-s // 2, s // 2) for s in shape]
        th = [2 * np.pi * m[a] / shape[a] for a in range(3)]
        wave = np.cos(th[0] * i + th[1] * j + th[2] * k + 0.7).reshape(-1, 1)
        lap = fd.laplacian(wave, shape, spacing)
        lam = -sum(fd.kinetic_symbol(np.array([th[a]]))[0] / spacing[a] ** 2 for a in range(3))
        np.testing.assert_allclose(lap, lam * wave, atol=1e-11 * abs(lam) + 1e-12)
    # a tuple grid of equal axes reproduces the cubic operator
    X = rng.standard_normal((10 ** 3, 2))
    np.testing.assert_allclose(fd.laplacian(X, (10, 10, 10), (0.4, 0.4, 0.4)),
                               fd.laplacian(X, 10, 0.4), rtol=0, atol=1e-12)


def test_gradient_on_plane_waves_orthorhombic():
    shape, spacing = (8, 12, 10), (0.5, 0.3, 0.45)
    nx, ny, nz = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    a = fd.first_derivative_weights()
    for direction, coord in enumerate((i, j, k)):
        th = 2 * np.pi * 2 / shape[direction]
        wave = np.sin(th * coord).reshape(-1, 1)
        g = fd.gradient(wave, shape, spacing, direction)
        factor = sum(2 * a[kk] * np.sin(kk * th) for kk in range(1, 7)) / spacing[direction]
        np.testing.assert_allclose(g, factor * np.cos(th * coord).reshape(-1, 1), atol=1e-12)


def test_orthorhombic_free_spectrum_and_bound():
    p = _noncubic_problem()
    H = Hamiltonian(p)
    assert H.n_grid == 8 * 9 * 10
    assert abs(H.h ** 3 - (3.6 / 8) * (4.1 / 9) * (4.9 / 10)) < 1e-15
    rng = np.random.default_rng(5)
    u, v = rng.standard_normal((2, H.n_grid))
    assert abs(u @ H.apply(v) - H.apply(u) @ v) < 1e-12 * abs(u @ H.apply(v))
    ev_full = np.linalg.eigvalsh(H.dense())
    b = H.upper_bound()
    assert ev_full[-1] <= b <= 1.2 * ev_full[-1]
    H.veff = np.zeros_like(H.veff)
    H.gamma = np.zeros_like(H.gamma)
    ev = np.linalg.eigvalsh(H.dense())
    sx, sy, sz = (fd.kinetic_symbol(2 * np.pi * np.arange(m) / m) / (2 * hh ** 2)
                  for m, hh in zip(p.spec.shape, p.spec.spacing))
    ref = np.sort((sz[:, None, None] + sy[None, :, None] + sx[None, None, :]).ravel())
    np.testing.assert_allclose(ev, ref, atol=1e-11)
