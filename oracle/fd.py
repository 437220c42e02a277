"""Twelfth-order central finite differences on a periodic grid (oracle).

The paper discretises with twelfth-order accurate real-space finite
differences (Sec. 5).  Weights of the order-2p central second and first
derivatives are the closed forms of the Lagrange-interpolation stencil
(Fornberg):

  second derivative  w_0 = -2 sum_{k=1}^{p} 1/k^2,
                     w_k = 2 (-1)^{k+1} (p!)^2 / (k^2 (p-k)! (p+k)!)
  first derivative   a_k = (-1)^{k+1} (p!)^2 / (k (p-k)! (p+k)!)

so that f''(x) ~ (1/h^2) sum_{|k|<=p} w_|k| f(x+kh) and
f'(x) ~ (1/h) sum_{k=1}^{p} a_k (f(x+kh) - f(x-kh)).
"""

from __future__ import annotations

from fractions import Fraction
from math import factorial

import numpy as np

P = 6  # radius of the twelfth-order stencil


def second_derivative_weights(p: int = P) -> np.ndarray:
    w = [Fraction(0)] * (p + 1)
    for k in range(1, p + 1):
        w[k] = Fraction(2 * (-1) ** (k + 1) * factorial(p) ** 2,
                        k * k * factorial(p - k) * factorial(p + k))
    w[0] = -2 * sum(Fraction(1, k * k) for k in range(1, p + 1))
    return np.array([float(x) for x in w])


def first_derivative_weights(p: int = P) -> np.ndarray:
    a = [Fraction(0)] * (p + 1)
    for k in range(1, p + 1):
        a[k] = Fraction((-1) ** (k + 1) * factorial(p) ** 2,
                        k * factorial(p - k) * factorial(p + k))
    return np.array([float(x) for x in a])


def _axes(n, h):
    """Per-axis points (nx, ny, nz) and spacings (hx, hy, hz) from an int/float
    (cubic grid) or from 3-tuples (orthorhombic grid, Sec. 2's rectangular
    domain)."""
    shape = (n, n, n) if np.isscalar(n) else tuple(int(v) for v in n)
    spacing = (h, h, h) if np.isscalar(h) else tuple(float(v) for v in h)
    return shape, spacing


def _as_grid(X: np.ndarray, n) -> np.ndarray:
    """(N_grid, k) -> (n_z, n_y, n_x, k) view for flat index i + nx(j + ny k)."""
    nx, ny, nz = _axes(n, 1.0)[0]
    return X.reshape(nz, ny, nx, -1)


def laplacian(X: np.ndarray, n, h) -> np.ndarray:
    """Periodic discrete Laplacian of every column of X (N_grid, k).

    n, h: points and spacing per axis (ints/floats for a cubic grid)."""
    w = second_derivative_weights()
    G = _as_grid(X, n)
    if np.isscalar(n) and np.isscalar(h):
        out = 3.0 * w[0] * G
        for axis in range(3):
            for k in range(1, P + 1):
                out = out + w[k] * (np.roll(G, k, axis=axis) + np.roll(G, -k, axis=axis))
        return (out / (h * h)).reshape(X.shape)
    _, spacing = _axes(n, h)
    out = np.zeros_like(G)
    for axis in range(3):  # grid view axis 0, 1, 2 = z, y, x
        ha = spacing[2 - axis]
        part = w[0] * G
        for k in range(1, P + 1):
            part = part + w[k] * (np.roll(G, k, axis=axis) + np.roll(G, -k, axis=axis))
        out = out + part / (ha * ha)
    return out.reshape(X.shape)


def gradient(X: np.ndarray, n, h, direction: int) -> np.ndarray:
    """Periodic first derivative along x (0), y (1) or z (2) of every column.

    n, h: points and spacing per axis (ints/floats for a cubic grid)."""
    a = first_derivative_weights()
    axis = 2 - direction  # grid view is (z, y, x, k)
    hd = _axes(n, h)[1][direction]
    G = _as_grid(X, n)
    out = np.zeros_like(G)
    for k in range(1, P + 1):
        # f(x + kh) sits at roll(..., -k)
        out = out + a[k] * (np.roll(G, -k, axis=axis) - np.roll(G, k, axis=axis))
    return (out / hd).reshape(X.shape)


def kinetic_symbol(theta: np.ndarray) -> np.ndarray:
    """s(theta) = -w_0 - 2 sum_k w_k cos(k theta): -h^2 Lap_h e^{i theta x/h} / e^{..} per axis."""
    w = second_derivative_weights()
    s = -w[0] * np.ones_like(theta)
    for k in range(1, P + 1):
        s = s - 2.0 * w[k] * np.cos(k * theta)
    return s
