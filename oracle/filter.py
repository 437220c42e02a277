"""Scaled Chebyshev filter of the auxiliary orbitals (oracle).

The paper generates each SCF iteration's auxiliary orbitals by Chebyshev
filtering the previous ones (Sec. 4, citing Zhou, Saad, Tiago & Chelikowsky
2006).  The filter is the degree-m Chebyshev polynomial of the first kind on
the interval [a, b] to be damped, mapped by L(t) = (t - c)/e with
c = (a+b)/2, e = (b-a)/2, and normalised so the polynomial equals 1 at the
point a0 below the interval:

    p_m(t) = T_m(L(t)) / T_m(L(a0)).

It is evaluated with the three-term recurrence of T_m applied to the block,
carrying the normalisation in the scalars s_k = T_{k-1}(L(a0)) / T_k(L(a0)):
    s_1 = e/(a0 - c),  s_{k+1} = 1 / (2/s_1 - s_k),
    Y_1 = (s_1/e) (H - c) X,
    Y_{k+1} = (2 s_{k+1}/e) (H - c) Y_k - s_k s_{k+1} Y_{k-1}.
"""

from __future__ import annotations

import numpy as np


def chebyshev_filter(H, X: np.ndarray, degree: int, a: float, b: float,
                     a0: float) -> np.ndarray:
    """Return p_m(H) X for the block X (N_grid, k)."""
    if degree < 1:
        return X.copy()
    e = (b - a) / 2.0
    c = (b + a) / 2.0
    s1 = e / (a0 - c)
    s = s1
    y_prev = X
    y = (s1 / e) * (H.apply(X) - c * X)
    for _ in range(2, degree + 1):
        s_next = 1.0 / (2.0 / s1 - s)
        y_next = (2.0 * s_next / e) * (H.apply(y) - c * y) - (s * s_next) * y_prev
        y_prev, y = y, y_next
        s = s_next
    return y


def filter_polynomial(t: np.ndarray, degree: int, a: float, b: float,
                      a0: float) -> np.ndarray:
    """Scalar values of the same recurrence at points t (for spectral checks)."""
    t = np.asarray(t, dtype=np.float64)
    e = (b - a) / 2.0
    c = (b + a) / 2.0
    s1 = e / (a0 - c)
    s = s1
    y_prev = np.ones_like(t)
    y = (s1 / e) * (t - c)
    for _ in range(2, degree + 1):
        s_next = 1.0 / (2.0 / s1 - s)
        y_next = (2.0 * s_next / e) * (t - c) * y - (s * s_next) * y_prev
        y_prev, y = y, y_next
        s = s_next
    return y
