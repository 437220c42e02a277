"""Alternating Anderson-Richardson (AAR) linear solver (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 5 solves the electrostatic (Poisson) equation and applies the real-space
Kerker preconditioner with AAR (Suryanarayana, Pratapa & Pask, 2019): a
stationary Richardson iteration on the preconditioned residual, with an
Anderson extrapolation over the last m iterates on every p-th iteration.  With
f_k = M^{-1} (b - A x_k) (M the Jacobi preconditioner, diag A) and the
difference pairs dX_j = x_{j+1} - x_j, dF_j = f_{j+1} - f_j of the last m
iterations:
    x_{k+1} = x_k + omega f_k                                  ((k+1) mod p != 0)
    x_{k+1} = x_k + beta f_k - (dX + beta dF) gamma_k,         ((k+1) mod p == 0)
    gamma_k = argmin || f_k - dF gamma ||_2
(normal equations with the same 1e-12 tr/m shift as the Pulay mixing).
Readings (the paper gives no parameters): omega = beta = 0.6, m = 7, p = 6;
iterate until ||b - A x|| <= tol ||b||.
"""

from __future__ import annotations

from typing import Callable, Tuple

import numpy as np

REG = 1e-12


def aar(apply_a: Callable[[np.ndarray], np.ndarray], b: np.ndarray, x0: np.ndarray,
        diag: float, tol: float, max_iter: int, omega: float = 0.6, beta: float = 0.6,
        history: int = 7, period: int = 6) -> Tuple[np.ndarray, int, float]:
    """Returns (x, iterations, ||b - A x|| / ||b||)."""
    x = np.asarray(x0, dtype=np.float64).copy()
    bn = float(np.linalg.norm(b))
    r = b - apply_a(x)
    f = r / diag
    dX, dF = [], []
    x_prev = f_prev = None
    for k in range(max_iter + 1):
        rn = float(np.linalg.norm(r))
        if rn <= tol * bn:
            return x, k, rn / bn if bn > 0 else 0.0
        if k == max_iter:
            break
        if x_prev is not None:
            dX.append(x - x_prev)
            dF.append(f - f_prev)
            if len(dX) > history:
                dX.pop(0)
                dF.pop(0)
        x_prev, f_prev = x.copy(), f.copy()
        if (k + 1) % period == 0 and dX:
            Fm = np.stack(dF, axis=1)
            Xm = np.stack(dX, axis=1)
            A = Fm.T @ Fm
            m = A.shape[0]
            A = A + REG * np.trace(A) / m * np.eye(m)
            gamma = np.linalg.solve(A, Fm.T @ f)
            x = x + beta * f - (Xm + beta * Fm) @ gamma
        else:
            x = x + omega * f
        r = b - apply_a(x)
        f = r / diag
    raise RuntimeError("aar: no convergence")
