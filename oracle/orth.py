"""Orthonormalisation of the filtered block (oracle).

The paper orthonormalises the filtered orbitals with SPARC's CheFSI kernel
without naming the method (Sec. 4).  Reading taken here: Cholesky QR repeated
once (CholQR2) in the discrete inner product <u, v> = h^3 u^T v:

    G = h^3 X^T X,  G = R^T R (R upper triangular, positive diagonal),
    Phi = X R^{-1};  then the same again on Phi.

Phi spans the columns of X and satisfies h^3 Phi^T Phi = I.  With positive
diagonals Phi equals the Householder Q of X with its column signs fixed, times
h^{-3/2}.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla


class NotPositiveDefinite(ValueError):
    pass


def cholqr(X: np.ndarray, h: float) -> np.ndarray:
    G = h ** 3 * (X.T @ X)
    G = 0.5 * (G + G.T)
    try:
        R = sla.cholesky(G, lower=False)
    except np.linalg.LinAlgError as exc:
        raise NotPositiveDefinite(str(exc)) from exc
    # Phi R = X  ->  Phi = X R^{-1}  (triangular solve from the right)
    return sla.solve_triangular(R, X.T, trans="T", lower=False).T


def cholqr2(X: np.ndarray, h: float) -> np.ndarray:
    return cholqr(cholqr(X, h), h)
