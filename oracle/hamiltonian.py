"""Discrete Kohn-Sham Hamiltonian with fixed effective potential (oracle).

H = -1/2 Lap_h + V_eff + V_nl (Eq. KSeqn), where the nonlocal part is the
Kleinman-Bylander sum over atoms and channels of gamma_Jl |chi~_Jlm><chi~_Jlm|
with periodically extended projectors (Eq. nonlocaloperator).  On the grid the
bra is a quadrature with weight h^3:  V_nl x = sum_p gamma_p chi_p (h^3 chi_p^T x).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fd


class Hamiltonian:
    def __init__(self, problem, veff=None):
        """veff: effective potential on the grid (default: the problem's fixed one)."""
        self.n = problem.n
        self.h = problem.h  # volume element h^3 = hx hy hz
        # points and spacings per axis for the FD operators (scalars on a cubic grid)
        self.fd_n = getattr(problem, "fd_n", problem.n)
        self.fd_h = getattr(problem, "fd_h", problem.h)
        self.n_grid = problem.n_grid
        self.veff = np.asarray(problem.veff if veff is None else veff, dtype=np.float64)
        pr = problem.proj
        n_proj = len(pr["gamma"])
        cols = np.repeat(np.arange(n_proj), np.diff(pr["offsets"]))
        # chi: N_grid x N_proj sparse matrix of projector values
        self.chi = sp.csc_matrix((pr["values"], (pr["indices"], cols)),
                                 shape=(self.n_grid, n_proj))
        self.gamma = np.asarray(pr["gamma"], dtype=np.float64)
        self.atom = np.asarray(pr["atom"])

    def projections(self, X: np.ndarray) -> np.ndarray:
        """h^3 chi^T X: integrals of every projector against every column."""
        return self.h ** 3 * (self.chi.T @ X)

    def apply(self, X: np.ndarray) -> np.ndarray:
        """H X for a block X of shape (N_grid, k) (or a single vector)."""
        vec = X.ndim == 1
        Xb = X[:, None] if vec else X
        Y = -0.5 * fd.laplacian(Xb, self.fd_n, self.fd_h)
        Y = Y + self.veff[:, None] * Xb
        C = self.projections(Xb)
        Y = Y + self.chi @ (self.gamma[:, None] * C)
        return Y[:, 0] if vec else Y

    def dense(self) -> np.ndarray:
        """Explicit N_grid x N_grid matrix (tiny grids only)."""
        return self.apply(np.eye(self.n_grid))

    def upper_bound(self) -> float:
        """Closed-form upper bound on the spectrum of H.

        kinetic: sum over the axes of max_theta s(theta)/(2 h_a^2), attained at theta = pi;
        local: max V_eff; nonlocal: sum of gamma_p h^3 |chi_p|^2 over gamma_p > 0
        (each gamma_p |chi_p><chi_p| is positive semidefinite with that norm).
        """
        s_pi = float(fd.kinetic_symbol(np.array([np.pi]))[0])
        if np.isscalar(self.fd_h):
            kin = 3.0 * s_pi / (2.0 * self.h ** 2)
        else:
            kin = sum(s_pi / (2.0 * ha ** 2) for ha in self.fd_h)
        norms = self.h ** 3 * np.asarray(self.chi.multiply(self.chi).sum(axis=0)).ravel()
        nl = float(np.sum(np.where(self.gamma > 0, self.gamma * norms, 0.0)))
        return kin + float(self.veff.max()) + nl
