"""Pulay (Anderson) mixing of the self-consistent density (oracle).

The paper accelerates its SCF iterations with Pulay-type mixing (Sec. 5); the
workloads here use plain Pulay mixing on the density.  With input densities
rho_in^k, residuals F^k = rho_out^k - rho_in^k and the last m <= history
difference pairs dR_j = rho_in^{j+1} - rho_in^j, dF_j = F^{j+1} - F^j:

    gamma = argmin || F^k - dF gamma ||_2
          (normal equations (dF^T dF + eps I) gamma = dF^T F^k,
           eps = 1e-12 tr(dF^T dF) / m keeps them definite)
    rho_in^{k+1} = rho_in^k + beta F^k - (dR + beta dF) gamma

which is the residual-minimising combination of the stored iterates followed
by a linear-mixing step of weight beta.  The first step (no history) is
linear mixing.  On a linear fixed-point map in n unknowns, with history >= n,
this reaches the fixed point in at most n + 1 steps (pin).

The paper's SCF uses Kerker-preconditioned periodic Pulay mixing (Sec. 5):
the Pulay extrapolation runs only on every period-th call and the other calls
are preconditioned linear mixing; the history of difference pairs is updated
on every call.  With the Kerker preconditioner P = (-Lap_h + k0^2)^{-1}(-Lap_h)
(damps the long-wavelength residual, removes its mean) and gamma = 0 on the
linear calls:
    rho_bar = rho_in^k - dR gamma,   F_bar = F^k - dF gamma,
    rho_in^{k+1} = rho_bar + beta P F_bar,
which for P = I and period 1 is the Pulay step above.  P is diagonal in the
discrete Fourier basis, with eigenvalue lam / (lam + k0^2), lam the symbol of
-Lap_h; k0 <= 0 means P = I.
"""

from __future__ import annotations

from typing import List, Optional

import numpy as np

from . import fd

REG = 1e-12


class Pulay:
    def __init__(self, history: int = 7, beta: float = 0.3):
        self.history = history
        self.beta = beta
        self.prev_in: Optional[np.ndarray] = None
        self.prev_f: Optional[np.ndarray] = None
        self.dR: List[np.ndarray] = []
        self.dF: List[np.ndarray] = []

    def mix(self, rho_in: np.ndarray, rho_out: np.ndarray) -> np.ndarray:
        F = rho_out - rho_in
        if self.prev_in is not None:
            self.dR.append(rho_in - self.prev_in)
            self.dF.append(F - self.prev_f)
            if len(self.dR) > self.history:
                self.dR.pop(0)
                self.dF.pop(0)
        self.prev_in = rho_in.copy()
        self.prev_f = F.copy()
        nxt = rho_in + self.beta * F
        if self.dR:
            dF = np.stack(self.dF, axis=1)
            dR = np.stack(self.dR, axis=1)
            A = dF.T @ dF
            m = A.shape[0]
            A = A + REG * np.trace(A) / m * np.eye(m)
            gamma = np.linalg.solve(A, dF.T @ F)
            nxt = nxt - (dR + self.beta * dF) @ gamma
        return nxt


def kerker(F: np.ndarray, n: int, h: float, k0: float) -> np.ndarray:
    """P F with P = (-Lap_h + k0^2)^{-1} (-Lap_h) on the periodic n^3 grid."""
    if k0 <= 0:
        return F.copy()
    s = fd.kinetic_symbol(2.0 * np.pi * np.fft.fftfreq(n)) / (h * h)
    lam = s[:, None, None] + s[None, :, None] + s[None, None, :]
    Fk = np.fft.fftn(F.reshape(n, n, n))
    return np.real(np.fft.ifftn(Fk * (lam / (lam + k0 * k0)))).reshape(F.shape)


class PeriodicPulay(Pulay):
    """Kerker-preconditioned periodic Pulay mixing on an n^3 grid of spacing h.

    restart: the restarted form (Sec. 5 names restarted periodic Pulay): the
    stored difference pairs are discarded after every Pulay extrapolation, so
    each extrapolation uses only the pairs gathered since the previous one
    (period - 1 pairs the first time, period afterwards; history >= period)."""

    def __init__(self, n: int, h: float, history: int = 7, beta: float = 0.3, period: int = 2,
                 k0: float = 1.0, restart: bool = False):
        super().__init__(history, beta)
        if restart and period > history:
            raise ValueError("restarted periodic Pulay needs period <= history")
        self.n, self.h, self.period, self.k0 = n, h, period, k0
        self.restart = restart
        self.calls = 0

    def mix(self, rho_in: np.ndarray, rho_out: np.ndarray) -> np.ndarray:
        F = rho_out - rho_in
        if self.prev_in is not None:
            self.dR.append(rho_in - self.prev_in)
            self.dF.append(F - self.prev_f)
            if len(self.dR) > self.history:
                self.dR.pop(0)
                self.dF.pop(0)
        self.prev_in = rho_in.copy()
        self.prev_f = F.copy()
        self.calls += 1
        rbar, fbar = rho_in, F
        if self.dR and self.calls % self.period == 0:
            dF = np.stack(self.dF, axis=1)
            dR = np.stack(self.dR, axis=1)
            A = dF.T @ dF
            m = A.shape[0]
            A = A + REG * np.trace(A) / m * np.eye(m)
            gamma = np.linalg.solve(A, dF.T @ F)
            rbar = rho_in - dR @ gamma
            fbar = F - dF @ gamma
            if self.restart:
                self.dR, self.dF = [], []
        return rbar + self.beta * kerker(fbar, self.n, self.h, self.k0)
