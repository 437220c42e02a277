"""Pseudocharge electrostatics on the periodic grid (oracle).

The paper's real-space formulation (Sec. 2) gathers the long-range part of the
local pseudopotentials and the Hartree potential into one electrostatic
potential V_c, the solution of a periodic Poisson problem with the electron
density plus the atoms' pseudocharges as source, discretised with the same
twelfth-order finite differences:

    -Lap_h V_c = 4 pi (rho + b),   b = sum_I b_I,
    b_I(x) = -Z (pi rc^2)^(-3/2) sum_L exp(-|x - R_I - L|^2 / rc^2)

(b_I is the Gaussian charge whose potential is -Z erf(r/rc)/r).  A neutral
cell has zero-mean rho + b; the mean is removed before the solve and V_c is
returned with zero mean.  The short-range core term of each atom,
v_core(r) = -c exp(-r^2 / w2), is added directly as a periodic image sum.

Energies and forces (integrals are h^3-weighted grid sums):
  E_es = 1/2 int (rho + b) V_c - E_self,  E_self = sum_I Z^2 / (sqrt(2 pi) rc)
         (the continuum self-energy of each Gaussian charge);
  f_I  = int grad b_I(x) V_c(x) dx + int rho(x) grad v_core,I(x) dx
         (the derivative of E_es + int rho v_core with respect to R_I, since
         b_I and v_core,I depend on x - R_I).

The Gaussian factors separate per axis, so every field is a product of three
one-dimensional periodic sums.

Poisson by diagonalisation: the FD Laplacian is diagonal in the discrete
Fourier basis with eigenvalue -sum_axes s(theta_a)/h^2 (s the stencil symbol of
``fd.kinetic_symbol``), so the exact solution of the discrete system is one
forward and one inverse FFT.

Ewald (pin only): the energy of point charges with a neutralising background,
split by erfc / erf at parameter eta; the result is independent of eta.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

from . import fd


def periodic_gauss_1d(x: np.ndarray, r0: float, a: float, w2: float, moment: int = 0):
    """sum over images n of d^moment exp(-d^2/w2), d = x - r0 - n a (terms < e^-50 dropped)."""
    d0 = x - r0
    d0 = d0 - a * np.round(d0 / a)
    reach = math.sqrt(50.0 * w2)
    m = int(math.ceil(reach / a)) + 1
    out = np.zeros_like(x, dtype=np.float64)
    for img in range(-m, m + 1):
        d = d0 - img * a
        out += d ** moment * np.exp(-d * d / w2)
    return out


def _separable_field(n: int, a: float, pos: np.ndarray, w2: float, deriv_axis=None):
    """Per atom: prod_axes G_axis (or the derivative along deriv_axis), (N_atoms, N_grid)."""
    x = np.arange(n) * (a / n)
    out = np.empty((len(pos), n ** 3))
    for i, p in enumerate(pos):
        f = [periodic_gauss_1d(x, p[k], a, w2) for k in range(3)]
        if deriv_axis is not None:
            # d/dx exp(-(x - R)^2/w2) = -2 (x - R)/w2 exp(...)
            f[deriv_axis] = -2.0 / w2 * periodic_gauss_1d(x, p[deriv_axis], a, w2, moment=1)
        out[i] = (f[2][:, None, None] * f[1][None, :, None] * f[0][None, None, :]).reshape(-1)
    return out


def pseudocharge(n: int, a: float, pos: np.ndarray, z: float, rc: float) -> np.ndarray:
    pref = -z * (math.pi * rc * rc) ** -1.5
    return pref * _separable_field(n, a, pos, rc * rc).sum(axis=0)


def core_potential(n: int, a: float, pos: np.ndarray, amp: float, w2: float) -> np.ndarray:
    return -amp * _separable_field(n, a, pos, w2).sum(axis=0)


def self_energy(n_atoms: int, z: float, rc: float) -> float:
    return n_atoms * z * z / (math.sqrt(2.0 * math.pi) * rc)


def poisson_fft(source: np.ndarray, n: int, a: float) -> np.ndarray:
    """Zero-mean V with -Lap_h V = 4 pi (source - mean(source)), exactly (FFT)."""
    h = a / n
    theta = 2.0 * np.pi * np.fft.fftfreq(n)
    s = fd.kinetic_symbol(theta) / (h * h)
    lam = s[:, None, None] + s[None, :, None] + s[None, None, :]
    f = np.fft.fftn(np.asarray(source, dtype=np.float64).reshape(n, n, n))
    lam[0, 0, 0] = 1.0
    vhat = 4.0 * np.pi * f / lam
    vhat[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(vhat)).reshape(-1)


def electrostatic_energy(rho, b, vc, h: float, e_self: float) -> float:
    return float(0.5 * h ** 3 * np.sum((rho + b) * vc) - e_self)


def local_forces(n: int, a: float, pos: np.ndarray, z: float, rc: float, amp: float,
                 w2: float, rho: np.ndarray, vc: np.ndarray) -> np.ndarray:
    h3 = (a / n) ** 3
    pref = -z * (math.pi * rc * rc) ** -1.5
    f = np.zeros((len(pos), 3))
    for ax in range(3):
        gb = pref * _separable_field(n, a, pos, rc * rc, deriv_axis=ax)
        gc = -amp * _separable_field(n, a, pos, w2, deriv_axis=ax)
        f[:, ax] = h3 * (gb @ vc + gc @ rho)
    return f


def ewald_energy(pos: np.ndarray, q: np.ndarray, a: float, eta: float) -> float:
    """Point charges q at pos in a cubic cell of edge a, with a neutralising background."""
    omega = a ** 3
    q = np.asarray(q, dtype=np.float64)
    # real space: images until erfc(eta r) < 1e-17
    rcut = 6.2 / eta
    m = int(math.ceil(rcut / a)) + 1
    e_real = 0.0
    rng = range(-m, m + 1)
    for i in range(len(pos)):
        for j in range(len(pos)):
            d0 = pos[i] - pos[j]
            for l1 in rng:
                for l2 in rng:
                    for l3 in rng:
                        if i == j and l1 == 0 and l2 == 0 and l3 == 0:
                            continue
                        r = np.linalg.norm(d0 + a * np.array([l1, l2, l3]))
                        if r < rcut:
                            e_real += 0.5 * q[i] * q[j] * erfc(eta * r) / r
    # reciprocal space: until exp(-G^2/(4 eta^2)) < 1e-17
    gcut = 2.0 * eta * math.sqrt(39.2)
    k = int(math.ceil(gcut * a / (2.0 * math.pi)))
    e_rec = 0.0
    for k1 in range(-k, k + 1):
        for k2 in range(-k, k + 1):
            for k3 in range(-k, k + 1):
                if k1 == 0 and k2 == 0 and k3 == 0:
                    continue
                g = 2.0 * math.pi / a * np.array([k1, k2, k3])
                g2 = float(g @ g)
                if g2 > gcut * gcut:
                    continue
                s = np.sum(q * np.exp(1j * (pos @ g)))
                e_rec += 2.0 * math.pi / omega * math.exp(-g2 / (4.0 * eta * eta)) / g2 * abs(s) ** 2
    e_self = -eta / math.sqrt(math.pi) * float(np.sum(q * q))
    e_bg = -math.pi * float(np.sum(q)) ** 2 / (2.0 * omega * eta * eta)
    return e_real + e_rec + e_self + e_bg
