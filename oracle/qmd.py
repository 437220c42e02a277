"""Born-Oppenheimer molecular dynamics with SQ3 forces (oracle).

The paper's application runs (Sec. 5) are quantum molecular dynamics: at every
ionic step the electronic problem is solved self-consistently and the
Hellmann-Feynman forces move the ions.  Here:

  * velocity Verlet (NVE):  v += (dt/2) f/M;  R += dt v;  f = f(R);  v += (dt/2) f/M;
  * initial velocities Maxwell-Boltzmann at temperature T (v_i = sqrt(T/M) N(0,1),
    seeded), with the centre-of-mass velocity removed;
  * total energy E = F(R) + (1/2) sum M v^2, F the electronic free energy
    (including the ion-ion part through the pseudocharges); its drift per atom
    measures the integration.

Units: Hartree atomic units; 1 fs = 41.341374575751 a.u. of time; aluminium
mass 26.9815385 u = 26.9815385 * 1822.888486 electron masses.

Isokinetic ensemble (Sec. 5 runs the transport calculations with a Gaussian
thermostat): dv/dt = f/M - alpha v with alpha = f.v / (M v.v) over all 3N
components keeps the kinetic energy fixed.  With f held over a kick of
length tau the flow has a closed form (Zhang's isokinetic integrator):
with g = f/M, c = v0.v0, a = g.v0/c, b = g.g/c and s(t) solving
s'' = a + b s, s(0) = 0, s'(0) = 1,
    s(tau)  = a (cosh(w) - 1)/b + sinh(w)/sqrt(b),   w = sqrt(b) tau,
    s'(tau) = a sinh(w)/sqrt(b) + cosh(w),
    v(tau)  = (v0 + g s(tau)) / s'(tau),
and |v(tau)| = |v0| exactly (s'^2 = 1 + 2 a s + b s^2).  The isokinetic
velocity Verlet replaces each half kick by this flow.  The start velocities
are the Maxwell-Boltzmann draw rescaled to K = (3N - 3) T / 2.

Pins (tests): time reversibility (forward n steps, flip v, forward n steps
returns to the start) and second-order energy error under an exact-gradient
force field; the Maxwell-Boltzmann draw has zero momentum; the isokinetic
kick against a high-order numerical integration of its differential
equation, and the kinetic energy of an isokinetic trajectory.
"""

from __future__ import annotations

from typing import Callable, List, Tuple

import numpy as np

FS = 41.341374575751
AMU = 1822.888486
M_AL = 26.9815385 * AMU
EV = 1.0 / 27.211386245988


def maxwell_boltzmann(n_atoms: int, mass: float, temperature: float, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    v = np.sqrt(temperature / mass) * rng.standard_normal((n_atoms, 3))
    return v - v.mean(axis=0)


def kinetic_energy(v: np.ndarray, mass: float) -> float:
    return 0.5 * mass * float(np.sum(v * v))


def verlet(x: np.ndarray, v: np.ndarray, f: np.ndarray, mass: float, dt: float,
           force: Callable[[np.ndarray], Tuple[np.ndarray, float]], steps: int):
    """steps of velocity Verlet; force(x) -> (forces, potential energy).

    Returns the final (x, v, f) and the total energy after each step."""
    x, v, f = x.copy(), v.copy(), f.copy()
    energies: List[float] = []
    for _ in range(steps):
        v = v + 0.5 * dt * f / mass
        x = x + dt * v
        f, e_pot = force(x)
        v = v + 0.5 * dt * f / mass
        energies.append(e_pot + kinetic_energy(v, mass))
    return x, v, f, energies


def isokinetic_start(n_atoms: int, mass: float, temperature: float, seed: int) -> np.ndarray:
    """Maxwell-Boltzmann draw rescaled to the kinetic energy (3N - 3) T / 2."""
    v = maxwell_boltzmann(n_atoms, mass, temperature, seed)
    k = kinetic_energy(v, mass)
    return v * np.sqrt(0.5 * (3 * n_atoms - 3) * temperature / k)


def isokinetic_kick(v: np.ndarray, f: np.ndarray, mass: float, tau: float) -> np.ndarray:
    """Exact isokinetic flow over time tau with the force f held fixed."""
    u0 = np.asarray(v, dtype=np.float64).ravel()
    g = np.asarray(f, dtype=np.float64).ravel() / mass
    c = float(u0 @ u0)
    a = float(g @ u0) / c
    b = float(g @ g) / c
    w = np.sqrt(b) * tau
    # sinh(w)/w and (cosh(w) - 1)/w^2 = (sinh(w/2)/(w/2))^2 / 2, both 1-safe at w = 0
    sinhc = np.sinh(w) / w if w > 0 else 1.0
    half = np.sinh(0.5 * w) / (0.5 * w) if w > 0 else 1.0
    s = a * tau * tau * 0.5 * half * half + tau * sinhc
    sdot = a * tau * sinhc + np.cosh(w)
    return ((u0 + g * s) / sdot).reshape(np.shape(v))


def isokinetic_verlet(x: np.ndarray, v: np.ndarray, f: np.ndarray, mass: float, dt: float,
                      force: Callable[[np.ndarray], Tuple[np.ndarray, float]], steps: int):
    """steps of isokinetic velocity Verlet; returns (x, v, f) and the potential
    energy after each step (the kinetic energy stays at its start value)."""
    x, v, f = x.copy(), v.copy(), f.copy()
    energies: List[float] = []
    for _ in range(steps):
        v = isokinetic_kick(v, f, mass, 0.5 * dt)
        x = x + dt * v
        f, e_pot = force(x)
        v = isokinetic_kick(v, f, mass, 0.5 * dt)
        energies.append(e_pot)
    return x, v, f, energies
