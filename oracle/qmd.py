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

Pins (tests): time reversibility (forward n steps, flip v, forward n steps
returns to the start) and second-order energy error under an exact-gradient
force field; the Maxwell-Boltzmann draw has zero momentum.
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
