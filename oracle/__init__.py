"""Plain FP64 CPU oracle of the density-kernel hot path.

TEST INFRASTRUCTURE ONLY.  This package is a slow, deliberately simple NumPy
implementation of what the GPU library computes, written from the paper
(arXiv 2112.08639, Secs. 2-4).  It is imported only by ``tests/``, by
``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of ``bench.py``.
The product path never calls it, and it shares no code with the library: its
only common dependency is the seeded input generator in ``workloads``.

Modules
  fd          twelfth-order central-difference weights and operators
  hamiltonian H = -1/2 Lap_h + V_eff + sum_p gamma_p |chi_p><chi_p|
  filter      scaled Chebyshev filter of the auxiliary orbitals
  orth        CholQR2 orthonormalisation (h^3 Phi^T Phi = I)
  foe         Chebyshev Fermi-operator expansion of the density kernel,
              Fermi level, band and entropy energies
  density     density and Hellmann-Feynman forces from Phi and D_s
  sq3         the whole non-self-consistent evaluation
  xc          LDA exchange-correlation (Perdew-Wang 1992)
  electrostatics  pseudocharges, core term, FD Poisson by FFT, Ewald (pin)
  mixing      Pulay mixing of the density
  scf         the self-consistent loop around the SQ3 steps
  mlp         learned start density: descriptors, network, gradients, Adam
  qmd         velocity-Verlet molecular dynamics, Maxwell-Boltzmann start
  stress      kinetic and nonlocal terms of the Hellmann-Feynman stress
  transport   Green-Kubo self-diffusion and viscosity from MD series
  linsolve    alternating Anderson-Richardson (AAR) linear solver

Every function was checked against something other than itself (closed forms,
dense diagonalisation, library routines, invariants); see tests/test_oracle_*.
"""

from . import fd, hamiltonian, filter, orth, foe, density, sq3  # noqa: F401
from . import xc, electrostatics, mixing, scf, mlp, qmd, stress, transport  # noqa: F401
from . import linsolve  # noqa: F401
