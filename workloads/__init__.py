"""Seeded synthetic inputs for the density-kernel hot path.

This package builds the *problem* both the library and the CPU oracle are
given: a periodic cubic cell of jittered fcc atoms, the fixed effective
potential on the grid, the Kleinman-Bylander projector tables, the per-atom
local-potential gradient fields, and the random start block.  It contains none
of the method's arithmetic (no Hamiltonian application, no filtering, no
orthonormalisation, no Fermi-operator expansion); random numbers the method
consumes are drawn here and passed in as inputs.
"""

from .cells import (  # noqa: F401
    CONFIGS,
    CellSpec,
    Problem,
    custom_spec,
    make_problem,
    spec_for,
)
