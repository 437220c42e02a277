"""Molecular dynamics on the GPU against the oracle (needs a GPU).

Three velocity-Verlet steps of a 4-atom cell (12^3 grid, N_s = 24, kT = 0.1 Ha,
a subspace whose upper edge is unoccupied so that every SCF converges), with
each ionic step warm-started from the previous orbitals and density.  The
FP64 GPU trajectory (positions, total energies, SCF iteration counts) must
follow the oracle's.  A second case checks energy conservation over a short
mixed-precision run.
"""

import numpy as np
import pytest
import torch

from oracle import qmd as oqmd
from oracle.scf import LocalModel as OModel
from oracle.scf import scf as oscf
from workloads import custom_spec, make_problem
from workloads.cells import CORE_AMP, CORE_W2, PROJ_CHANNELS, PROJ_CUTOFF_REL, RC_LOC, Z_VALENCE

pytestmark = pytest.mark.gpu

MODEL = (Z_VALENCE, RC_LOC, CORE_AMP, CORE_W2)
SPEC = custom_spec("md12", 98, 6.0, 1, 12, 24, 0.1, filter_degree=16, filter_passes=4,
                   n_pl=0, noise=False)


def _problem(pos=None):
    return make_problem(SPEC, positions=pos)


STEPS, DT_FS = 3, 0.5


@pytest.fixture(scope="module")
def oracle_run():
    """The oracle's trajectory on the GPU path's schedule (each ionic step warm-started
    from the previous orbitals and density)."""
    p0 = _problem()
    T = 10 * oqmd.EV
    state = {}
    model = OModel(*MODEL)

    def force(x):
        p = _problem(x)
        if state:
            r = oscf(p, model, tol=1e-6, max_iter=60, first_passes=1, X0=state["Phi"],
                     rho0=state["rho"])
        else:
            r = oscf(p, model, tol=1e-6, max_iter=60)
        state.update(Phi=r.Phi, rho=r.rho, iters=state.get("iters", []) + [r.iterations])
        return r.forces, r.free_energy

    f0, e0 = force(p0.positions)
    v0 = oqmd.maxwell_boltzmann(len(p0.positions), oqmd.M_AL, T, 7000)
    x, v, f, energies = oqmd.verlet(p0.positions, v0, f0, oqmd.M_AL, DT_FS * oqmd.FS, force, STEPS)
    return {"x": x, "energies": energies, "e0": e0 + oqmd.kinetic_energy(v0, oqmd.M_AL),
            "iters": state["iters"], "p0": p0}


@pytest.mark.parametrize("tables", ["host", "device"])
def test_qmd_matches_oracle(oracle_run, tables):
    # host: tables from the workload generator at every step (dk_set_projectors);
    # device: built from the positions by dk_set_projector_model
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_08639_amd.pipeline import ProjectorModel
    from paper_2112_08639_amd.qmd import EV, qmd
    from paper_2112_08639_amd.scf import LocalModel

    p0 = oracle_run["p0"]
    kw = dict(steps=STEPS, dt_fs=DT_FS, temperature=10 * EV, scf_tol=1e-6, scf_max_iter=60)
    if tables == "host":
        traj = qmd(p0, _problem, LocalModel(*MODEL), "fp64", **kw)
    else:
        traj = qmd(p0, None, LocalModel(*MODEL), "fp64",
                   projectors=ProjectorModel(PROJ_CHANNELS, PROJ_CUTOFF_REL), **kw)
    assert traj.scf_iterations == oracle_run["iters"]
    np.testing.assert_allclose(traj.positions[-1], oracle_run["x"], atol=1e-10)
    np.testing.assert_allclose(traj.energies[1:], oracle_run["energies"], atol=1e-8)
    assert abs(traj.energies[0] - oracle_run["e0"]) < 1e-8
    # the atoms moved
    assert np.abs(traj.positions[-1] - p0.positions).max() > 1e-3


def test_qmd_mixed_conserves_energy():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_08639_amd.qmd import EV, qmd
    from paper_2112_08639_amd.scf import LocalModel

    p0 = _problem()
    traj = qmd(p0, _problem, LocalModel(*MODEL), "mixed", steps=6, dt_fs=0.5,
               temperature=10 * EV, scf_tol=1e-6, scf_max_iter=60)
    e = np.array(traj.energies)
    ke = np.array(traj.kinetic)
    # total energy steady to a small fraction of the kinetic energy exchanged
    assert np.abs(e - e[0]).max() < 0.05 * (ke.max() - ke.min()) + 1e-5
