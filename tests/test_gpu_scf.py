"""Parity of the self-consistent-field entry points with the FP64 oracle (needs a GPU).

Atom fields, the CG Poisson solve (against the exact FFT solution of the same
FD system), LDA exchange-correlation, the effective potential with its energy
integrals, Pulay mixing and Kerker-preconditioned periodic Pulay mixing over
several calls, local forces, and a whole SCF run (with either mixing) on a small cell (same iteration count, density, free energy and forces as the
oracle; the mixed path to the accuracy budgets).  Grids: 20^3 (several
reduction blocks) and a ragged 15^3.
"""

import numpy as np
import pytest
import torch

from oracle import electrostatics as es
from oracle import xc as oxc
from oracle.mixing import PeriodicPulay, Pulay
from oracle.scf import LocalModel as OModel
from oracle.scf import effective_potential, scf as oscf
from workloads import custom_spec, make_problem
from workloads.cells import CORE_AMP, CORE_W2, RC_LOC, Z_VALENCE

pytestmark = pytest.mark.gpu

MODEL = (Z_VALENCE, RC_LOC, CORE_AMP, CORE_W2)


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_08639_amd import _lib
    _lib.load()
    return _lib


def _problem(n, n_s=40, kT=0.1, index=96):
    spec = custom_spec(f"scf{n}", index, 7.6, 1, n, n_s, kT, filter_degree=16, filter_passes=4,
                       n_pl=0, noise=False)
    return make_problem(spec)


@pytest.fixture(scope="module", params=[20, 15])
def cell(request):
    return _problem(request.param)


def _ctx(p, precision="fp64"):
    from paper_2112_08639_amd.pipeline import Context
    ctx = Context(p, precision)
    ctx.ensure_workspace(p.n_s, 64)
    return ctx


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def test_local_fields_and_start_density(L, cell):
    p = cell
    ctx = _ctx(p)
    L.dk_set_atoms(ctx.h, p.positions, *MODEL)
    b = torch.zeros(p.n_grid, dtype=torch.float64, device="cuda")
    vc = torch.zeros_like(b)
    L.dk_get_local_fields(ctx.h, b, vc)
    b_ref = es.pseudocharge(p.n, p.spec.a, p.positions, Z_VALENCE, RC_LOC)
    vc_ref = es.core_potential(p.n, p.spec.a, p.positions, CORE_AMP, CORE_W2)
    np.testing.assert_allclose(b.cpu().numpy(), b_ref, atol=1e-13 * np.abs(b_ref).max())
    np.testing.assert_allclose(vc.cpu().numpy(), vc_ref, atol=1e-13 * np.abs(vc_ref).max())
    rho = torch.zeros_like(b)
    L.dk_start_density(ctx.h, rho)
    assert abs(p.h ** 3 * (rho.sum().item() + b_ref.sum())) < 1e-12
    # discrete charge: N_e up to the Gaussian's aliasing on the grid (Poisson summation)
    assert abs(p.h ** 3 * rho.sum().item() - p.n_e) < 1e-9
    ctx.close()


def test_poisson_matches_fft_solution(L, cell):
    p = cell
    ctx = _ctx(p)
    rng = np.random.default_rng(17)
    src = rng.standard_normal(p.n_grid) + 0.3
    v = torch.zeros(p.n_grid, dtype=torch.float64, device="cuda")
    it, rr = L.dk_poisson(ctx.h, _dev(src), v, tol=1e-13, max_iter=5000)
    ref = es.poisson_fft(src, p.n, p.spec.a)
    got = v.cpu().numpy()
    assert rr <= 1e-13 and 0 < it < 5000
    np.testing.assert_allclose(got, ref, atol=1e-10 * np.abs(ref).max())
    assert abs(got.mean()) < 1e-13 * np.abs(ref).max()
    # warm start from the solution: converged on entry, nothing moves
    it2, _ = L.dk_poisson(ctx.h, _dev(src), v, tol=1e-10)
    assert it2 == 0
    np.testing.assert_allclose(v.cpu().numpy(), got, atol=1e-14 * np.abs(ref).max())
    # iteration limit reported, not silently truncated
    w = torch.zeros_like(v)
    with pytest.raises(L.DkError) as e:
        L.dk_poisson(ctx.h, _dev(src), w, tol=1e-13, max_iter=3)
    assert e.value.name == "DK_ERR_CONVERGENCE"
    ctx.close()


def test_xc_matches_oracle(L):
    p = _problem(15)
    ctx = _ctx(p)
    rng = np.random.default_rng(5)
    rho = np.exp(rng.uniform(np.log(1e-6), np.log(5.0), p.n_grid))
    rho[:7] = [0.0, -1e-9, 1e-21, 1e-19, 1e-12, 1e3, 1e-3]
    v = torch.zeros(p.n_grid, dtype=torch.float64, device="cuda")
    e_xc = L.dk_xc(ctx.h, _dev(rho), v)
    eps_ref, v_ref = oxc.lda(rho)
    np.testing.assert_allclose(v.cpu().numpy(), v_ref, rtol=1e-13, atol=1e-300)
    e_ref = p.h ** 3 * np.sum(rho * eps_ref)
    assert abs(e_xc - e_ref) < 1e-12 * abs(e_ref)
    ctx.close()


def test_scf_potential_terms(L, cell):
    p = cell
    ctx = _ctx(p)
    L.dk_set_atoms(ctx.h, p.positions, *MODEL)
    model = OModel(*MODEL)
    b = es.pseudocharge(p.n, p.spec.a, p.positions, Z_VALENCE, RC_LOC)
    vcore = es.core_potential(p.n, p.spec.a, p.positions, CORE_AMP, CORE_W2)
    rng = np.random.default_rng(8)
    rho = -b * (1.0 + 0.2 * rng.uniform(-1, 1, p.n_grid)) + 0.01
    rho *= p.n_e / (p.h ** 3 * rho.sum())
    vc_ref, vxc_ref, veff_ref, terms_ref = effective_potential(p, model, rho, b, vcore)
    vc = torch.zeros(p.n_grid, dtype=torch.float64, device="cuda")
    veff = torch.zeros_like(vc)
    t = L.dk_scf_potential(ctx.h, _dev(rho), vc, veff, tol=1e-13)
    scale = np.abs(veff_ref).max()
    np.testing.assert_allclose(vc.cpu().numpy(), vc_ref, atol=1e-10 * scale)
    np.testing.assert_allclose(veff.cpu().numpy(), veff_ref, atol=1e-10 * scale)
    for k in ("e_xc", "int_rho_vc", "int_rho_vxc", "e_es"):
        assert abs(getattr(t, k) - terms_ref[k]) < 1e-9 * max(1.0, abs(terms_ref[k])), k
    # the context potential is now veff: the upper bound sees its maximum
    ub = L.dk_spectrum_upper_bound(ctx.h)
    assert ub > veff_ref.max()
    ctx.close()


def test_pulay_sequence_matches_oracle(L):
    p = _problem(15)
    ctx = _ctx(p)
    rng = np.random.default_rng(12)
    n = p.n_grid
    history = 3
    mixer = Pulay(history=history, beta=0.3)
    state = torch.empty(L.dk_pulay_bytes(ctx.h, history) // 8 + 1, dtype=torch.float64, device="cuda")
    M = 0.4 * rng.standard_normal((n, 6)) @ rng.standard_normal((6, n)) / n
    c = rng.standard_normal(n)
    x = rng.standard_normal(n)
    nxt = torch.zeros(n, dtype=torch.float64, device="cuda")
    for k in range(6):  # more calls than the history: the ring buffer wraps
        out = M @ x + c + 0.01 * np.sin(x)
        ref = mixer.mix(x, out)
        res = L.dk_pulay_mix(ctx.h, state, history, k, 0.3, _dev(x), _dev(out), nxt)
        assert abs(res - np.linalg.norm(out - x) / np.linalg.norm(out)) < 1e-13
        np.testing.assert_allclose(nxt.cpu().numpy(), ref, atol=1e-11 * np.abs(ref).max())
        x = ref
    with pytest.raises(L.DkError):
        L.dk_pulay_mix(ctx.h, state, history, 0, 0.3, nxt, _dev(x), nxt)  # aliasing
    ctx.close()


@pytest.mark.parametrize("period,k0,restart,solver", [(2, 1.1, False, "cg"), (3, 0.6, False, "cg"),
                                                      (1, 0.0, False, "cg"), (2, 1.1, True, "cg"),
                                                      (3, 0.6, True, "aar"), (1, 0.8, True, "aar")])
def test_kerker_pulay_sequence_matches_oracle(L, period, k0, restart, solver):
    # restart: the pairs are discarded after every extrapolation (slots refill
    # from 0); solver: the Kerker solve by CG or AAR (the oracle applies P
    # exactly in Fourier space)
    p = _problem(15)
    ctx = _ctx(p)
    if solver == "aar":
        L.dk_set_linear_solver(ctx.h, L.DK_SOLVER_AAR)
    rng = np.random.default_rng(13)
    n = p.n_grid
    history = 3
    mixer = PeriodicPulay(p.n, p.h, history=history, beta=0.3, period=period, k0=k0,
                          restart=restart)
    state = torch.empty(L.dk_kerker_pulay_bytes(ctx.h, history) // 8 + 1, dtype=torch.float64,
                        device="cuda")
    M = 0.4 * rng.standard_normal((n, 6)) @ rng.standard_normal((6, n)) / n
    c = rng.standard_normal(n)
    x = rng.standard_normal(n)
    nxt = torch.zeros(n, dtype=torch.float64, device="cuda")
    for k in range(7):  # more calls than the history: the ring buffer wraps
        out = M @ x + c + 0.01 * np.sin(x)
        ref = mixer.mix(x, out)
        res = L.dk_kerker_pulay_mix(ctx.h, state, history, k, period, 0.3, k0, 1e-13, _dev(x),
                                    _dev(out), nxt, restart=restart)
        assert abs(res - np.linalg.norm(out - x) / np.linalg.norm(out)) < 1e-13
        np.testing.assert_allclose(nxt.cpu().numpy(), ref, atol=1e-10 * np.abs(ref).max())
        x = ref
    with pytest.raises(L.DkError):
        L.dk_kerker_pulay_mix(ctx.h, state, history, 0, 0, 0.3, k0, 1e-12, _dev(x), _dev(x), nxt)
    with pytest.raises(L.DkError) as e:  # restarts need period <= history
        L.dk_kerker_pulay_mix(ctx.h, state, history, 0, 4, 0.3, k0, 1e-12, _dev(x), _dev(x + 1),
                              nxt, restart=True)
    assert e.value.name == "DK_ERR_ARG"
    ctx.close()


def test_aar_poisson_matches_oracle(L, cell):
    # AAR on the FD Poisson problem: the oracle's AAR (same parameters, same
    # iteration count up to one step at the threshold) and the exact FFT solution
    from oracle import fd as ofd
    from oracle.linsolve import aar
    p = cell
    ctx = _ctx(p)
    L.dk_set_linear_solver(ctx.h, L.DK_SOLVER_AAR, 0.6, 0.6, 7, 6)
    rng = np.random.default_rng(19)
    src = rng.standard_normal(p.n_grid) + 0.3
    v = torch.zeros(p.n_grid, dtype=torch.float64, device="cuda")
    print(f"dk_poisson AAR {p.n}^3", flush=True)
    it, rr = L.dk_poisson(ctx.h, _dev(src), v, tol=1e-11, max_iter=20000)
    w = ofd.second_derivative_weights()
    b = 4.0 * np.pi * (src - src.mean())
    x, it_ref, rr_ref = aar(lambda u: -ofd.laplacian(u[:, None], p.n, p.h)[:, 0], b,
                            np.zeros(p.n_grid), -3.0 * w[0] / p.h ** 2, 1e-11, 20000)
    ref = es.poisson_fft(src, p.n, p.spec.a)
    got = v.cpu().numpy()
    assert rr <= 1e-11 and abs(it - it_ref) <= 1, (it, it_ref)
    np.testing.assert_allclose(got, ref, atol=1e-9 * np.abs(ref).max())
    np.testing.assert_allclose(got, x - x.mean(), atol=1e-9 * np.abs(ref).max())
    with pytest.raises(L.DkError) as e:
        L.dk_poisson(ctx.h, _dev(src), torch.zeros_like(v), tol=1e-13, max_iter=5)
    assert e.value.name == "DK_ERR_CONVERGENCE"
    with pytest.raises(L.DkError) as e:
        L.dk_set_linear_solver(ctx.h, L.DK_SOLVER_AAR, 0.6, 0.6, 9, 6)
    assert e.value.name == "DK_ERR_ARG"
    ctx.close()


def test_electrostatic_stress_matches_oracle(L, cell):
    from oracle import stress as ostress
    p = cell
    ctx = _ctx(p)
    zeros = torch.zeros(p.n_grid, dtype=torch.float64, device="cuda")
    with pytest.raises(L.DkError) as err:   # no atoms yet
        L.dk_electrostatic_stress(ctx.h, zeros, zeros)
    assert err.value.name == "DK_ERR_STATE"
    L.dk_set_atoms(ctx.h, p.positions, *MODEL)
    rng = np.random.default_rng(22)
    rho = 0.05 + 0.01 * rng.random(p.n_grid)
    rho *= len(p.positions) * Z_VALENCE / (p.h ** 3 * rho.sum())
    b = torch.zeros(p.n_grid, dtype=torch.float64, device="cuda")
    L.dk_get_local_fields(ctx.h, b, None)
    v = torch.zeros(p.n_grid, dtype=torch.float64, device="cuda")
    L.dk_poisson(ctx.h, _dev(rho) + b, v, tol=1e-13, max_iter=5000)
    got = L.dk_electrostatic_stress(ctx.h, _dev(rho), v)
    want = ostress.electrostatic_stress(p.n, p.spec.a, p.positions, *MODEL, rho)
    np.testing.assert_allclose(got, want, atol=1e-10 * np.abs(want).max())
    ctx.close()


def test_local_forces_match_oracle(L, cell):
    p = cell
    ctx = _ctx(p)
    L.dk_set_atoms(ctx.h, p.positions, *MODEL)
    rng = np.random.default_rng(21)
    rho = 0.05 + 0.01 * rng.standard_normal(p.n_grid)
    vc = rng.standard_normal(p.n_grid)
    f = L.dk_local_forces(ctx.h, _dev(rho), _dev(vc), len(p.positions))
    ref = es.local_forces(p.n, p.spec.a, p.positions, Z_VALENCE, RC_LOC, CORE_AMP, CORE_W2, rho, vc)
    np.testing.assert_allclose(f, ref, atol=1e-12 * np.abs(ref).max())
    ctx.close()


@pytest.fixture(scope="module")
def scf_ref():
    p = _problem(20)
    return p, oscf(p, OModel(*MODEL), tol=1e-6, max_iter=40)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_scf_run_matches_oracle(L, scf_ref, precision):
    from paper_2112_08639_amd.scf import LocalModel, scf
    p, ref = scf_ref
    assert ref.converged
    got = scf(p, LocalModel(*MODEL), precision, tol=1e-6, max_iter=40)
    assert got.converged
    rho = got.rho.cpu().numpy()
    drho = p.h ** 3 * np.abs(rho - ref.rho).sum() / p.n_e
    n_atoms = len(p.positions)
    if precision == "fp64":
        assert got.iterations == ref.iterations
        np.testing.assert_allclose(got.residuals, ref.residuals, rtol=1e-4, atol=1e-12)
        assert drho < 1e-10
        assert abs(got.free_energy - ref.free_energy) < 1e-10 * abs(ref.free_energy)
        assert abs(got.mu - ref.mu) < 1e-10
        np.testing.assert_allclose(got.forces, ref.forces, atol=1e-9)
    else:
        # mixed: the converged result, not the path, is compared
        assert abs(got.iterations - ref.iterations) <= 3
        assert drho < 1e-5
        assert abs(got.free_energy - ref.free_energy) / n_atoms < 1e-5
        assert np.abs(got.forces - ref.forces).max() < 1e-4
    # mixed: the FP32 block is orthonormal to ~1e-7, so is the electron count
    assert abs(p.h ** 3 * rho.sum() - p.n_e) < (1e-9 if precision == "fp64" else 1e-6 * p.n_e)


@pytest.mark.parametrize("restart,solver", [(False, "cg"), (True, "aar")])
def test_scf_kerker_matches_oracle(L, restart, solver):
    from paper_2112_08639_amd.scf import LocalModel, scf
    p = _problem(20)
    kw = dict(mixing="kerker", period=2, k0=1.0, restart=restart)
    ref = oscf(p, OModel(*MODEL), tol=1e-6, max_iter=40, **kw)
    assert ref.converged
    print(f"scf kerker restart={restart} solver={solver}", flush=True)
    got = scf(p, LocalModel(*MODEL), "fp64", tol=1e-6, max_iter=40, kerker_tol=1e-13,
              poisson_tol=1e-12, solver=solver, **kw)
    assert got.converged
    assert got.iterations == ref.iterations
    np.testing.assert_allclose(got.residuals, ref.residuals, rtol=1e-4, atol=1e-12)
    rho = got.rho.cpu().numpy()
    assert p.h ** 3 * np.abs(rho - ref.rho).sum() / p.n_e < 1e-10
    assert abs(got.free_energy - ref.free_energy) < 1e-10 * abs(ref.free_energy)
