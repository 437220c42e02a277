"""Parity with the oracle at N_s = 2048 (needs a GPU).

Above N_s = 1024 the libdk products switch to their large-matrix forms: the
Gram and projection split-K over ~32768 workgroups (more than 256 output
tiles), the spectral-bound squarings and the Chebyshev recurrence on 64 x 64
tiles, and a Cholesky of 64 diagonal blocks.  These tests run each entry point
of the electronic step at that size on a 20^3 grid (8000 points: N_s < N_grid,
125 K-blocks of 64 with a ragged split), in both precisions, element by element
against the FP64 oracle on the same seeded inputs.

Tolerances: FP64 to a relative 1e-12 (1e-10 for the forces, whose nonlocal
term is a difference of products); the mixed path to its precision (the block
is FP32, so every product is FP32-level; the projection is two-piece
split-BF16, 2^-16 per product).
"""

import numpy as np
import pytest
import torch

from oracle import density as odens
from oracle import foe as ofoe
from oracle import sq3 as osq3
from oracle.hamiltonian import Hamiltonian
from oracle.orth import cholqr2
from workloads import custom_spec, make_problem

pytestmark = pytest.mark.gpu

N_S = 2048


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_08639_amd import _lib
    _lib.load()
    return _lib


@pytest.fixture(scope="module")
def case():
    """Problem, a seeded block with column scales 1..10, its CholQR2 and H_s."""
    spec = custom_spec("ns2048", 98, 7.6, 1, 20, N_S, 5.0, noise=True)
    p = make_problem(spec, with_block=False)
    rng = np.random.default_rng(11)
    X = rng.standard_normal((p.n_grid, N_S)) * np.logspace(0, 1, N_S)
    H = Hamiltonian(p)
    Phi = cholqr2(X, p.h)
    Hs = osq3.project(H, Phi)
    return {"p": p, "H": H, "X": X, "Phi": Phi, "Hs": Hs}


@pytest.fixture(scope="module")
def kernel_ref(case):
    return ofoe.density_kernel(case["Hs"], 0.4 * N_S, case["p"].spec.kT, 0)


def _ctx(p, precision, n_pl=0):
    from paper_2112_08639_amd.pipeline import Context
    ctx = Context(p, precision)
    ctx.ensure_workspace(N_S, n_pl)
    return ctx


def _dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_orthonormalize_2048(L, case, precision):
    p, ref = case["p"], case["Phi"]
    ctx = _ctx(p, precision)
    print(f"dk_orthonormalize N_s={N_S} grid 20^3 {precision}", flush=True)
    Xd = _dev(case["X"].T, ctx.dtype)
    L.dk_orthonormalize(ctx.h, Xd)
    got = Xd.double().cpu().numpy().T
    if precision == "fp64":
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    else:
        G = p.h ** 3 * got.T @ got
        assert np.abs(G - np.eye(N_S)).max() < 2e-5
        assert np.abs(got - ref).max() < 2e-4 * np.abs(ref).max()
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_project_and_bounds_2048(L, case, precision):
    p, ref = case["p"], case["Hs"]
    ctx = _ctx(p, precision)
    print(f"dk_project + dk_spectral_bounds N_s={N_S} {precision}", flush=True)
    Xd = _dev(case["Phi"].T, ctx.dtype)
    Hs = torch.zeros((N_S, N_S), dtype=torch.float64, device="cuda")
    L.dk_project(ctx.h, Xd, Hs)
    got = Hs.cpu().numpy()
    scale = np.abs(ref).max()
    tol = 1e-12 if precision == "fp64" else 1e-4
    assert np.abs(got - ref).max() < tol * scale, np.abs(got - ref).max() / scale
    assert np.array_equal(got, got.T)
    lo, hi, it = L.dk_spectral_bounds(ctx.h, Hs)
    ev = np.linalg.eigvalsh(got)
    assert abs(lo - ev[0]) < 1e-12 * np.abs(ev).max()
    assert abs(hi - ev[-1]) < 1e-12 * np.abs(ev).max()
    assert 0 < it <= 96
    ctx.close()


def test_density_kernel_2048(L, case, kernel_ref):
    # the tail rule picks the degree; recurrence, traces, Fermi level and D_s
    # on 64 x 64 tiles
    p, ref = case["p"], kernel_ref
    ctx = _ctx(p, "fp64")
    print(f"dk_density_kernel N_s={N_S} n_pl=0", flush=True)
    Hd = _dev(case["Hs"])
    Dd = torch.zeros_like(Hd)
    tau = torch.zeros(L.DK_TAIL_MAX_DEGREE + 1, dtype=torch.float64, device="cuda")
    info = L.dk_density_kernel(ctx.h, Hd, 0.4 * N_S, p.spec.kT, 0, Dd, tau)
    assert info.n_pl == ref.n_pl
    assert abs(info.mu - ref.mu) < 1e-12 * max(1, abs(ref.mu))
    np.testing.assert_allclose(tau.cpu().numpy()[:ref.n_pl + 1], ref.tau, rtol=0,
                               atol=1e-10 * N_S)
    np.testing.assert_allclose(Dd.cpu().numpy(), ref.D, rtol=0, atol=1e-12)
    assert abs(info.e_band - ref.e_band) < 1e-11 * abs(ref.e_band)
    assert abs(info.e_ent - ref.e_ent) < 1e-11 * abs(ref.e_ent)
    assert abs(info.n_count - 0.4 * N_S) < 1e-9
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_density_and_forces_2048(L, case, kernel_ref, precision):
    p, H, Phi, D = case["p"], case["H"], case["Phi"], kernel_ref.D
    rho_ref = odens.density(Phi, D)
    f_ref = odens.nonlocal_forces(H, Phi, D, len(p.positions))
    ctx = _ctx(p, precision)
    print(f"dk_density + dk_forces N_s={N_S} {precision}", flush=True)
    Xd = _dev(Phi.T, ctx.dtype)
    Dd = _dev(D)
    rho = torch.zeros(p.n_grid, dtype=torch.float64, device="cuda")
    L.dk_density(ctx.h, Xd, Dd, rho)
    got = rho.cpu().numpy()
    f = L.dk_forces(ctx.h, Xd, Dd, rho, None, len(p.positions))
    fscale = np.abs(f_ref).max()
    if precision == "fp64":
        np.testing.assert_allclose(got, rho_ref, rtol=0, atol=1e-12 * rho_ref.max())
        np.testing.assert_allclose(f, f_ref, rtol=0, atol=1e-10 * fscale)
    else:
        assert np.abs(got - rho_ref).max() < 1e-6 * rho_ref.max()
        assert np.abs(f - f_ref).max() < 1e-5 * fscale
    ctx.close()
