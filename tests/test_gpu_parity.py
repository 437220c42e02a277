"""Parity of every libdk entry point with the FP64 oracle (needs a GPU).

Each call goes through the C ABI (ctypes binding) on seeded inputs shared with
the oracle.  FP64 results must agree to a relative 1e-10 (most to ~1e-13);
the mixed path (FP32 blocks, FP32 stencil/projectors, split-BF16 products)
to the budgets of the accuracy targets: h^3 sum |drho| / N_e <= 1e-5, band
free energy <= 1e-5 Ha/atom, forces <= 1e-4 Ha/bohr.

Cases: the 4-atom workload (24^3 grid, several 64-row tiles), a ragged
10^3 grid with N_s = 20 (no dimension a multiple of a tile), and edge cases.
"""

import numpy as np
import pytest
import torch

from oracle import density as odens
from oracle import foe as ofoe
from oracle import sq3 as osq3
from oracle.filter import chebyshev_filter
from oracle.hamiltonian import Hamiltonian
from oracle.orth import cholqr2
from workloads import custom_spec, make_problem, spec_for

pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def L():
    _need_gpu()
    from paper_2112_08639_amd import _lib
    _lib.load()
    return _lib


@pytest.fixture(scope="module")
def al4():
    return make_problem(spec_for("al4"))


@pytest.fixture(scope="module")
def ragged():
    spec = custom_spec("ragged", 95, 5.0, 1, 10, 20, 1.0, filter_degree=6, filter_passes=2,
                       n_pl=80, basis="fcc")
    return make_problem(spec)


def _ctx(problem, precision="fp64", n_s=None, n_pl=200):
    from paper_2112_08639_amd.pipeline import Context
    ctx = Context(problem, precision)
    ctx.ensure_workspace(n_s or problem.n_s, n_pl)
    return ctx


def _dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _orth_block(problem, n_s, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((problem.n_grid, n_s))
    return cholqr2(X, problem.h)


@pytest.mark.parametrize("name", ["al4", "ragged"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_apply_h(L, al4, ragged, name, precision):
    p = al4 if name == "al4" else ragged
    H = Hamiltonian(p)
    X = np.random.default_rng(1).standard_normal((p.n_grid, 7))
    ref = H.apply(X)
    ctx = _ctx(p, precision, n_s=7)
    dt = ctx.dtype
    Xd = _dev(X.T, dt)
    Yd = torch.zeros_like(Xd)
    L.dk_apply_h(ctx.h, Xd, Yd)
    got = Yd.double().cpu().numpy().T
    tol = 1e-12 if precision == "fp64" else 2e-5
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err < tol, err
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_apply_h_many_projectors(L, precision):
    # 108 atoms on a 36^3 grid: 432 projectors, so the projector integrals use
    # 128-row tiles over 64-projector mask rows, and about 10% of the (64-projector,
    # 64-point) blocks are empty; a tile may skip a block only when both of its
    # mask rows are empty there
    spec = custom_spec("al108c", 96, 7.6, 3, 36, 6, 5.0, noise=False)
    p = make_problem(spec, with_block=False)
    H = Hamiltonian(p)
    X = np.random.default_rng(21).standard_normal((p.n_grid, 6))
    ref = H.apply(X)
    from paper_2112_08639_amd.pipeline import Context
    ctx = Context(p, precision)
    ctx.ensure_workspace(6, 16)
    dt = ctx.dtype
    Xd = _dev(X.T, dt)
    Yd = torch.zeros_like(Xd)
    L.dk_apply_h(ctx.h, Xd, Yd)
    got = Yd.double().cpu().numpy().T
    tol = 1e-12 if precision == "fp64" else 2e-5
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err < tol, err
    ctx.close()


# More than 64 atom groups: the projector integrals run over the compact
# supports (chunks of 64-point blocks, union of live groups per chunk).  The
# dense case (108 atoms in a 13.5 bohr cell on 24^3, each 64-point block
# reaching ~70 of the 108 atoms) also exercises blocks with more live groups
# than one chunk holds (32 in FP64, 64 mixed), which are split over several
# single-block chunks; the sparse case (108 atoms, 36^3) the multi-block chunks.
@pytest.mark.parametrize("case", ["dense", "sparse"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_apply_h_compact_supports(L, case, precision):
    if case == "dense":
        spec = custom_spec("cs108d", 89, 4.5, 3, 24, 6, 5.0, noise=True)
    else:
        spec = custom_spec("cs108s", 88, 7.6, 3, 36, 6, 5.0, noise=True)
    p = make_problem(spec, with_block=False)
    H = Hamiltonian(p)
    X = np.random.default_rng(23).standard_normal((p.n_grid, 70))
    ref = H.apply(X)
    from paper_2112_08639_amd.pipeline import Context
    ctx = Context(p, precision)
    ctx.ensure_workspace(70, 16)
    print(f"dk_apply_h compact supports {case} {precision}", flush=True)
    Xd = _dev(X.T, ctx.dtype)
    Yd = torch.zeros_like(Xd)
    L.dk_apply_h(ctx.h, Xd, Yd)
    got = Yd.double().cpu().numpy().T
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err < (1e-12 if precision == "fp64" else 2e-5), err
    # the nonlocal term alone, to its own scale (H - H_local)
    Hl = Hamiltonian(p)
    Hl.gamma = np.zeros_like(Hl.gamma)
    nl_ref = ref - Hl.apply(X)
    nl_got = got - Hl.apply(X)
    err_nl = np.abs(nl_got - nl_ref).max() / np.abs(nl_ref).max()
    assert err_nl < (1e-11 if precision == "fp64" else 1e-4), err_nl
    ctx.close()


# Stencil forms by plane size.  FP32: 8^2 and 20^2 take the fixed-pitch plane
# kernel (at ny = 8 the rows 2..5 carry both periodic copies, at nx = 8 every x
# segment both), 32^2 and 48^2 the DPP kernel (x halo by row rotations over 16
# lanes of 2 or 3 points), 64^2 the whole-plane kernel of 1024 threads, 72^2 and 96^2 the
# slab form with workgroups of at most 768 threads (several row slabs per plane
# with periodic halo rows), 88^2 the slab form with 968 threads.  FP64 (2-point
# vectors): every plane takes the slab form; 24^2 and 48^2 at most 768 threads,
# 72^2 (864) and 96^2 (960) the 1024-thread form.
@pytest.mark.parametrize("n,precision", [(8, "mixed"), (20, "mixed"), (32, "mixed"),
                                         (48, "mixed"), (64, "mixed"),
                                         (72, "mixed"), (96, "mixed"), (88, "mixed"),
                                         (24, "fp64"), (48, "fp64"), (72, "fp64"),
                                         (96, "fp64")])
def test_apply_h_large_plane(L, n, precision):
    spec = custom_spec(f"plane{n}", 99, 7.6, 1, n, 3, 1.0, noise=False)
    p = make_problem(spec, with_block=False)
    H = Hamiltonian(p)
    X = np.random.default_rng(4).standard_normal((p.n_grid, 3))
    ref = H.apply(X)
    from paper_2112_08639_amd.pipeline import Context
    ctx = Context(p, precision)
    ctx.ensure_workspace(3, 16)
    print(f"dk_apply_h plane {n}^2 {precision}", flush=True)
    Xd = _dev(X.T, ctx.dtype)
    Yd = torch.zeros_like(Xd)
    L.dk_apply_h(ctx.h, Xd, Yd)
    got = Yd.double().cpu().numpy().T
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err < (1e-12 if precision == "fp64" else 2e-5), err
    ctx.close()


# The mixed filter: the fused beta Y_{k-1} update of the stencil writes over
# Y_{k-1} in place.  24^2 takes the fixed-pitch plane kernel, 48^2 the DPP
# kernel, 64^2 the 1024-thread plane kernel, 72^2 the slab kernel.  FP32 block: the relative
# error of a degree-m filter grows like m times the FP32 rounding of one
# application against the damped-interval amplification.
@pytest.mark.parametrize("n", [24, 48, 64, 72])
def test_filter_mixed(L, n):
    spec = custom_spec(f"filt{n}", 94, 7.6, 1, n, 5, 1.0, noise=True)
    p = make_problem(spec, with_block=False)
    H = Hamiltonian(p)
    Phi = _orth_block(p, 5, 12)
    b = H.upper_bound()
    a0, a, m = -3.0, 8.0, 6
    ref = chebyshev_filter(H, Phi, m, a, b, a0)
    from paper_2112_08639_amd.pipeline import Context
    ctx = Context(p, "mixed")
    ctx.ensure_workspace(5, 16)
    print(f"dk_filter mixed plane {n}^2", flush=True)
    Xd = _dev(Phi.T, torch.float32)
    L.dk_filter(ctx.h, Xd, m, a, b, a0)
    got = Xd.double().cpu().numpy().T
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err < 1e-5, err
    ctx.close()


# The mixed filter with 128 projectors (32 groups, the three-piece integrals over
# 128-row tiles and the scatter over the per-block group lists): 18^3 points
# end in a partial 64-point tile, 70 columns in a partial 64-column tile.
def test_filter_mixed_projectors(L):
    spec = custom_spec("filtp", 93, 7.6, 2, 18, 70, 1.0, noise=True)
    p = make_problem(spec, with_block=False)
    H = Hamiltonian(p)
    Phi = _orth_block(p, 70, 14)
    b = H.upper_bound()
    a0, a, m = -3.0, 8.0, 5
    ref = chebyshev_filter(H, Phi, m, a, b, a0)
    from paper_2112_08639_amd.pipeline import Context
    ctx = Context(p, "mixed")
    ctx.ensure_workspace(70, 16)
    print("dk_filter mixed 18^3, 128 projectors, N_s = 70", flush=True)
    Xd = _dev(Phi.T, torch.float32)
    L.dk_filter(ctx.h, Xd, m, a, b, a0)
    got = Xd.double().cpu().numpy().T
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"max relative error {err:.3e}", flush=True)
    assert err < 1e-5, err
    ctx.close()


# The mixed filter over compact supports (more than 64 atom groups): its steps
# take the two-piece split-BF16 integrals (x = hi + lo, three products).
@pytest.mark.parametrize("case", ["dense", "sparse"])
def test_filter_mixed_compact_supports(L, case):
    if case == "dense":
        spec = custom_spec("cs108d", 89, 4.5, 3, 24, 70, 5.0, noise=True)
    else:
        spec = custom_spec("cs108s", 88, 7.6, 3, 36, 70, 5.0, noise=True)
    p = make_problem(spec, with_block=False)
    H = Hamiltonian(p)
    Phi = _orth_block(p, 70, 15)
    b = H.upper_bound()
    a0, a, m = -3.0, 8.0, 4
    ref = chebyshev_filter(H, Phi, m, a, b, a0)
    from paper_2112_08639_amd.pipeline import Context
    ctx = Context(p, "mixed")
    ctx.ensure_workspace(70, 16)
    print(f"dk_filter mixed compact supports {case}", flush=True)
    Xd = _dev(Phi.T, torch.float32)
    L.dk_filter(ctx.h, Xd, m, a, b, a0)
    got = Xd.double().cpu().numpy().T
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"max relative error {err:.3e}", flush=True)
    assert err < 1e-5, err
    ctx.close()


@pytest.mark.parametrize("name", ["al4", "ragged"])
def test_filter(L, al4, ragged, name):
    p = al4 if name == "al4" else ragged
    H = Hamiltonian(p)
    Phi = _orth_block(p, 9, 2)
    b = H.upper_bound()
    a0, a, m = -0.5, 6.0, 7
    ref = chebyshev_filter(H, Phi, m, a, b, a0)
    ctx = _ctx(p, "fp64", n_s=9)
    assert abs(ctx.upper - b) < 1e-12 * b
    Xd = _dev(Phi.T)
    L.dk_filter(ctx.h, Xd, m, a, b, a0)
    got = Xd.cpu().numpy().T
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err < 1e-11, err
    ctx.close()


@pytest.mark.parametrize("name", ["al4", "ragged"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_orthonormalize(L, al4, ragged, name, precision):
    p = al4 if name == "al4" else ragged
    n_s = 40 if name == "al4" else 20
    X = np.random.default_rng(3).standard_normal((p.n_grid, n_s)) @ np.diag(np.logspace(0, 2, n_s))
    ref = cholqr2(X, p.h)
    ctx = _ctx(p, precision, n_s=n_s)
    Xd = _dev(X.T, ctx.dtype)
    L.dk_orthonormalize(ctx.h, Xd)
    got = Xd.double().cpu().numpy().T
    if precision == "fp64":
        np.testing.assert_allclose(got, ref, atol=1e-12 * np.abs(ref).max())
    else:
        G = p.h ** 3 * got.T @ got
        assert np.abs(G - np.eye(n_s)).max() < 1e-5
        assert np.abs(got - ref).max() < 1e-4 * np.abs(ref).max()
    ctx.close()


@pytest.mark.parametrize("name", ["al4", "ragged"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_project_and_bounds(L, al4, ragged, name, precision):
    p = al4 if name == "al4" else ragged
    n_s = 64 if name == "al4" else 20
    Phi = _orth_block(p, n_s, 4)
    ref = osq3.project(Hamiltonian(p), Phi)
    ctx = _ctx(p, precision, n_s=n_s)
    Xd = _dev(Phi.T, ctx.dtype)
    Hs = torch.zeros((n_s, n_s), dtype=torch.float64, device="cuda")
    L.dk_project(ctx.h, Xd, Hs)
    got = Hs.cpu().numpy()
    scale = np.abs(ref).max()
    tol = 1e-12 if precision == "fp64" else 1e-4
    assert np.abs(got - ref).max() < tol * scale
    assert np.array_equal(got, got.T)
    lo, hi, it = L.dk_spectral_bounds(ctx.h, Hs)
    ev = np.linalg.eigvalsh(got)
    assert abs(lo - ev[0]) < 1e-12 * np.abs(ev).max()
    assert abs(hi - ev[-1]) < 1e-12 * np.abs(ev).max()
    assert 0 <= it <= 96
    ctx.close()


@pytest.mark.parametrize("n_s,n_pl,sigma", [(64, 120, 1.0), (20, 80, 0.3), (150, 60, 2.0)])
def test_density_kernel(L, al4, n_s, n_pl, sigma):
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((n_s, n_s)))
    lam = np.sort(rng.uniform(-3, 9, n_s))
    Hs = (Q * lam) @ Q.T
    Hs = 0.5 * (Hs + Hs.T)
    n_e = 0.6 * n_s
    ref = ofoe.density_kernel(Hs, n_e, sigma, n_pl)
    ctx = _ctx(al4, "fp64", n_s=n_s, n_pl=n_pl)
    Hd = _dev(Hs)
    Dd = torch.zeros_like(Hd)
    tau = torch.zeros(n_pl + 1, dtype=torch.float64, device="cuda")
    info = L.dk_density_kernel(ctx.h, Hd, n_e, sigma, n_pl, Dd, tau)
    assert abs(info.mu - ref.mu) < 1e-12 * max(1, abs(ref.mu))
    assert abs(info.lam_min - ref.lam_min) < 1e-12 * 10 and abs(info.lam_max - ref.lam_max) < 1e-12 * 10
    np.testing.assert_allclose(tau.cpu().numpy(), ref.tau, atol=1e-10 * n_s)
    np.testing.assert_allclose(Dd.cpu().numpy(), ref.D, atol=1e-12)
    assert abs(info.e_band - ref.e_band) < 1e-11 * max(1, abs(ref.e_band))
    assert abs(info.e_ent - ref.e_ent) < 1e-11 * max(1, abs(ref.e_ent))
    assert abs(info.n_count - n_e) < 1e-10
    eb, ee = L.dk_energy(ctx.h, tau, n_pl, info.mu, info.chi, info.xi, sigma)
    assert abs(eb - ref.e_band) < 1e-11 * max(1, abs(ref.e_band))
    assert abs(ee - ref.e_ent) < 1e-11 * max(1, abs(ref.e_ent))
    ctx.close()


def _random_spectrum_hs(ns, lo, hi, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((ns, ns)))
    Hs = (Q * np.sort(rng.uniform(lo, hi, ns))) @ Q.T
    return 0.5 * (Hs + Hs.T)


@pytest.mark.parametrize("sigma", [2.0, 1.0, 0.3])
def test_density_kernel_tail_rule(L, al4, sigma):
    # n_pl = 0: degree from the coefficient-tail rule, identical choice to the oracle's
    n_s = 40
    Hs = _random_spectrum_hs(n_s, -5.0, 6.0, 21)
    n_e = 31.0
    ref = ofoe.density_kernel(Hs, n_e, sigma, 0)
    ctx = _ctx(al4, "fp64", n_s=n_s, n_pl=0)
    Hd = _dev(Hs)
    Dd = torch.zeros_like(Hd)
    tau = torch.zeros(L.DK_TAIL_MAX_DEGREE + 1, dtype=torch.float64, device="cuda")
    info = L.dk_density_kernel(ctx.h, Hd, n_e, sigma, 0, Dd, tau)
    assert info.n_pl == ref.n_pl
    assert abs(info.mu - ref.mu) < 1e-12 * max(1, abs(ref.mu))
    np.testing.assert_allclose(tau.cpu().numpy()[:ref.n_pl + 1], ref.tau, atol=1e-10 * n_s)
    np.testing.assert_allclose(Dd.cpu().numpy(), ref.D, atol=1e-12)
    eb, ee = L.dk_energy(ctx.h, tau, info.n_pl, info.mu, info.chi, info.xi, sigma)
    assert abs(eb - ref.e_band) < 1e-11 * max(1, abs(ref.e_band))
    assert abs(ee - ref.e_ent) < 1e-11 * max(1, abs(ref.e_ent))
    # a temperature too low for degree 256 is reported, not truncated
    Ds2 = torch.zeros_like(Hd)
    with pytest.raises(L.DkError) as e:
        L.dk_density_kernel(ctx.h, Hd, n_e, 0.01, 0, Ds2, tau)
    assert e.value.name == "DK_ERR_CONVERGENCE"
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_density_and_forces(L, al4, precision):
    p = al4
    n_s = 64
    Phi = _orth_block(p, n_s, 6)
    H = Hamiltonian(p)
    Hs = osq3.project(H, Phi)
    dk = ofoe.density_kernel(Hs, p.n_e, p.spec.kT, 120)
    rho_ref = odens.density(Phi, dk.D)
    f_ref = odens.local_forces(rho_ref, p.gradv, p.h) + odens.nonlocal_forces(H, Phi, dk.D, 4)
    ctx = _ctx(p, precision, n_s=n_s)
    Xd = _dev(Phi.T, ctx.dtype)
    Dd = _dev(dk.D)
    rho = torch.zeros(p.n_grid, dtype=torch.float64, device="cuda")
    L.dk_density(ctx.h, Xd, Dd, rho)
    got = rho.cpu().numpy()
    gv = _dev(p.gradv)
    f = L.dk_forces(ctx.h, Xd, Dd, rho, gv, 4)
    if precision == "fp64":
        np.testing.assert_allclose(got, rho_ref, atol=1e-12 * rho_ref.max())
        np.testing.assert_allclose(f, f_ref, atol=1e-11)
    else:
        assert p.h ** 3 * np.abs(got - rho_ref).sum() / p.n_e < 1e-5
        # three-piece split of the Phi D product: FP32-level density (the block is FP32)
        assert np.abs(got - rho_ref).max() < 1e-6 * rho_ref.max()
        assert np.abs(f - f_ref).max() < 1e-4
    ctx.close()


def test_full_al4_fp64_matches_oracle(L, al4):
    from paper_2112_08639_amd.pipeline import evaluate
    ref = osq3.run(al4)
    got = evaluate(al4, "fp64")
    rho = got.rho.cpu().numpy()
    assert np.abs(rho - ref.rho).max() < 1e-10 * ref.rho.max()
    assert abs(got.info["mu"] - ref.dk.mu) < 1e-10 * max(1, abs(ref.dk.mu))
    assert abs(got.e_band - ref.e_band) < 1e-10 * abs(ref.e_band)
    assert abs(got.e_ent - ref.e_ent) < 1e-10 * abs(ref.e_ent)
    assert np.abs(got.forces - ref.forces).max() < 1e-10 * np.abs(ref.forces).max() + 1e-13
    for (a0g, ag, bg), (a0r, ar, br) in zip(got.bounds, ref.bounds):
        assert abs(a0g - a0r) < 1e-11 * abs(ar) and abs(ag - ar) < 1e-11 * abs(ar)
        assert abs(bg - br) < 1e-12 * br
    # invariants
    assert abs(al4.h ** 3 * rho.sum() - al4.n_e) < 1e-10
    ev = np.linalg.eigvalsh(got.Ds.cpu().numpy())
    assert ev.min() > -1e-10 and ev.max() < 1 + 1e-10


def test_full_al4_mixed_within_budget(L, al4):
    from paper_2112_08639_amd.pipeline import evaluate
    ref = osq3.run(al4)
    got = evaluate(al4, "mixed")
    rho = got.rho.cpu().numpy()
    n_at = len(al4.positions)
    assert al4.h ** 3 * np.abs(rho - ref.rho).sum() / al4.n_e <= 1e-5
    assert abs(got.free_energy - ref.free_energy) / n_at <= 1e-5
    assert np.abs(got.forces - ref.forces).max() <= 1e-4


def test_full_ragged_fp64(L, ragged):
    from paper_2112_08639_amd.pipeline import evaluate
    ref = osq3.run(ragged)
    got = evaluate(ragged, "fp64")
    rho = got.rho.cpu().numpy()
    assert np.abs(rho - ref.rho).max() < 1e-10 * ref.rho.max()
    assert abs(got.free_energy - ref.free_energy) < 1e-10 * abs(ref.free_energy)
    assert np.abs(got.forces - ref.forces).max() < 1e-10 * np.abs(ref.forces).max() + 1e-13


# ------------------------------------------------------------------ errors --

def test_error_paths(L, al4):
    ctx = _ctx(al4, "fp64", n_s=8)
    X = np.random.default_rng(9).standard_normal((al4.n_grid, 8))
    X[:, 5] = X[:, 2]  # rank deficient
    Xd = _dev(X.T)
    with pytest.raises(L.DkError) as e:
        L.dk_orthonormalize(ctx.h, Xd)
    assert e.value.name == "DK_ERR_NOT_SPD"
    Hs = torch.eye(8, dtype=torch.float64, device="cuda")
    Ds = torch.zeros_like(Hs)
    with pytest.raises(L.DkError) as e:
        L.dk_density_kernel(ctx.h, Hs, 16.0, 1.0, 20, Ds)
    assert e.value.name == "DK_ERR_FERMI"
    with pytest.raises(L.DkError) as e:
        L.dk_filter(ctx.h, Xd, 5, 2.0, 1.0, 0.0)
    assert e.value.name == "DK_ERR_ARG"
    # H_s a multiple of the identity: xi = 1, D = (N_e / 2 N_s) I
    info = L.dk_density_kernel(ctx.h, 3.0 * Hs, 6.0, 1.0, 20, Ds)
    np.testing.assert_allclose(Ds.cpu().numpy(), 6.0 / 16.0 * np.eye(8), atol=1e-13)
    assert abs(info.mu - (3.0 - np.log(16.0 / 6.0 - 1.0))) < 1e-12
    # NaN potential
    bad = torch.as_tensor(al4.veff, device="cuda").clone()
    bad[17] = float("nan")
    with pytest.raises(L.DkError) as e:
        L.dk_set_potential(ctx.h, bad)
    assert e.value.name == "DK_ERR_NONFINITE"
    ctx.close()


def test_workspace_too_small(L, al4):
    from paper_2112_08639_amd.pipeline import Context
    ctx = Context(al4, "fp64")
    small = torch.empty(1024, dtype=torch.float64, device="cuda")
    L.dk_set_workspace(ctx.h, small)
    Xd = _dev(np.random.default_rng(1).standard_normal((8, al4.n_grid)))
    with pytest.raises(L.DkError) as e:
        L.dk_orthonormalize(ctx.h, Xd)
    assert e.value.name == "DK_ERR_ALLOC"
    ctx.close()


def test_single_column(L, al4):
    ctx = _ctx(al4, "fp64", n_s=1)
    X = _dev(np.random.default_rng(2).standard_normal((1, al4.n_grid)))
    L.dk_orthonormalize(ctx.h, X)
    assert abs(al4.h ** 3 * float((X * X).sum()) - 1.0) < 1e-13
    Hs = torch.zeros((1, 1), dtype=torch.float64, device="cuda")
    L.dk_project(ctx.h, X, Hs)
    Ds = torch.zeros_like(Hs)
    info = L.dk_density_kernel(ctx.h, Hs, 1.0, 1.0, 10, Ds)
    assert abs(float(Ds[0, 0]) - 0.5) < 1e-13
    assert abs(info.mu - float(Hs[0, 0])) < 1e-12
    ctx.close()


# ------------------------------------------------------- orthorhombic grid --
# nx != ny != nz and lx != ly != lz (spacings 0.34, 0.35, 0.31 bohr): per-axis
# stencil weights, periodic wraps and index strides, the per-axis kinetic
# bound, and the forces' per-axis first differences.

@pytest.fixture(scope="module")
def ortho():
    spec = custom_spec("ortho", 93, 7.6, 1, 16, 24, 1.0, filter_degree=8, filter_passes=2,
                       n_pl=80, basis="fcc", dims=(16, 20, 28), lens=(5.44, 7.0, 8.68))
    pos = np.array([[0.4, 0.3, 0.9], [2.9, 3.8, 1.2], [1.1, 4.6, 5.3], [4.2, 1.7, 7.1]])
    return make_problem(spec, positions=pos)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_apply_h_orthorhombic(L, ortho, precision):
    p = ortho
    H = Hamiltonian(p)
    X = np.random.default_rng(8).standard_normal((p.n_grid, 5))
    ref = H.apply(X)
    ctx = _ctx(p, precision, n_s=5)
    assert abs(ctx.upper - H.upper_bound()) < 1e-12 * ctx.upper
    print(f"dk_apply_h 16x20x28 {precision}", flush=True)
    Xd = _dev(X.T, ctx.dtype)
    Yd = torch.zeros_like(Xd)
    L.dk_apply_h(ctx.h, Xd, Yd)
    got = Yd.double().cpu().numpy().T
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err < (1e-12 if precision == "fp64" else 2e-5), err
    ctx.close()


def test_filter_orthorhombic(L, ortho):
    p = ortho
    H = Hamiltonian(p)
    Phi = _orth_block(p, 9, 13)
    b = H.upper_bound()
    a0, a, m = -1.0, 7.0, 7
    ref = chebyshev_filter(H, Phi, m, a, b, a0)
    ctx = _ctx(p, "fp64", n_s=9)
    print("dk_filter 16x20x28 fp64", flush=True)
    Xd = _dev(Phi.T)
    L.dk_filter(ctx.h, Xd, m, a, b, a0)
    got = Xd.cpu().numpy().T
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err < 1e-11, err
    ctx.close()


def test_full_orthorhombic(L, ortho):
    from paper_2112_08639_amd.pipeline import evaluate
    ref = osq3.run(ortho)
    print("evaluate 16x20x28 fp64 and mixed", flush=True)
    got = evaluate(ortho, "fp64")
    rho = got.rho.cpu().numpy()
    assert np.abs(rho - ref.rho).max() < 1e-10 * ref.rho.max()
    assert abs(got.free_energy - ref.free_energy) < 1e-10 * abs(ref.free_energy)
    assert np.abs(got.forces - ref.forces).max() < 1e-10 * np.abs(ref.forces).max() + 1e-13
    assert abs(ortho.h ** 3 * rho.sum() - ortho.n_e) < 1e-10
    mix = evaluate(ortho, "mixed")
    n_at = len(ortho.positions)
    assert ortho.h ** 3 * np.abs(mix.rho.cpu().numpy() - ref.rho).sum() / ortho.n_e <= 1e-5
    assert abs(mix.free_energy - ref.free_energy) / n_at <= 1e-5
    assert np.abs(mix.forces - ref.forces).max() <= 1e-4
