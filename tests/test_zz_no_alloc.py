"""dk_density_noalloc against dk_density (needs a GPU).

The no-allocation variant shares the kernels of dk_density and keeps the
per-tile row partials in the library's static device scratch.  Two calls in a
row, the second with a smaller problem (fewer columns, then a smaller grid on
another context), must each give dk_density's result on the same inputs; the
context used for the variant never gets a workspace.  A problem beyond the
scratch is refused on the host.
"""

import numpy as np
import pytest
import torch

from workloads import custom_spec, make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_08639_amd import _lib
    _lib.load()
    return _lib


def _inputs(p, n_s, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n_s, p.n_grid))
    A = rng.standard_normal((n_s, n_s))
    return X, 0.5 * (A + A.T) / n_s


def _pair(L, p, precision, n_s, seed):
    """(dk_density on a context with a workspace, dk_density_noalloc on one without)."""
    from paper_2112_08639_amd.pipeline import Context
    X, D = _inputs(p, n_s, seed)
    dt = torch.float64 if precision == "fp64" else torch.float32
    Xd = torch.as_tensor(X, dtype=dt, device="cuda").contiguous()
    Dd = torch.as_tensor(D, dtype=torch.float64, device="cuda").contiguous()
    ref_ctx = Context(p, precision)
    ref_ctx.ensure_workspace(n_s, 16)
    rho_ref = torch.zeros(p.n_grid, dtype=torch.float64, device="cuda")
    L.dk_density(ref_ctx.h, Xd, Dd, rho_ref)
    ref_ctx.close()
    ctx = Context(p, precision)  # no workspace
    rho = torch.full((p.n_grid,), float("nan"), dtype=torch.float64, device="cuda")
    print(f"dk_density_noalloc {precision} N_grid={p.n_grid} n_s={n_s}", flush=True)
    L.dk_density_noalloc(ctx.h, Xd, Dd, rho)
    ctx.close()
    return rho_ref.cpu().numpy(), rho.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_density_twice(L, precision):
    big = make_problem(custom_spec("na24", 91, 7.6, 1, 24, 8, 1.0, noise=False),
                       with_block=False)
    small = make_problem(custom_spec("na16", 92, 5.0, 1, 16, 8, 1.0, basis="sc", noise=False),
                         with_block=False)
    # 200 columns on 24^3 (4 column tiles, ragged), then 70 on the same grid,
    # then 33 on 16^3: each call leaves partials the next must not read
    for p, n_s, seed in ((big, 200, 1), (big, 70, 2), (small, 33, 3)):
        ref, got = _pair(L, p, precision, n_s, seed)
        assert np.all(np.isfinite(got))
        # same kernels on the same inputs: identical up to rounding (bitwise here)
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_noalloc_refuses_beyond_scratch(L):
    from paper_2112_08639_amd.pipeline import Context
    p = make_problem(custom_spec("na24b", 91, 7.6, 1, 24, 8, 1.0, noise=False),
                     with_block=False)
    ctx = Context(p, "fp64")
    # 24^3 x ceil(n_s/64) doubles > 128 MiB needs n_s > 64 * 1214
    n_s = 64 * 1300
    X = torch.zeros((1, p.n_grid), dtype=torch.float64, device="cuda")
    D = torch.zeros((1, 1), dtype=torch.float64, device="cuda")
    rho = torch.zeros(p.n_grid, dtype=torch.float64, device="cuda")
    import ctypes as C
    lib = L.load()
    st = lib.dk_density_noalloc(ctx.h, C.c_void_p(X.data_ptr()), p.n_grid, n_s,
                                C.c_void_p(D.data_ptr()), C.c_void_p(rho.data_ptr()))
    assert L.STATUS[st] == "DK_ERR_ARG"
    assert b"static scratch" in lib.dk_last_error(ctx.h)
    ctx.close()
