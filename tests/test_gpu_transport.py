"""Green-Kubo entry points against the oracle (needs a GPU).

dk_time_correlation and dk_deviatoric_stress on seeded series, element by
element: FP64 sums in another order, so to a relative 1e-12 of the largest
entry.  Sizes span several 256-lane strides with a ragged tail; edge cases:
max_lag = n_steps (one origin at the last lag), a single component, and the
argument errors.
"""

import numpy as np
import pytest
import torch

from oracle import transport as otr
from workloads import custom_spec, make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_08639_amd.pipeline import Context
    p = make_problem(custom_spec("gk", 90, 5.0, 1, 12, 4, 1.0, basis="sc", noise=False),
                     with_block=False)
    c = Context(p, "fp64")
    yield c
    c.close()


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("T,n,K", [(613, 96, 200), (50, 1, 50), (1, 5, 1), (2000, 15, 700)])
def test_time_correlation_matches_oracle(ctx, T, n, K):
    from paper_2112_08639_amd import _lib as L
    rng = np.random.default_rng(T + n)
    s = rng.standard_normal((T, n)) + 0.3
    dt, scale = 0.37, 2.5
    print(f"dk_time_correlation T={T} n_comp={n} max_lag={K}", flush=True)
    integral = torch.zeros(K, dtype=torch.float64, device="cuda")
    corr, _ = L.dk_time_correlation(ctx.h, _dev(s), K, dt, scale, integral=integral)
    ref = otr.time_correlation(s, K)
    ref_i = scale * otr.running_integral(ref, dt)
    np.testing.assert_allclose(corr.cpu().numpy(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    np.testing.assert_allclose(integral.cpu().numpy(), ref_i, rtol=0,
                               atol=1e-12 * max(1.0, np.abs(ref_i).max()))


def test_deviatoric_stress_matches_oracle(ctx):
    from paper_2112_08639_amd import _lib as L
    rng = np.random.default_rng(5)
    T, N, mass = 37, 70, 3.1
    sig = rng.standard_normal((T, 3, 3))
    sig = 0.5 * (sig + sig.transpose(0, 2, 1))
    v = rng.standard_normal((T, N, 3))
    vol = ctx.problem.spec.volume
    got = L.dk_deviatoric_stress(ctx.h, _dev(sig), _dev(v), mass).cpu().numpy()
    total = np.stack([sig[t] - otr.ionic_momentum_flux(v[t], mass, vol) for t in range(T)])
    ref = otr.deviatoric_components(total)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    got0 = L.dk_deviatoric_stress(ctx.h, _dev(sig)).cpu().numpy()
    np.testing.assert_allclose(got0, otr.deviatoric_components(sig), rtol=0, atol=1e-15)


def test_transport_argument_errors(ctx):
    from paper_2112_08639_amd import _lib as L
    s = torch.zeros((10, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(L.DkError) as e:
        L.dk_time_correlation(ctx.h, s, 11)
    assert e.value.name == "DK_ERR_ARG"
    with pytest.raises(L.DkError) as e:
        L.dk_time_correlation(ctx.h, s, 0)
    assert e.value.name == "DK_ERR_ARG"
    with pytest.raises(L.DkError) as e:
        L.dk_time_correlation(ctx.h, s, 5, 0.0, 1.0,
                              integral=torch.zeros(5, dtype=torch.float64, device="cuda"))
    assert e.value.name == "DK_ERR_ARG"
