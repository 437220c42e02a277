"""Parity of the learned-start entry points with the FP64 oracle (needs a GPU).

Descriptors (FP32 output) against the oracle's image sums; channel statistics;
the loss gradient by backpropagation in FP32 MFMA mode (tight) and in BF16
mode (to BF16 rounding); Adam; the normalised predicted density; and a short
training run whose loss falls.  Batch sizes span several 64-point tiles with
a ragged tail.
"""

import numpy as np
import pytest
import torch

from oracle import mlp as omlp
from workloads import custom_spec, make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_08639_amd import _lib
    _lib.load()
    return _lib


@pytest.fixture(scope="module")
def cell():
    spec = custom_spec("mlp15", 97, 7.6, 1, 15, 8, 1.0, basis="fcc", noise=False)
    return make_problem(spec)


def _ctx(p):
    from paper_2112_08639_amd.pipeline import Context
    return Context(p, "fp64")


def _f32(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def _f64(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def test_descriptors_and_stats(L, cell):
    p = cell
    ctx = _ctx(p)
    w = omlp.widths(32, 0.5, 4.0)
    d = torch.empty(p.n_grid * 32, dtype=torch.float32, device="cuda")
    L.dk_descriptors(ctx.h, p.positions, w, d)
    ref = omlp.descriptors(p.n, p.spec.a, p.positions, w)
    got = d.cpu().numpy().reshape(p.n_grid, 32)
    np.testing.assert_allclose(got, ref, rtol=2e-7, atol=1e-30)
    mean = torch.zeros(32, dtype=torch.float64, device="cuda")
    inv = torch.zeros_like(mean)
    L.dk_descriptor_stats(ctx.h, d, p.n_grid, 32, mean, inv)
    g64 = got.astype(np.float64)
    np.testing.assert_allclose(mean.cpu().numpy(), g64.mean(axis=0), rtol=1e-12)
    np.testing.assert_allclose(inv.cpu().numpy(), 1.0 / g64.std(axis=0), rtol=1e-10)
    ctx.close()


def _batch(n_in, P, seed):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((P, n_in)).astype(np.float32)
    t = rng.uniform(0.2, 3.0, P).astype(np.float32)
    return u, t


@pytest.mark.parametrize("mode", ["f32", "bf16"])
def test_loss_gradient_matches_oracle(L, cell, mode):
    ctx = _ctx(cell)
    shapes = omlp.layer_shapes(32, 64, 3)
    theta = omlp.init_params(shapes, 5000).astype(np.float32).astype(np.float64)
    P = 1000
    u, t = _batch(32, P, 3)
    loss_ref, g_ref = omlp.loss_and_grad(theta, shapes, u.astype(np.float64), t.astype(np.float64))
    shape = L.MlpShape(32, 64, 3)
    assert L.dk_mlp_param_count(shape) == omlp.param_count(shapes)
    ws = torch.empty(L.dk_mlp_workspace_bytes(shape, P) // 4 + 64, dtype=torch.float32, device="cuda")
    grad = torch.zeros(len(theta), dtype=torch.float32, device="cuda")
    m = L.DK_MLP_F32 if mode == "f32" else L.DK_MLP_BF16
    loss = L.dk_mlp_loss_grad(ctx.h, shape, m, _f32(theta), _f32(u.reshape(-1)), _f32(t), P, grad, ws)
    g = grad.cpu().numpy().astype(np.float64)
    # element by element, per layer (W then b), against the largest entry of
    # that layer's W or b gradient: FP32 MFMA to FP32 rounding, BF16 operands
    # (2^-8 relative) to a few BF16 units
    tol = 1e-5 if mode == "f32" else 3e-2
    off = 0
    for n_out, n_in in shapes:
        for size in (n_out * n_in, n_out):
            gl, rl = g[off:off + size], g_ref[off:off + size]
            err = np.abs(gl - rl).max() / np.abs(rl).max()
            assert err < tol, (n_out, n_in, size, err)
            off += size
    assert off == len(g_ref)
    if mode == "f32":
        assert abs(loss - loss_ref) < 1e-5 * loss_ref
    else:
        assert abs(loss - loss_ref) < 2e-2 * loss_ref
    y = torch.zeros(P, dtype=torch.float64, device="cuda")
    L.dk_mlp_forward(ctx.h, shape, m, _f32(theta), _f32(u.reshape(-1)), P, y, ws)
    y_ref, _, _ = omlp.forward(theta, shapes, u.astype(np.float64))
    tol = 1e-5 if mode == "f32" else 2e-2
    np.testing.assert_allclose(y.cpu().numpy(), y_ref, rtol=tol, atol=tol * np.abs(y_ref).max())
    ctx.close()


def test_adam_matches_oracle(L, cell):
    ctx = _ctx(cell)
    rng = np.random.default_rng(7)
    n = 1000
    th = rng.standard_normal(n).astype(np.float32).astype(np.float64)
    m = np.zeros(n)
    v = np.zeros(n)
    dth, dm, dv = _f32(th), _f32(m), _f32(v)
    for t in range(1, 4):
        g = (rng.standard_normal(n) * 10.0 ** rng.uniform(-6, 0, n)).astype(np.float32).astype(np.float64)
        th, m, v = omlp.adam_step(th, m, v, g, t)
        L.dk_adam_step(ctx.h, dth, dm, dv, _f32(g), t)
    np.testing.assert_allclose(dth.cpu().numpy(), th, rtol=1e-6, atol=1e-7)
    ctx.close()


def test_predicted_density(L, cell):
    p = cell
    ctx = _ctx(p)
    w = omlp.widths(32, 0.5, 4.0)
    d = torch.empty(p.n_grid * 32, dtype=torch.float32, device="cuda")
    L.dk_descriptors(ctx.h, p.positions, w, d)
    mean = torch.zeros(32, dtype=torch.float64, device="cuda")
    inv = torch.zeros_like(mean)
    L.dk_descriptor_stats(ctx.h, d, p.n_grid, 32, mean, inv)
    shape = L.MlpShape(32, 64, 3)
    shapes = omlp.layer_shapes(32, 64, 3)
    theta = omlp.init_params(shapes, 11).astype(np.float32).astype(np.float64)
    ws = torch.empty(L.dk_mlp_workspace_bytes(shape, 1) // 4 + 64, dtype=torch.float32, device="cuda")
    rho = torch.zeros(p.n_grid, dtype=torch.float64, device="cuda")
    L.dk_mlp_density(ctx.h, shape, L.DK_MLP_F32, _f32(theta), d, mean, inv, p.n_e, rho, ws)
    dd = d.cpu().numpy().reshape(p.n_grid, 32).astype(np.float64)
    u = (dd - mean.cpu().numpy()) * inv.cpu().numpy()
    ref = omlp.density(theta, shapes, u, p.n_e, p.h)
    got = rho.cpu().numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-5)
    assert abs(p.h ** 3 * got.sum() - p.n_e) < 1e-10
    ctx.close()


def test_training_reduces_loss(L, cell):
    from paper_2112_08639_amd.learned import LearnedStart, MlpConfig
    p = cell
    ctx = _ctx(p)
    cfg = MlpConfig(batch=2000, steps=150, lr=3e-3)
    ls = LearnedStart(ctx.h, p.n_grid, p.spec.a ** 3, p.n_e, cfg, max_snapshots=2)
    # target: a smooth function of the atomic environment (the normalised
    # widest descriptor), two snapshots of displaced atoms
    for s in range(2):
        pos = p.positions + 0.3 * np.random.default_rng(s).standard_normal(p.positions.shape)
        d = ls.descriptors(pos)
        rho = d.view(p.n_grid, 32)[:, 31].to(torch.float64).contiguous()
        rho = rho * (p.n_e / (p.h ** 3 * rho.sum()))
        ls.add_snapshot(pos, rho)
    log = ls.fit()
    assert np.mean(log.losses[-10:]) < 0.2 * np.mean(log.losses[:10])
    r0 = ls.predict(p.positions)
    assert abs(p.h ** 3 * r0.sum().item() - p.n_e) < 1e-9
    ctx.close()
