"""Pins of the stress oracle (CPU only).

* Kinetic term: for plane waves on the periodic grid the twelfth-order first
  difference acts by the closed-form symbol kappa(k) = (2/h) sum_p a_p sin(p k h),
  so -2 sum_i int d_a phi_i d_b phi~_i reduces to -2 sum_i D_ii kappa_a kappa_b
  (cross terms between different waves vanish by discrete orthogonality).
* Nonlocal term: under a homogeneous strain F = I + eps that carries atoms and
  grid points along (orbital values scaled by det(F)^(-1/2) so that they stay
  normalised, D fixed), the nonlocal energy becomes
      E_nl(eps) = det(F) 2 sum_p gamma_p sum_ik D_ik c_pi(eps) c_pk(eps),
      c_pi(eps) = h^3 sum_x chi_p(F (x - R - L)) phi_i(x),
  and its derivative at eps = 0 equals |Omega| sigma^III_ab (integrate the
  d_a phi~ term of Eq. stressIIIRe by parts).  The test evaluates E_nl(eps)
  from the projector functions themselves (Gaussians times 1 or x, y, z), not
  from the tables, and differentiates by central differences; the two sides
  differ only by the finite-difference error of d_a on the smooth moments.
  Each l = 1 shell is complete (x, y, z with one gamma), so E_nl is invariant
  under rotations and the tensor is symmetric.
"""

import math

import numpy as np

from oracle import fd
from oracle import stress as ostress
from oracle.hamiltonian import Hamiltonian
from workloads import custom_spec, make_problem
from workloads.cells import PROJ_CHANNELS


def _plane_waves(n, h, ks):
    a = n * h
    g = np.arange(n) * h
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    cols = []
    c = math.sqrt(2.0 / a ** 3)
    for k in ks:
        kv = 2.0 * np.pi * np.asarray(k, dtype=float) / a
        ph = pts @ kv
        cols.append(c * np.cos(ph))
        cols.append(c * np.sin(ph))
    return np.stack(cols, axis=1), [2.0 * np.pi * np.asarray(k, dtype=float) / a for k in ks]


def _kappa(kv, h):
    w = fd.first_derivative_weights()
    return np.array([(2.0 / h) * sum(w[p] * math.sin(p * kc * h) for p in range(1, 7))
                     for kc in kv])


def test_kinetic_stress_plane_waves():
    n, h = 12, 0.55
    ks = [(1, 0, 0), (0, 2, 1), (1, -1, 3), (2, 1, -1), (-3, 2, 2)]
    Phi, kvs = _plane_waves(n, h, ks)
    # orthonormal with the h^3 weight
    np.testing.assert_allclose(h ** 3 * Phi.T @ Phi, np.eye(Phi.shape[1]), atol=1e-12)
    rng = np.random.default_rng(7)
    A = rng.standard_normal((Phi.shape[1], Phi.shape[1]))
    D = 0.5 * (A + A.T)
    got = ostress.kinetic_stress(Phi, D, n, h)
    vol = (n * h) ** 3
    want = np.zeros((3, 3))
    for j, kv in enumerate(kvs):
        kap = _kappa(kv, h)
        want += -2.0 * (D[2 * j, 2 * j] + D[2 * j + 1, 2 * j + 1]) * np.outer(kap, kap)
    want /= vol
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-13 * np.abs(want).max())


def _norm(l, rc):
    a0 = (2.0 / (np.pi * rc * rc)) ** 0.75
    return a0 if l == 0 else a0 * 2.0 / rc


def _e_nl_strained(p, Phi, D, eps):
    """Nonlocal energy with atoms and grid carried by F = I + eps."""
    F = np.eye(3) + eps
    n, h, a = p.n, p.h, p.spec.a
    g = np.arange(n) * h
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    Phit = Phi @ D
    e = 0.0
    for R in p.positions:
        funcs = []
        for (l, rc, gam) in PROJ_CHANNELS:
            nm = _norm(l, rc)
            vals = np.zeros((len(pts), 1 if l == 0 else 3))
            # images beyond one cell from the home cell are more than 7 bohr
            # from every grid point: their Gaussians are below 1e-11
            for L in np.ndindex(3, 3, 3):
                shift = (np.asarray(L) - 1) * a
                d = (pts - R - shift) @ F.T
                gau = nm * np.exp(-np.sum(d * d, axis=1) / (rc * rc))
                if l == 0:
                    vals[:, 0] += gau
                else:
                    vals += gau[:, None] * d
            for m in range(vals.shape[1]):
                funcs.append((gam, vals[:, m]))
        for gam, chi in funcs:
            c = h ** 3 * (chi @ Phi)
            ct = h ** 3 * (chi @ Phit)
            e += 2.0 * gam * np.dot(c, ct)
    return np.linalg.det(F) * e


def test_nonlocal_stress_is_the_strain_derivative():
    spec = custom_spec("stress", 60, 7.6, 1, 24, 6, 1.0, noise=False)
    p = make_problem(spec, with_block=False)
    H = Hamiltonian(p)
    rng = np.random.default_rng(8)
    Phi = rng.standard_normal((p.n_grid, 5))
    A = rng.standard_normal((5, 5))
    D = 0.5 * (A + A.T)
    got = ostress.nonlocal_stress(H, p.proj, Phi, D)
    vol = p.spec.a ** 3
    step = 1e-4
    want = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            e = np.zeros((3, 3))
            e[a, b] = step
            want[a, b] = (_e_nl_strained(p, Phi, D, e) - _e_nl_strained(p, Phi, D, -e)) / (2 * step)
    want /= vol
    scale = np.abs(want).max()
    err = np.abs(got - want).max() / scale
    # measured 6e-6: the twelfth-order difference error on the moments and the
    # 1e-8 cutoff of the tables
    assert err < 2e-5, err
    # the delta_ab term is large against the tolerance (dropping it would fail)
    e_nl = 2.0 * np.sum((H.h ** 3 * (H.chi.T @ (Phi @ D))) * (H.gamma[:, None] * H.projections(Phi)))
    assert abs(e_nl / vol) / scale > 1e-2


def test_xc_stress_is_the_strain_derivative():
    # E_xc(eps) = det F h^3 sum (rho / det F) eps_xc(rho / det F) for a diagonal strain
    from oracle import xc
    n, h = 10, 0.45
    g = np.arange(n) * h * 2 * np.pi / (n * h)
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    rho = (0.02 + 0.015 * np.cos(x) * np.sin(2 * y) + 0.01 * np.cos(z + x) ** 2).ravel()
    got = ostress.xc_stress(rho, n, h)
    vol = (n * h) ** 3

    def e_xc(t):
        det = 1.0 + t
        return det * h ** 3 * float(np.sum((rho / det) * xc.lda(rho / det)[0]))

    step = 1e-5
    d = (e_xc(step) - e_xc(-step)) / (2 * step) / vol
    np.testing.assert_allclose(np.diag(got), d, rtol=1e-8)
    assert np.all(got - np.diag(np.diag(got)) == 0.0)
    assert abs(d) > 1e-4   # the term is not trivially small


def test_electrostatic_stress_is_the_strain_derivative():
    # diagonal strain of the discrete pseudocharge + core energy: grid spacing
    # h (1 + eps), atoms and cell carried along, rho -> rho / det F; the exact
    # derivative uses the Poisson operator's second difference where the
    # stress form has products of first differences, so that difference (an
    # FD-consistency term, 5e-6 of the entries here) is added back
    from oracle import electrostatics as es
    n, a = 16, 6.0
    z, rc, amp, w2 = 3.0, 1.0, 1.5, 0.8
    pos = np.array([[1.1, 2.0, 1.7], [4.0, 3.1, 4.6]])
    x = np.arange(n) * a / n
    zz, yy, xx = np.meshgrid(x, x, x, indexing="ij")
    rho = (0.05 + 0.02 * np.cos(2 * np.pi * xx / a) * np.sin(2 * np.pi * yy / a)
           + 0.01 * np.cos(2 * np.pi * (zz + xx) / a)).ravel()
    rho *= 2 * z / (rho.sum() * (a / n) ** 3)

    def energy(eps):
        F = 1.0 + eps
        h = a / n * F
        xs = [np.arange(n) * h[k] for k in range(3)]

        def field(width2, pref):
            out = np.zeros(n ** 3)
            for p in pos:
                f = [es.periodic_gauss_1d(xs[k], p[k] * F[k], a * F[k], width2) for k in range(3)]
                out += (f[2][:, None, None] * f[1][None, :, None] * f[0][None, None, :]).reshape(-1)
            return pref * out

        b = field(rc * rc, -z * (np.pi * rc * rc) ** -1.5)
        vcore = field(w2, -amp)
        rp = rho / np.prod(F)
        th = 2 * np.pi * np.fft.fftfreq(n)
        sy = [fd.kinetic_symbol(th) / h[k] ** 2 for k in range(3)]
        lam = sy[2][:, None, None] + sy[1][None, :, None] + sy[0][None, None, :]
        fk = np.fft.fftn((rp + b).reshape(n, n, n))
        lam[0, 0, 0] = 1.0
        vk = 4 * np.pi * fk / lam
        vk[0, 0, 0] = 0.0
        V = np.real(np.fft.ifftn(vk)).reshape(-1)
        return 0.5 * np.prod(h) * np.sum((rp + b) * V) + np.prod(h) * np.sum(rp * vcore)

    got = ostress.electrostatic_stress(n, a, pos, z, rc, amp, w2, rho)
    h = a / n
    V = es.poisson_fft(rho + es.pseudocharge(n, a, pos, z, rc), n, a)
    w = fd.second_derivative_weights()
    G = V.reshape(n, n, n)
    step = 1e-5
    for ax in range(3):
        e = np.zeros(3)
        e[ax] = step
        num = (energy(e) - energy(-e)) / (2 * step) / a ** 3
        d2 = w[0] * G
        for k in range(1, 7):
            d2 = d2 + w[k] * (np.roll(G, k, axis=2 - ax) + np.roll(G, -k, axis=2 - ax))
        dv = fd.gradient(V[:, None], n, h, ax)[:, 0]
        fix = h ** 3 * (np.sum(V * (-d2.reshape(-1) / h ** 2)) - np.sum(dv * dv)) / (4 * np.pi) / a ** 3
        assert abs(got[ax, ax] + fix - num) < 1e-9 * abs(num), (ax, got[ax, ax], fix, num)
        assert abs(fix) < 1e-5 * abs(num)


def test_electrostatic_moment_fields_against_image_sums():
    # the separable moments sum_L d_a G(d) d_b against a direct 3-D image sum
    n, a, w2 = 6, 4.0, 0.9
    pos = np.array([[0.3, 3.5, 1.9]])
    x = np.arange(n) * a / n
    zz, yy, xx = np.meshgrid(x, x, x, indexing="ij")
    pts = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    for ax in range(3):
        for bx in range(3):
            want = np.zeros(n ** 3)
            for L in np.ndindex(9, 9, 9):
                d = pts - pos[0] - (np.asarray(L) - 4) * a
                g = np.exp(-np.sum(d * d, axis=1) / w2)
                want += -2.0 * d[:, ax] / w2 * g * d[:, bx]
            got = ostress._moment_field(n, a, pos, w2, ax, bx)
            np.testing.assert_allclose(got, want, atol=1e-13 * np.abs(want).max())
