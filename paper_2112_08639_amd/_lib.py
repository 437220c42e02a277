"""ctypes binding of libdk (include/dk.h).

Argument marshalling only: every function here forwards to the C entry point
of the same name; device arrays are torch tensors on the context's GPU, whose
data pointers are passed straight through.  The library must be built
(``python -m paper_2112_08639_amd.build``); importing this module fails loudly
otherwise.
"""

from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdk.so")

DK_PREC_FP64 = 0
DK_PREC_MIXED = 1
DK_TAIL_MAX_DEGREE = 256

STATUS = {0: "DK_OK", 1: "DK_ERR_ARG", 2: "DK_ERR_DEVICE", 3: "DK_ERR_ALLOC", 4: "DK_ERR_NOT_SPD",
          5: "DK_ERR_FERMI", 6: "DK_ERR_NONFINITE", 7: "DK_ERR_STATE", 8: "DK_ERR_CONVERGENCE"}


class DkError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class FermiInfo(C.Structure):
    _fields_ = [("mu", C.c_double), ("lam_min", C.c_double), ("lam_max", C.c_double),
                ("chi", C.c_double), ("xi", C.c_double), ("e_band", C.c_double),
                ("e_ent", C.c_double), ("n_count", C.c_double), ("n_pl", C.c_int),
                ("bisect_iters", C.c_int), ("bound_steps", C.c_int), ("reserved", C.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class LocalModel(C.Structure):
    _fields_ = [("z", C.c_double), ("rc", C.c_double), ("core_amp", C.c_double),
                ("core_w2", C.c_double)]


class ScfTerms(C.Structure):
    _fields_ = [("e_xc", C.c_double), ("int_rho_vc", C.c_double), ("int_rho_vxc", C.c_double),
                ("e_es", C.c_double), ("poisson_relres", C.c_double), ("poisson_iters", C.c_int),
                ("reserved", C.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class MlpShape(C.Structure):
    _fields_ = [("n_in", C.c_int), ("hidden", C.c_int), ("n_hidden_layers", C.c_int)]


DK_MLP_BF16 = 0
DK_MLP_F32 = 1

EXPORTS = {
    "dk_version": (C.c_int, []),
    "dk_status_name": (C.c_char_p, [C.c_int]),
    "dk_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.c_int, C.c_int, C.c_double,
                            C.c_double, C.c_double, C.c_int, C.c_int, C.c_void_p]),
    "dk_destroy": (C.c_int, [C.c_void_p]),
    "dk_last_error": (C.c_char_p, [C.c_void_p]),
    "dk_set_potential": (C.c_int, [C.c_void_p, C.c_void_p]),
    "dk_set_projectors": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p]),
    "dk_set_projector_model": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.c_double]),
    "dk_spectrum_upper_bound": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "dk_workspace_bytes": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int,
                                     C.POINTER(C.c_size_t)]),
    "dk_set_workspace": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "dk_apply_h": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int]),
    "dk_filter": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_double,
                            C.c_double, C.c_double]),
    "dk_orthonormalize": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int]),
    "dk_project": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int, C.c_void_p]),
    "dk_spectral_bounds": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.POINTER(C.c_double),
                                     C.POINTER(C.c_double), C.POINTER(C.c_int)]),
    "dk_density_kernel": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_double, C.c_double,
                                    C.c_int, C.c_void_p, C.c_void_p, C.POINTER(FermiInfo)]),
    "dk_density": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int, C.c_void_p,
                             C.c_void_p]),
    "dk_density_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int, C.c_void_p,
                             C.c_void_p]),
    "dk_energy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_double, C.c_double, C.c_double,
                            C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "dk_forces": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int, C.c_void_p, C.c_void_p,
                            C.c_void_p, C.c_int, C.c_void_p]),
    "dk_stress": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int, C.c_void_p, C.c_void_p,
                            C.c_void_p]),
    "dk_electrostatic_stress": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dk_set_atoms": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.POINTER(LocalModel)]),
    "dk_get_local_fields": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "dk_start_density": (C.c_int, [C.c_void_p, C.c_void_p]),
    "dk_poisson": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int,
                             C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "dk_xc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "dk_scf_potential": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                   C.c_int, C.POINTER(ScfTerms)]),
    "dk_pulay_bytes": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_size_t)]),
    "dk_pulay_mix": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_int, C.c_double,
                               C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "dk_kerker_pulay_bytes": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_size_t)]),
    "dk_kerker_pulay_mix": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_int, C.c_int,
                                      C.c_int, C.c_double, C.c_double, C.c_double, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "dk_set_linear_solver": (C.c_int, [C.c_void_p, C.c_int, C.c_double, C.c_double, C.c_int,
                                       C.c_int]),
    "dk_local_forces": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dk_verlet_kick": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_double,
                                 C.c_double]),
    "dk_isokinetic_kick": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_double,
                                     C.c_double]),
    "dk_verlet_drift": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_double]),
    "dk_kinetic_energy": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_double,
                                    C.POINTER(C.c_double)]),
    "dk_mlp_param_count": (C.c_int, [C.POINTER(MlpShape), C.POINTER(C.c_int64)]),
    "dk_mlp_workspace_bytes": (C.c_int, [C.POINTER(MlpShape), C.c_int64, C.POINTER(C.c_size_t)]),
    "dk_descriptors": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "dk_descriptor_stats": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int, C.c_void_p,
                                      C.c_void_p]),
    "dk_mlp_gather": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_int64,
                                C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p]),
    "dk_mlp_loss_grad": (C.c_int, [C.c_void_p, C.POINTER(MlpShape), C.c_int, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                   C.POINTER(C.c_double), C.c_void_p, C.c_size_t]),
    "dk_mlp_forward": (C.c_int, [C.c_void_p, C.POINTER(MlpShape), C.c_int, C.c_void_p, C.c_void_p,
                                 C.c_int64, C.c_void_p, C.c_void_p, C.c_size_t]),
    "dk_adam_step": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_int, C.c_double, C.c_double, C.c_double,
                               C.c_double]),
    "dk_mlp_density": (C.c_int, [C.c_void_p, C.POINTER(MlpShape), C.c_int, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p,
                                 C.c_size_t]),
    "dk_get_timings": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int]),
    "dk_profile_enable": (C.c_int, [C.c_void_p, C.c_int]),
    "dk_profile_read": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "dk_time_correlation": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int, C.c_int,
                                      C.c_double, C.c_double, C.c_void_p, C.c_void_p]),
    "dk_deviatoric_stress": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_double,
                                       C.c_int64, C.c_void_p]),
    "dk_free_energy": (C.c_int, [C.c_void_p, C.POINTER(ScfTerms), C.c_double, C.c_double,
                                 C.POINTER(C.c_double), C.c_void_p]),
}

KERNEL_KINDS = ["stencil", "nl_gather", "nl_scatter", "gram", "project", "cholesky",
                "orth_apply", "bounds", "foe_gemm", "fermi", "density", "forces", "other",
                "poisson", "scf_fields", "mix", "stress"]

_LIB = None


def load() -> C.CDLL:
    """Load libdk.so (built in-tree); raise if it is missing."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not built: run `python -m paper_2112_08639_amd.build`")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(None)


def _check(handle, status: int) -> None:
    if status != 0:
        msg = load().dk_last_error(handle) if handle else b""
        raise DkError(status, (msg or b"").decode())


def _block_args(X):
    """(pointer, ld, n_s) of a (n_s, N_grid) block whose rows are contiguous."""
    assert X.dim() == 2 and X.stride(1) == 1, "block must be (n_s, N_grid) with contiguous rows"
    return _ptr(X), X.stride(0), X.shape[0]


# ---------------------------------------------------------------- entry points

def dk_version() -> int:
    return load().dk_version()


def dk_create(nx, ny, nz, lx, ly, lz, precision=DK_PREC_FP64, device=0, stream=None):
    h = C.c_void_p()
    st = C.c_void_p(stream.cuda_stream if stream is not None else None)
    _check(None, load().dk_create(C.byref(h), nx, ny, nz, lx, ly, lz, precision, device, st))
    return h


def dk_destroy(h) -> None:
    load().dk_destroy(h)


def dk_set_potential(h, veff) -> None:
    assert veff.dtype == torch.float64 and veff.is_contiguous()
    _check(h, load().dk_set_potential(h, _ptr(veff)))


def dk_set_projectors(h, offsets, indices, values, gamma, atom, n_atoms) -> None:
    """Host arrays (numpy): int64 offsets, int32 indices, float64 values/gamma, int32 atom."""
    import numpy as np
    o = np.ascontiguousarray(offsets, dtype=np.int64)
    i = np.ascontiguousarray(indices, dtype=np.int32)
    v = np.ascontiguousarray(values, dtype=np.float64)
    g = np.ascontiguousarray(gamma, dtype=np.float64)
    a = np.ascontiguousarray(atom, dtype=np.int32)
    n_proj = len(g)
    _check(h, load().dk_set_projectors(h, n_proj, n_atoms, o.ctypes.data_as(C.c_void_p),
                                       i.ctypes.data_as(C.c_void_p), v.ctypes.data_as(C.c_void_p),
                                       g.ctypes.data_as(C.c_void_p), a.ctypes.data_as(C.c_void_p)))


def dk_set_projector_model(h, positions, channels, cutoff_rel) -> None:
    """Device-built projector tables.  positions: host (n_atoms, 3) bohr;
    channels: sequence of (l, rc, gamma), the same for every atom."""
    import numpy as np
    pos = np.ascontiguousarray(positions, dtype=np.float64).reshape(-1, 3)
    ch = list(channels)
    ls = np.ascontiguousarray([c[0] for c in ch], dtype=np.int32)
    rc = np.ascontiguousarray([c[1] for c in ch], dtype=np.float64)
    g = np.ascontiguousarray([c[2] for c in ch], dtype=np.float64)
    _check(h, load().dk_set_projector_model(h, len(pos), pos.ctypes.data_as(C.c_void_p), len(ch),
                                            ls.ctypes.data_as(C.c_void_p),
                                            rc.ctypes.data_as(C.c_void_p),
                                            g.ctypes.data_as(C.c_void_p), float(cutoff_rel)))


def dk_spectrum_upper_bound(h) -> float:
    b = C.c_double()
    _check(h, load().dk_spectrum_upper_bound(h, C.byref(b)))
    return b.value


def dk_workspace_bytes(h, n_s, ld, n_pl) -> int:
    b = C.c_size_t()
    _check(h, load().dk_workspace_bytes(h, n_s, ld, n_pl, C.byref(b)))
    return b.value


def dk_set_workspace(h, ws) -> None:
    _check(h, load().dk_set_workspace(h, _ptr(ws), ws.numel() * ws.element_size() if ws is not None else 0))


def dk_apply_h(h, X, Y) -> None:
    px, ld, ns = _block_args(X)
    assert Y.shape == X.shape and Y.stride(0) == ld
    _check(h, load().dk_apply_h(h, px, _ptr(Y), ld, ns))


def dk_filter(h, X, degree, a, b, a0) -> None:
    px, ld, ns = _block_args(X)
    _check(h, load().dk_filter(h, px, ld, ns, degree, a, b, a0))


def dk_orthonormalize(h, X) -> None:
    px, ld, ns = _block_args(X)
    _check(h, load().dk_orthonormalize(h, px, ld, ns))


def dk_project(h, X, Hs) -> None:
    px, ld, ns = _block_args(X)
    assert Hs.dtype == torch.float64 and Hs.numel() == ns * ns and Hs.is_contiguous()
    _check(h, load().dk_project(h, px, ld, ns, _ptr(Hs)))


def dk_spectral_bounds(h, Hs):
    ns = Hs.shape[0]
    lo, hi, it = C.c_double(), C.c_double(), C.c_int()
    _check(h, load().dk_spectral_bounds(h, _ptr(Hs), ns, C.byref(lo), C.byref(hi), C.byref(it)))
    return lo.value, hi.value, it.value


def dk_density_kernel(h, Hs, n_e, sigma, n_pl, Ds, tau=None) -> FermiInfo:
    ns = Hs.shape[0]
    info = FermiInfo()
    _check(h, load().dk_density_kernel(h, _ptr(Hs), ns, float(n_e), float(sigma), int(n_pl),
                                       _ptr(Ds), _ptr(tau), C.byref(info)))
    return info


def dk_density(h, X, Ds, rho) -> None:
    px, ld, ns = _block_args(X)
    _check(h, load().dk_density(h, px, ld, ns, _ptr(Ds), _ptr(rho)))


def dk_density_noalloc(h, X, Ds, rho) -> None:
    px, ld, ns = _block_args(X)
    _check(h, load().dk_density_noalloc(h, px, ld, ns, _ptr(Ds), _ptr(rho)))


def dk_energy(h, tau, n_pl, mu, chi, xi, sigma):
    eb, ee = C.c_double(), C.c_double()
    _check(h, load().dk_energy(h, _ptr(tau), n_pl, mu, chi, xi, sigma, C.byref(eb), C.byref(ee)))
    return eb.value, ee.value


def dk_forces(h, X, Ds, rho, gradv, n_atoms):
    import numpy as np
    px, ld, ns = _block_args(X)
    f = np.zeros(3 * n_atoms)
    _check(h, load().dk_forces(h, px, ld, ns, _ptr(Ds), _ptr(rho), _ptr(gradv), n_atoms,
                               f.ctypes.data_as(C.c_void_p)))
    return f.reshape(n_atoms, 3)


def dk_stress(h, X, Ds):
    """Kinetic and nonlocal stress terms, each a 3 x 3 host array (Ha/bohr^3)."""
    import numpy as np
    px, ld, ns = _block_args(X)
    kin = np.zeros(9)
    nl = np.zeros(9)
    _check(h, load().dk_stress(h, px, ld, ns, _ptr(Ds), kin.ctypes.data_as(C.c_void_p),
                               nl.ctypes.data_as(C.c_void_p)))
    return kin.reshape(3, 3), nl.reshape(3, 3)


def dk_electrostatic_stress(h, rho, vc):
    """Electrostatic stress terms, a 3 x 3 host array (Ha/bohr^3)."""
    import numpy as np
    sig = np.zeros(9)
    _check(h, load().dk_electrostatic_stress(h, _f64(rho, "rho"), _f64(vc, "vc"),
                                             sig.ctypes.data_as(C.c_void_p)))
    return sig.reshape(3, 3)


def _f64(t, name):
    assert t.dtype == torch.float64 and t.is_contiguous(), f"{name} must be contiguous float64"
    return _ptr(t)


def dk_set_atoms(h, positions, z, rc, core_amp, core_w2) -> None:
    import numpy as np
    pos = np.ascontiguousarray(positions, dtype=np.float64).reshape(-1, 3)
    m = LocalModel(z, rc, core_amp, core_w2)
    _check(h, load().dk_set_atoms(h, len(pos), pos.ctypes.data_as(C.c_void_p), C.byref(m)))


def dk_get_local_fields(h, b=None, vcore=None) -> None:
    _check(h, load().dk_get_local_fields(h, _ptr(b), _ptr(vcore)))


def dk_start_density(h, rho) -> None:
    _check(h, load().dk_start_density(h, _f64(rho, "rho")))


def dk_poisson(h, src, v, tol=1e-10, max_iter=5000):
    it, rr = C.c_int(), C.c_double()
    _check(h, load().dk_poisson(h, _f64(src, "src"), _f64(v, "v"), tol, max_iter, C.byref(it),
                                C.byref(rr)))
    return it.value, rr.value


def dk_xc(h, rho, vxc) -> float:
    e = C.c_double()
    _check(h, load().dk_xc(h, _f64(rho, "rho"), _f64(vxc, "vxc"), C.byref(e)))
    return e.value


def dk_scf_potential(h, rho, vc, veff, tol=1e-10, max_iter=5000) -> ScfTerms:
    t = ScfTerms()
    _check(h, load().dk_scf_potential(h, _f64(rho, "rho"), _f64(vc, "vc"), _f64(veff, "veff"),
                                      tol, max_iter, C.byref(t)))
    return t


def dk_pulay_bytes(h, history) -> int:
    b = C.c_size_t()
    _check(h, load().dk_pulay_bytes(h, history, C.byref(b)))
    return b.value


def dk_pulay_mix(h, state, history, it, beta, rho_in, rho_out, rho_next) -> float:
    r = C.c_double()
    _check(h, load().dk_pulay_mix(h, _ptr(state), state.numel() * state.element_size(), history,
                                  it, beta, _f64(rho_in, "in"), _f64(rho_out, "out"),
                                  _f64(rho_next, "next"), C.byref(r)))
    return r.value


def dk_kerker_pulay_bytes(h, history) -> int:
    b = C.c_size_t()
    _check(h, load().dk_kerker_pulay_bytes(h, history, C.byref(b)))
    return b.value


DK_SOLVER_CG = 0
DK_SOLVER_AAR = 1


def dk_set_linear_solver(h, solver, omega=0.6, beta=0.6, history=7, period=6) -> None:
    _check(h, load().dk_set_linear_solver(h, solver, omega, beta, history, period))


def dk_kerker_pulay_mix(h, state, history, it, period, beta, k0, tol, rho_in, rho_out,
                        rho_next, restart=False) -> float:
    r = C.c_double()
    _check(h, load().dk_kerker_pulay_mix(h, _ptr(state), state.numel() * state.element_size(),
                                         history, it, period, 1 if restart else 0, beta, k0, tol,
                                         _f64(rho_in, "in"), _f64(rho_out, "out"),
                                         _f64(rho_next, "next"), C.byref(r)))
    return r.value


def dk_local_forces(h, rho, vc, n_atoms):
    import numpy as np
    f = np.zeros(3 * n_atoms)
    _check(h, load().dk_local_forces(h, _f64(rho, "rho"), _f64(vc, "vc"),
                                     f.ctypes.data_as(C.c_void_p)))
    return f.reshape(n_atoms, 3)


def _f32(t, name):
    assert t.dtype == torch.float32 and t.is_contiguous(), f"{name} must be contiguous float32"
    return _ptr(t)


def _nbytes(t):
    return t.numel() * t.element_size()


def dk_verlet_kick(h, v, f, half_dt, mass) -> None:
    _check(h, load().dk_verlet_kick(h, v.numel() // 3, _f64(v, "v"), _f64(f, "f"), half_dt, mass))


def dk_isokinetic_kick(h, v, f, tau, mass) -> None:
    _check(h, load().dk_isokinetic_kick(h, v.numel() // 3, _f64(v, "v"), _f64(f, "f"), tau, mass))


def dk_verlet_drift(h, x, v, dt) -> None:
    _check(h, load().dk_verlet_drift(h, x.numel() // 3, _f64(x, "x"), _f64(v, "v"), dt))


def dk_kinetic_energy(h, v, mass) -> float:
    e = C.c_double()
    _check(h, load().dk_kinetic_energy(h, v.numel() // 3, _f64(v, "v"), mass, C.byref(e)))
    return e.value


def dk_mlp_param_count(shape: MlpShape) -> int:
    n = C.c_int64()
    _check(None, load().dk_mlp_param_count(C.byref(shape), C.byref(n)))
    return n.value


def dk_mlp_workspace_bytes(shape: MlpShape, n_points: int) -> int:
    b = C.c_size_t()
    _check(None, load().dk_mlp_workspace_bytes(C.byref(shape), n_points, C.byref(b)))
    return b.value


def dk_descriptors(h, positions, widths, desc) -> None:
    import numpy as np
    pos = np.ascontiguousarray(positions, dtype=np.float64).reshape(-1, 3)
    w = np.ascontiguousarray(widths, dtype=np.float64)
    _check(h, load().dk_descriptors(h, len(pos), pos.ctypes.data_as(C.c_void_p), len(w),
                                    w.ctypes.data_as(C.c_void_p), _f32(desc, "desc")))


def dk_descriptor_stats(h, desc, n_points, n_w, mean, inv_std) -> None:
    _check(h, load().dk_descriptor_stats(h, _f32(desc, "desc"), n_points, n_w, _f64(mean, "mean"),
                                         _f64(inv_std, "inv_std")))


def dk_mlp_gather(h, desc, rho, n_w, idx, n_pts, mean, inv_std, scale, u, t) -> None:
    if idx is not None:
        assert idx.dtype == torch.int64 and idx.is_contiguous()
    _check(h, load().dk_mlp_gather(h, _f32(desc, "desc"), _ptr(rho), n_w, _ptr(idx), n_pts,
                                   _f64(mean, "mean"), _f64(inv_std, "inv_std"), scale,
                                   _f32(u, "u"), _ptr(t)))


def dk_mlp_loss_grad(h, shape, mode, params, u, t, n_pts, grad, ws) -> float:
    loss = C.c_double()
    _check(h, load().dk_mlp_loss_grad(h, C.byref(shape), mode, _f32(params, "params"), _f32(u, "u"),
                                      _f32(t, "t"), n_pts, _ptr(grad), C.byref(loss), _ptr(ws),
                                      _nbytes(ws)))
    return loss.value


def dk_mlp_forward(h, shape, mode, params, u, n_pts, y, ws) -> None:
    _check(h, load().dk_mlp_forward(h, C.byref(shape), mode, _f32(params, "params"), _f32(u, "u"),
                                    n_pts, _f64(y, "y"), _ptr(ws), _nbytes(ws)))


def dk_adam_step(h, params, m, v, grad, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8) -> None:
    _check(h, load().dk_adam_step(h, params.numel(), _f32(params, "params"), _f32(m, "m"),
                                  _f32(v, "v"), _f32(grad, "grad"), t, lr, b1, b2, eps))


def dk_mlp_density(h, shape, mode, params, desc, mean, inv_std, n_e, rho, ws) -> None:
    _check(h, load().dk_mlp_density(h, C.byref(shape), mode, _f32(params, "params"),
                                    _f32(desc, "desc"), _f64(mean, "mean"),
                                    _f64(inv_std, "inv_std"), n_e, _f64(rho, "rho"), _ptr(ws),
                                    _nbytes(ws)))


def dk_get_timings(h):
    arr = (C.c_double * 8)()
    _check(h, load().dk_get_timings(h, arr, 8))
    return list(arr)


def dk_profile_enable(h, on=True) -> None:
    _check(h, load().dk_profile_enable(h, 1 if on else 0))


def dk_profile_read(h):
    """{kind: (total_ms, launches)} for every kernel kind with launches."""
    ms = (C.c_double * len(KERNEL_KINDS))()
    cnt = (C.c_int64 * len(KERNEL_KINDS))()
    _check(h, load().dk_profile_read(h, ms, cnt))
    return {KERNEL_KINDS[i]: (ms[i], cnt[i]) for i in range(len(KERNEL_KINDS)) if cnt[i] > 0}


def dk_time_correlation(h, series, max_lag, dt=0.0, scale=1.0, corr=None, integral=None):
    """series: device FP64 (T, n_comp).  Returns (corr, integral) device tensors."""
    T, n = series.shape
    assert series.dtype == torch.float64 and series.is_contiguous()
    if corr is None:
        corr = torch.zeros(max_lag, dtype=torch.float64, device=series.device)
    _check(h, load().dk_time_correlation(h, _ptr(series), T, n, max_lag, dt, scale, _ptr(corr),
                                         _ptr(integral)))
    return corr, integral


def dk_deviatoric_stress(h, sigma, v=None, mass=0.0):
    """sigma: device FP64 (T, 3, 3); v: device FP64 (T, N, 3) or None.  Returns (T, 5)."""
    T = sigma.shape[0]
    assert sigma.dtype == torch.float64 and sigma.is_contiguous()
    n_atoms = 0
    if v is not None:
        assert v.dtype == torch.float64 and v.is_contiguous() and v.shape[0] == T
        n_atoms = v.shape[1]
    s = torch.zeros((T, 5), dtype=torch.float64, device=sigma.device)
    _check(h, load().dk_deviatoric_stress(h, _ptr(sigma), _ptr(v), n_atoms, mass, T, _ptr(s)))
    return s


def dk_free_energy(h, terms, e_band, e_ent, xc_stress=False):
    """Harris-Foulkes free energy from dk_scf_potential's terms; with xc_stress
    also the exchange-correlation stress term (3 x 3 host array)."""
    import numpy as np
    F = C.c_double()
    st = np.zeros(9) if xc_stress else None
    _check(h, load().dk_free_energy(h, C.byref(terms), e_band, e_ent, C.byref(F),
                                    st.ctypes.data_as(C.c_void_p) if xc_stress else None))
    return (F.value, st.reshape(3, 3)) if xc_stress else F.value
