"""C-ABI boundary checks that need no GPU.

* libdk.so loads and exports every function include/dk.h declares;
* argument errors are reported on the host before any device work;
* without a GPU, dk_create reports DK_ERR_DEVICE.
"""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dk.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dk_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2112_08639_amd import _lib
    return _lib.load()


def test_header_declares_the_hot_path():
    names = _declared()
    for fn in ["dk_create", "dk_destroy", "dk_filter", "dk_orthonormalize", "dk_project",
               "dk_density_kernel", "dk_density", "dk_energy", "dk_forces",
               "dk_spectral_bounds", "dk_set_potential", "dk_set_projectors",
               "dk_workspace_bytes", "dk_set_workspace"]:
        assert fn in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2112_08639_amd import _lib
    assert set(_declared()) <= set(_lib.EXPORTS)


def test_version_and_status_names(lib):
    assert lib.dk_version() >= 100
    assert lib.dk_status_name(0) == b"DK_OK"
    assert lib.dk_status_name(4) == b"DK_ERR_NOT_SPD"
    assert lib.dk_status_name(99) == b"DK_ERR_UNKNOWN"


def test_create_rejects_bad_grids_on_host(lib):
    h = C.c_void_p()
    # stencil radius 6 needs at least 7 points per axis; checked before any device query
    assert lib.dk_create(C.byref(h), 6, 24, 24, 7.6, 7.6, 7.6, 0, 0, None) == 1
    assert lib.dk_create(C.byref(h), 24, 24, 24, -1.0, 7.6, 7.6, 0, 0, None) == 1
    assert lib.dk_create(C.byref(h), 24, 24, 24, 7.6, 7.6, 7.6, 5, 0, None) == 1
    assert lib.dk_create(None, 24, 24, 24, 7.6, 7.6, 7.6, 0, 0, None) == 1
    assert not h.value


def test_null_context_is_an_argument_error(lib):
    assert lib.dk_filter(None, None, 0, 0, 1, 0.0, 1.0, -1.0) == 1
    assert lib.dk_destroy(None) == 0
    assert lib.dk_last_error(None) == b"null context"


def test_no_device_reports_device_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert lib.dk_create(C.byref(h), 24, 24, 24, 7.6, 7.6, 7.6, 0, 0, None) == 2


def test_new_entry_points_reject_null_context(lib):
    f = C.c_double()
    assert lib.dk_poisson(None, None, None, 1e-10, 10, None, None) == 1
    assert lib.dk_xc(None, None, None, C.byref(f)) == 1
    assert lib.dk_scf_potential(None, None, None, None, 1e-10, 10, None) == 1
    assert lib.dk_pulay_mix(None, None, 0, 7, 0, 0.3, None, None, None, C.byref(f)) == 1
    assert lib.dk_local_forces(None, None, None, None) == 1
    assert lib.dk_verlet_kick(None, 4, None, None, 1.0, 1.0) == 1
    assert lib.dk_adam_step(None, 10, None, None, None, None, 1, 1e-3, 0.9, 0.999, 1e-8) == 1
    assert lib.dk_set_projector_model(None, 1, None, 1, None, None, None, 1e-8) == 1
    assert lib.dk_stress(None, None, 0, 1, None, None, None) == 1
    assert lib.dk_electrostatic_stress(None, None, None, None) == 1
    assert lib.dk_isokinetic_kick(None, 4, None, None, 1.0, 1.0) == 1
    assert lib.dk_kerker_pulay_mix(None, None, 0, 7, 0, 2, 0, 0.3, 1.0, 1e-10, None, None, None,
                                   C.byref(f)) == 1
    assert lib.dk_set_linear_solver(None, 1, 0.6, 0.6, 7, 6) == 1
    assert lib.dk_time_correlation(None, None, 10, 3, 5, 0.1, 1.0, None, None) == 1
    assert lib.dk_deviatoric_stress(None, None, None, 0, 1.0, 4, None) == 1
    assert lib.dk_density_noalloc(None, None, 100, 4, None, None) == 1
    b = C.c_size_t()
    assert lib.dk_kerker_pulay_bytes(None, 7, C.byref(b)) == 1


def test_mlp_shape_queries_match_the_oracle(lib):
    from oracle import mlp as omlp
    from paper_2112_08639_amd import _lib
    for n_in, hidden, layers in [(32, 64, 3), (5, 7, 1), (16, 64, 8)]:
        shape = _lib.MlpShape(n_in, hidden, layers)
        assert _lib.dk_mlp_param_count(shape) == omlp.param_count(
            omlp.layer_shapes(n_in, hidden, layers))
        assert _lib.dk_mlp_workspace_bytes(shape, 1000) > 0
    n = C.c_int64()
    assert lib.dk_mlp_param_count(C.byref(_lib.MlpShape(32, 65, 3)), C.byref(n)) == 1  # > 64 wide
    assert lib.dk_mlp_param_count(C.byref(_lib.MlpShape(32, 64, 9)), C.byref(n)) == 1  # > 8 layers
    b = C.c_size_t()
    assert lib.dk_mlp_workspace_bytes(C.byref(_lib.MlpShape(32, 64, 3)), 0, C.byref(b)) == 1
