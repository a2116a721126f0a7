"""The C-ABI library loads, exports every declared entry point and rejects
bad arguments before touching the device (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2503_12557_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    return binding, binding.load()


def test_header_declarations_are_exported():
    binding, lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "pepsmin.h")).read()
    declared = set(re.findall(r"^\s*(?:peps_status|void|const char\*|size_t)\s+(\w+)\(", hdr, re.M))
    assert declared == set(binding.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_create_rejects_bad_geometry():
    binding, lib = _lib()
    h = ctypes.c_void_p()
    for g, code in [((1, 4, 2, 2, 2, 0), 1), ((4, 4, 3, 2, 2, 0), 2), ((4, 4, 2, 0, 2, 0), 1),
                    ((4, 4, 2, 2, 2, 9), 1), ((4, 4, 2, 8, 64, 0), 2), ((40, 4, 2, 2, 2, 0), 1),
                    ((4, 4, 2, 6, 48, 4), 2), ((4, 4, 2, 2, 2, -1), 1)]:
        geom = binding.Geom(*g)
        st = lib.peps_create(ctypes.byref(geom), ctypes.byref(h))
        assert st == code, (g, st, lib.peps_last_error())
        assert lib.peps_last_error()
    assert lib.peps_create(None, ctypes.byref(h)) == 1


def test_null_context_is_rejected():
    binding, lib = _lib()
    assert lib.peps_set_hamiltonian(None, 0, None, None, None, 0, None, None, None) == 1
    assert lib.minsr_step(None, None, None, 4, None, 1e-4, 1e-12, None, None, None) == 1
    assert lib.peps_amplitude(None, None, None, 1, None, None, None, None) == 1
    assert lib.peps_num_params(None) == 0
    assert lib.peps_env_cache_bytes(None, 4) == 0
    assert lib.peps_local_energy_strict(None, None, None, 1, None, None, None) == 1
    assert lib.peps_set_truncation(None, 1e-4) == 1
    assert lib.peps_direct_sample(None, None, 4, 4, 1, 1, 0, None, None, None, None, None) == 1
    assert lib.peps_vmc_step(None, None, 0, 1, 1, 0, 1, 1, 0, 0.1, 1e-4, 1e-12, None, None,
                             None, None, None) == 1


def test_null_arguments_of_the_newer_entry_points():
    binding, lib = _lib()
    assert lib.peps_set_compression(None, 1) == 1
    assert lib.peps_set_minsr_solver(None, 1) == 1
    assert lib.minsr_step_noalloc(None, None, None, 4, None, 1e-4, 1e-12, None, None, None) == 1
    assert lib.peps_sample(None, None, 2, 4, 1, 0, 1, 0, 0, None, None, None, None, None) == 1
    assert lib.made_train(None, None, None, 8, 1, 4, 0, 1e-3, 0.9, 0.999, 1e-8, 0, None, None,
                          None, None) == 1
    assert lib.peps_tau_int(None, 4, 8, 0, 5.0, None, None, None) == 1
    assert lib.peps_rotate_basis(None, None, 1, None, None) == 1
    assert lib.peps_energy_diag(None, None, 4, None, None) == 1
