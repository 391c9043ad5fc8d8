"""CPU checks of the C-ABI library: it builds for gfx950, loads, and exports
every function include/ensfem.h declares (no compute call without a GPU)."""
import ctypes
import os

import pytest

from paper_2101_09059_amd import ensfem


def _lib_path():
    if not os.path.exists(ensfem.LIB_PATH):
        from paper_2101_09059_amd import build
        build.build()
    return ensfem.LIB_PATH


def test_header_lists_the_boundary():
    names = ensfem.header_functions()
    for f in ("ens_create", "ens_set_mesh", "ens_set_ensemble", "ens_step", "ens_read_qoi",
              "ens_apply", "ens_moments", "ens_save", "ens_load"):
        assert f in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    missing = [n for n in ensfem.header_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares a signature for every exported function
    assert set(ensfem.header_functions()) <= set(ensfem._SIGS)


def test_null_context_is_rejected_without_a_gpu():
    lib = ensfem.load_library(_lib_path())
    assert lib.ens_destroy(None) == ensfem.ENS_EINVAL
    assert lib.ens_set_material(None, 0.3, 1.0, 1.0, 0.0) == ensfem.ENS_EINVAL
    assert lib.ens_last_error(None) == b"null context"
