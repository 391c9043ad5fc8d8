"""CPU checks of the C-ABI library: it builds for gfx950, loads, exports
every function the headers declare, and rejects NULL handles and outputs
before any device call (no compute call without a GPU)."""
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


def _zero_args(argtypes):
    out = []
    for t in argtypes:
        if t in (ctypes.c_double, ctypes.c_float):
            out.append(0.0)
        elif t in (ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t):
            out.append(0)
        elif isinstance(t, type) and issubclass(t, ctypes.Structure):
            out.append(t())
        else:
            out.append(None)
    return out


CREATORS = {"ens_create", "ens_batch_create", "sur_create", "spde_create"}


def test_every_entry_point_rejects_a_null_handle():
    """Error behaviour of the boundary: a NULL context, batch, network or
    sampler is ENS_EINVAL (or a message, for *_last_error) from every entry
    point, with no device call."""
    lib = ensfem.load_library(_lib_path())
    checked = 0
    for name, (res, argtypes) in ensfem._SIGS.items():
        if name in CREATORS or name == "sur_cv_moments":
            continue
        rc = getattr(lib, name)(None, *_zero_args(argtypes[1:]))
        if res is ctypes.c_char_p:
            assert rc and rc.startswith(b"null"), name
        else:
            assert rc == ensfem.ENS_EINVAL, (name, rc)
        checked += 1
    assert checked >= 50


def test_creators_reject_a_null_output_and_missing_devices_are_reported():
    lib = ensfem.load_library(_lib_path())
    assert lib.ens_create(0, None) == ensfem.ENS_EINVAL
    assert lib.ens_batch_create(None, 0, None) == ensfem.ENS_EINVAL
    assert lib.sur_create(0, 0, 0, 0, 0, 0, None) == ensfem.ENS_EINVAL
    assert lib.spde_create(0, None) == ensfem.ENS_EINVAL
    assert lib.sur_cv_moments(None, None, 0, 0, None, None, 0, None, None, None, None) == ensfem.ENS_EINVAL
    h = ctypes.c_void_p()
    rc = lib.ens_create(0, ctypes.byref(h))
    if rc == ensfem.ENS_OK:  # a GPU is present: nothing to report
        assert lib.ens_destroy(h) == ensfem.ENS_OK
    else:
        assert rc == ensfem.ENS_EDEVICE and h.value is None
