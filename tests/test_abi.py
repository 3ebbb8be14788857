"""Host-side checks of the C-ABI library: it loads without a GPU, exports
every function include/kf.h declares, and rejects bad arguments before any
device work."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kf.h")
LIB = os.path.join(ROOT, "paper_1906_02253_amd", "libkfmi.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(kf_[a-z0-9_]+)\s*\(", text, re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libkfmi.so is not built: run __graft_entry__.build()")
    return C.CDLL(LIB)


def test_header_declares_core_entry_points():
    names = declared_functions()
    for f in ("kf_create", "kf_destroy", "kf_propagate", "kf_fit", "kf_seed"):
        assert f in names


def test_every_declared_symbol_is_exported(lib):
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_argument_validation_without_device(lib):
    lib.kf_create.restype = C.c_int
    lib.kf_create.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]
    assert lib.kf_create(None, None, 0, None) == -1
    out = C.c_void_p()
    assert lib.kf_create(C.byref(out), None, 3, None) == -1
    lib.kf_last_error_global.restype = C.c_char_p
    assert b"layers" in lib.kf_last_error_global()
    lib.kf_fit.restype = C.c_int
    lib.kf_fit.argtypes = [C.c_void_p] * 6 + [C.c_int, C.c_void_p]
    assert lib.kf_fit(None, None, None, None, None, 0, 0, None) == -1


def test_batched_and_autotune_validation_without_device(lib):
    """The graph and autotuning entry points reject a null context before any
    device work."""
    for f, n in (("kf_find_batched", 13), ("kf_autotune", 13), ("kf_clean_seeds", 8),
                 ("kf_remove_duplicates", 7), ("kf_find_noalloc", 12)):
        fn = getattr(lib, f)
        fn.restype = C.c_int
        fn.argtypes = [C.c_void_p] * n
        assert fn(*([None] * n)) == -1, f
    lib.kf_get_find_config.restype = C.c_int
    lib.kf_get_find_config.argtypes = [C.c_void_p] * 3
    assert lib.kf_get_find_config(None, None, None) == -1
    lib.kf_timings.restype = C.c_int
    lib.kf_timings.argtypes = [C.c_void_p] * 2
    assert lib.kf_timings(None, None) == -1


def test_mlp_entry_points_validate_without_device(lib):
    for f, n in (("kf_mlp_load", 2), ("kf_mlp_get", 2), ("kf_mlp_features", 6),
                 ("kf_mlp_forward", 6), ("kf_mlp_grad", 10), ("kf_mlp_train", 11),
                 ("kf_mlp_targets", 7)):
        fn = getattr(lib, f)
        fn.restype = C.c_int
        fn.argtypes = [C.c_void_p] * n
        assert fn(*([None] * n)) == -1, f


def test_cleaning_thresholds_validated_without_device(lib):
    """kf_create rejects seed-cleaning thresholds wider than a seed cell (or
    negative) before touching the device."""
    from paper_1906_02253_amd.binding import KfLayer, KfParams
    lib.kf_create.restype = C.c_int
    lib.kf_create.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]
    lay = (KfLayer * 1)()
    lay[0] = KfLayer(0, 128, 32, 0, 10.0, -20.0, 20.0, 0.0, 0.01, 0.05)
    for bad in (dict(clean_deta=0.1), dict(clean_dphi=0.1), dict(clean_dc=-1.0),
                dict(clean_deta=-0.01)):
        kw = dict(clean_deta=0.01, clean_dphi=0.01, clean_dc=0.05)
        kw.update(bad)
        prm = KfParams(3.8, 30.0, 1e-4, 0.13957, 6, 10, 2, 3, 0.0, 2.0, kw["clean_deta"],
                       kw["clean_dphi"], kw["clean_dc"], 0.5)
        out = C.c_void_p()
        assert lib.kf_create(C.byref(out), lay, 1, C.byref(prm)) == -1, bad


def test_steering_material_entry_points_validate_without_device(lib):
    """kf_set_steering and kf_set_material reject a null context before any
    device work."""
    for f, n in (("kf_set_steering", 3), ("kf_set_material", 2)):
        fn = getattr(lib, f)
        fn.restype = C.c_int
        fn.argtypes = [C.c_void_p] * n
        assert fn(*([None] * n)) == -1, f
