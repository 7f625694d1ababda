"""Host-only checks of the C ABI: the library loads, exports every function that
include/tensornet.h declares, and rejects bad requests before touching a GPU."""

import ctypes
import os
import re

import pytest

from paper_2402_17660_amd import _lib as L
from synth import make_weights, write_blob

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(tn_[a-z_0-9]+)\s*\(", src))
    return names


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("tn_model_create", "tn_build_neighbors", "tn_energy", "tn_energy_forces"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    names = declared_functions()
    assert names, "no declarations found"
    for name in names:
        assert hasattr(lib, name), name
        assert name in L.PROTOTYPES, f"binding lacks a prototype for {name}"


def test_status_strings():
    assert L.status_string(0) == "ok"
    assert "blob" in L.status_string(L.TN_E_BLOB)
    assert "box" in L.status_string(L.TN_E_BOX)


def test_blob_rejected_on_host():
    lib = L.lib()
    blob = write_blob(make_weights(16, 8, 1, 100, seed=0), 16, 8, 1, 100, 4.5)
    h = ctypes.c_void_p()
    bad = b"XXXXXXXX" + blob[8:]
    buf = ctypes.create_string_buffer(bad, len(bad))
    assert lib.tn_model_create(ctypes.cast(buf, ctypes.c_void_p), len(bad), 0, ctypes.byref(h)) == L.TN_E_BLOB
    buf = ctypes.create_string_buffer(blob, len(blob))
    assert lib.tn_model_create(ctypes.cast(buf, ctypes.c_void_p), len(blob) - 8, 0, ctypes.byref(h)) == L.TN_E_BLOB
    assert lib.tn_model_create(None, 0, 0, ctypes.byref(h)) == L.TN_E_ARG


def test_box_validation_on_host():
    lib = L.lib()
    small = (ctypes.c_double * 9)(8.0, 0, 0, 0, 8.0, 0, 0, 0, 8.0)
    tilted = (ctypes.c_double * 9)(20.0, 1.0, 0, 0, 20.0, 0, 0, 0, 20.0)      # not lower triangular
    unreduced = (ctypes.c_double * 9)(20.0, 0, 0, 12.0, 20.0, 0, 0, 0, 20.0)  # |b_x| > a_x / 2
    flat = (ctypes.c_double * 9)(20.0, 0, 0, 0, 20.0, 0, 10.0, 10.0, 8.5)     # height c_z < 2 r_c
    triclinic = (ctypes.c_double * 9)(20.0, 0, 0, 5.0, 19.0, 0, -4.0, 6.0, 18.0)
    ok = (ctypes.c_double * 9)(20.0, 0, 0, 0, 20.0, 0, 0, 0, 20.0)
    cast = lambda a: ctypes.cast(a, ctypes.c_void_p)
    assert lib.tn_neighbor_workspace_bytes(100, 1000, cast(small), 4.5) == 0
    assert lib.tn_neighbor_workspace_bytes(100, 1000, cast(tilted), 4.5) == 0
    assert lib.tn_neighbor_workspace_bytes(100, 1000, cast(unreduced), 4.5) == 0
    assert lib.tn_neighbor_workspace_bytes(100, 1000, cast(flat), 4.5) == 0
    assert lib.tn_neighbor_workspace_bytes(100, 1000, cast(triclinic), 4.5) > 0
    assert lib.tn_neighbor_workspace_bytes(100, 1000, cast(ok), 4.5) > 0
    assert lib.tn_neighbor_workspace_bytes(100, 1000, None, 4.5) > 0
    one = ctypes.c_void_p(1)   # never dereferenced: the call fails validation first
    rc = lib.tn_build_neighbors(None, 10, one, 0, one, cast(small), 4.5, 100, one, one, one, one, 1 << 20)
    assert rc == L.TN_E_BOX
    rc = lib.tn_build_neighbors(None, 10, one, 0, one, cast(tilted), 4.5, 100, one, one, one, one, 1 << 20)
    assert rc == L.TN_E_ARG
    rc = lib.tn_build_neighbors(None, 10, one, 0, one, cast(unreduced), 4.5, 100, one, one, one, one, 1 << 20)
    assert rc == L.TN_E_ARG
    rc = lib.tn_build_neighbors(None, 10, one, 0, one, cast(flat), 4.5, 100, one, one, one, one, 1 << 20)
    assert rc == L.TN_E_BOX
    rc = lib.tn_build_neighbors(None, 10, one, 0, one, cast(ok), 4.5, 100, one, one, one, one, 16)
    assert rc == L.TN_E_WORKSPACE


def test_neighbor_method_validation_on_host():
    lib = L.lib()
    ok = (ctypes.c_double * 9)(20.0, 0, 0, 0, 20.0, 0, 0, 0, 20.0)
    cast = lambda a: ctypes.cast(a, ctypes.c_void_p)
    one = ctypes.c_void_p(1)   # never dereferenced: the call fails validation first
    args = (None, 10, one, 0, one)
    rc = lib.tn_build_neighbors_method(*args, cast(ok), 4.5, 100, one, one, one, one, 1 << 20, 7)
    assert rc == L.TN_E_ARG
    rc = lib.tn_build_neighbors_method(*args, None, 4.5, 100, one, one, one, one, 1 << 20, L.TN_NBR_CELL)
    assert rc == L.TN_E_UNSUPPORTED
    # the brute force in a box still validates the box and the workspace
    small = (ctypes.c_double * 9)(8.0, 0, 0, 0, 8.0, 0, 0, 0, 8.0)
    rc = lib.tn_build_neighbors_method(*args, cast(small), 4.5, 100, one, one, one, one, 1 << 20, L.TN_NBR_BRUTE)
    assert rc == L.TN_E_BOX
    rc = lib.tn_build_neighbors_method(*args, cast(ok), 4.5, 100, one, one, one, one, 16, L.TN_NBR_BRUTE)
    assert rc == L.TN_E_WORKSPACE


def test_pair_variant_queries_on_host():
    lib = L.lib()
    assert lib.tn_pair_variant_count(L.TN_FP32) >= 2
    assert lib.tn_pair_variant_count(L.TN_BF16) >= 2
    assert lib.tn_pair_variant_count(L.TN_FP64) == 0
    assert lib.tn_model_set_pair_variant(None, L.TN_FP32, 0, 0) == L.TN_E_ARG


def test_training_entry_points_reject_bad_requests_on_host():
    lib = L.lib()
    assert lib.tn_param_count(None) == -1
    assert lib.tn_train_workspace_bytes(None, 10, 1, 100, None, L.TN_FP64) == 0
    one = ctypes.c_void_p(1)   # never dereferenced: every call below fails its argument checks first
    head = (None, None, 10, 1, one, one, one, None, 100)
    tail = (one, one, 1.0, 1.0, one, one, one, one, one, one, one, 1 << 20)
    assert lib.tn_train_grad(*head, L.TN_FP64, *tail) == L.TN_E_ARG   # null model
    assert lib.tn_train_grad(one, None, -1, 1, one, one, one, None, 100, L.TN_FP64, *tail) == L.TN_E_ARG
    assert lib.tn_train_grad(one, None, 10, 1, one, one, one, None, 100, L.TN_BF16, *tail) == L.TN_E_UNSUPPORTED
    no_ref = (one, None, 1.0, 1.0, one, one, one, one, one, one, one, 1 << 20)
    assert lib.tn_train_grad(one, None, 10, 1, one, one, one, None, 100, L.TN_FP64, *no_ref) == L.TN_E_ARG
    bad_w = (one, one, float("nan"), 1.0, one, one, one, one, one, one, one, 1 << 20)
    assert lib.tn_train_grad(one, None, 10, 1, one, one, one, None, 100, L.TN_FP64, *bad_w) == L.TN_E_ARG
    too_many = (1 << 30) + 1   # pair budgets above 2^30 are refused, as for tn_energy_forces
    assert lib.tn_train_grad(one, None, 10, 1, one, one, one, None, too_many, L.TN_FP64, *tail) == L.TN_E_ARG
