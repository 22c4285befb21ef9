"""The C ABI library loads and exports every symbol include/octrack.h
declares; host-side argument checks answer without touching a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "octrack.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ot_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def ot():
    import paper_2605_20565_amd as m
    return m


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("ot_build_tree", "ot_locate", "ot_interpolate", "ot_spread", "ot_track", "ot_grad_pos",
              "ot_interp_grad_pos", "ot_spread_grad_pos", "ot_spread_workspace_bytes",
              "ot_batch_plan_create", "ot_batch_run", "ot_destroy_tree", "ot_strerror", "ot_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(ot):
    out = subprocess.run(["nm", "-D", "--defined-only", ot.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (ot_[a-z_]+)\b", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    for n in _declared():
        assert hasattr(ot.lib, n)


def test_strerror_and_host_side_validation(ot):
    L = ot.lib
    assert L.ot_strerror(0) == b"success"
    assert L.ot_strerror(-2) == b"leaves do not tile the unit cube"
    h = ctypes.c_void_p()
    desc = ot.TreeDesc(1, 3, 1)
    assert L.ot_build_tree(None, None, 10, ctypes.byref(desc), None, None, ctypes.byref(h)) == -1
    assert b"bad arguments" in L.ot_last_error()
    # level range and capacity are checked before any device work
    dummy = ctypes.c_void_p(0x1000)
    bad = ot.TreeDesc(1, 22, 1)
    assert L.ot_build_tree(dummy, dummy, 10, ctypes.byref(bad), None, None, ctypes.byref(h)) == -4
    assert L.ot_build_tree(dummy, dummy, (1 << 26) + 1, ctypes.byref(desc), None, None, ctypes.byref(h)) == -7
    assert L.ot_locate(None, dummy, 0, 10, dummy, None) == -1
    assert L.ot_encode_keys(None, 0, 30, None, None) == -4
    assert L.ot_encode_keys(None, 0, 5, None, None) == 0
    off = (ctypes.c_int64 * 2)(0, 5)
    ops = (ctypes.c_int32 * 1)(7)
    assert L.ot_batch_plan_create(None, off, ops, 1, 0, 0, None, ctypes.byref(h)) == -1


def test_mdf_host_side_validation(ot):
    L = ot.lib
    assert L.ot_mdf_workspace_bytes(None, 10, 0) == -1
    assert L.ot_mdf(None, None, None, None, 0, 10, 3, 1.0, 1.0, 1, None, None, None, None) == -1
    assert b"tree is NULL" in L.ot_last_error()


def test_body_sums_host_side_validation(ot):
    L = ot.lib
    assert L.ot_body_sums(None, None, 10, None, 2, None, None, 1.0, 0, 1, None, None, None) == -1
    assert L.ot_body_sums(None, None, 10, None, 0, None, None, 1.0, 0, 1, None, None, None) == 0
    assert L.ot_body_sums(None, None, -1, None, 1, None, None, 1.0, 0, 1, None, None, None) == -1


def test_migration_host_side_validation(ot):
    L = ot.lib
    assert L.ot_relocate(None, None, 0, 5, None, None, None) == -1
    assert L.ot_leaf_splitters(None, 4, None, None) == -1
    assert L.ot_find_owner(None, 0, 5, 1, None, 0, 10, None, None, None) == -1
    assert L.ot_find_owner(None, 4, 22, 1, None, 0, 10, None, None, None) == -4


def test_particle_step_host_side_validation(ot):
    L = ot.lib
    assert L.ot_particle_step(None, None, None, None, None, None, None, 0, 1, None, None) == -1
    dummy = ctypes.c_void_p(0x1000)
    args = [dummy] * 8
    assert L.ot_particle_sort(None, 0, 10, *args, None, None, None, None) == -1
    assert b"tree is NULL" in L.ot_last_error()
    assert L.ot_particle_sort(dummy, 0, -1, *args, None, None, None, None) == -1
    assert L.ot_particle_sort(dummy, 0, 10, *args, None, None, ctypes.c_void_p(0x1001), None) == -1
    assert b"256-byte aligned" in L.ot_last_error()
    assert L.ot_particle_sort(dummy, 0, 10, None, *args[1:], None, None, None, None) == -1
    assert L.ot_particle_sort_workspace_bytes(1000) >= 1000 * 24
    # an output that is also an input (or another output) is refused
    d2 = [ctypes.c_void_p(0x1000 + 0x100 * i) for i in range(8)]
    assert L.ot_particle_sort(dummy, 0, 10, *d2[:4], d2[0], *d2[5:], None, None, None, None) == -1
    assert b"distinct" in L.ot_last_error()
    assert L.ot_particle_sort(dummy, 0, 10, *d2[:4], d2[4], d2[4], *d2[6:], None, None, None, None) == -1


def test_backward_host_side_validation(ot):
    L = ot.lib
    dummy = ctypes.c_void_p(0x1000)
    # both outputs NULL: nothing to compute
    assert L.ot_interp_backward(dummy, dummy, dummy, dummy, None, 0, 10, 1, 0, None, None, None, None) == -1
    assert b"both outputs are NULL" in L.ot_last_error()
    assert L.ot_spread_backward(dummy, dummy, dummy, dummy, None, 0, 10, None, None, None) == -1
    # no tree
    assert L.ot_interp_backward(None, dummy, dummy, dummy, None, 0, 10, 1, 0, dummy, dummy, None, None) == -1
    assert b"tree is NULL" in L.ot_last_error()
    assert L.ot_spread_backward(None, dummy, dummy, dummy, None, 0, 10, dummy, None, None) == -1
    # no points: nothing per point to compute, whatever the outputs
    assert L.ot_spread_backward(dummy, dummy, dummy, None, None, 0, 0, None, None, None) == 0


def test_ids_and_workspace_host_side_validation(ot):
    """The calls that take caller host ids and a spreading workspace check
    their arguments before any device work."""
    L = ot.lib
    dummy = ctypes.c_void_p(0x1000)
    assert L.ot_spread_workspace_bytes(None) == 0
    assert L.ot_interpolate(None, dummy, dummy, dummy, 0, 10, dummy, None) == -1
    assert L.ot_spread(None, dummy, dummy, dummy, 0, 10, 1, 0, dummy, None, None) == -1
    for fn in (L.ot_grad_pos, L.ot_interp_grad_pos, L.ot_spread_grad_pos):
        assert fn(None, dummy, dummy, dummy, dummy, 0, 10, dummy, None) == -1
        assert b"tree is NULL" in L.ot_last_error()


def test_batch_gradient_ops_host_side_validation(ot):
    L = ot.lib
    h = ctypes.c_void_p()
    off = (ctypes.c_int64 * 3)(0, 5, 9)
    for bad in ((9, 9), (14, 14), (16, 16), (7, 8), (12, 3)):   # not gradient sets / mixed with forward ops
        ops = (ctypes.c_int32 * 2)(*bad)
        assert L.ot_batch_plan_create(ctypes.c_void_p(0x1000), off, ops, 2, 0, 0, None, ctypes.byref(h)) == -1
    assert L.ot_batch_run_grad(None, None, None, None, None, None, None, None, None) == -1
