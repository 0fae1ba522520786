"""The C boundary loads and exports every function include/dg.h declares
(CPU only: no compute call is made)."""
import ctypes
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dg.h")
LIB = os.path.join(ROOT, "paper_2109_09527_amd", "libdg.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z_]+)\s*\(", text)))


def _ensure_built():
    if not os.path.exists(LIB):
        from paper_2109_09527_amd import build
        build.build()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["dg_create", "dg_destroy", "dg_apply_batch", "dg_add_vertex", "dg_remove_vertex",
                 "dg_contains_vertex", "dg_add_edge", "dg_remove_edge", "dg_contains_edge",
                 "dg_snapshot_acquire", "dg_snapshot_release", "dg_bfs", "dg_sssp", "dg_bc",
                 "dg_query_batch", "dg_server_start", "dg_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    _ensure_built()
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(dg_\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


def test_library_loads_and_resolves_symbols():
    _ensure_built()
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        getattr(lib, n)


def test_op_record_layout_matches_header():
    from paper_2109_09527_amd.synth import OP_DTYPE
    assert OP_DTYPE.itemsize == 16
    assert [OP_DTYPE.fields[f][1] for f in ("type", "u", "v", "w")] == [0, 4, 8, 12]


def test_invalid_create_reports_without_device():
    """dg_create validates its config before touching the device."""
    _ensure_built()
    from paper_2109_09527_amd import dg
    cfg = dg.Config(0, 0, 10, 8, 0, 0)
    h = ctypes.c_void_p()
    assert dg.lib.dg_create(ctypes.byref(cfg), ctypes.byref(h)) == dg.E_INVALID_ARG
    cfg = dg.Config(1 << 24, 0, 1 << 10, 8, 0, 0)     # (V-1) * w_max overflows int32
    assert dg.lib.dg_create(ctypes.byref(cfg), ctypes.byref(h)) == dg.E_INVALID_ARG
    assert b"int32" in dg.lib.dg_last_error(None)
