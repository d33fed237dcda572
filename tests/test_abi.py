"""CPU checks of the C-ABI library: it loads and exports every entry point
declared in include/sph.h (no compute calls without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "sph.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_entry_points():
    syms = declared_symbols()
    for s in ("sph_build_neighbors", "sph_rates", "sph_adapt", "sph_step", "sph_bg_update",
              "sph_mref_lookup", "sph_create", "sph_workspace_bytes"):
        assert s in syms


def test_library_exports_all_declared():
    lib_path = os.path.join(ROOT, "paper_2107_01276_amd", "libsph.so")
    if not os.path.exists(lib_path):
        pytest.skip("libsph.so not built")
    lib = ctypes.CDLL(lib_path)
    for s in declared_symbols():
        assert hasattr(lib, s), s
    lib.sph_version.restype = ctypes.c_int
    assert lib.sph_version() >= 10000


def test_binding_symbols_match_header():
    import paper_2107_01276_amd as P
    assert set(P.EXPORTS) == set(declared_symbols())


def test_workspace_bytes_and_invalid_config():
    import paper_2107_01276_amd as P
    lib = P.load_library()
    cfg = P.Config(h_lo=0.02, h_hi=0.02)
    c = cfg.c()
    b1 = lib.sph_workspace_bytes(ctypes.byref(c), 1000)
    b2 = lib.sph_workspace_bytes(ctypes.byref(c), 100000)
    assert 0 < b1 < b2
    bad = P.Config(h_lo=-1.0).c()
    assert lib.sph_workspace_bytes(ctypes.byref(bad), 1000) == 0
    h = ctypes.c_void_p()
    # a workspace that is too small is rejected before any device work
    assert lib.sph_create(ctypes.byref(c), 1000, None, 0, None, ctypes.byref(h)) == P.SPH_E_NOMEM


def test_checkpoint_size():
    """sph_export_bytes: a 64-byte header, then eight double arrays, the
    int64 ledger and the int32 kinds per particle; negative n is refused."""
    lib_path = os.path.join(ROOT, "paper_2107_01276_amd", "libsph.so")
    if not os.path.exists(lib_path):
        pytest.skip("libsph.so not built")
    lib = ctypes.CDLL(lib_path)
    lib.sph_export_bytes.restype = ctypes.c_size_t
    lib.sph_export_bytes.argtypes = [ctypes.c_int64]
    for n in (0, 1, 1000, 123457):
        assert lib.sph_export_bytes(n) == 64 + n * (8 * 8 + 8 + 4)
    assert lib.sph_export_bytes(-1) == 0
