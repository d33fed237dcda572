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


def test_timestep_matches_oracle(orc):
    """sph_timestep (eq. timestep in the library, a host computation) equals
    the oracle's for the configurations of the workloads, to the last bit or
    one rounding of the quotients; h_min <= 0 takes the config's h_lo."""
    import numpy as np

    import paper_2107_01276_amd as P
    import workloads as W
    lib_path = os.path.join(ROOT, "paper_2107_01276_amd", "libsph.so")
    if not os.path.exists(lib_path):
        pytest.skip("libsph.so not built")
    for s in (W.tgv(50, seed=1), W.tgv(30, re=1000.0), W.gresho_chan(40)):
        prm = s["params"]
        cfg = P.Config(h_lo=s["h_min"], h_hi=s["h_min"], cs=prm["cs"], nu=prm["nu"],
                       u_ref=s["u_ref"])
        ref = orc.timestep(s["h_min"], s["u_ref"], prm["cs"], prm["nu"])
        assert P.timestep(cfg) == pytest.approx(ref, rel=4e-16, abs=0)
        assert P.timestep(cfg, 2 * s["h_min"]) == pytest.approx(
            orc.timestep(2 * s["h_min"], s["u_ref"], prm["cs"], prm["nu"]), rel=4e-16, abs=0)
    # the channel of the benchmark: the paper's cylinder runs give
    # dt = 0.25 h_min / (U + c_s) (the viscous bound is looser there)
    s = W.channel_cylinder(seed=2)
    prm = s["params"]
    cfg = P.Config(h_lo=s["h_min"], h_hi=s["h_min"], cs=prm["cs"], nu=prm["nu"], u_ref=s["u_ref"])
    assert P.timestep(cfg) == pytest.approx(0.25 * s["h_min"] / (s["u_ref"] + prm["cs"]),
                                            rel=4e-16)
    assert P.timestep(P.Config(h_lo=0.01, h_hi=0.01, cs=-1.0, u_ref=1.0)) == 0.0


def test_bg_init_passes_matches_oracle(orc):
    """sph_bg_init_passes (the initialisation's pass count of section 3.3, a
    host computation) equals the oracle's: 3 per size level, an exact power
    of C_r not rounded up a level, and 0 without a valid range."""
    import paper_2107_01276_amd as P
    lib_path = os.path.join(ROOT, "paper_2107_01276_amd", "libsph.so")
    if not os.path.exists(lib_path):
        pytest.skip("libsph.so not built")
    for ds_min, ds_max, cr in ((0.01, 0.64, 1.05), (0.0025, 0.25, 1.05), (0.01, 2.5, 1.05),
                               (0.1, 0.4, 1.2), (0.01, 0.02, 1.2), (0.1, 0.1, 1.2)):
        cfg = P.Config(h_lo=0.01, h_hi=0.01, ds_min=ds_min, ds_max=ds_max, cr=cr)
        assert P.bg_init_passes(cfg) == orc.bg_init_passes(ds_min, ds_max, cr), (ds_min, ds_max)
    # ln 64 / ln 1.05 = 85.24: 86 levels; 1.2^2 = 1.44 exactly two levels
    assert P.bg_init_passes(P.Config(h_lo=0.01, h_hi=0.01, ds_min=0.01, ds_max=0.64, cr=1.05)) == 258
    assert P.bg_init_passes(P.Config(h_lo=0.01, h_hi=0.01, ds_min=0.25, ds_max=0.36, cr=1.2)) == 6
    for bad in (dict(ds_min=0.0, ds_max=1.0, cr=1.05), dict(ds_min=0.5, ds_max=0.1, cr=1.05),
                dict(ds_min=0.1, ds_max=1.0, cr=1.0)):
        assert P.bg_init_passes(P.Config(h_lo=0.01, h_hi=0.01, **bad)) == 0
