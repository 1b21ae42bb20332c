"""The C-ABI library loads and exports every entry point include/mmc.h declares
(no compute call: runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_symbols_exported():
    from paper_2106_05593_amd import mmc
    hdr = open(os.path.join(ROOT, "include", "mmc.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    names = set(re.findall(r"\b(mmc_[a-z_0-9]+)\s*\(", hdr))
    assert len(names) >= 20
    lib = ctypes.CDLL(mmc.SO)
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert names == set(mmc.EXPORTS)


def test_status_strings_and_arg_errors():
    from paper_2106_05593_amd import mmc
    L = mmc.lib()
    assert L.mmc_status_str(0) == b"ok"
    assert L.mmc_status_str(-1) == b"invalid argument"
    # NULL arguments are rejected before any device call
    h = ctypes.c_void_p()
    assert L.mmc_create(None, None, None, None, None, ctypes.byref(h)) == mmc.MMC_ERR_ARG
    assert b"NULL" in L.mmc_last_error()
    g = mmc.mmc_grid(0, 4, 1)
    cs = mmc.mmc_cellsize(1e-9, 1e-9, 1e-9)
    mat = mmc.mmc_material(Ms0=1e6, A0=1e-11, K1=0, Tc=700, mu_atomic=mmc.MUB, mf=1)
    mat.easy_axis[2] = 1.0
    run = mmc.mmc_run(T=300.0, cone_deg=30, refresh_per_sweep=2)
    assert L.mmc_create(ctypes.byref(g), ctypes.byref(cs), ctypes.byref(mat), ctypes.byref(run), None,
                        ctypes.byref(h)) == mmc.MMC_ERR_ARG
    g.nx = 4
    run.T = -1.0
    assert L.mmc_create(ctypes.byref(g), ctypes.byref(cs), ctypes.byref(mat), ctypes.byref(run), None,
                        ctypes.byref(h)) == mmc.MMC_ERR_DOMAIN
    run.T = 300.0
    run.cone_deg = 0
    assert L.mmc_create(ctypes.byref(g), ctypes.byref(cs), ctypes.byref(mat), ctypes.byref(run), None,
                        ctypes.byref(h)) == mmc.MMC_ERR_ARG
    assert L.mmc_sweep(None, 1) == mmc.MMC_ERR_ARG
    assert L.mmc_batch_create(None, 0, ctypes.byref(h)) == mmc.MMC_ERR_ARG


def test_missing_library_fails_loudly(monkeypatch):
    """No CPU fallback: without the built library every call raises."""
    import pytest
    from paper_2106_05593_amd import mmc
    monkeypatch.setattr(mmc, "SO", os.path.join(ROOT, "no_such_dir", "libmmc.so"))
    monkeypatch.setattr(mmc, "_lib", None)
    with pytest.raises(ImportError):
        mmc.lib()
    with pytest.raises(ImportError):
        mmc.Chain((4, 4, 1), (5e-9,) * 3, Ms0=1e6, A0=1e-11, K1=0.0, Tc=700.0, T=300.0)


def test_header_is_plain_c(tmp_path):
    """include/mmc.h compiles as strict C99 (and as C++): the ABI takes plain
    C types only."""
    import shutil
    import subprocess
    import pytest
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    src = tmp_path / "use.c"
    src.write_text('#include "mmc.h"\nint main(void) { mmc_ctx* c = 0; mmc_stats st; (void)c; (void)st; return 0; }\n')
    inc = os.path.join(ROOT, "include")
    for cmd in (["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only", "-I", inc, str(src)],
                ["g++", "-std=c++17", "-Wall", "-Werror", "-fsyntax-only", "-x", "c++", "-I", inc, str(src)]):
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
