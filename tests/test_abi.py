"""The C-ABI library loads and exports every entry point its headers declare (CPU-only)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1708_03188_amd", "libsgm.so")


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b(sgm_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_header_declares_entry_points():
    names = _declared()
    for n in ("sgm_plan_create", "sgm_forward", "sgm_backward", "sgm_helmholtz_solve", "sgm_helmholtz_solve_physical",
              "sgm_biharmonic_solve"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsgm.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsgm.so not built")
def test_status_strings_and_argument_errors_without_gpu():
    from paper_1708_03188_amd import _lib
    lib = _lib.load()
    assert lib.sgm_status_string(0) == b"ok"
    assert lib.sgm_status_string(-2) == b"unsupported size"
    assert lib.sgm_status_string(-6) == b"singular system"
    assert lib.sgm_version() >= 1
    # A null descriptor is rejected before any device call.
    assert lib.sgm_plan_create(None, None, None) == -1
    assert b"null" in lib.sgm_last_error()
    # so are null plans and arrays on the solve entry points
    assert lib.sgm_helmholtz_solve(None, 0.0, None, None, None) == -1
    assert lib.sgm_helmholtz_solve_physical(None, 0.0, None, None, None) == -1
    assert b"null" in lib.sgm_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsgm.so not built")
def test_fno_create_rejects_sizes_before_any_device_call():
    from paper_1708_03188_amd import _lib
    lib = _lib.load()
    out = ctypes.c_void_p()
    # 2 * modes > H
    d = _lib.FNODesc(H=16, W=16, width=32, modes=9, layers=4, hidden=128, max_batch=1)
    assert lib.sgm_fno_create(ctypes.byref(d), 1, ctypes.byref(out)) == -1
    assert b"modes" in lib.sgm_last_error()
    # the spectral buffers' element count (max_batch * 4 * modes^2 * width) must stay below 2^31
    d = _lib.FNODesc(H=256, W=256, width=32, modes=16, layers=4, hidden=128, max_batch=1 << 20)
    assert lib.sgm_fno_create(ctypes.byref(d), 1, ctypes.byref(out)) == -1
    assert b"2^31" in lib.sgm_last_error()
    assert not out.value


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsgm.so not built")
def test_autotune_cache_path_follows_environment(monkeypatch):
    from paper_1708_03188_amd.api import autotune_cache_path
    monkeypatch.setenv("SGM_TUNE_CACHE", "/tmp/some/where/tune.txt")
    assert autotune_cache_path() == "/tmp/some/where/tune.txt"
    monkeypatch.setenv("SGM_TUNE_CACHE", "off")
    assert autotune_cache_path() == ""
    monkeypatch.delenv("SGM_TUNE_CACHE")
    monkeypatch.setenv("XDG_CACHE_HOME", "/tmp/xdg")
    assert autotune_cache_path() == "/tmp/xdg/libsgm/tune.txt"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsgm.so not built")
def test_plain_c_consumer_compiles_links_and_runs(tmp_path):
    # The header must be valid C99 (no C++ or HIP types across the boundary) and the
    # library usable from C alone; the program only makes calls that need no GPU.
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    exe = str(tmp_path / "abi_consumer")
    libdir = os.path.dirname(LIB)
    subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I" + os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "abi_consumer.c"), "-L" + libdir, "-lsgm", "-Wl,-rpath," + libdir,
                    "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert "ok" in r.stdout


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    # the product path has no fallback: without the built library every entry into
    # the binding raises instead of computing anything another way
    from paper_1708_03188_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libsgm.so"))
    with pytest.raises(_lib.SgmError, match="not found"):
        _lib.load()
    from paper_1708_03188_amd import api
    with pytest.raises(_lib.SgmError, match="not found"):
        api.Plan("dirichlet", 8, 4)
