"""The host-side plan-table builders (long-double Chebyshev/Shen and Legendre
tables, twiddles, radix factorisation) built with AddressSanitizer and
UndefinedBehaviorSanitizer and run over every basis and a range of sizes, on the
CPU (the builders are plain C++; the HIP headers are only needed for types)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1708_03188_amd", "csrc")
ROCM_INC = "/opt/rocm/include"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(ROCM_INC), reason="needs g++ and the HIP headers")
def test_table_builders_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_tables_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I" + ROCM_INC, "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           os.path.join(CSRC, "tables.cpp"), os.path.join(CSRC, "legendre_tables.cpp"),
           os.path.join(ROOT, "tests", "host_tables_check.cpp"), "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), (r.stdout[-2000:], r.stderr[-3000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
