"""The band kernel's tile dispatch order (border tiles first, then interior
tiles in XCD-contiguous ranges) is a bijection on the tiles of a band: built
as a host-only program against the library and run on the CPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2010_04868_amd")


def test_tile_order_is_a_border_first_bijection():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    if not os.path.exists(os.path.join(LIBDIR, "libtvstencil.so")):
        pytest.skip("library not built")
    out_dir = os.path.join(ROOT, "_build")
    os.makedirs(out_dir, exist_ok=True)
    exe = os.path.join(out_dir, "tile_order_check")
    src = os.path.join(ROOT, "tests", "tile_order_check.cpp")
    r = subprocess.run([hipcc, "-O1", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                        "-I", os.path.join(ROOT, "include"), src, "-o", exe,
                        "-L", LIBDIR, "-ltvstencil", f"-Wl,-rpath,{LIBDIR}"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout
