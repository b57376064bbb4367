"""Host-side tables of the PML row-band sweep (k_wave_pml_band): compiles
tests/pml_band_tables_check.cpp against libfwi.so and runs it on assorted
geometries (reflecting top or not, 0-10 layer cells, 2-8 bands, widths that
need more halo words than one thread can hold).  No GPU is used: the program
checks the tables and the kernel's index formulas on the host."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2603_16393_amd")


def test_pml_band_tables(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc is not installed")
    if not os.path.exists(os.path.join(PKG, "libfwi.so")):
        pytest.skip("libfwi.so is not built")
    exe = str(tmp_path / "pml_band_tables_check")
    cmd = [hipcc, "-O1", "-std=c++17", f"-I{ROOT}/include", f"-I{PKG}/csrc",
           os.path.join(ROOT, "tests", "pml_band_tables_check.cpp"), f"-L{PKG}", "-lfwi", f"-Wl,-rpath,{PKG}",
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-2000:]
    assert "fails: 0" in r.stdout
