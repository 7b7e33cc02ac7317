"""Plan-time staging windows of the staged resample + FFT kernel, checked on
the CPU: tests/stage_windows_check.cpp replays every LDS write and read of
the kernel for several geometries (4K at every sub-transform length, square,
odd and ragged frames) and counts reads outside the staged pixels; geometries
whose windows exceed the kernel's staging buffer must be refused (the plan
then uses the direct gather)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


def test_staging_windows_cover_every_tap(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc missing")
    exe = str(tmp_path / "stage_windows_check")
    subprocess.check_call([HIPCC, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I",
                           os.path.join(ROOT, "paper_2304_14492_amd", "csrc"),
                           os.path.join(ROOT, "tests", "stage_windows_check.cpp"), "-o", exe],
                          stderr=subprocess.DEVNULL)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failure(s)" in r.stdout
    # 4K and the smaller frames are served; the coarse 4096^2 / 300-ring and 3000^2 grids are refused
    assert r.stdout.count("planner ok") == 5 and r.stdout.count("REFUSED") == 2
