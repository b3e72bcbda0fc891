"""The fused tile kernels' addressing (region walks, plane masks, tile origins;
paper_2405_14903_amd/csrc/nf_tile.h) enumerated on the host for grids with
ragged tiles along every axis: coverage, element indices and bounds."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_tile_walks_cover_and_stay_in_bounds(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path / "tile_walks_check"
    subprocess.run([cxx, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_2405_14903_amd", "csrc"),
                    os.path.join(HERE, "tile_walks_check.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout[-2000:]
    assert out.stdout.strip().endswith("OK")
