"""Host check of the tile-box layout that the sorted deposit stores and its gather pass
reads (paper_2410_20501_amd/csrc/tile_box.h): compiled with the host compiler against a
stand-in for the HIP runtime header (the functions are plain host/device arithmetic)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2410_20501_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs a host C++ compiler")
def test_tile_box_layout(tmp_path):
    stub = tmp_path / "hip"
    stub.mkdir()
    (stub / "hip_runtime.h").write_text("#pragma once\n#define __host__\n#define __device__\n")
    exe = tmp_path / "tile_box_check"
    subprocess.run(["g++", "-std=c++17", "-O1", f"-I{tmp_path}", f"-I{CSRC}",
                    os.path.join(HERE, "tile_box_check.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout
