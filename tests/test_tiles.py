"""Last-phase tile selections (csrc/fw_tiles.h, the code the kernels include),
checked on the host: each launch visits every selected tile exactly once, a
round's launch selects every tile outside its block row and column, and the
lookahead split (block row / column r + 1 first, then the rest) partitions it."""
import os
import subprocess

from conftest import ROOT


def test_tile_selections(tmp_path):
    exe = str(tmp_path / "tiles_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-Werror", "-o", exe,
                    os.path.join(ROOT, "tests", "tiles_check.cpp")], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(out.stdout)
    assert out.returncode == 0, out.stdout
    assert " 0 failures" in out.stdout
