"""The kernels' tile addressing, replayed on the CPU (tests/native/tile_walk_check.cpp)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_tile_walk_addressing(tmp_path):
    exe = str(tmp_path / "tile_walk")
    subprocess.run(["g++", "-O1", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", os.path.join(ROOT, "paper_1308_1343_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "tile_walk_check.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "tile walk OK" in r.stdout
