"""Host test of the library's geometry upload cache: the upload logic
(csrc/ss_geom_upload.hpp, HIP-free) is compiled with g++ against device
operations that fail on demand, and every failure must leave the cache
invalid so that the next call uploads again (no GPU needed)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_upload_cache_is_invalid_after_every_failure(tmp_path):
    exe = tmp_path / "geom_upload_test"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-fsanitize=address,undefined",
                    "-I", os.path.join(ROOT, "paper_2511_11078_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host", "geom_upload_test.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout
