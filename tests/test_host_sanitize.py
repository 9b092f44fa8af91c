"""Host AddressSanitizer / UndefinedBehaviorSanitizer build of the library's
host code (validation of the C-ABI arguments, determinant compaction, the
integral checks, the Jacobi eigensolver of the Dyall set-up, the estimators
formed from accumulated sums), sanitizers on the host code only, run on the CPU
without any GPU call (tests/host_sanitize_main.hip)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc")
def test_host_code_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "host_sanitize")
    cmd = ["hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fno-gpu-sanitize",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "include"), "-o", exe, os.path.join(HERE, "host_sanitize_main.hip")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "clean" in r.stdout, r.stdout
