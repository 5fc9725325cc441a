"""Host-side native code under AddressSanitizer and UndefinedBehaviorSanitizer:
the service's admission scheduler against a mock allocator, and the C oracle
driven through its entry points.  Built with g++/gcc (no device code)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, tmp_path, name):
    exe = str(tmp_path / name)
    subprocess.run(cmd + ["-o", exe], check=True, capture_output=True, text=True)
    res = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    print(res.stdout[-2000:], res.stderr[-4000:])
    assert res.returncode == 0, res.stderr[-4000:]
    return res.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_scheduler_against_mock_allocator(tmp_path):
    out = _run(["g++", "-std=c++17", "-Wall", "-Wextra", "-Werror"] + SAN +
               [os.path.join(HERE, "native", "test_scheduler.cpp")], tmp_path, "sched")
    assert "all checks passed" in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_entry_points_under_sanitizers(tmp_path):
    src = [os.path.join(ROOT, "oracle", f) for f in sorted(os.listdir(os.path.join(ROOT, "oracle")))
           if f.endswith(".c")]
    # serial build (the OpenMP pragmas are ignored): the sanitizers see one thread
    out = _run(["gcc", "-std=gnu11", "-Wall", "-Wextra", "-Werror", "-Wno-unknown-pragmas"] + SAN +
               ["-I", os.path.join(ROOT, "oracle"), os.path.join(HERE, "native",
                                                                 "test_oracle_san.c")] +
               src + ["-lm"], tmp_path, "oracle_san")
    assert "all checks passed" in out
