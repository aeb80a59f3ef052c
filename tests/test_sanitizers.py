"""The project's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(gcc/g++, host code only): the generator, the oracle and the server's
admission queue, driven by tests/sanitize_driver.cpp.  Any sanitizer report
aborts the driver (-fno-sanitize-recover)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all"]


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host compiler")
def test_host_code_is_sanitizer_clean(tmp_path):
    objs = []
    for src in ("xdrop_oracle.c", "banded_oracle.c"):
        obj = str(tmp_path / (src + ".o"))
        subprocess.check_call(["gcc", "-std=c11", "-c", os.path.join(ROOT, "oracle", src),
                               "-o", obj] + FLAGS)
        objs.append(obj)
    exe = str(tmp_path / "sanitize_driver")
    subprocess.check_call(["g++", "-std=c++17", os.path.join(HERE, "sanitize_driver.cpp"),
                           "-I" + os.path.join(ROOT, "oracle"),
                           "-I" + os.path.join(ROOT, "paper_2001_10049_amd", "csrc"),
                           "-o", exe, "-pthread"] + FLAGS + objs)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    res = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stderr[-3000:]
    assert "0 failures" in res.stdout
