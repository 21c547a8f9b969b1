"""The CPU oracle, the seeded input generator and the C ABI's host-side
validation built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
host code only) and run through tests/asan_driver.cpp: every function over
edge-case inputs, with a few results the definitions fix checked on the way.
Any out-of-bounds access, leak, overflow or other undefined behaviour aborts
the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


@pytest.mark.skipif(not (shutil.which("gcc") and shutil.which("g++")), reason="gcc/g++ not available")
def test_oracle_synth_and_validation_under_asan_ubsan(tmp_path):
    objs = []
    for src, cc, std in ((os.path.join(ROOT, "oracle", "igsp_oracle.c"), "gcc", "-std=c99"),
                         (os.path.join(ROOT, "synth", "synth.c"), "gcc", "-std=c99"),
                         (os.path.join(ROOT, "paper_2603_08661_amd", "csrc", "validate.cpp"), "g++", "-std=c++17"),
                         (os.path.join(ROOT, "tests", "asan_driver.cpp"), "g++", "-std=c++17")):
        obj = tmp_path / (os.path.basename(src) + ".o")
        subprocess.run([cc, std, *SAN, "-c", src, "-o", str(obj)], check=True, capture_output=True, text=True)
        objs.append(str(obj))
    exe = tmp_path / "asan_driver"
    subprocess.run(["g++", *SAN, *objs, "-o", str(exe), "-lm"], check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:halt_on_error=1:detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "all checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
