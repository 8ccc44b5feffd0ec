"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU):
the library's table derivations (basis-change rows, orbit templates, fold
tables) and the oracle, each built with gcc/g++ and the sanitizers and run
at small sizes by its own driver (tests/sanitize/).  Any report fails the
run (-fno-sanitize-recover)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1807_10058_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, exe, tmp):
    subprocess.check_call(cmd, cwd=tmp)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], cwd=tmp, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-2000:] + r.stderr[-4000:]


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_library_host_code(tmp_path):
    exe = str(tmp_path / "lib_host")
    srcs = [os.path.join(CSRC, f) for f in ("asp_tables.cpp", "orbit_blocks.cpp", "fold_plan.cpp")]
    cmd = ["g++", "-std=c++17", "-pthread"] + SAN + ["-I", os.path.join(ROOT, "include"), "-I", CSRC,
                                                    os.path.join(ROOT, "tests", "sanitize", "lib_host_driver.cpp")] + \
        srcs + ["-o", exe]
    _run(cmd, exe, str(tmp_path))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle(tmp_path):
    exe = str(tmp_path / "oracle")
    cmd = ["gcc", "-std=gnu11"] + SAN + [os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                                      os.path.join(ROOT, "oracle", "fcc_oracle.c"), "-lm", "-o", exe]
    _run(cmd, exe, str(tmp_path))
