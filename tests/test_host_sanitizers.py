"""The host side of the library (the table builder: validation, phase fold,
merge, grouping, the group index and the occupation form of the diagonal;
and the host entry points) built without device code under AddressSanitizer
and UndefinedBehaviorSanitizer, and the host-table tests run against that
build in a child process.  Any out-of-bounds access, use after free or
undefined operation aborts the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2506_23809_amd", "csrc")


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_table_builder_under_address_and_ub_sanitizers(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    sys.path.insert(0, os.path.join(ROOT, "paper_2506_23809_amd"))
    import build as nqs_build
    lib = str(tmp_path / "libnqs_host_asan.so")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fPIC", "-shared", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           *[os.path.join(CSRC, f) for f in nqs_build.HOST_SOURCES], "-o", lib]
    subprocess.check_call(cmd)
    env = dict(os.environ)
    env["NQS_LIBRARY"] = lib
    env["LD_PRELOAD"] = asan + (":" + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    child = subprocess.run(
        [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
         os.path.join(ROOT, "tests", "test_host_table.py"),
         "-k", "table_groups or merges or rejections"],
        cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = child.stdout + child.stderr
    assert child.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    # both table workloads, the merge order and every rejection ran
    assert "4 passed" in out and "failed" not in out, out[-2000:]
