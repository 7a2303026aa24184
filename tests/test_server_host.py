"""The docking server's host code (worker thread, locks, admission, cancel, retirement, destroy
with work pending) and the batch paths, built for the CPU against an emulated HIP runtime
(tests/hostmock) and run under ThreadSanitizer and under AddressSanitizer + UBSan.  Four client
threads submit, wait, poll, cancel and release requests while another docks the same requests
through md_dock and md_dock_batch; every result of a request must equal every other."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2203_02096_amd", "csrc")
MOCK = os.path.join(ROOT, "tests", "hostmock")
HOST_SOURCES = ["api.cpp", "autotune.cpp", "ligand_prep.cpp", "schedule.cpp", "server.cpp"]


def _clang():
    for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++")):
        if c and os.path.exists(c):
            return c
    return None


def _build(out_dir, sanitize):
    cxx = _clang()
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", f"-fsanitize={sanitize}",
             "-I", MOCK, "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    srcs = [os.path.join(CSRC, s) for s in HOST_SOURCES] + [os.path.join(MOCK, "mock_runtime.cpp"),
                                                            os.path.join(MOCK, "server_stress.cpp")]
    procs, objs = [], []
    for s in srcs:
        o = os.path.join(out_dir, os.path.basename(s) + ".o")
        objs.append(o)
        procs.append(subprocess.Popen([cxx, *flags, "-c", s, "-o", o], stdout=subprocess.PIPE,
                                      stderr=subprocess.STDOUT, text=True))
    for p, s in zip(procs, srcs):
        out, _ = p.communicate()
        assert p.returncode == 0, f"compiling {s}:\n{out}"
    exe = os.path.join(out_dir, "server_stress")
    subprocess.run([cxx, f"-fsanitize={sanitize}", *objs, "-lpthread", "-o", exe], check=True)
    return exe


@pytest.mark.parametrize("sanitize", ["thread", "address,undefined"])
def test_server_host_code_under_sanitizers(tmp_path, sanitize):
    if _clang() is None:
        pytest.skip("clang++ not available")
    exe = _build(str(tmp_path), sanitize)
    env = dict(os.environ)
    env["TSAN_OPTIONS"] = "halt_on_error=1 second_deadlock_stack=1"
    env["ASAN_OPTIONS"] = "halt_on_error=1 detect_leaks=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1 print_stacktrace=1"
    r = subprocess.run([exe, "3"], capture_output=True, text=True, timeout=300, env=env)
    sys.stdout.write(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "WARNING: ThreadSanitizer" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
    assert "; 0 failures" in r.stdout
