"""The request server's host code (scheduler thread, admission, uploads,
cancel and deadlines, latency accounting) compiled for the CPU against a
stub HIP runtime (tests/cpp/stub), with a model of the batched kernel:
plain, under ThreadSanitizer and under AddressSanitizer/UBSan.  No device
involved."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "cpp", "test_server_host.cpp")
INC = ["-I", os.path.join(ROOT, "tests", "cpp", "stub"), "-I", os.path.join(ROOT, "include"),
       "-I", os.path.join(ROOT, "paper_2205_01313_amd", "csrc")]
WARN = ["-Wall", "-Wno-unknown-pragmas"]


def build_and_run(tmp_path, name, cxx, flags, timeout=600):
    exe = tmp_path / name
    subprocess.run([cxx, "-O1", "-g", "-std=c++17", *flags, "-x", "c++", *INC, SRC, "-o", str(exe), "-lpthread"],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=timeout)
    return r


def test_server_host_code(tmp_path):
    r = build_and_run(tmp_path, "server_host", "g++", [*WARN, "-Wno-subobject-linkage", "-Werror"])
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr


def test_server_host_code_under_thread_sanitizer(tmp_path):
    """ThreadSanitizer from the ROCm LLVM toolchain (GCC 11's runtime misses
    mutex releases inside timed condition-variable waits and reports races
    that cannot happen)."""
    clang = "/opt/rocm/llvm/bin/clang++"
    if not os.path.exists(clang):
        clang = shutil.which("clang++")
    if not clang:
        pytest.skip("no clang++ with a ThreadSanitizer runtime")
    r = build_and_run(tmp_path, "server_host_tsan", clang, ["-fsanitize=thread", *WARN])
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-6000:]
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr[-3000:]


def test_server_host_code_under_address_sanitizer(tmp_path):
    r = build_and_run(tmp_path, "server_host_asan", "g++",
                      ["-fsanitize=address,undefined", "-fno-sanitize-recover", *WARN, "-Wno-subobject-linkage"])
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr[-3000:]
