"""Host bookkeeping of the request server (device-memory arena and FIFO
admission by memory), unit-tested on the CPU with g++: no device involved."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_arena_and_admission(tmp_path):
    exe = tmp_path / "test_arena"
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-Werror",
                    os.path.join(ROOT, "tests", "cpp", "test_arena.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr


def test_arena_under_host_sanitizers(tmp_path):
    exe = tmp_path / "test_arena_asan"
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover",
                    os.path.join(ROOT, "tests", "cpp", "test_arena.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr


def test_entry_point_guard_maps_exceptions_to_status(tmp_path):
    """The wrapper around every C entry point: a thrown std::bad_alloc (forced
    by capping the address space), a length error and any other exception
    become status codes; nothing escapes into std::terminate."""
    exe = tmp_path / "test_guard"
    subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "cpp", "test_guard.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
