"""The C-ABI library loads without a GPU and exports every function that
include/pso.h declares; the binding declares exactly those."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pso[0-9]*_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def libpath():
    from paper_2205_01313_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        from paper_2205_01313_amd import build
        build.build()
    return _native.LIB_PATH


def test_library_exports_every_declared_symbol(libpath):
    names = declared("pso.h")
    assert "pso_create" in names and "pso_run" in names
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (pso[0-9]*_[a-z0-9_]+)$", out, flags=re.M))
    missing = [n for n in names if n not in exported]
    assert not missing, missing


def test_binding_declares_exactly_the_header(libpath):
    from paper_2205_01313_amd import _native
    assert sorted(_native.SIGNATURES) == declared("pso.h")
    lib = _native.load()
    for n in _native.SIGNATURES:
        assert getattr(lib, n) is not None


def test_pure_host_entry_points_without_gpu(libpath):
    """Calls that touch no device: sizes and argument rejection."""
    import ctypes
    from paper_2205_01313_amd import _native
    lib = _native.load()
    N, D = 1 << 20, 32
    b = lib.pso_workspace_bytes(N, D)
    assert b >= 3 * N * D * 4 + N * 4
    assert lib.pso_workspace_bytes(0, 4) == 0 and lib.pso_workspace_bytes(4, 0) == 0
    assert lib.pso_workspace_bytes((1 << 30) + 1, 1) == 0
    h = ctypes.c_void_p()
    bounds = (ctypes.c_float * 2)(-1.0, 1.0)
    assert lib.pso_create(9, 16, 2, bounds, 0.7, 1.4, 1.4, 0.2, 0, ctypes.byref(h)) == _native.PSO_EINVAL
    assert b"fitness" in lib.pso_last_error()
    assert lib.pso_create(2, 16, 1, bounds, 0.7, 1.4, 1.4, 0.2, 0, ctypes.byref(h)) == _native.PSO_EINVAL
    bad = (ctypes.c_float * 2)(1.0, -1.0)
    assert lib.pso_create(0, 16, 2, bad, 0.7, 1.4, 1.4, 0.2, 0, ctypes.byref(h)) == _native.PSO_EINVAL
    assert lib.pso_create(0, 16, 2, bounds, 0.7, 1.4, 1.4, 0.0, 0, ctypes.byref(h)) == _native.PSO_EINVAL
    assert lib.pso_create(0, 16, 2, bounds, float("nan"), 1.4, 1.4, 0.2, 0, ctypes.byref(h)) == _native.PSO_EINVAL
    assert lib.pso_destroy(None) == _native.PSO_EINVAL
    assert lib.pso_step(None) == _native.PSO_EINVAL
    assert lib.pso_run(None, 1, 0.0, 0.0, None, None, None, None) == _native.PSO_EINVAL
    shape = _native.PsoBatchShape(256, 0, 1 << 17)
    assert lib.pso_batch_get_shape(None, ctypes.byref(shape)) == _native.PSO_EINVAL
    assert lib.pso_batch_set_shape(None, ctypes.byref(shape)) == _native.PSO_EINVAL
    assert lib.pso_batch_autotune(None, 8, None) == _native.PSO_EINVAL
    b = (ctypes.c_float * 2)(-1.0, 1.0)
    h64 = ctypes.c_void_p()
    assert lib.pso64_create(9, 16, 2, b, 0.7, 1.4, 1.4, 0.2, 0, ctypes.byref(h64)) == _native.PSO_EINVAL
    assert lib.pso64_create(0, 0, 2, b, 0.7, 1.4, 1.4, 0.2, 0, ctypes.byref(h64)) == _native.PSO_EINVAL
    assert lib.pso64_destroy(None) == _native.PSO_EINVAL
    assert lib.pso64_step(None) == _native.PSO_EINVAL
    assert lib.pso64_eval(None, None, 1, None) == _native.PSO_EINVAL


def test_batch_limits_rejected_before_any_allocation(libpath):
    """Counts beyond a batch's limits fail with a status, on the host, before
    anything is allocated or any device is touched."""
    import ctypes
    from paper_2205_01313_amd import _native
    lib = _native.load()
    descs = (_native.PsoDesc * 1)()
    h = ctypes.c_void_p()
    assert lib.pso_batch_create(descs, 0, None, ctypes.byref(h)) == _native.PSO_EINVAL
    assert lib.pso_batch_create(descs, (1 << 24) + 1, None, ctypes.byref(h)) == _native.PSO_EINVAL
    assert lib.pso_batch_create(descs, 1 << 31, None, ctypes.byref(h)) == _native.PSO_EINVAL
    assert b"count" in lib.pso_last_error()
