"""Global-best particle swarm optimisation on AMD Instinct MI355X (gfx950).

A thin binding of libpso.so (include/pso.h): every function below marshals
arguments for the C entry point of the same name; all computation happens in
the library's HIP kernels.  PyTorch is used only for device memory and
streams (pso_create_in with a torch tensor and torch's current stream).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _native
from ._native import (PSO_ACKLEY, PSO_ASYNC, PSO_CUBIC, PSO_EAGAIN, PSO_ECANCELED, PSO_EDEVICE,  # noqa: F401
                      PSO_EINVAL, PSO_ENOMEM, PSO_ESTATE, PSO_ETIMEDOUT, PSO_OK, PSO_PERSISTENT, PSO_RASTRIGIN,
                      PSO_REDUCE, PSO_REDUCE_UNROLLED, PSO_ROSENBROCK, PSO_SPHERE, PSO_SYNC)

FITNESS = {"sphere": PSO_SPHERE, "rastrigin": PSO_RASTRIGIN, "rosenbrock": PSO_ROSENBROCK,
           "ackley": PSO_ACKLEY, "cubic": PSO_CUBIC}


class PsoError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _native.load().pso_last_error().decode(errors="replace")
        super().__init__(f"{where} -> {code}: {msg}")
        self.code = code


def _check(code: int, where: str) -> int:
    if code != PSO_OK:
        raise PsoError(code, where)
    return code


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def fitness_id(f) -> int:
    return FITNESS[f] if isinstance(f, str) else int(f)


def lib():
    return _native.load()


def pso_workspace_bytes(N: int, D: int) -> int:
    return int(lib().pso_workspace_bytes(N, D))


def pso_create(fitness, N, D, bounds, w, c1, c2, vmax, seed) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    b = (ctypes.c_float * 2)(*bounds)
    _check(lib().pso_create(fitness_id(fitness), N, D, b, w, c1, c2, vmax, seed, ctypes.byref(h)), "pso_create")
    return h


def pso_create_in(fitness, N, D, bounds, w, c1, c2, vmax, seed, dev_ptr: int, nbytes: int, stream_ptr: int):
    h = ctypes.c_void_p()
    b = (ctypes.c_float * 2)(*bounds)
    _check(lib().pso_create_in(fitness_id(fitness), N, D, b, w, c1, c2, vmax, seed, ctypes.c_void_p(dev_ptr),
                               nbytes, ctypes.c_void_p(stream_ptr), ctypes.byref(h)), "pso_create_in")
    return h


def pso_set_shift(h, shift):
    if shift is None:
        return _check(lib().pso_set_shift(h, None), "pso_set_shift")
    s = np.ascontiguousarray(shift, np.float32)
    return _check(lib().pso_set_shift(h, _fptr(s)), "pso_set_shift")


def pso_set_variant(h, variant: int):
    return _check(lib().pso_set_variant(h, variant), "pso_set_variant")


def pso_set_max_lead(h, max_lead: int):
    return _check(lib().pso_set_max_lead(h, int(max_lead)), "pso_set_max_lead")


def pso_reset(h):
    return _check(lib().pso_reset(h), "pso_reset")


def pso_step(h):
    return _check(lib().pso_step(h), "pso_step")


def pso_run(h, max_iter, D, tol=0.0, f_star=0.0):
    val = ctypes.c_float()
    pos = np.empty(D, np.float32)
    git = ctypes.c_int64()
    done = ctypes.c_int64()
    _check(lib().pso_run(h, max_iter, tol, f_star, ctypes.byref(val), _fptr(pos), ctypes.byref(git),
                         ctypes.byref(done)), "pso_run")
    return dict(gbest_fit=np.float32(val.value), gbest_pos=pos, gbest_iter=git.value, iters=done.value)


def pso_get_best(h, D):
    val = ctypes.c_float()
    pos = np.empty(D, np.float32)
    git = ctypes.c_int64()
    t = ctypes.c_int64()
    _check(lib().pso_get_best(h, ctypes.byref(val), _fptr(pos), ctypes.byref(git), ctypes.byref(t)), "pso_get_best")
    return dict(gbest_fit=np.float32(val.value), gbest_pos=pos, gbest_iter=git.value, t=t.value)


def pso_get_history(h, t0, count):
    out = np.empty(count, np.uint64)
    _check(lib().pso_get_history(h, t0, count, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))),
           "pso_get_history")
    return out


def pso_get_state(h, N, D):
    st = dict(x=np.empty(D * N, np.float32), v=np.empty(D * N, np.float32), p=np.empty(D * N, np.float32),
              pf=np.empty(N, np.float32), gpos=np.empty(D, np.float32))
    key = ctypes.c_uint64()
    git = ctypes.c_int64()
    t = ctypes.c_int64()
    _check(lib().pso_get_state(h, _fptr(st["x"]), _fptr(st["v"]), _fptr(st["p"]), _fptr(st["pf"]),
                               ctypes.byref(key), _fptr(st["gpos"]), ctypes.byref(git), ctypes.byref(t)),
           "pso_get_state")
    st.update(gkey=key.value, giter=git.value, t=t.value)
    return st


def pso_set_state(h, st):
    arrs = {k: np.ascontiguousarray(st[k], np.float32) for k in ("x", "v", "p", "pf", "gpos")}
    return _check(lib().pso_set_state(h, _fptr(arrs["x"]), _fptr(arrs["v"]), _fptr(arrs["p"]), _fptr(arrs["pf"]),
                                       int(st["gkey"]), _fptr(arrs["gpos"]), int(st["giter"]), int(st["t"])),
                  "pso_set_state")


def pso_get_counters(h):
    n = ctypes.c_uint64()
    _check(lib().pso_get_counters(h, ctypes.byref(n)), "pso_get_counters")
    return dict(pbest_improvements=n.value)


def pso_get_async_counters(h):
    n, f = ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib().pso_get_async_counters(h, ctypes.byref(n), ctypes.byref(f)), "pso_get_async_counters")
    return dict(tiles=n.value, fresh_tiles=f.value)


def pso_sync(h):
    return _check(lib().pso_sync(h), "pso_sync")


def pso_destroy(h):
    return _check(lib().pso_destroy(h), "pso_destroy")


def _descs(specs):
    """Array of pso_desc from objects with fitness, N, D, box, w, c1, c2, vmax,
    seed, shift, T (max_iter), tol, f_star; keeps the shift arrays alive."""
    arr = (_native.PsoDesc * len(specs))()
    keep = []
    for k, sp in enumerate(specs):
        d = arr[k]
        d.fitness_id = fitness_id(sp.fitness)
        d.D, d.N = int(sp.D), int(sp.N)
        d.bounds[0], d.bounds[1] = sp.box
        d.w, d.c1, d.c2, d.vmax = sp.w, sp.c1, sp.c2, sp.vmax
        d.seed = int(sp.seed)
        if getattr(sp, "shift", None) is not None:
            sh = np.ascontiguousarray(sp.shift, np.float32)
            keep.append(sh)
            d.shift = sh.ctypes.data
        else:
            d.shift = None
        d.max_iter = int(sp.T)
        d.tol = float(getattr(sp, "tol", 0.0) or 0.0)
        d.f_star = float(getattr(sp, "f_star", 0.0) or 0.0)
    return arr, keep


class Swarm64:
    """A swarm computed in binary64 (pso64_*): same parameters as Swarm."""

    def __init__(self, fitness, N, D, bounds, w, c1, c2, vmax, seed, shift=None):
        self.N, self.D = int(N), int(D)
        self.h = ctypes.c_void_p()
        b = (ctypes.c_float * 2)(*bounds)
        _check(lib().pso64_create(fitness_id(fitness), self.N, self.D, b, float(w), float(c1), float(c2), float(vmax),
                                  int(seed), ctypes.byref(self.h)), "pso64_create")
        if shift is not None:
            sh = np.ascontiguousarray(shift, np.float32)
            _check(lib().pso64_set_shift(self.h, sh.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
                   "pso64_set_shift")

    def step(self, n=1):
        for _ in range(n):
            _check(lib().pso64_step(self.h), "pso64_step")

    def reset(self):
        _check(lib().pso64_reset(self.h), "pso64_reset")

    def run(self, max_iter, tol=0.0, f_star=0.0):
        val, git, done = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
        pos = np.empty(self.D)
        dp = ctypes.POINTER(ctypes.c_double)
        _check(lib().pso64_run(self.h, int(max_iter), float(tol), float(f_star), ctypes.byref(val),
                               pos.ctypes.data_as(dp), ctypes.byref(git), ctypes.byref(done)), "pso64_run")
        return dict(gbest_fit=val.value, gbest_pos=pos, gbest_iter=git.value, iters=done.value)

    def eval(self, points):
        """The swarm's fitness (binary64, with its shift) at points (M x D)."""
        pts = np.ascontiguousarray(np.asarray(points, np.float64).reshape(-1, self.D))
        out = np.empty(pts.shape[0])
        dp = ctypes.POINTER(ctypes.c_double)
        _check(lib().pso64_eval(self.h, pts.ctypes.data_as(dp), pts.shape[0], out.ctypes.data_as(dp)), "pso64_eval")
        return out

    def state(self):
        N, D = self.N, self.D
        out = dict(x=np.empty(D * N), v=np.empty(D * N), p=np.empty(D * N), pf=np.empty(N))
        gi, t = ctypes.c_int64(), ctypes.c_int64()
        dp = ctypes.POINTER(ctypes.c_double)
        _check(lib().pso64_get_state(self.h, out["x"].ctypes.data_as(dp), out["v"].ctypes.data_as(dp),
                                     out["p"].ctypes.data_as(dp), out["pf"].ctypes.data_as(dp), ctypes.byref(gi),
                                     ctypes.byref(t)), "pso64_get_state")
        out["gbest_idx"], out["t"] = gi.value, t.value
        return out

    def close(self):
        if getattr(self, "h", None):
            _check(lib().pso64_destroy(self.h), "pso64_destroy")
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent swarms run by one persistent launch (pso_batch_*)."""

    def __init__(self, specs, stream=None):
        self.specs = list(specs)
        self._arr, self._keep = _descs(self.specs)
        self.h = ctypes.c_void_p()
        sp = None if stream is None else ctypes.c_void_p(int(stream.cuda_stream))
        _check(lib().pso_batch_create(self._arr, len(self.specs), sp, ctypes.byref(self.h)), "pso_batch_create")

    def launch(self):
        _check(lib().pso_batch_launch(self.h), "pso_batch_launch")

    @property
    def shape(self):
        """Current tiles and schedule: dict(lanes, grid, part_work, stage_kib)."""
        sh = _native.PsoBatchShape()
        _check(lib().pso_batch_get_shape(self.h, ctypes.byref(sh)), "pso_batch_get_shape")
        return dict(lanes=sh.lanes, grid=sh.grid, part_work=sh.part_work, stage_kib=sh.stage_kib)

    def set_shape(self, lanes, grid=0, part_work=1 << 17, stage_kib=0):
        """stage_kib > 0: each part's state in that many KiB of LDS for a
        whole launch (lanes 256, 512 or 1024); 0: streamed from device memory."""
        sh = _native.PsoBatchShape(int(lanes), int(grid), int(part_work), int(stage_kib), 0)
        _check(lib().pso_batch_set_shape(self.h, ctypes.byref(sh)), "pso_batch_set_shape")

    def autotune(self, probe_iters=8):
        """Times every candidate shape on probe_iters iterations and keeps
        the fastest (pso_batch_autotune); returns it."""
        sh = _native.PsoBatchShape()
        _check(lib().pso_batch_autotune(self.h, int(probe_iters), ctypes.byref(sh)), "pso_batch_autotune")
        return dict(lanes=sh.lanes, grid=sh.grid, part_work=sh.part_work, stage_kib=sh.stage_kib)

    def results(self, positions=True):
        n = len(self.specs)
        res = (_native.PsoResult * n)()
        pos = [np.empty(int(sp.D), np.float32) for sp in self.specs] if positions else None
        for k in range(n):
            res[k].gbest_pos = pos[k].ctypes.data if positions else None
        _check(lib().pso_batch_results(self.h, res), "pso_batch_results")
        out = []
        for k in range(n):
            out.append(dict(gbest_fit=np.float32(res[k].gbest_value), gbest_iter=res[k].gbest_iter,
                            iters=res[k].iters, gbest_pos=pos[k] if positions else None))
        return out

    def close(self):
        if getattr(self, "h", None):
            _check(lib().pso_batch_destroy(self.h), "pso_batch_destroy")
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Request server with continuous batching (pso_server_*)."""

    def __init__(self, mem_budget: int, chunk_updates: int = 0):
        self.h = ctypes.c_void_p()
        _check(lib().pso_server_create(int(mem_budget), int(chunk_updates), ctypes.byref(self.h)),
               "pso_server_create")
        self._D = {}

    def submit(self, spec) -> int:
        arr, keep = _descs([spec])
        t = ctypes.c_uint64()
        _check(lib().pso_server_submit(self.h, arr, ctypes.byref(t)), "pso_server_submit")
        self._D[t.value] = int(spec.D)
        return t.value

    def poll(self, ticket):
        """None while pending; else dict(gbest_fit, gbest_pos, gbest_iter, iters, latency_ms)."""
        D = self._D.get(ticket, 0)
        res = _native.PsoResult()
        pos = np.empty(D, np.float32)
        res.gbest_pos = pos.ctypes.data if D else None
        lat = ctypes.c_double()
        rc = lib().pso_server_poll(self.h, ticket, ctypes.byref(res), ctypes.byref(lat))
        if rc == PSO_EAGAIN:
            return None
        self._D.pop(ticket, None)
        _check(rc, "pso_server_poll")
        return dict(gbest_fit=np.float32(res.gbest_value), gbest_pos=pos, gbest_iter=res.gbest_iter,
                    iters=res.iters, latency_ms=lat.value)

    def cancel(self, ticket):
        _check(lib().pso_server_cancel(self.h, int(ticket)), "pso_server_cancel")

    def set_deadline(self, ticket, timeout_ms):
        _check(lib().pso_server_set_deadline(self.h, int(ticket), float(timeout_ms)), "pso_server_set_deadline")

    def stats(self):
        c = _native.PsoServerCounters()
        _check(lib().pso_server_stats(self.h, ctypes.byref(c)), "pso_server_stats")
        return {f: getattr(c, f) for f, _ in c._fields_}

    def close(self):
        if getattr(self, "h", None):
            _check(lib().pso_server_destroy(self.h), "pso_server_destroy")
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pso_batch_run(specs):
    with Batch(specs) as b:
        b.launch()
        return b.results()


def _run_descs(fn, specs, *extra):
    specs = list(specs)
    arr, keep = _descs(specs)
    n = len(specs)
    res = (_native.PsoResult * n)()
    pos = [np.empty(int(sp.D), np.float32) for sp in specs]
    for k in range(n):
        res[k].gbest_pos = pos[k].ctypes.data
    _check(getattr(lib(), fn)(arr, n, res, *extra), fn)
    del keep
    return [dict(gbest_fit=np.float32(res[k].gbest_value), gbest_iter=res[k].gbest_iter, iters=res[k].iters,
                 gbest_pos=pos[k]) for k in range(n)]


def pso_batch_run_c(specs):
    """The C call pso_batch_run (create, launch, results, destroy in one)."""
    return _run_descs("pso_batch_run", specs)


def pso_batch_run_static(specs, stream=None):
    """pso_batch_run_static: the same batch with every device buffer in the
    library's fixed per-device scratch (no allocation); `stream` is a torch
    stream or None for the device's null stream."""
    sp = None if stream is None else ctypes.c_void_p(int(stream.cuda_stream))
    return _run_descs("pso_batch_run_static", specs, sp)


class Swarm:
    """One swarm on the GPU: owns its handle; parameters as in Table 1."""

    def __init__(self, fitness, N, D, bounds, w, c1, c2, vmax, seed, shift=None, variant=PSO_SYNC,
                 workspace=None, stream=None):
        self.N, self.D = int(N), int(D)
        if workspace is None:
            self.h = pso_create(fitness, N, D, bounds, w, c1, c2, vmax, seed)
        else:
            # torch tensor (device memory) + torch stream
            self._ws = workspace
            sp = 0 if stream is None else int(stream.cuda_stream)
            self.h = pso_create_in(fitness, N, D, bounds, w, c1, c2, vmax, seed, int(workspace.data_ptr()),
                                   int(workspace.numel() * workspace.element_size()), sp)
        if shift is not None:
            pso_set_shift(self.h, shift)
        if variant != PSO_SYNC:
            pso_set_variant(self.h, variant)

    def set_max_lead(self, max_lead):
        pso_set_max_lead(self.h, max_lead)

    def step(self, n=1):
        for _ in range(n):
            pso_step(self.h)

    def run(self, max_iter, tol=0.0, f_star=0.0):
        return pso_run(self.h, max_iter, self.D, tol, f_star)

    def reset(self):
        pso_reset(self.h)

    def best(self):
        return pso_get_best(self.h, self.D)

    def history(self, t0, count):
        return pso_get_history(self.h, t0, count)

    def state(self):
        return pso_get_state(self.h, self.N, self.D)

    def set_state(self, st):
        pso_set_state(self.h, st)

    def sync(self):
        pso_sync(self.h)

    def counters(self):
        return pso_get_counters(self.h)

    def async_counters(self):
        return pso_get_async_counters(self.h)

    def close(self):
        if getattr(self, "h", None):
            pso_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
