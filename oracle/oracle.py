"""ctypes binding of the C oracle in pso_oracle.c (test infrastructure).

The oracle is a plain CPU implementation of cuPSO's global-best PSO (Wang et
al., SAC'22): Step 1 initialisation and Steps 2-5 of Alg. 1 (Sec. 2.1, Eq. 1
and Eq. 2), with the global best synchronised once per iteration as in the
parallel PSO of Sec. 2.2.  Only tests, the smoke check and the benchmark's CPU
baseline use it; the GPU library shares no code with it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pso_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

FITNESS = {"sphere": 0, "rastrigin": 1, "rosenbrock": 2, "ackley": 3, "cubic": 4}
TAG_VEL = 0
TAG_INIT = 1

CFLAGS = ["-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(out: str = LIB, src: str = SRC) -> str:
    """Compile pso_oracle.c with gcc into liboracle.so."""
    tmp = out + ".tmp"
    subprocess.run(["gcc", *CFLAGS, src, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, out)
    return out


class Problem(ctypes.Structure):
    _fields_ = [
        ("fitness_id", ctypes.c_int32),
        ("D", ctypes.c_int32),
        ("N", ctypes.c_int64),
        ("lo", ctypes.c_float),
        ("hi", ctypes.c_float),
        ("w", ctypes.c_float),
        ("c1", ctypes.c_float),
        ("c2", ctypes.c_float),
        ("vmax", ctypes.c_float),
        ("seed", ctypes.c_uint64),
        ("shift", ctypes.c_void_p),
        ("nthreads", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("PSO_ORACLE_LIB", LIB)
        if path == LIB and not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(path)
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        L.oracle_philox4x32_10.argtypes = [P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32)]
        L.oracle_uniform_f32.argtypes = [ctypes.c_uint32]
        L.oracle_uniform_f32.restype = ctypes.c_float
        L.oracle_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                  ctypes.c_int32, P(ctypes.c_float)]
        L.oracle_cospi_f32.argtypes = [ctypes.c_float]
        L.oracle_cospi_f32.restype = ctypes.c_float
        L.oracle_exp_f32.argtypes = [ctypes.c_float]
        L.oracle_exp_f32.restype = ctypes.c_float
        L.oracle_cospi_f32_array.argtypes = [vp, vp, ctypes.c_int64]
        L.oracle_exp_f32_array.argtypes = [vp, vp, ctypes.c_int64]
        L.oracle_fitness_f32_batch.argtypes = [P(Problem), vp, ctypes.c_int64, vp]
        L.oracle_fitness_f64_batch.argtypes = [P(Problem), vp, ctypes.c_int64, vp]
        L.oracle_key_f32.argtypes = [ctypes.c_float, ctypes.c_uint32]
        L.oracle_key_f32.restype = ctypes.c_uint64
        L.oracle_key_value_f32.argtypes = [ctypes.c_uint64]
        L.oracle_key_value_f32.restype = ctypes.c_float
        L.oracle_constants_f32.argtypes = [P(ctypes.c_float)]
        L.oracle_key_f32_array.argtypes = [vp, vp, vp, ctypes.c_int64]
        L.oracle_init_f32.argtypes = [P(Problem), vp, vp, vp, vp, vp, P(ctypes.c_uint64)]
        L.oracle_step_f32.argtypes = [P(Problem), ctypes.c_uint64, vp, vp, vp, vp, vp, P(ctypes.c_uint64)]
        L.oracle_step_f32.restype = ctypes.c_int
        L.oracle_step_serial_immediate_f32.argtypes = L.oracle_step_f32.argtypes
        L.oracle_step_serial_immediate_f32.restype = ctypes.c_int
        L.oracle_run_f32.argtypes = [P(Problem), ctypes.c_int64, ctypes.c_float, ctypes.c_float, ctypes.c_int,
                                     vp, vp, vp, vp, vp, vp, P(ctypes.c_int64)]
        L.oracle_run_f32.restype = ctypes.c_int64
        L.oracle_init_f64.argtypes = [P(Problem), vp, vp, vp, vp, vp, P(ctypes.c_int64)]
        L.oracle_step_f64.argtypes = [P(Problem), ctypes.c_uint64, vp, vp, vp, vp, vp, P(ctypes.c_int64)]
        L.oracle_step_f64.restype = ctypes.c_int
        L.oracle_run_f64.argtypes = [P(Problem), ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                     vp, vp, vp, vp, vp, vp, vp, P(ctypes.c_int64)]
        L.oracle_run_f64.restype = ctypes.c_int64
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def fitness_id(f) -> int:
    return FITNESS[f] if isinstance(f, str) else int(f)


class Swarm:
    """Parameters of one swarm (Table 1) plus the shift vector, in the form
    the oracle takes.  Keeps the shift array alive for the C side."""

    def __init__(self, fitness, N, D, lo, hi, w, c1, c2, vmax, seed, shift=None, nthreads=0):
        self.fitness_id = fitness_id(fitness)
        self.N, self.D = int(N), int(D)
        self.shift = None if shift is None else np.ascontiguousarray(shift, dtype=np.float32)
        if self.shift is not None:
            assert self.shift.shape == (self.D,)
        self.problem = Problem(self.fitness_id, self.D, self.N, lo, hi, w, c1, c2, vmax, int(seed),
                               None if self.shift is None else self.shift.ctypes.data, int(nthreads), 0)
        self.params = dict(fitness=self.fitness_id, N=self.N, D=self.D, lo=lo, hi=hi, w=w, c1=c1, c2=c2,
                           vmax=vmax, seed=int(seed))

    @property
    def pref(self):
        return ctypes.byref(self.problem)

    # ---- binary32 mode -------------------------------------------------
    def init_f32(self):
        N, D = self.N, self.D
        st = dict(x=np.empty(D * N, np.float32), v=np.empty(D * N, np.float32),
                  p=np.empty(D * N, np.float32), pf=np.empty(N, np.float32),
                  gpos=np.empty(D, np.float32))
        gk = ctypes.c_uint64(0)
        lib().oracle_init_f32(self.pref, _ptr(st["x"]), _ptr(st["v"]), _ptr(st["p"]), _ptr(st["pf"]),
                              _ptr(st["gpos"]), ctypes.byref(gk))
        st["gkey"] = gk.value
        return st

    def step_f32(self, st, t, serial_immediate=False):
        gk = ctypes.c_uint64(st["gkey"])
        fn = lib().oracle_step_serial_immediate_f32 if serial_immediate else lib().oracle_step_f32
        changed = fn(self.pref, int(t), _ptr(st["x"]), _ptr(st["v"]), _ptr(st["p"]), _ptr(st["pf"]),
                     _ptr(st["gpos"]), ctypes.byref(gk))
        st["gkey"] = gk.value
        return bool(changed)

    def run_f32(self, T, tol=0.0, f_star=0.0, serial_immediate=False):
        N, D = self.N, self.D
        out = dict(x=np.empty(D * N, np.float32), v=np.empty(D * N, np.float32),
                   p=np.empty(D * N, np.float32), pf=np.empty(N, np.float32),
                   gpos=np.empty(D, np.float32), hist=np.zeros(T + 1, np.uint64))
        giter = ctypes.c_int64(0)
        iters = lib().oracle_run_f32(self.pref, int(T), tol, f_star, int(serial_immediate),
                                     _ptr(out["x"]), _ptr(out["v"]), _ptr(out["p"]), _ptr(out["pf"]),
                                     _ptr(out["gpos"]), _ptr(out["hist"]), ctypes.byref(giter))
        out["hist"] = out["hist"][: iters + 1]
        out["iters"] = int(iters)
        out["giter"] = int(giter.value)
        out["gkey"] = int(out["hist"][-1])
        out["gbest_fit"] = key_value(out["gkey"])
        out["gbest_idx"] = out["gkey"] & 0xFFFFFFFF
        return out

    # ---- binary64 mode -------------------------------------------------
    def run_f64(self, T, tol=0.0, f_star=0.0):
        N, D = self.N, self.D
        out = dict(x=np.empty(D * N), v=np.empty(D * N), p=np.empty(D * N), pf=np.empty(N),
                   gpos=np.empty(D), hist_f=np.zeros(T + 1), hist_i=np.zeros(T + 1, np.int64))
        giter = ctypes.c_int64(0)
        iters = lib().oracle_run_f64(self.pref, int(T), tol, f_star, _ptr(out["x"]), _ptr(out["v"]),
                                     _ptr(out["p"]), _ptr(out["pf"]), _ptr(out["gpos"]), _ptr(out["hist_f"]),
                                     _ptr(out["hist_i"]), ctypes.byref(giter))
        out["hist_f"] = out["hist_f"][: iters + 1]
        out["hist_i"] = out["hist_i"][: iters + 1]
        out["iters"] = int(iters)
        out["giter"] = int(giter.value)
        out["gbest_fit"] = float(out["hist_f"][-1])
        out["gbest_idx"] = int(out["hist_i"][-1])
        return out

    # ---- fitness -------------------------------------------------------
    def fitness_f32(self, pts):
        """pts: (M, D) array of positions -> (M,) binary32 fitness."""
        pts = np.asarray(pts, np.float32)
        M = pts.shape[0]
        soa = np.ascontiguousarray(pts.T)
        out = np.empty(M, np.float32)
        lib().oracle_fitness_f32_batch(self.pref, _ptr(soa), M, _ptr(out))
        return out

    def fitness_f64(self, pts):
        pts = np.asarray(pts, np.float64)
        M = pts.shape[0]
        soa = np.ascontiguousarray(pts.T)
        out = np.empty(M, np.float64)
        lib().oracle_fitness_f64_batch(self.pref, _ptr(soa), M, _ptr(out))
        return out


def philox(key, ctr):
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    o = (ctypes.c_uint32 * 4)()
    lib().oracle_philox4x32_10(k, c, o)
    return tuple(o)


def uniform(u):
    return lib().oracle_uniform_f32(int(u))


def draw(seed, tag, t, i, d):
    o = (ctypes.c_float * 2)()
    lib().oracle_draw(int(seed), int(tag), int(t), int(i), int(d), o)
    return np.float32(o[0]), np.float32(o[1])


def cospi_f32(y):
    y = np.ascontiguousarray(y, np.float32)
    out = np.empty_like(y)
    lib().oracle_cospi_f32_array(_ptr(y), _ptr(out), y.size)
    return out


def exp_f32(x):
    x = np.ascontiguousarray(x, np.float32)
    out = np.empty_like(x)
    lib().oracle_exp_f32_array(_ptr(x), _ptr(out), x.size)
    return out


def constants():
    """COS_C (6), SIN_C (5), EXP_C (9), LN2_HI, LN2_LO, LOG2E of the built library."""
    o = (ctypes.c_float * 23)()
    lib().oracle_constants_f32(o)
    v = [float(t) for t in o]
    return dict(cos=v[0:6], sin=v[6:11], exp=v[11:20], ln2_hi=v[20], ln2_lo=v[21], log2e=v[22])


def key(f, i):
    return lib().oracle_key_f32(float(np.float32(f)), int(i))


def keys(f, idx):
    f = np.ascontiguousarray(f, np.float32)
    idx = np.ascontiguousarray(idx, np.uint32)
    out = np.empty(f.size, np.uint64)
    lib().oracle_key_f32_array(_ptr(f), _ptr(idx), _ptr(out), f.size)
    return out


def key_value(k):
    return np.float32(lib().oracle_key_value_f32(int(k)))
