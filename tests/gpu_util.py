"""Helpers shared by the GPU tests: run the same swarm on the GPU (through
the C ABI) and in the oracle, and compare."""
import numpy as np

import oracle
import paper_2205_01313_amd as pso


def oracle_swarm(spec, nthreads=0):
    return oracle.Swarm(spec.fitness, spec.N, spec.D, spec.lo, spec.hi, spec.w, spec.c1, spec.c2, spec.vmax,
                        spec.seed, shift=spec.shift, nthreads=nthreads)


def gpu_swarm(spec, variant=pso.PSO_SYNC):
    return pso.Swarm(spec.fitness, spec.N, spec.D, (spec.lo, spec.hi), spec.w, spec.c1, spec.c2, spec.vmax,
                     spec.seed, shift=spec.shift, variant=variant)


def announce(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def assert_state_equal(g, o, N, D, cols=None):
    """Bit-exact comparison of x, v, p, pf, gbest position (optionally on a
    subset of particle columns)."""
    for k in ("x", "v", "p"):
        a = g[k].reshape(D, N)
        b = o[k].reshape(D, N)
        if cols is not None:
            a, b = a[:, cols], b[:, cols]
        bad = np.argwhere(a.view(np.uint32) != b.view(np.uint32))
        assert bad.size == 0, f"{k} differs at (d, i) {bad[:5].tolist()}: {a[tuple(bad[0])]} vs {b[tuple(bad[0])]}"
    a, b = (g["pf"], o["pf"]) if cols is None else (g["pf"][cols], o["pf"][cols])
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), "pf differs"
    assert np.array_equal(g["gpos"].view(np.uint32), o["gpos"].view(np.uint32)), "gbest position differs"
