"""pso_run of a swarm small enough for one workgroup: its whole state staged
in that workgroup's LDS for the run (the default where it fits) against the
one-workgroup run that reads it from device memory every iteration
(PSO_BLOCK_STAGED=0) and against the oracle -- bit for bit: the state, the
gbest, its iteration, the per-iteration history, the pbest improvement count
and the stop rule, across runs that continue each other."""
import numpy as np
import pytest

import paper_2205_01313_amd as pso
from paper_2205_01313_amd import workloads as wl
from tests.gpu_util import announce, assert_state_equal, gpu_swarm, oracle_swarm

pytestmark = pytest.mark.gpu


def run_twice(spec, T, tol, f_star):
    with gpu_swarm(spec) as g:
        r1 = g.run(T // 3, tol=tol, f_star=f_star)
        r2 = g.run(T - T // 3, tol=tol, f_star=f_star)
        st = g.state()
        t = st["t"]
        hist = g.history(1, t) if t > 0 else np.zeros(0, np.uint64)
        return r1, r2, st, hist, g.counters()["pbest_improvements"]


@pytest.mark.parametrize("fit,N,D", [("sphere", 1024, 2), ("rastrigin", 300, 17), ("ackley", 1000, 33),
                                     ("rosenbrock", 77, 64), ("cubic", 4097, 1), ("sphere", 1, 1),
                                     ("rastrigin", 2047, 3)])
def test_staged_block_run_equals_streamed_and_oracle(monkeypatch, fit, N, D):
    T = 90
    spec = wl.SwarmSpec(fit, N, D, T, seed=N * 7 + D, shift_amplitude=2.0)
    tol, f_star = (1e-3, 0.0) if fit == "sphere" else (0.0, 0.0)
    announce(f"staged one-workgroup run {fit} N={N} D={D}")
    monkeypatch.setenv("PSO_GANG", "0")  # the one-workgroup run, where a gang would overtake it
    monkeypatch.delenv("PSO_BLOCK_STAGED", raising=False)
    s1, s2, st, hist, imp = run_twice(spec, T, tol, f_star)
    monkeypatch.setenv("PSO_BLOCK_STAGED", "0")
    q1, q2, qt, qhist, qimp = run_twice(spec, T, tol, f_star)
    for a, b in ((s1, q1), (s2, q2)):
        assert a["gbest_fit"] == b["gbest_fit"] and a["gbest_iter"] == b["gbest_iter"] and a["iters"] == b["iters"]
        assert np.array_equal(a["gbest_pos"], b["gbest_pos"])
    assert st["t"] == qt["t"] and st["gkey"] == qt["gkey"]
    assert np.array_equal(hist, qhist) and imp == qimp
    assert_state_equal(st, qt, N, D)
    o = oracle_swarm(spec, 8).run_f32(T, tol=tol, f_star=f_star)
    assert s1["iters"] + s2["iters"] == o["iters"] and s2["gbest_fit"] == o["gbest_fit"]
    assert s2["gbest_iter"] == o["giter"] and np.array_equal(s2["gbest_pos"], o["gpos"])


@pytest.mark.parametrize("fit,N,D", [("cubic", 16384, 1), ("sphere", 9000, 2), ("rastrigin", 20001, 1),
                                     ("rosenbrock", 12000, 2), ("ackley", 65536, 2), ("rastrigin", 16384, 8),
                                     ("rosenbrock", 9000, 5), ("ackley", 20000, 16), ("sphere", 30001, 3),
                                     ("cubic", 4097, 1), ("rastrigin", 2049, 4)])
def test_gang_run_equals_step_launches_and_oracle(monkeypatch, fit, N, D):
    """Swarms with D <= 16 too large for one workgroup's LDS run as a gang of
    co-resident workgroups (one particle per lane, a step-tagged meeting per
    iteration): the same bits as the graph-replayed step launches (PSO_GANG=0)
    and as the oracle, across runs that continue each other."""
    T = 90
    spec = wl.SwarmSpec(fit, N, D, T, seed=N * 5 + D, shift_amplitude=2.0)
    tol, f_star = (1e-3, 0.0) if fit == "sphere" else (0.0, 0.0)
    announce(f"gang run {fit} N={N} D={D}")
    monkeypatch.delenv("PSO_GANG", raising=False)
    s1, s2, st, hist, imp = run_twice(spec, T, tol, f_star)
    monkeypatch.setenv("PSO_GANG", "0")
    q1, q2, qt, qhist, qimp = run_twice(spec, T, tol, f_star)
    for a, b in ((s1, q1), (s2, q2)):
        assert a["gbest_fit"] == b["gbest_fit"] and a["gbest_iter"] == b["gbest_iter"] and a["iters"] == b["iters"]
        assert np.array_equal(a["gbest_pos"], b["gbest_pos"])
    assert st["t"] == qt["t"] and st["gkey"] == qt["gkey"]
    assert np.array_equal(hist, qhist) and imp == qimp
    assert_state_equal(st, qt, N, D)
    o = oracle_swarm(spec, 8).run_f32(T, tol=tol, f_star=f_star)
    assert s1["iters"] + s2["iters"] == o["iters"] and s2["gbest_fit"] == o["gbest_fit"]
    assert s2["gbest_iter"] == o["giter"] and np.array_equal(s2["gbest_pos"], o["gpos"])
