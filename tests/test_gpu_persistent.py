"""Fully asynchronous persistent variant (PSO_PERSISTENT): one launch runs
every iteration of a pso_run, each workgroup iterating its own particles with
no barrier between iterations.  Its trajectory is not deterministic, so it is
judged as the asynchronous variant is: invariants that every correct run
satisfies (checked after runs with unbounded, small and zero staleness),
the stop rule, and the final-fitness distribution against the synchronous
variant."""
import numpy as np
import pytest

import oracle
import paper_2205_01313_amd as pso
from paper_2205_01313_amd import workloads as wl
from tests.gpu_util import announce, gpu_swarm, oracle_swarm
from tests.test_gpu_async import check_invariants

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("fit,N,D", [("rastrigin", 1, 3), ("sphere", 1000, 5), ("ackley", 30000, 17),
                                     ("rosenbrock", 300000, 8), ("cubic", 4097, 1)])
@pytest.mark.parametrize("lead", [0, 3, 1 << 40])
def test_invariants_after_persistent_runs(fit, N, D, lead):
    spec = wl.SwarmSpec(fit, N, D, 40, seed=N + D, shift_amplitude=1.0)
    announce(f"persistent {fit} N={N} D={D} lead={lead}")
    osw = oracle_swarm(spec, nthreads=16)
    with gpu_swarm(spec, variant=pso.PSO_PERSISTENT) as g:
        g.set_max_lead(lead)
        prev = g.state()
        r = g.run(25)
        st = g.state()
        assert r["iters"] == 25 and st["t"] == 25
        check_invariants(spec, st, prev, osw)
        assert r["gbest_fit"] == oracle.key_value(st["gkey"])
        assert 0 <= r["gbest_iter"] <= 25
        # the history: non-increasing, ending at the run's gbest
        h = g.history(1, 25)
        assert np.all(h[1:] <= h[:-1]) and h[-1] == st["gkey"]
        # a second run continues the iteration count; pso_step runs one
        r2 = g.run(10)
        g.step()
        st2 = g.state()
        assert r2["iters"] == 10 and st2["t"] == 36
        check_invariants(spec, st2, st, None)
        h2 = g.history(1, 36)
        assert np.all(h2[1:] <= h2[:-1]) and h2[-1] == st2["gkey"]


def test_persistent_stop_rule():
    spec = wl.SwarmSpec("sphere", 200000, 4, 2000, seed=2)
    announce("persistent stop rule")
    with gpu_swarm(spec, variant=pso.PSO_PERSISTENT) as g:
        r = g.run(2000, tol=1e-3, f_star=0.0)
        st = g.state()
    assert r["gbest_fit"] < 1e-3 and r["iters"] < 2000
    assert oracle.key_value(st["gkey"]) == st["pf"].min()


def test_persistent_reaches_the_synchronous_quality():
    """Rastrigin D=32, N=2^18, 200 iterations, 8 seeds: medians of the final
    fitness within a factor of 1.5 of the synchronous variant's."""
    fs = {pso.PSO_SYNC: [], pso.PSO_PERSISTENT: []}
    for variant in fs:
        for seed in range(8):
            spec = wl.SwarmSpec("rastrigin", 1 << 18, 32, 200, seed=seed, box=(-5.12, 5.12), vmax=1.024)
            with gpu_swarm(spec, variant=variant) as g:
                fs[variant].append(float(g.run(spec.T)["gbest_fit"]))
    s, a = np.array(fs[pso.PSO_SYNC]), np.array(fs[pso.PSO_PERSISTENT])
    print(f"\nsync {np.percentile(s, [0, 50, 100])}  persistent {np.percentile(a, [0, 50, 100])}")
    assert np.all(np.isfinite(a))
    assert np.median(a) <= 1.5 * np.median(s) and np.median(s) <= 1.5 * np.median(a)
