"""GPU parity of the synchronous gbest PSO step against the oracle.

The synchronous path computes exactly the oracle's binary32 definition, so
the comparison is bit for bit: the gbest key of every iteration (fitness and
index), the iteration of the last gbest change, and the full state
(x, v, pbest position, pbest fitness, gbest position)."""
import numpy as np
import pytest

import paper_2205_01313_amd as pso
from paper_2205_01313_amd import workloads as wl
from tests.gpu_util import announce, assert_state_equal, gpu_swarm, oracle_swarm

pytestmark = pytest.mark.gpu


def run_both(spec, T, nthreads=0, compare_state=True):
    announce(f"{spec.fitness} N={spec.N} D={spec.D} T={T} seed={spec.seed}")
    o = oracle_swarm(spec, nthreads).run_f32(T)
    with gpu_swarm(spec) as g:
        r = g.run(T)
        hist = g.history(0, T + 1)
        st = g.state()
    bad = np.flatnonzero(hist != o["hist"])
    assert bad.size == 0, f"gbest key differs first at iteration {bad[0]}: {hist[bad[0]]:x} vs {o['hist'][bad[0]]:x}"
    assert r["iters"] == T and st["t"] == T
    assert r["gbest_iter"] == o["giter"]
    assert r["gbest_fit"] == o["gbest_fit"]
    assert st["gkey"] == o["gkey"]
    if compare_state:
        assert_state_equal(st, o, spec.N, spec.D)
    return o, st


def test_small_sphere_full_run():
    """Sphere D=2, N=1024, 1000 iterations, seed 0: whole trajectory."""
    o, st = run_both(wl.small_sphere(), 1000)
    assert o["gbest_fit"] < 1e-10


@pytest.mark.parametrize("fit", wl.FITNESS_NAMES)
@pytest.mark.parametrize("N,D", [(1, 3), (63, 1), (257, 2), (1000, 7), (4099, 32), (777, 33), (300, 70)])
def test_ragged_shapes_all_fitness(fit, N, D):
    if fit == "rosenbrock" and D < 2:
        pytest.skip("Rosenbrock needs D >= 2")
    spec = wl.SwarmSpec(fit, N, D, 40, seed=N * 31 + D, shift_amplitude=2.0)
    run_both(spec, 40, nthreads=8)


def test_golden_rastrigin_trajectory():
    """Same run as tests/golden/rastrigin_d32_n4096_t50_seed1.txt."""
    from tests.test_oracle_golden import load
    giter, hist = load("rastrigin_d32_n4096_t50_seed1.txt")
    spec = wl.SwarmSpec("rastrigin", 4096, 32, 50, seed=1, box=(-5.12, 5.12), vmax=1.024)
    announce("golden rastrigin N=4096 D=32 T=50")
    with gpu_swarm(spec) as g:
        r = g.run(50)
        h = g.history(0, 51)
    assert np.array_equal(h, hist)
    assert r["gbest_iter"] == giter


@pytest.mark.parametrize("seed", [0, 1])
def test_large_rastrigin_full_run(seed):
    """The benchmark's workload in full -- Rastrigin D=32, N=2^20, all 200
    iterations (Alg. 1 Steps 2-5 with the per-iteration gbest of Sec. 2.2)
    -- for seeds 0 and 1: the gbest key of every iteration, the iteration of
    the last change and the final x, v, pbest position, pbest fitness and
    gbest position, bit for bit."""
    spec = wl.large_rastrigin(seed=seed)
    run_both(spec, spec.T, nthreads=16)


@pytest.mark.parametrize("mk", [wl.deep_rosenbrock, wl.deep_ackley])
def test_deep_d128_full_run(mk):
    """Rosenbrock and shifted Ackley, D=128, N=65536, all 2000 iterations
    (the split step): the whole trajectory and the final state, bit for bit."""
    spec = mk(seed=0)
    run_both(spec, spec.T, nthreads=16)


@pytest.mark.parametrize("split,phases", [("0", None), ("1", None), ("1", "1"), ("1", "2")])
@pytest.mark.parametrize("fit", wl.FITNESS_NAMES)
@pytest.mark.parametrize("N,D", [(4099, 16), (2050, 17), (3001, 33), (1025, 130), (701, 200), (129, 512)])
def test_split_and_plain_steps_equal_oracle(monkeypatch, split, phases, fit, N, D):
    """The step launched per iteration, forced onto the plain kernel (four
    particles per lane) or the split kernel (lanes share a particle's
    dimensions, terms folded in order from LDS), the latter in one phase or
    in two (each half of the dimensions staged and folded in turn, the
    running sum carried over): all bit-exact against the oracle, over ragged
    particle counts, odd D, one to 64 chunks per quad."""
    monkeypatch.setenv("PSO_STEP_SPLIT", split)
    if phases is not None:
        monkeypatch.setenv("PSO_SPLIT_PHASES", phases)
    T = 30
    spec = wl.SwarmSpec(fit, N, D, T, seed=N + 7 * D, shift_amplitude=2.0)
    announce(f"split={split} phases={phases} {fit} N={N} D={D} T={T}")
    o = oracle_swarm(spec, 8).run_f32(T)
    with gpu_swarm(spec) as g:
        g.step(T)
        hist = g.history(0, T + 1)
        st = g.state()
        b = g.best()
    bad = np.flatnonzero(hist != o["hist"])
    assert bad.size == 0, f"gbest key differs first at iteration {bad[0]}"
    assert b["gbest_iter"] == o["giter"] and st["t"] == T
    assert_state_equal(st, o, N, D)


@pytest.mark.parametrize("fit", wl.FITNESS_NAMES)
@pytest.mark.parametrize("N,D", [(4099, 16), (2050, 17), (3001, 33), (1025, 130), (701, 200), (129, 512),
                                 (1000, 128), (70, 3)])
def test_one_particle_per_lane_step_equals_oracle(monkeypatch, fit, N, D):
    """The step with one particle per lane and the rows of the next dimension
    pairs loaded ahead (forced with PSO_STEP_ONE=1): bit-exact against the
    oracle over ragged particle counts and odd D, including a D fixed at
    compile time (128) and a prefetch ring longer than the dimension pairs."""
    if fit == "rosenbrock" and D < 2:
        pytest.skip("Rosenbrock needs D >= 2")
    monkeypatch.setenv("PSO_STEP_ONE", "1")
    T = 30
    spec = wl.SwarmSpec(fit, N, D, T, seed=3 * N + D, shift_amplitude=2.0)
    announce(f"one particle per lane {fit} N={N} D={D} T={T}")
    o = oracle_swarm(spec, 8).run_f32(T)
    with gpu_swarm(spec) as g:
        g.step(T)
        hist = g.history(0, T + 1)
        st = g.state()
        b = g.best()
    bad = np.flatnonzero(hist != o["hist"])
    assert bad.size == 0, f"gbest key differs first at iteration {bad[0]}"
    assert b["gbest_iter"] == o["giter"] and st["t"] == T
    assert_state_equal(st, o, N, D)


def test_step_by_step_equals_run():
    spec = wl.SwarmSpec("ackley", 3000, 9, 25, seed=5, shift_amplitude=3.0)
    announce("step vs run")
    with gpu_swarm(spec) as a, gpu_swarm(spec) as b:
        a.run(25)
        for _ in range(25):
            b.step()
        sa, sb = a.state(), b.state()
    for k in ("x", "v", "p", "pf", "gpos"):
        assert np.array_equal(sa[k], sb[k]), k
    assert sa["gkey"] == sb["gkey"] and sa["giter"] == sb["giter"] and sa["t"] == sb["t"] == 25


def test_stop_rule_matches_oracle():
    spec = wl.SwarmSpec("sphere", 2048, 4, 600, seed=7)
    announce("stop rule")
    o = oracle_swarm(spec).run_f32(600, tol=1e-4, f_star=0.0)
    assert o["iters"] < 600
    with gpu_swarm(spec) as g:
        r = g.run(600, tol=1e-4, f_star=0.0)
        st = g.state()
        # a second run with the rule already met runs nothing
        r2 = g.run(50, tol=1e-4, f_star=0.0)
    assert r["iters"] == o["iters"]
    assert r["gbest_fit"] == o["gbest_fit"] and r["gbest_iter"] == o["giter"]
    assert np.array_equal(r["gbest_pos"], o["gpos"])
    assert_state_equal(st, o, spec.N, spec.D)
    assert r2["iters"] == 0


def test_checkpoint_resume_repeats_uninterrupted_run():
    spec = wl.SwarmSpec("rastrigin", 5000, 12, 30, seed=11)
    announce("checkpoint/resume")
    with gpu_swarm(spec) as a:
        a.run(30)
        full = a.state()
    with gpu_swarm(spec) as b:
        b.run(17)
        ck = b.state()
    with gpu_swarm(wl.SwarmSpec("rastrigin", 5000, 12, 30, seed=11)) as c:
        c.set_state(ck)
        c.run(13)
        res = c.state()
    for k in ("x", "v", "p", "pf", "gpos"):
        assert np.array_equal(res[k], full[k]), k
    assert res["gkey"] == full["gkey"] and res["giter"] == full["giter"] and res["t"] == 30


def test_reset_repeats_and_shift_reinitialises():
    spec = wl.SwarmSpec("ackley", 1500, 6, 20, seed=2, shift_amplitude=4.0)
    announce("reset/shift")
    with gpu_swarm(spec) as g:
        g.run(20)
        a = g.state()
        g.reset()
        g.run(20)
        b = g.state()
        pso.pso_set_shift(g.h, None)
        s0 = g.state()
    for k in ("x", "v", "p", "pf", "gpos"):
        assert np.array_equal(a[k], b[k]), k
    assert s0["t"] == 0
    o = oracle_swarm(wl.SwarmSpec("ackley", 1500, 6, 0, seed=2)).run_f32(0)
    assert_state_equal(s0, o, 1500, 6)


def test_caller_workspace_and_torch_stream():
    import torch
    spec = wl.SwarmSpec("rosenbrock", 3333, 5, 30, seed=4)
    announce("pso_create_in with torch memory and stream")
    nbytes = pso.pso_workspace_bytes(spec.N, spec.D)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    o = oracle_swarm(spec).run_f32(30)
    g = pso.Swarm(spec.fitness, spec.N, spec.D, spec.box, spec.w, spec.c1, spec.c2, spec.vmax, spec.seed,
                  workspace=ws, stream=stream)
    try:
        g.run(30)
        st = g.state()
    finally:
        g.close()
    assert st["gkey"] == o["gkey"]
    assert_state_equal(st, o, spec.N, spec.D)


def test_large_seed_and_single_particle():
    spec = wl.SwarmSpec("cubic", 1, 1, 50, seed=(1 << 63) + 12345)
    run_both(spec, 50)


def test_history_window_errors():
    spec = wl.SwarmSpec("sphere", 64, 2, 5, seed=0)
    with gpu_swarm(spec) as g:
        g.run(5)
        with pytest.raises(pso.PsoError) as e:
            g.history(0, 7)
        assert e.value.code == pso.PSO_ESTATE


def test_improvement_counter_matches_oracle():
    """pso_get_counters counts Step 4 improvements; the oracle's count is the
    number of pf decreases over the same iterations (grid and one-workgroup
    paths)."""
    for spec in (wl.SwarmSpec("rastrigin", 70000, 6, 15, seed=8), wl.SwarmSpec("ackley", 900, 5, 15, seed=8)):
        osw = oracle_swarm(spec, nthreads=16)
        st = osw.init_f32()
        n = 0
        for t in range(1, spec.T + 1):
            prev = st["pf"].copy()
            osw.step_f32(st, t)
            n += int(np.count_nonzero(st["pf"] < prev))
        with gpu_swarm(spec) as g:
            g.run(spec.T)
            assert g.counters()["pbest_improvements"] == n


@pytest.mark.parametrize("variant", [pso.PSO_REDUCE, pso.PSO_REDUCE_UNROLLED])
@pytest.mark.parametrize("fit,N,D", [("rastrigin", 70001, 32), ("cubic", 2048, 1), ("ackley", 5000, 7)])
def test_two_kernel_reduction_comparator_equals_oracle(variant, fit, N, D):
    """The paper's parallel-reduction comparator (two kernels per iteration)
    computes exactly the synchronous gbest PSO."""
    spec = wl.SwarmSpec(fit, N, D, 30, seed=N + D, shift_amplitude=1.0)
    announce(f"reduction comparator variant={variant} {fit} N={N} D={D}")
    o = oracle_swarm(spec, nthreads=16).run_f32(spec.T)
    with gpu_swarm(spec, variant=variant) as g:
        r = g.run(spec.T)
        h = g.history(0, spec.T + 1)
        st = g.state()
    assert np.array_equal(h, o["hist"])
    assert r["gbest_iter"] == o["giter"]
    assert_state_equal(st, o, spec.N, spec.D)


@pytest.mark.parametrize("fit,N,D", [("cubic", 16384, 1), ("rastrigin", 30000, 5), ("ackley", 5000, 40)])
def test_run_graph_replays_equal_oracle_and_direct_launches(monkeypatch, fit, N, D):
    """pso_run replays a captured graph of step launches: several pso_run
    calls (each several replays plus direct launches), eager pso_step work
    and host synchronisations between them, with and without the stop rule;
    after each call the whole gbest trajectory so far equals the oracle's, and
    the final state equals the same calls with every step launched directly
    (PSO_RUN_GRAPH=0)."""
    spec = wl.SwarmSpec(fit, N, D, 200, seed=N + D, shift_amplitude=1.0)
    announce(f"run graph {fit} N={N} D={D}")
    o = oracle_swarm(spec, 16).run_f32(129)
    states = {}
    for mode in ("1", "0"):
        monkeypatch.setenv("PSO_RUN_GRAPH", mode)
        with gpu_swarm(spec) as g:
            t = 0
            for n, eager in ((37, 3), (40, 0), (17, 5), (24, 3)):
                r = g.run(n)
                t += n
                assert r["iters"] == n
                assert np.array_equal(g.history(0, t + 1), o["hist"][: t + 1]), (mode, t)
                g.step(eager)
                g.sync()
                t += eager
                assert np.array_equal(g.history(0, t + 1), o["hist"][: t + 1]), (mode, t)
            states[mode] = g.state()
            assert states[mode]["t"] == 129
        assert_state_equal(states[mode], o, N, D)
    # the stop rule over replays: the same stopping iteration as the oracle
    monkeypatch.setenv("PSO_RUN_GRAPH", "1")
    f_star = float(o["gbest_fit"])
    tol = abs(f_star) * 1e-5 + 1e-6
    os_ = oracle_swarm(spec, 16).run_f32(200, tol=tol, f_star=f_star)
    assert os_["iters"] <= 129
    with gpu_swarm(spec) as g:
        r = g.run(200, tol=tol, f_star=f_star)
    assert r["iters"] == os_["iters"] and r["gbest_fit"] == os_["gbest_fit"]
