"""Batches: many swarms of uneven N, D and fitness in one persistent launch.
Each swarm must compute exactly what it computes alone (pso_create +
pso_run, synchronous) -- bit for bit -- and the oracle's result."""
import numpy as np
import pytest

import paper_2205_01313_amd as pso
from paper_2205_01313_amd import workloads as wl
from tests.gpu_util import announce, gpu_swarm, oracle_swarm

pytestmark = pytest.mark.gpu


def mixed_specs(n, seed, max_iter=60):
    rng = np.random.default_rng(seed)
    specs = []
    for k in range(n):
        fit = wl.FITNESS_NAMES[int(rng.integers(0, 4))]
        N = int(np.exp(rng.uniform(np.log(1), np.log(3000))))
        D = int(rng.integers(1, 40))
        if fit == "rosenbrock":
            D = max(D, 2)
        sp = wl.SwarmSpec(fit, N, D, int(rng.integers(0, max_iter)), seed=int(rng.integers(0, 2**40)),
                          shift_amplitude=float(rng.uniform(0, 5)))
        if k % 5 == 0:
            sp.tol, sp.f_star = 1e-2, 0.0
        specs.append(sp)
    return specs


def alone(sp):
    with gpu_swarm(sp) as g:
        r = g.run(sp.T, tol=getattr(sp, "tol", 0.0), f_star=getattr(sp, "f_star", 0.0))
    return r


def test_batch_equals_each_swarm_alone():
    specs = mixed_specs(150, 1)
    announce("batch of 150 vs alone")
    res = pso.pso_batch_run(specs)
    for sp, r in zip(specs, res):
        a = alone(sp)
        assert r["gbest_fit"] == a["gbest_fit"], sp
        assert r["gbest_iter"] == a["gbest_iter"], sp
        assert r["iters"] == a["iters"], sp
        assert np.array_equal(r["gbest_pos"], a["gbest_pos"]), sp


def test_batch_equals_oracle():
    specs = mixed_specs(40, 2)
    announce("batch of 40 vs oracle")
    res = pso.pso_batch_run(specs)
    for sp, r in zip(specs, res):
        o = oracle_swarm(sp, nthreads=8).run_f32(sp.T, tol=getattr(sp, "tol", 0.0), f_star=getattr(sp, "f_star", 0.0))
        assert r["gbest_fit"] == o["gbest_fit"], sp
        assert r["gbest_iter"] == o["giter"] and r["iters"] == o["iters"], sp
        assert np.array_equal(r["gbest_pos"], o["gpos"]), sp


def test_batch_relaunch_repeats():
    specs = mixed_specs(64, 3)
    with pso.Batch(specs) as b:
        b.launch()
        r1 = b.results()
        b.launch()
        r2 = b.results()
    for a, c in zip(r1, r2):
        assert a["gbest_fit"] == c["gbest_fit"] and np.array_equal(a["gbest_pos"], c["gbest_pos"])


def test_batch_single_and_tiny():
    specs = [wl.SwarmSpec("sphere", 1, 1, 10, seed=3)]
    r = pso.pso_batch_run(specs)[0]
    o = oracle_swarm(specs[0]).run_f32(10)
    assert r["gbest_fit"] == o["gbest_fit"] and r["iters"] == 10


def test_batch_rejects_bad_descriptor():
    specs = [wl.SwarmSpec("sphere", 16, 2, 5), wl.SwarmSpec("rosenbrock", 16, 1, 5)]
    with pytest.raises(pso.PsoError) as e:
        pso.pso_batch_run(specs)
    assert e.value.code == pso.PSO_EINVAL and "descriptor 1" in str(e.value)


def test_large_swarms_split_into_parts_equal_alone_and_oracle():
    """Swarms large enough to be split over several workgroups (parts meet
    once per iteration) compute the same bits as alone and as the oracle."""
    specs = [wl.SwarmSpec("rastrigin", 50000, 16, 25, seed=1, shift_amplitude=1.0),
             wl.SwarmSpec("ackley", 20000, 33, 20, seed=2, shift_amplitude=2.0),
             wl.SwarmSpec("rosenbrock", 30001, 40, 15, seed=3),
             wl.SwarmSpec("sphere", 300, 4, 25, seed=4)]
    specs[1].tol, specs[1].f_star = 5.0, 0.0
    announce("batch with multi-part swarms")
    res = pso.pso_batch_run(specs)
    for sp, r in zip(specs, res):
        a = alone(sp)
        assert r["gbest_fit"] == a["gbest_fit"] and r["iters"] == a["iters"], sp
        assert r["gbest_iter"] == a["gbest_iter"] and np.array_equal(r["gbest_pos"], a["gbest_pos"]), sp
        o = oracle_swarm(sp, nthreads=16).run_f32(sp.T, tol=getattr(sp, "tol", 0.0), f_star=getattr(sp, "f_star", 0.0))
        assert r["gbest_fit"] == o["gbest_fit"] and np.array_equal(r["gbest_pos"], o["gpos"]), sp


def test_every_shape_and_the_autotuner_give_the_same_results():
    """Lanes 64/128/256, part sizes that split the large swarms, a small and the
    full grid: bit-identical results; the autotuner picks one of them and
    leaves the batch ready to run."""
    specs = mixed_specs(40, 21)
    specs += [wl.SwarmSpec("rastrigin", 6000, 48, 30, seed=900, shift_amplitude=1.0),
              wl.SwarmSpec("ackley", 9000, 20, 30, seed=901, shift_amplitude=1.0)]
    announce(f"batch shapes, {len(specs)} swarms")
    ref = None
    with pso.Batch(specs) as b:
        for lanes in (64, 128, 256):
            for grid, pw in ((0, 1 << 17), (7, 1 << 14)):
                b.set_shape(lanes, grid, pw)
                sh = b.shape
                assert sh["lanes"] == lanes and sh["part_work"] == pw and sh["grid"] >= 1
                b.launch()
                res = b.results()
                if ref is None:
                    ref = res
                for r, q in zip(res, ref):
                    assert r["gbest_fit"] == q["gbest_fit"] and r["gbest_iter"] == q["gbest_iter"]
                    assert np.array_equal(r["gbest_pos"], q["gbest_pos"])
        chosen = b.autotune(probe_iters=3)
        assert chosen["lanes"] in (64, 128, 256, 512, 1024) and chosen["grid"] >= 1
        b.launch()
        res = b.results()
    for r, q in zip(res, ref):
        assert r["gbest_fit"] == q["gbest_fit"] and np.array_equal(r["gbest_pos"], q["gbest_pos"])
    # the oracle agrees on two of them
    for k in (0, len(specs) - 1):
        o = oracle_swarm(specs[k], 8).run_f32(specs[k].T)
        assert ref[k]["gbest_fit"] == o["gbest_fit"] and ref[k]["gbest_iter"] == o["giter"]


@pytest.mark.parametrize("lanes,kib", [(512, 78), (1024, 78), (1024, 158)])
def test_lds_staged_shapes_equal_streamed_and_oracle(lanes, kib):
    """LDS-staged shapes (each part's state in LDS for the whole launch, the
    iteration split into per-(quad, dimension pair) updates and an in-order
    fold): bit-identical to the streamed shape and to the oracle, with swarms
    of one part and of many (at 78 KiB the Rastrigin swarm takes 59 parts
    that meet every iteration), ragged N, D = 1 and the stop rule (whose
    swarms take the unsplit iteration)."""
    specs = mixed_specs(30, 31)
    specs += [wl.SwarmSpec("rastrigin", 6001, 48, 20, seed=910, shift_amplitude=1.0),
              wl.SwarmSpec("ackley", 9003, 20, 20, seed=911, shift_amplitude=1.0),
              wl.SwarmSpec("rosenbrock", 2050, 64, 15, seed=912),
              wl.SwarmSpec("cubic", 4097, 1, 25, seed=913),
              wl.SwarmSpec("sphere", 5, 3, 30, seed=914)]
    specs[-2].tol, specs[-2].f_star = 1e3, -5e5
    announce(f"staged batch lanes={lanes} kib={kib}, {len(specs)} swarms")
    with pso.Batch(specs) as b:
        b.set_shape(256, 0, 1 << 17)
        assert b.shape["stage_kib"] == 0
        b.launch()
        ref = b.results()
        try:
            b.set_shape(lanes, 0, 0, stage_kib=kib)
        except pso.PsoError as e:
            if kib > 78 and e.code == pso.PSO_EINVAL and "exceed the LDS" in str(e):
                pytest.skip(f"{kib} KiB of LDS per workgroup not available on this device")
            raise
        sh = b.shape
        assert sh["lanes"] == lanes and sh["stage_kib"] == kib and sh["grid"] >= 1
        for rep in range(2):
            b.launch()
            res = b.results()
            for sp, r, q in zip(specs, res, ref):
                assert r["gbest_fit"] == q["gbest_fit"] and r["gbest_iter"] == q["gbest_iter"], (rep, sp)
                assert r["iters"] == q["iters"] and np.array_equal(r["gbest_pos"], q["gbest_pos"]), (rep, sp)
    for k in (len(specs) - 5, len(specs) - 4, len(specs) - 2, 3):
        sp = specs[k]
        o = oracle_swarm(sp, 16).run_f32(sp.T, tol=getattr(sp, "tol", 0.0), f_star=getattr(sp, "f_star", 0.0))
        assert ref[k]["gbest_fit"] == o["gbest_fit"] and ref[k]["gbest_iter"] == o["giter"], sp
        assert np.array_equal(ref[k]["gbest_pos"], o["gpos"]), sp


def test_lds_staged_shape_rejections():
    """More staged KiB than the LDS holds, unsupported lanes or a negative
    budget: EINVAL, and the batch keeps working under its previous shape."""
    specs = [wl.SwarmSpec("rastrigin", 100, 64, 5, seed=1), wl.SwarmSpec("sphere", 50, 2, 5, seed=2)]
    with pso.Batch(specs) as b:
        before = b.shape
        for lanes, kib in ((256, 100000), (128, 38), (256, -1)):
            with pytest.raises(pso.PsoError) as e:
                b.set_shape(lanes, 0, 0, stage_kib=kib)
            assert e.value.code == pso.PSO_EINVAL
        assert b.shape == before
        b.launch()
        r = b.results()
    o = oracle_swarm(specs[0]).run_f32(5)
    assert r[0]["gbest_fit"] == o["gbest_fit"]


def test_graph_replays_equal_the_direct_launch(monkeypatch):
    """pso_batch_launch captures the launch into a HIP graph once and replays
    it: three replays, with other eager GPU work and synchronisations between
    them, each give exactly the results of a direct (uncaptured) launch."""
    import torch
    specs = mixed_specs(60, 33)
    specs.append(wl.SwarmSpec("rastrigin", 7000, 40, 25, seed=77, shift_amplitude=1.0))  # several parts
    announce("batch graph replays")
    monkeypatch.setenv("PSO_BATCH_GRAPH", "0")
    with pso.Batch(specs) as b:
        b.launch()
        ref = b.results()
    monkeypatch.delenv("PSO_BATCH_GRAPH")
    other = wl.SwarmSpec("sphere", 5000, 6, 20, seed=3)
    with pso.Batch(specs) as b:
        for rep in range(3):
            b.launch()
            res = b.results()
            for r, q in zip(res, ref):
                assert r["gbest_fit"] == q["gbest_fit"] and r["gbest_iter"] == q["gbest_iter"], rep
                assert r["iters"] == q["iters"] and np.array_equal(r["gbest_pos"], q["gbest_pos"]), rep
            # unrelated eager work between replays
            with gpu_swarm(other) as g:
                g.run(other.T)
            x = torch.ones(1 << 20, device="cuda")
            torch.cuda.synchronize()
            assert float(x.sum()) == float(1 << 20)


def test_full_batched_workload_sampled_against_oracle():
    """The batched workload at full size (4096 swarms, N log-uniform in
    [32, 8192], D in {2..64}, 500 iterations) in the launch configuration the
    benchmark times (the default shape: LDS-staged where every swarm fits):
    a 256-swarm subset -- every 16th swarm, plus the largest and smallest
    state -- equals the oracle bit for bit."""
    specs = wl.batch_specs()
    announce("full batched workload, 4096 swarms x 500 iterations")
    with pso.Batch(specs) as b:
        assert b.shape["stage_kib"] > 0
        b.launch()
        res = b.results()
    sizes = [sp.N * sp.D for sp in specs]
    picks = set(range(0, len(specs), 16)) | {int(np.argmax(sizes)), int(np.argmin(sizes))}
    for k in sorted(picks):
        sp, r = specs[k], res[k]
        o = oracle_swarm(sp, nthreads=16).run_f32(sp.T)
        assert r["iters"] == sp.T == o["iters"], k
        assert r["gbest_fit"] == o["gbest_fit"] and r["gbest_iter"] == o["giter"], (k, sp.fitness, sp.N, sp.D)
        assert np.array_equal(r["gbest_pos"], o["gpos"]), k


@pytest.mark.parametrize("seed", [41, 42])
def test_random_batches_staged_equal_streamed(seed):
    """Random batches -- N from 1 to 20 000 (N*D <= 400 000), D from 1 to
    200, every fitness, iteration limits from 0 to 80, a stop rule on a
    third of the swarms --
    give the same bits under the staged default (1024 lanes, as much staged
    state as fits beside the widest swarm's vectors), a staged shape of two
    workgroups per compute unit, and the streamed shape."""
    rng = np.random.default_rng(seed)
    specs = []
    for k in range(120):
        fit = wl.FITNESS_NAMES[int(rng.integers(0, 5))]
        N = int(np.exp(rng.uniform(0, np.log(20000))))
        D = int(np.exp(rng.uniform(0, np.log(200))))
        if fit == "rosenbrock":
            D = max(D, 2)
        N = min(N, 400000 // D)  # every swarm fits a staged launch's workgroups
        sp = wl.SwarmSpec(fit, N, D, int(rng.integers(0, 81)), seed=int(rng.integers(0, 2**40)),
                          shift_amplitude=float(rng.uniform(0, 3)))
        if k % 3 == 0:
            sp.tol, sp.f_star = float(10.0 ** rng.uniform(-3, 1)), 0.0
        specs.append(sp)
    announce(f"random batch seed={seed}: staged vs streamed")
    out = []
    with pso.Batch(specs) as b:
        full = b.shape["stage_kib"]  # the default: as much staged state as fits beside 2 x 200 floats
        assert 150 <= full < 158
        for lanes, pw, kib in ((1024, 0, full), (512, 0, full // 2), (256, 1 << 17, 0)):
            b.set_shape(lanes, 0, pw, stage_kib=kib)
            b.launch()
            out.append(b.results())
    for res in out[1:]:
        for sp, r, q in zip(specs, res, out[0]):
            assert r["gbest_fit"] == q["gbest_fit"] or (np.isnan(r["gbest_fit"]) and np.isnan(q["gbest_fit"])), sp
            assert r["gbest_iter"] == q["gbest_iter"] and r["iters"] == q["iters"], sp
            assert np.array_equal(r["gbest_pos"], q["gbest_pos"]), sp


def test_staged_launch_streams_swarms_too_large_to_stage():
    """Under a staged shape, swarms whose staged parts would outnumber the
    workgroups (or are too wide for a tiny budget) stream in a second kernel
    of the same launch, after the staged ones: every result equals the
    streamed shape's and, on a sample, the oracle."""
    specs = [wl.SwarmSpec("rastrigin", 400000, 40, 6, seed=51, shift_amplitude=1.0),
             wl.SwarmSpec("ackley", 120001, 64, 8, seed=52, shift_amplitude=1.0)]
    specs += mixed_specs(40, 53, max_iter=40)
    announce("staged launch with streamed swarms")
    with pso.Batch(specs) as b:
        b.set_shape(256, 0, 1 << 17)
        b.launch()
        ref = b.results()
        outs = []
        for lanes, kib in ((1024, 150), (512, 1)):  # 1 KiB: only the smallest swarms stage
            b.set_shape(lanes, 0, 0, stage_kib=kib)
            b.launch()
            outs.append(b.results())
    for res in outs:
        for sp, r, q in zip(specs, res, ref):
            assert r["gbest_fit"] == q["gbest_fit"] and r["gbest_iter"] == q["gbest_iter"], sp
            assert r["iters"] == q["iters"] and np.array_equal(r["gbest_pos"], q["gbest_pos"]), sp
    for k in (0, 1, 5):
        sp = specs[k]
        o = oracle_swarm(sp, 16).run_f32(sp.T, tol=getattr(sp, "tol", 0.0), f_star=getattr(sp, "f_star", 0.0))
        assert ref[k]["gbest_fit"] == o["gbest_fit"] and np.array_equal(ref[k]["gbest_pos"], o["gpos"]), sp
