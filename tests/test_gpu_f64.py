"""The binary64 path against the oracle's binary64 mode.

Sphere, Rosenbrock and Cubic use only +, -, * and / in double, so the state
after a run (x, v, pbest position and fitness, gbest index and iteration) is
compared bit for bit on every path: one workgroup (256 or 1024 lanes), the
persistent gang of workgroups that meet once per iteration, one grid launch
per iteration, and step by step.  Rastrigin and Ackley call cos and exp, whose device
and host implementations may differ in the last bit: after one iteration the
state is compared within 1e-12 relative, and after a longer run the
invariants of the method are checked (bounds, velocity limit, pbest fitness
equal to F(pbest position), gbest = lowest-index minimum of the pbest
fitness)."""
import numpy as np
import pytest

import oracle
import paper_2205_01313_amd as pso
from paper_2205_01313_amd import workloads as wl
from tests.gpu_util import announce, oracle_swarm

pytestmark = pytest.mark.gpu


def gpu64(spec):
    return pso.Swarm64(spec.fitness, spec.N, spec.D, (spec.lo, spec.hi), spec.w, spec.c1, spec.c2, spec.vmax,
                       spec.seed, shift=spec.shift)


def assert_equal64(g, o, what=("x", "v", "p", "pf")):
    for k in what:
        a, b = np.asarray(g[k]), np.asarray(o[k])
        bad = np.flatnonzero(a.view(np.uint64) != b.view(np.uint64))
        assert bad.size == 0, f"{k} differs at {bad[:5].tolist()}: {a[bad[0]]!r} vs {b[bad[0]]!r}"


@pytest.mark.parametrize("fit", ["sphere", "rosenbrock", "cubic"])
@pytest.mark.parametrize("N,D,how", [(500, 7, "run"), (300, 1, "run"), (3001, 9, "run"), (777, 13, "step"),
                                     (64, 2, "run")])
def test_exact_functions_bit_for_bit(fit, N, D, how):
    if fit == "rosenbrock" and D < 2:
        pytest.skip("Rosenbrock needs D >= 2")
    T = 50
    spec = wl.SwarmSpec(fit, N, D, T, seed=N * 13 + D, shift_amplitude=2.0)
    announce(f"f64 {fit} N={N} D={D} {how}")
    o = oracle_swarm(spec, 8).run_f64(T)
    with gpu64(spec) as g:
        if how == "run":
            r = g.run(T)
            assert r["iters"] == T and r["gbest_iter"] == o["giter"]
            assert r["gbest_fit"] == o["gbest_fit"]
            assert np.array_equal(r["gbest_pos"].view(np.uint64), o["gpos"].view(np.uint64))
        else:
            g.step(T)
        st = g.state()
    assert st["t"] == T and st["gbest_idx"] == o["gbest_idx"]
    assert_equal64(st, o)


def set_path(monkeypatch, path):
    """block, grid, gang (each workgroup's slice in LDS where it fits) or
    gang_unstaged (the slices in device memory)."""
    monkeypatch.setenv("PSO64_PATH", "gang" if path.startswith("gang") else path)
    if path == "gang_unstaged":
        monkeypatch.setenv("PSO64_GANG_STAGED", "0")
    else:
        monkeypatch.delenv("PSO64_GANG_STAGED", raising=False)


@pytest.mark.parametrize("path", ["block", "gang", "gang_unstaged", "grid"])
@pytest.mark.parametrize("fit,N,D", [("cubic", 2049, 1), ("rosenbrock", 1500, 6), ("sphere", 700, 3),
                                     ("cubic", 20000, 1)])
def test_every_run_path_bit_for_bit(monkeypatch, path, fit, N, D):
    set_path(monkeypatch, path)
    T = 60
    spec = wl.SwarmSpec(fit, N, D, T, seed=7 * N + D, shift_amplitude=1.5)
    announce(f"f64 path={path} {fit} N={N} D={D}")
    o = oracle_swarm(spec, 8).run_f64(T)
    with gpu64(spec) as g:
        r1 = g.run(T // 3)
        r2 = g.run(T - T // 3)
        st = g.state()
    assert r1["iters"] + r2["iters"] == T and st["t"] == T
    assert r2["gbest_fit"] == o["gbest_fit"] and r2["gbest_iter"] == o["giter"]
    assert np.array_equal(r2["gbest_pos"].view(np.uint64), o["gpos"].view(np.uint64))
    assert_equal64(st, o)


@pytest.mark.parametrize("staged", ["1", "0"])
@pytest.mark.parametrize("fit,N,D,tol", [("cubic", 4096, 1, 0.0), ("cubic", 33, 1, 0.0), ("cubic", 1500, 1, 0.0),
                                         ("rosenbrock", 300, 6, 0.0), ("sphere", 100, 3, 0.0),
                                         ("sphere", 2000, 4, 0.0), ("sphere", 900, 2, 1e-3),
                                         ("sphere", 900, 2, 1e-5)])
def test_one_workgroup_run_in_lds_and_in_memory(monkeypatch, staged, fit, N, D, tol):
    """The one-workgroup run with the swarm's state in LDS for the whole
    run (256 or 1024 lanes, the one-dimensional form, up to four particles
    per lane with a ragged last round) and with it in device memory; Sphere
    N = 2000, D = 4 does not fit LDS and takes the second form either way.
    Bit for bit against the oracle's binary64 mode, over two runs (the state
    is stored back after the first and loaded again), with a stop rule."""
    monkeypatch.setenv("PSO64_PATH", "block")
    monkeypatch.setenv("PSO64_BLOCK_STAGED", staged)
    T = 80
    spec = wl.SwarmSpec(fit, N, D, T, seed=5 * N + D, shift_amplitude=2.5)
    announce(f"f64 block staged={staged} {fit} N={N} D={D} tol={tol}")
    o = oracle_swarm(spec, 8).run_f64(T, tol=tol, f_star=0.0)
    with gpu64(spec) as g:
        r1 = g.run(T // 4, tol=tol, f_star=0.0)
        r2 = g.run(T - r1["iters"], tol=tol, f_star=0.0) if r1["iters"] == T // 4 else r1
        st = g.state()
    assert st["t"] == o["iters"] and st["gbest_idx"] == o["gbest_idx"]
    assert r2["gbest_fit"] == o["gbest_fit"] and r2["gbest_iter"] == o["giter"]
    assert np.array_equal(r2["gbest_pos"].view(np.uint64), o["gpos"].view(np.uint64))
    assert_equal64(st, o)


GRID_FORMS = {"narrow": dict(PSO64_WIDE="0", PSO64_SPLIT="0"), "wide": dict(PSO64_WIDE="1", PSO64_SPLIT="0"),
              "split": dict(PSO64_SPLIT="1"), "split_p64": dict(PSO64_SPLIT="1", PSO64_SPLIT_P="64"),
              "split_p16": dict(PSO64_SPLIT="1", PSO64_SPLIT_P="16")}


@pytest.mark.parametrize("form", list(GRID_FORMS))
@pytest.mark.parametrize("fit,N,D", [("sphere", 5001, 7), ("rosenbrock", 3001, 33), ("cubic", 2049, 1),
                                     ("rosenbrock", 999, 2), ("sphere", 130, 64), ("cubic", 77, 120)])
def test_grid_step_forms_bit_for_bit(monkeypatch, form, fit, N, D):
    """The grid step with one particle per lane (each new pbest position
    written at once), with two (16-byte accesses, new pbest positions
    deferred into the next iteration's pass), and split (several lanes per
    particle, each over a chunk of its dimensions, the fitness terms folded
    in dimension order by one lane; pbest positions deferred; 4, 16 or 64
    particles per workgroup, a ragged last one): step by step, then continued
    by pso64_run on the path the shape takes (the one-workgroup and gang
    paths first complete the deferred positions), bit for bit against the
    oracle's binary64 mode."""
    for k, v in GRID_FORMS[form].items():
        monkeypatch.setenv(k, v)
    T1, T2 = 20, 25
    spec = wl.SwarmSpec(fit, N, D, T1 + T2, seed=3 * N + D, shift_amplitude=1.0)
    announce(f"f64 grid form={form} {fit} N={N} D={D}")
    o = oracle_swarm(spec, 8).run_f64(T1 + T2)
    with gpu64(spec) as g:
        g.step(T1)
        mid = g.state()
        r = g.run(T2)
        st = g.state()
    assert mid["t"] == T1 and st["t"] == T1 + T2
    assert r["gbest_fit"] == o["gbest_fit"] and r["gbest_iter"] == o["giter"]
    assert np.array_equal(r["gbest_pos"].view(np.uint64), o["gpos"].view(np.uint64))
    assert st["gbest_idx"] == o["gbest_idx"]
    assert_equal64(st, o)


@pytest.mark.parametrize("fit", ["rastrigin", "ackley"])
def test_split_step_transcendental_close(monkeypatch, fit):
    """Rastrigin and Ackley (device cos and exp) through the split step at a
    shape of the paper's 120-dimensional rows: within 1e-12 relative of the
    oracle's binary64 mode after one iteration, and the same state as the
    one-particle-per-lane step after five (the same device functions)."""
    spec = wl.SwarmSpec(fit, 300, 120, 5, seed=17, shift_amplitude=1.0)
    announce(f"f64 split {fit} N=300 D=120")
    o = oracle_swarm(spec, 8).run_f64(1)
    states = {}
    for form in ("split", "narrow"):
        for k in ("PSO64_WIDE", "PSO64_SPLIT", "PSO64_SPLIT_P"):
            monkeypatch.delenv(k, raising=False)
        for k, v in GRID_FORMS[form].items():
            monkeypatch.setenv(k, v)
        with gpu64(spec) as g:
            g.step(1)
            one = g.state()
            g.step(4)
            states[form] = g.state()
        if form == "split":
            for key in ("x", "v", "pf"):
                np.testing.assert_allclose(one[key], o[key], rtol=1e-12, atol=1e-300)
    assert_equal64(states["split"], states["narrow"])


def test_large_swarm_wide_step_bit_for_bit():
    """A swarm large enough to take the two-particles-per-lane grid step by
    default (Sphere, N = 2^18, D = 32, 6 iterations): the state bit for bit."""
    T = 6
    spec = wl.SwarmSpec("sphere", 1 << 18, 32, T, seed=41, shift_amplitude=3.0)
    announce("f64 wide default N=2^18 D=32")
    o = oracle_swarm(spec, 16).run_f64(T)
    with gpu64(spec) as g:
        r = g.run(T)
        st = g.state()
    assert r["gbest_fit"] == o["gbest_fit"] and r["gbest_iter"] == o["giter"]
    assert st["gbest_idx"] == o["gbest_idx"]
    assert_equal64(st, o)


@pytest.mark.parametrize("path", ["block", "gang", "gang_unstaged", "grid"])
def test_stop_rule_on_every_path(monkeypatch, path):
    set_path(monkeypatch, path)
    spec = wl.SwarmSpec("sphere", 3000, 3, 500, seed=4)
    announce(f"f64 stop rule path={path}")
    o = oracle_swarm(spec, 8).run_f64(500, tol=1e-2, f_star=0.0)
    assert o["iters"] < 500
    with gpu64(spec) as g:
        r = g.run(500, tol=1e-2, f_star=0.0)
        st = g.state()
    assert r["iters"] == o["iters"] and r["gbest_fit"] == o["gbest_fit"]
    assert_equal64(st, o)


def test_paper_shape_cubic_1d():
    """The paper's 1D problem: Cubic (Eq. 3, maximised there, minimised
    negated here) on [-100, 100], w = 1, c1 = c2 = 2, double; vmax 20."""
    spec = wl.SwarmSpec("cubic", 2048, 1, 3000, seed=3, box=(-100.0, 100.0), vmax=20.0, w=1.0, c1=2.0, c2=2.0)
    announce("f64 paper-shape cubic 1D N=2048 T=3000")
    o = oracle_swarm(spec, 8).run_f64(spec.T)
    with gpu64(spec) as g:
        r = g.run(spec.T)
        st = g.state()
    assert r["gbest_fit"] == o["gbest_fit"] and r["gbest_iter"] == o["giter"]
    assert_equal64(st, o)


def test_stop_rule_and_resume():
    spec = wl.SwarmSpec("sphere", 512, 4, 400, seed=9)
    announce("f64 stop rule")
    o = oracle_swarm(spec).run_f64(400, tol=1e-3, f_star=0.0)
    assert o["iters"] < 400
    with gpu64(spec) as g:
        r = g.run(400, tol=1e-3, f_star=0.0)
        assert r["iters"] == o["iters"] and r["gbest_fit"] == o["gbest_fit"]
        assert g.run(10, tol=1e-3, f_star=0.0)["iters"] == 0
        g.reset()
        a = g.run(30)
        g.reset()
        b1 = g.run(10)
        b2 = g.run(20)
    assert b1["iters"] + b2["iters"] == 30 and a["gbest_fit"] == b2["gbest_fit"]


@pytest.mark.parametrize("fit", ["rastrigin", "ackley"])
def test_transcendental_functions_close_then_invariants(fit):
    spec = wl.SwarmSpec(fit, 4000, 24, 1, seed=5, shift_amplitude=3.0)
    announce(f"f64 {fit} one iteration")
    o = oracle_swarm(spec, 8).run_f64(1)
    with gpu64(spec) as g:
        g.run(1)
        st = g.state()
    assert st["gbest_idx"] == o["gbest_idx"]
    assert_equal64(st, o, what=("x", "v"))
    np.testing.assert_allclose(st["pf"], o["pf"], rtol=1e-12, atol=1e-12)
    # a longer run: invariants of the method
    T = 200
    with gpu64(spec) as g:
        g.run(T)
        st = g.state()
    N, D = spec.N, spec.D
    x, v, p = (st[k].reshape(D, N) for k in ("x", "v", "p"))
    assert (x >= spec.lo).all() and (x <= spec.hi).all()
    assert (np.abs(v) <= np.float32(spec.vmax)).all()
    ref = oracle_swarm(spec, 8).fitness_f64(p.T)
    np.testing.assert_allclose(st["pf"], ref, rtol=1e-12, atol=1e-12)
    gi = st["gbest_idx"]
    assert st["pf"][gi] == st["pf"].min() and gi == int(np.flatnonzero(st["pf"] == st["pf"].min())[0])
    assert st["t"] == T


@pytest.mark.parametrize("fit", ["sphere", "rastrigin", "rosenbrock", "ackley", "cubic"])
def test_eval_matches_oracle(fit):
    """pso64_eval (the binary64 fitness with the swarm's shift, used to
    re-evaluate binary32 results): bit for bit against the oracle's binary64
    fitness for the functions of +, -, *, / only, within 1e-12 relative for
    those that call cos and exp."""
    D = 1 if fit == "cubic" else 37
    spec = wl.SwarmSpec(fit, 10, D, 1, seed=77, shift_amplitude=3.0)
    rng = np.random.default_rng(3)
    pts = rng.uniform(spec.lo, spec.hi, (500, D))
    pts[0] = spec.shift.astype(np.float64)  # the optimum (Rosenbrock: near it)
    with gpu64(spec) as g:
        got = g.eval(pts)
        assert g.eval(np.zeros((0, D))).shape == (0,)
    ref = oracle_swarm(spec).fitness_f64(pts)
    if fit in ("rastrigin", "ackley"):
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)
    else:
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
