"""Pins of the oracle's PSO iteration (Alg. 1 Steps 1-5, Eq. 1, Eq. 2) against
invariants, known minima, brute-force grid search and special cases of the
update equations that reduce to closed forms."""
import numpy as np
import pytest

import oracle

F32 = np.float32
W, C = 0.729, 1.49445
BOX = {"sphere": (-100.0, 100.0), "rastrigin": (-5.12, 5.12), "rosenbrock": (-30.0, 30.0),
       "ackley": (-32.768, 32.768), "cubic": (-100.0, 100.0)}


def mk(fit, N, D, seed=0, shift=None, w=W, c1=C, c2=C, vmax=None, box=None, nthreads=2):
    lo, hi = box or BOX[fit]
    vmax = vmax if vmax is not None else 0.1 * (hi - lo)
    return oracle.Swarm(fit, N, D, lo, hi, w, c1, c2, vmax, seed, shift=shift, nthreads=nthreads)


def check_invariants(sw, st, prev):
    N, D = sw.N, sw.D
    P = sw.problem
    x, v, p, pf = (st[k].reshape(D, N) if k != "pf" else st[k] for k in ("x", "v", "p", "pf"))
    assert np.all(x >= F32(P.lo)) and np.all(x <= F32(P.hi))
    assert np.all(np.abs(v) <= F32(P.vmax))
    # pf is the fitness of p, re-evaluated
    assert np.array_equal(sw.fitness_f32(p.T), pf)
    # gbest = lowest index among the smallest pbest fitness; gpos = p[:, gi]
    gf = oracle.key_value(st["gkey"])
    gi = st["gkey"] & 0xFFFFFFFF
    assert gf == pf.min()
    assert gi == int(np.flatnonzero(pf == pf.min())[0])
    assert np.array_equal(st["gpos"], p[:, gi])
    if prev is not None:
        assert np.all(pf <= prev["pf"])  # pbest never gets worse
        assert st["gkey"] <= prev["gkey"]  # gbest never gets worse
        moved = pf < prev["pf"]
        # pbest position changes exactly where pbest fitness improved, to the new x
        assert np.array_equal(p[:, moved], x[:, moved])
        assert np.array_equal(p[:, ~moved], prev["p"].reshape(D, N)[:, ~moved])


@pytest.mark.parametrize("fit,N,D", [("sphere", 64, 2), ("rastrigin", 100, 5), ("rosenbrock", 33, 7),
                                     ("ackley", 50, 3), ("cubic", 40, 1)])
def test_invariants_every_iteration(fit, N, D):
    rng = np.random.default_rng(N)
    sw = mk(fit, N, D, seed=N, shift=rng.uniform(-1, 1, D).astype(F32))
    st = sw.init_f32()
    check_invariants(sw, st, None)
    for t in range(1, 60):
        prev = {k: (val.copy() if isinstance(val, np.ndarray) else val) for k, val in st.items()}
        sw.step_f32(st, t)
        check_invariants(sw, st, prev)


def test_cfg_small_sphere_reaches_known_minimum():
    """Sphere, D=2, N=1024, 1000 iterations, w=0.729, c1=c2=1.49445, vmax 20."""
    r = mk("sphere", 1024, 2, vmax=20.0).run_f32(1000)
    assert r["gbest_fit"] < 1e-10
    assert r["iters"] == 1000
    assert np.all(r["hist"][1:] <= r["hist"][:-1])


@pytest.mark.parametrize("fit,opt", [("sphere", 0.0), ("rastrigin", 0.0), ("rosenbrock", 1.0), ("ackley", 0.0)])
def test_low_dim_instances_find_the_optimum(fit, opt):
    s = np.array([0.75, -1.25], F32)
    sw = mk(fit, 256, 2, seed=3, shift=s)
    r = sw.run_f32(400)
    assert r["gbest_fit"] < 1e-3
    np.testing.assert_allclose(r["gpos"], s + opt, atol=2e-2)


@pytest.mark.parametrize("fit", ["rastrigin", "ackley", "rosenbrock", "cubic"])
def test_brute_force_grid_d1_d2(fit):
    """PSO never reports a value below the true minimum over the box (grid
    minimum minus its Lipschitz slack) and gets at least as low as the grid."""
    lo, hi = BOX[fit]
    for D in (1, 2):
        n = 4001 if D == 1 else 1201
        g = np.linspace(lo, hi, n)
        h = g[1] - g[0]
        pts = (np.stack(np.meshgrid(*([g] * D), indexing="ij"), -1).reshape(-1, D)).astype(F32)
        sw = mk(fit, 256, D, seed=5)
        fgrid = sw.fitness_f64(pts.astype(np.float64))
        gmin = fgrid.min()
        # Lipschitz constant over the box, bounded from the formulas
        L = {"rastrigin": 2 * 5.12 + 20 * np.pi, "ackley": 20 * 0.2 + 2 * np.pi * np.e,
             "rosenbrock": 400 * 30 ** 3 + 400 * 30 + 2 * 31 + 200 * 30 * 2,
             "cubic": 3 * 100 ** 2 + 1.6 * 100 + 1000}[fit] * np.sqrt(D)
        r = sw.run_f32(300)
        f_at = sw.fitness_f64(r["gpos"][None, :].astype(np.float64))[0]
        assert f_at >= gmin - L * h * np.sqrt(D) / 2 - 1e-9
        assert r["gbest_fit"] <= gmin + 1e-3 * max(1.0, abs(gmin))


def test_determinism_and_thread_count_independence():
    a = mk("rastrigin", 777, 6, seed=9, nthreads=1).run_f32(40)
    b = mk("rastrigin", 777, 6, seed=9, nthreads=8).run_f32(40)
    for k in ("x", "v", "p", "pf", "gpos", "hist"):
        assert np.array_equal(a[k], b[k]), k
    assert a["giter"] == b["giter"]


def test_pure_inertia_moves_in_a_straight_line():
    """w=1, c1=c2=0: Eq. 1 leaves v unchanged, Eq. 2 moves x by v and the
    clamp stops it at the wall (v is not zeroed there)."""
    sw = mk("sphere", 16, 3, w=1.0, c1=0.0, c2=0.0, vmax=5.0, box=(-10.0, 10.0))
    st = sw.init_f32()
    x0, v0 = st["x"].copy(), st["v"].copy()
    xe = x0.copy()
    for t in range(1, 30):
        sw.step_f32(st, t)
        xe = np.minimum(np.maximum(xe + v0, F32(-10.0)), F32(10.0)).astype(F32)
        assert np.array_equal(st["v"], v0)
        assert np.array_equal(st["x"], xe)


def test_inertia_halves_velocity():
    """w=1/2, c1=c2=0: v_t = v_0 / 2^t exactly."""
    sw = mk("sphere", 8, 2, w=0.5, c1=0.0, c2=0.0, vmax=5.0, box=(-1e4, 1e4))
    st = sw.init_f32()
    v0 = st["v"].copy()
    for t in range(1, 20):
        sw.step_f32(st, t)
        assert np.array_equal(st["v"], (v0 * F32(0.5) ** t).astype(F32))


def test_cognitive_term_attracts_to_own_pbest_only():
    """w=0, c2=0: v = c1 r1 (pbest - x); after init pbest = x so nothing moves."""
    sw = mk("sphere", 32, 4, w=0.0, c1=1.5, c2=0.0)
    st = sw.init_f32()
    x0 = st["x"].copy()
    for t in range(1, 10):
        sw.step_f32(st, t)
        assert np.array_equal(st["x"], x0)
        assert np.all(st["v"] == 0.0)


def test_social_term_pulls_towards_gbest():
    """w=0, c1=0, c2=1: v = r2 (gbest - x) with r2 in [0,1): each coordinate
    moves towards the gbest position and never overshoots it; the gbest
    particle itself does not move."""
    N, D = 64, 3
    sw = mk("sphere", N, D, w=0.0, c1=0.0, c2=1.0, vmax=1e6)
    st = sw.init_f32()
    for t in range(1, 15):
        x_prev = st["x"].reshape(D, N).copy()
        g = st["gpos"].copy()
        gi = st["gkey"] & 0xFFFFFFFF
        sw.step_f32(st, t)
        x = st["x"].reshape(D, N)
        before = np.abs(x_prev - g[:, None])
        after = np.abs(x - g[:, None])
        assert np.all(after <= before)
        assert np.all(np.sign(x - x_prev) * np.sign(g[:, None] - x_prev) >= 0)
        assert np.array_equal(x[:, gi], x_prev[:, gi])
        # exact value with the oracle's own r2 draws
        for i in (0, N // 2, N - 1):
            for d in range(D):
                _, r2 = oracle.draw(0, oracle.TAG_VEL, t, i, d)
                # the w and c1 terms are signed zeros, which leave a sum unchanged
                vn = F32(r2 * F32(g[d] - x_prev[d, i]))
                assert x[d, i] == F32(x_prev[d, i] + vn)


def test_pbest_keeps_old_position_on_equal_fitness():
    """Step 4 updates pbest only on a strictly better fitness: a particle that
    moves from x = -1 to x = +1 on Sphere (equal fitness) keeps pbest -1."""
    sw = mk("sphere", 1, 1, w=1.0, c1=0.0, c2=0.0, vmax=4.0, box=(-10.0, 10.0))
    st = dict(x=np.array([-1.0], F32), v=np.array([2.0], F32), p=np.array([-1.0], F32),
              pf=np.array([1.0], F32), gpos=np.array([-1.0], F32), gkey=oracle.key(1.0, 0))
    sw.step_f32(st, 1)
    assert st["x"][0] == 1.0 and st["pf"][0] == 1.0
    assert st["p"][0] == -1.0 and st["gpos"][0] == -1.0


def test_velocity_and_position_clamps_hold():
    sw = mk("sphere", 200, 4, w=3.0, c1=4.0, c2=4.0, vmax=0.5, box=(-1.0, 1.0))
    st = sw.init_f32()
    for t in range(1, 20):
        sw.step_f32(st, t)
        assert np.all(np.abs(st["v"]) <= 0.5)
        assert np.all((st["x"] >= -1.0) & (st["x"] <= 1.0))


def test_serial_immediate_equals_sync_for_one_particle():
    a = mk("ackley", 1, 5, seed=4).run_f32(50)
    b = mk("ackley", 1, 5, seed=4).run_f32(50, serial_immediate=True)
    for k in ("x", "v", "p", "pf", "gpos", "hist"):
        assert np.array_equal(a[k], b[k])


def test_serial_immediate_keeps_invariants_and_converges():
    sw = mk("sphere", 128, 2, seed=1, vmax=20.0)
    r = sw.run_f32(300, serial_immediate=True)
    assert r["gbest_fit"] < 1e-6
    assert np.all(r["hist"][1:] <= r["hist"][:-1])


def test_stop_rule():
    sw = mk("sphere", 256, 2, seed=2, vmax=20.0)
    full = sw.run_f32(500)
    stop = sw.run_f32(500, tol=1e-4, f_star=0.0)
    assert stop["iters"] < 500
    assert stop["gbest_fit"] < 1e-4
    # the previous iteration had not reached the tolerance: stop is the first hit
    prev = oracle.key_value(stop["hist"][-2])
    assert abs(prev) >= 1e-4
    # and the trajectory up to there is the full run's
    assert np.array_equal(stop["hist"], full["hist"][: stop["iters"] + 1])


def test_f64_mode_tracks_f32_mode():
    """Same draws, same binary32 inputs: binary64 reaches the same basin."""
    sw = mk("rosenbrock", 512, 4, seed=6)
    a = sw.run_f32(200)
    b = sw.run_f64(200)
    assert b["gbest_fit"] <= 5.0 and a["gbest_fit"] <= 5.0
    # the first iterations agree closely before chaos separates the runs
    a5 = sw.run_f32(3)
    b5 = sw.run_f64(3)
    np.testing.assert_allclose(a5["x"], b5["x"], rtol=1e-5, atol=1e-4)
