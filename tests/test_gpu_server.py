"""Request server (continuous batching): every request's result is the same
bits as the same swarm run alone (pso_create + pso_run, synchronous), in any
mix and arrival pattern; admission never exceeds the memory budget."""
import threading
import time

import numpy as np
import pytest

import paper_2205_01313_amd as pso
from paper_2205_01313_amd import workloads as wl
from tests.gpu_util import announce, gpu_swarm, oracle_swarm
from tests.test_gpu_batch import mixed_specs

pytestmark = pytest.mark.gpu


def alone(sp):
    with gpu_swarm(sp) as g:
        return g.run(sp.T, tol=getattr(sp, "tol", 0.0), f_star=getattr(sp, "f_star", 0.0))


def wait_all(srv, tickets, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        assert time.time() - t0 < timeout, f"{len(out)}/{len(tickets)} done"
        time.sleep(0.001)
    return out


def check_same(specs, tickets, res):
    for sp, t in zip(specs, tickets):
        a = alone(sp)
        r = res[t]
        assert r["gbest_fit"] == a["gbest_fit"], sp
        assert r["gbest_iter"] == a["gbest_iter"] and r["iters"] == a["iters"], sp
        assert np.array_equal(r["gbest_pos"], a["gbest_pos"]), sp


@pytest.fixture(params=["staged", "staged_half_grid", "streamed"])
def server_mode(request, monkeypatch):
    """Requests that fit run in LDS-staged launches by default, each launch
    over every co-resident workgroup; staged_half_grid gives each launch
    half of them (PSO_SERVER_GRID=half); the last mode streams every
    request (PSO_SERVER_STAGED=0)."""
    monkeypatch.delenv("PSO_SERVER_GRID", raising=False)
    if request.param == "streamed":
        monkeypatch.setenv("PSO_SERVER_STAGED", "0")
    else:
        monkeypatch.delenv("PSO_SERVER_STAGED", raising=False)
    if request.param == "staged_half_grid":
        monkeypatch.setenv("PSO_SERVER_GRID", "half")
    return request.param


def test_results_equal_alone_with_staggered_arrivals(server_mode):
    specs = mixed_specs(120, 11, max_iter=300)
    announce(f"server ({server_mode}): 120 staggered requests")
    with pso.Server(1 << 30, chunk_updates=20000) as srv:
        tickets = []
        for k, sp in enumerate(specs):
            tickets.append(srv.submit(sp))
            if k % 10 == 9:
                time.sleep(0.002)  # let launches start between arrivals
        res = wait_all(srv, tickets)
        st = srv.stats()
    assert st["completed"] == len(specs) and st["rejected"] == 0
    assert st["launches"] > 1
    check_same(specs, tickets, res)


def test_small_budget_admits_in_stages_and_never_exceeds_it():
    specs = [wl.SwarmSpec("rastrigin", 2000, 16, 120, seed=k) for k in range(30)]
    need = pso.pso_workspace_bytes(2000, 16)
    budget = 3 * need  # a few swarms at a time
    announce("server: small budget")
    with pso.Server(budget, chunk_updates=2000*16*8) as srv:
        tickets = [srv.submit(sp) for sp in specs]
        res = wait_all(srv, tickets)
        st = srv.stats()
    assert st["completed"] == 30 and st["mem_peak"] <= budget and st["mem_used"] == 0
    check_same(specs[:6], tickets[:6], res)


def test_oversize_request_is_rejected_and_others_continue():
    big = wl.SwarmSpec("sphere", 100000, 64, 10, seed=1)
    small = wl.SwarmSpec("sphere", 64, 2, 10, seed=2)
    with pso.Server(1 << 20) as srv:
        tb = srv.submit(big)
        ts = srv.submit(small)
        t0 = time.time()
        while True:
            try:
                r = srv.poll(tb)
            except pso.PsoError as e:
                assert e.code == pso.PSO_ENOMEM
                break
            assert r is None and time.time() - t0 < 30
            time.sleep(0.001)
        rs = wait_all(srv, [ts])[ts]
        assert rs["iters"] == 10
        with pytest.raises(pso.PsoError) as e:
            srv.poll(987654)
        assert e.value.code == pso.PSO_EINVAL


def test_submit_from_two_threads():
    specs = mixed_specs(60, 12, max_iter=80)
    with pso.Server(1 << 30, chunk_updates=50000) as srv:
        tickets = [None] * len(specs)

        def worker(lo):
            for k in range(lo, len(specs), 2):
                tickets[k] = srv.submit(specs[k])

        th = [threading.Thread(target=worker, args=(i,)) for i in (0, 1)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        res = wait_all(srv, tickets)
    check_same(specs[:10], tickets[:10], res)


def test_large_requests_split_into_parts(server_mode):
    specs = [wl.SwarmSpec("rastrigin", 40000, 24, 40, seed=k, shift_amplitude=1.0) for k in range(3)]
    specs += mixed_specs(20, 13, max_iter=60)
    announce(f"server ({server_mode}) with multi-part requests")
    with pso.Server(1 << 30, chunk_updates=1 << 21) as srv:
        tickets = [srv.submit(sp) for sp in specs]
        res = wait_all(srv, tickets)
    check_same(specs, tickets, res)


def test_staged_and_streamed_requests_mixed():
    """Requests too large to stage (their parts would outnumber a staged
    launch's workgroups) or too wide (D > 64) run in streamed launches while
    the others run staged; every result equals the swarm alone."""
    specs = [wl.SwarmSpec("sphere", 300000, 32, 12, seed=21, shift_amplitude=1.0),
             wl.SwarmSpec("ackley", 150001, 40, 10, seed=22, shift_amplitude=1.0),
             wl.SwarmSpec("rastrigin", 3000, 100, 20, seed=23, shift_amplitude=1.0)]
    specs += mixed_specs(40, 14, max_iter=80)
    announce("server: staged and streamed requests")
    with pso.Server(1 << 31, chunk_updates=1 << 22) as srv:
        tickets = [srv.submit(sp) for sp in specs]
        res = wait_all(srv, tickets, timeout=240.0)
    check_same(specs, tickets, res)


def test_serving_workload_burst_sampled_against_alone():
    """Requests of the serving workload (N log-normal, median 512, up to
    16 384; D in [2, 64]; stop at |gbest| < 1e-4 or 1000 iterations) arriving
    as one burst, the saturated case of the benchmark: every request
    completes, sampled results equal the swarm run alone, and the oracle
    replays 200 of the requests bit for bit."""
    specs = wl.serving_specs(300, seed=5)
    announce("server: 300-request burst of the serving workload")
    with pso.Server(4 << 30) as srv:
        tickets = [srv.submit(sp) for sp in specs]
        res = wait_all(srv, tickets, timeout=240.0)
        st = srv.stats()
    assert st["completed"] == len(specs) and st["rejected"] == 0
    sample = list(range(0, len(specs), 23))
    check_same([specs[k] for k in sample], [tickets[k] for k in sample], res)
    # and the oracle replays a 200-request sample
    for k in range(200):
        sp, r = specs[k], res[tickets[k]]
        o = oracle_swarm(sp, nthreads=16).run_f32(sp.T, tol=sp.tol, f_star=sp.f_star)
        assert r["iters"] == o["iters"] and r["gbest_fit"] == o["gbest_fit"], (k, sp.fitness, sp.N, sp.D)
        assert r["gbest_iter"] == o["giter"] and np.array_equal(r["gbest_pos"], o["gpos"]), k


def test_burst_beyond_two_launches_uploads_before_each_launch(monkeypatch):
    """One part per workgroup per launch (PSO_SERVER_LAUNCH_WAVES=1) and a
    burst whose staged parts exceed both streams' launches together: most
    admitted swarms wait for a later launch, on either stream, and each must
    still start from its own uploaded item and loop state.  Every result
    equals the same batch run in one launch (itself equal to each swarm
    alone), and a sample equals the swarm alone."""
    monkeypatch.setenv("PSO_SERVER_LAUNCH_WAVES", "1")
    rng = np.random.default_rng(77)
    specs = []
    for k in range(700):
        fit = wl.FITNESS_NAMES[int(rng.integers(0, 4))]
        D = int(rng.integers(2, 17))
        sp = wl.SwarmSpec(fit, int(rng.integers(32, 600)), D, int(rng.integers(20, 120)), seed=1000 + k,
                          shift_amplitude=2.0)
        specs.append(sp)
    announce("server: 700-request burst, one part per workgroup per launch")
    with pso.Server(1 << 30) as srv:
        tickets = [srv.submit(sp) for sp in specs]
        res = wait_all(srv, tickets, timeout=240.0)
        st = srv.stats()
    assert st["completed"] == len(specs) and st["launches"] > 2
    ref = pso.pso_batch_run(specs)
    for sp, t, b in zip(specs, tickets, ref):
        r = res[t]
        assert r["gbest_fit"] == b["gbest_fit"] and r["iters"] == b["iters"], sp
        assert r["gbest_iter"] == b["gbest_iter"] and np.array_equal(r["gbest_pos"], b["gbest_pos"]), sp
    sample = list(range(0, len(specs), 35))
    check_same([specs[k] for k in sample], [tickets[k] for k in sample], res)


def wait_code(srv, ticket, timeout=60.0):
    """Polls until the request ends; returns (status code, result or None)."""
    t0 = time.time()
    while True:
        try:
            r = srv.poll(ticket)
        except pso.PsoError as e:
            return e.code, None
        if r is not None:
            return pso.PSO_OK, r
        assert time.time() - t0 < timeout
        time.sleep(0.001)


def test_cancel_and_deadlines_free_memory_and_others_continue():
    """A request that would run far longer than the test is cancelled while
    running; one waiting for memory behind it is cancelled at once; another
    passes its deadline while waiting; afterwards the budget is free and a
    new request's result equals the swarm alone."""
    big = wl.SwarmSpec("rastrigin", 200000, 32, 10 ** 7, seed=3)
    need = pso.pso_workspace_bytes(big.N, big.D)
    announce("server: cancel and deadlines")
    with pso.Server(int(need * 1.5)) as srv:
        t_run = srv.submit(big)
        while srv.stats()["launches"] < 2:
            time.sleep(0.001)
        t_wait = srv.submit(big)  # waits for memory
        t_q = srv.submit(big)
        srv.cancel(t_q)
        assert wait_code(srv, t_q)[0] == pso.PSO_ECANCELED
        srv.set_deadline(t_wait, 30.0)
        assert wait_code(srv, t_wait)[0] == pso.PSO_ETIMEDOUT
        srv.cancel(t_run)
        assert wait_code(srv, t_run)[0] == pso.PSO_ECANCELED
        with pytest.raises(pso.PsoError) as e:
            srv.cancel(t_run)  # forgotten after the poll
        assert e.value.code == pso.PSO_EINVAL
        st = srv.stats()
        assert st["cancelled"] == 2 and st["timed_out"] == 1 and st["mem_used"] == 0
        small = wl.SwarmSpec("ackley", 3000, 12, 150, seed=9, shift_amplitude=2.0)
        t = srv.submit(small)
        code, r = wait_code(srv, t)
        assert code == pso.PSO_OK
        with pytest.raises(pso.PsoError) as e:
            srv.cancel(t)  # finished and polled: unknown
        assert e.value.code == pso.PSO_EINVAL
    check_same([small], [t], {t: r})
