"""Benchmark of the global-best PSO step on one MI355X.

Workload: one synthetic swarm, Rastrigin, D = 32, N = 2^20 particles,
200 iterations, x0 ~ U[-5.12, 5.12], vmax = 1.024, w = 0.729,
c1 = c2 = 1.49445, Philox seed 0.  One benchmark step is one whole solve:
Step 1 (initialisation) plus 200 iterations, with all state resident in HBM.

Prints one JSON line: throughput in particle-dimension updates per second
(fitness included), the step kernel's roofline figures measured with HIP
events on the stream the kernels run on, and the CPU oracle's rate on a
bounded sample of the same workload.  Extra legs (same line): the
asynchronous variant on the same workload; a batch of 4096 uneven swarms in
one persistent launch with its speedup over a plain per-swarm pso_run loop
on a subset; and the request server under Poisson arrivals (p50/p99 latency
and throughput per arrival rate).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
COPY_BYTES = 256 << 20  # calibration copy: reads and writes this many bytes
SIMDS = 1024  # MI355X: 256 compute units x 4 SIMDs
CLOCK_MHZ = 2400.0


# Sources that define the grid step kernel: a counter summary taken on other
# sources is stale.
STEP_SOURCES = ["pso_device.hpp", "pso_aggregate.hpp", "pso_quad.hpp", "pso_kernels.hpp", "pso_kernels.hip"]


def source_digest() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2205_01313_amd", "csrc")
    for name in STEP_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def counters_from_profiles(kernel: str):
    """Per-launch counter figures of the step kernel from the committed
    rocprofv3 summary, if it was taken on the current step-kernel sources
    (else None): HBM bytes (FETCH_SIZE and WRITE_SIZE, each scaled by what it
    reads for a copy of known size) and VALU instructions (SQ_INSTS_VALU)."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    ent = rec.get("kernels", {}).get(kernel)
    if not ent or rec.get("source_digest") != source_digest():
        return None
    return ent


def host_cpu():
    """The host's CPU model, its logical CPUs, those this process may run on,
    and the OpenMP thread setting."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count() or 1
    return dict(cpu_model=model, logical_cpus=os.cpu_count(), cpus_allowed=allowed,
                omp_num_threads=os.environ.get("OMP_NUM_THREADS"))


def oracle_threads() -> int:
    """Threads for the oracle: every CPU this process may run on, at most the
    OpenMP setting of the environment (the CPU share of the machine)."""
    n = host_cpu()["cpus_allowed"]
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp and omp.isdigit() and int(omp) > 0:
        n = min(n, int(omp))
    return max(1, n)


def cpu_baseline(spec, iters: int, gpu_run=None):
    """The oracle (binary32 mode, OpenMP over particles on the CPU share of
    the host) on the first `iters` iterations of the same swarm, init
    excluded from the rate.  With gpu_run (the GPU's last timed solve of the
    same swarm: per-iteration gbest keys, gbest position, iteration of the
    last change, final state), the two runs are compared: every iteration's
    gbest key and the final state, bit for bit.  Then, on one core, the same
    problem at N = 65536 for 20 iterations in the synchronous mode and in the
    literal order of Alg. 1 (gbest updated inside the particle loop, the
    serial CPU baseline of the paper's tables)."""
    import numpy as np

    import oracle

    threads = oracle_threads()
    sw = oracle.Swarm(spec.fitness, spec.N, spec.D, spec.lo, spec.hi, spec.w, spec.c1, spec.c2, spec.vmax,
                      spec.seed, nthreads=threads)
    st = sw.init_f32()
    hist = [st["gkey"]]
    giter = 0
    t0 = time.perf_counter()
    for t in range(1, iters + 1):
        if sw.step_f32(st, t):
            giter = t
        hist.append(st["gkey"])
    dt = time.perf_counter() - t0
    out = dict(value=spec.N * spec.D * iters / dt, unit="particle·dim updates/s", cores=threads, kind="oracle",
               sample=f"first {iters} iterations of the same swarm (N={spec.N}, D={spec.D}), init excluded, "
                      f"{dt:.1f} s", host=host_cpu())
    if gpu_run is not None and iters == len(gpu_run["hist"]) - 1:
        hist = np.asarray(hist, np.uint64)
        eq = dict(history=bool(np.array_equal(hist, gpu_run["hist"])),
                  gbest_key=int(hist[-1]) == int(gpu_run["gkey"]),
                  gbest_iter=giter == int(gpu_run["giter"]),
                  gbest_pos=bool(np.array_equal(st["gpos"].view(np.uint32), gpu_run["gpos"].view(np.uint32))))
        for k in ("x", "v", "p", "pf"):
            eq[k] = bool(np.array_equal(st[k].view(np.uint32), gpu_run[k].view(np.uint32)))
        out["oracle_equal"] = all(eq.values())
        out["oracle_compare"] = eq
    n1, it1 = 65536, 20
    for name, serial in (("single_core", False), ("single_core_serial_alg1", True)):
        sw1 = oracle.Swarm(spec.fitness, n1, spec.D, spec.lo, spec.hi, spec.w, spec.c1, spec.c2, spec.vmax,
                           spec.seed, nthreads=1)
        st1 = sw1.init_f32()
        t1 = time.perf_counter()
        for t in range(1, it1 + 1):
            sw1.step_f32(st1, t, serial_immediate=serial)
        dt1 = time.perf_counter() - t1
        out[name] = dict(value=n1 * spec.D * it1 / dt1, cores=1,
                         sample=f"N={n1}, D={spec.D}, {it1} iterations, {dt1:.1f} s"
                                + (", gbest updated inside the particle loop" if serial else ""))
    return out


def timed_events(torch, stream, fn):
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b)


def copy_ceiling(torch, stream, nbytes=1 << 30, reps=5):
    """Device-to-device copy of nbytes (read nbytes + write nbytes), larger
    than the 256 MiB Infinity Cache so that HBM carries it: the bandwidth a
    plain streaming kernel reaches on this device (median of reps copies)."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ms = sorted(timed_events(torch, stream, lambda: dst.copy_(src)) for _ in range(reps))
    del src, dst
    return dict(bytes_per_copy=2 * nbytes, ms_median=ms[reps // 2], gbs=2 * nbytes / (ms[reps // 2] * 1e-3) / 1e9)


def async_leg(pso, torch, wl, spec, ws, stream, seeds=32):
    """Asynchronous variant on the same swarm: updates/s over one solve and
    its tiles (how many used a gbest published during the same iteration);
    the final-fitness distribution over 32 seeds of the synchronous,
    asynchronous and persistent variants (quantiles 0, 10, 50, 90, 100) and
    two-sample KS statistics against the synchronous one."""
    import numpy as np
    import scipy.stats
    sw = pso.Swarm(spec.fitness, spec.N, spec.D, spec.box, spec.w, spec.c1, spec.c2, spec.vmax, spec.seed,
                   variant=pso.PSO_ASYNC, workspace=ws, stream=stream)

    def solve():
        sw.reset()
        for _ in range(spec.T):
            pso.pso_step(sw.h)
    solve()
    ms = timed_events(torch, stream, solve)
    best = sw.best()
    tiles = sw.async_counters()
    sw.close()
    finals, fresh = {}, []
    for name, var in (("sync", pso.PSO_SYNC), ("async", pso.PSO_ASYNC), ("persistent", pso.PSO_PERSISTENT)):
        fs = []
        for seed in range(seeds):
            sp = wl.large_rastrigin(seed=seed)
            with pso.Swarm(sp.fitness, sp.N, sp.D, sp.box, sp.w, sp.c1, sp.c2, sp.vmax, sp.seed, variant=var,
                           workspace=ws, stream=stream) as g:
                fs.append(float(g.run(sp.T)["gbest_fit"]))
                if var == pso.PSO_ASYNC:
                    fresh.append(g.async_counters()["fresh_tiles"])
        finals[name] = np.array(fs)
    dist = {k: [float(q) for q in np.percentile(v, [0, 10, 50, 90, 100])] for k, v in finals.items()}
    ks = {}
    for k in ("async", "persistent"):
        r = scipy.stats.ks_2samp(finals["sync"], finals[k])
        ks[k] = dict(statistic=float(r.statistic), pvalue=float(r.pvalue))
    return dict(value=spec.N * spec.D * spec.T / (ms / 1e3), unit="particle·dim updates/s", ms_per_solve=ms,
                gbest=float(best["gbest_fit"]),
                tiles_per_workgroup=os.environ.get("PSO_ASYNC_TILES", "library default"),
                tiles=tiles["tiles"], fresh_tiles=tiles["fresh_tiles"],
                seeds_differing_from_sync=int(np.sum(finals["sync"] != finals["async"])),
                fresh_tiles_per_seed_min=int(min(fresh)),
                final_fitness_quantiles_32_seeds=dist, ks_vs_sync=ks)


def small_leg(pso, torch, wl, stream):
    """Small Sphere (D=2, N=1024, 1000 iterations): microseconds per
    iteration, (a) as one pso_run (the whole run inside one workgroup) and
    (b) as one pso_step launch per iteration; median of 5 solves each."""
    spec = wl.small_sphere()
    ws = torch.empty(pso.pso_workspace_bytes(spec.N, spec.D), dtype=torch.uint8, device="cuda")
    sw = pso.Swarm(spec.fitness, spec.N, spec.D, spec.box, spec.w, spec.c1, spec.c2, spec.vmax, spec.seed,
                   workspace=ws, stream=stream)

    def run():
        sw.reset()
        sw.run(spec.T)

    def steps():
        sw.reset()
        for _ in range(spec.T):
            pso.pso_step(sw.h)
    run()
    steps()
    us_run = sorted(timed_events(torch, stream, run) * 1e3 / spec.T for _ in range(5))
    us_step = sorted(timed_events(torch, stream, steps) * 1e3 / spec.T for _ in range(5))
    best = sw.best()
    sw.close()
    return dict(workload="Sphere D=2 N=1024, 1000 iterations", us_per_iteration_run=us_run[2],
                us_per_iteration_step_launches=us_step[2], gbest=float(best["gbest_fit"]),
                updates_per_s_run=spec.N * spec.D / (us_run[2] * 1e-6))


def deep_leg(pso, torch, wl, stream):
    """Deep workloads (D=128, N=65536, 2000 iterations): Rosenbrock, and
    Ackley with a shift; updates/s and the step kernel's share of the HBM
    roofline on algorithmic bytes.  Their 100 MB state fits the 256 MiB
    Infinity Cache, so the fraction can exceed what HBM alone would allow.
    The binary32 result's error: its gbest position re-evaluated in binary64,
    and the same run in binary64."""
    import numpy as np
    out = {}
    for spec in (wl.deep_rosenbrock(0), wl.deep_ackley(0)):
        ws = torch.empty(pso.pso_workspace_bytes(spec.N, spec.D), dtype=torch.uint8, device="cuda")
        sw = pso.Swarm(spec.fitness, spec.N, spec.D, spec.box, spec.w, spec.c1, spec.c2, spec.vmax, spec.seed,
                       shift=spec.shift, workspace=ws, stream=stream)

        def solve():
            sw.reset()
            for _ in range(spec.T):
                pso.pso_step(sw.h)
        solve()
        ms = timed_events(torch, stream, solve)
        rho = sw.counters()["pbest_improvements"] / (spec.N * spec.T)
        best = sw.best()
        sw.close()
        us = ms * 1e3 / spec.T
        alg = spec.N * spec.D * (20.0 + 4.0 * rho) + spec.N * (4.0 + 4.0 * rho)
        # the same run in binary64 (the binary64 path computes the reference
        # definition in double): the binary32 result's error against it
        with pso.Swarm64(spec.fitness, spec.N, spec.D, spec.box, spec.w, spec.c1, spec.c2, spec.vmax, spec.seed,
                         shift=spec.shift) as g64:
            t0 = time.perf_counter()
            r64 = g64.run(spec.T)
            s64 = time.perf_counter() - t0
            # the binary32 gbest position re-evaluated in binary64
            f32_at64 = float(g64.eval(np.asarray(best["gbest_pos"], np.float64)[None, :])[0])
        f32 = float(best["gbest_fit"])
        f64 = float(r64["gbest_fit"])
        out[spec.fitness] = dict(value=spec.N * spec.D * spec.T / (ms / 1e3), unit="particle·dim updates/s",
                                 us_per_iteration=us, hbm_frac=alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                                 pbest_improvement_rate=rho, gbest=f32, gbest_f64=f64,
                                 gbest_pos_reevaluated_f64=f32_at64, fitness_eval_err=abs(f32 - f32_at64),
                                 abs_err_vs_f64=abs(f32 - f64), rel_err_vs_f64=abs(f32 - f64) / max(abs(f64), 1e-300),
                                 f64_run_s=s64)
    return out


def latency_leg(pso):
    """Latency-bound swarms (binary32 Cubic 1D, N = 1024 / 4096 / 16384,
    20 000 iterations; w = 1, c1 = c2 = 2, [-100, 100], vmax 20): microseconds
    per iteration of a pso_run, synchronous against the fully asynchronous
    persistent variant (one launch, no barrier between iterations)."""
    rows = []
    for N in (1024, 4096, 16384):
        row = dict(N=N, D=1, iterations=20000)
        for name, var in (("sync", pso.PSO_SYNC), ("persistent", pso.PSO_PERSISTENT)):
            with pso.Swarm("cubic", N, 1, (-100.0, 100.0), 1.0, 2.0, 2.0, 20.0, 0, variant=var) as g:
                g.run(200)
                g.reset()
                t0 = time.perf_counter()
                r = g.run(20000)
                s = time.perf_counter() - t0
            row[name + "_us_per_iteration"] = s / 20000 * 1e6
            row[name + "_gbest"] = float(r["gbest_fit"])
        rows.append(row)
    return dict(precision="f32", rows=rows)


# The paper's experiments (Sec. 5, Tables 2-4): binary64, Cubic (Eq. 3, on
# [-100, 100]), w = 1, c1 = c2 = 2; vmax is not stated there (0.1 of the box
# here).  The paper's own Queue Lock (1D) and Queue (120D) seconds on its
# GPU are printed beside each row as context.
PAPER_ROWS = [  # N, D, iterations, paper seconds
    (32, 1, 100000, 0.216), (256, 1, 100000, 0.222), (1024, 1, 100000, 0.227), (2048, 1, 100000, 0.230),
    (4096, 1, 100000, 0.265), (16384, 1, 100000, 0.417), (65536, 1, 100000, 1.026), (131072, 1, 100000, 2.759),
    (128, 120, 5000, 0.487), (1024, 120, 2000, 0.225), (8192, 120, 1000, 0.191), (32768, 120, 1000, 0.570),
    (131072, 120, 800, 1.744)]


def paper_leg(pso):
    """Replay of the paper's shapes through the binary64 path (pso64_run),
    seconds per run (after one untimed warm-up run of 200 iterations)."""
    rows = []
    for N, D, T, paper_s in PAPER_ROWS:
        with pso.Swarm64("cubic", N, D, (-100.0, 100.0), 1.0, 2.0, 2.0, 20.0, 0) as g:
            g.run(min(T, 200))
            g.reset()
            t0 = time.perf_counter()
            g.run(T)
            s = time.perf_counter() - t0
        rows.append(dict(N=N, D=D, iterations=T, s=s, us_per_iteration=s / T * 1e6,
                         updates_per_s=N * D * T / s, paper_s_context=paper_s))
    return dict(precision="f64", fitness="cubic", rows=rows)


def batched_leg(pso, torch, wl, stream):
    """4096 swarms (N log-uniform in [32, 8192], D in {2..64}, four fitness
    functions with shifts, 500 iterations) in one persistent launch, its
    shape (lanes, workgroups, part size, LDS staging) picked by the
    autotuner, and the streamed kernel's time on the same batch; then every
    swarm of the batch run alone, as the plain loop (one swarm after another,
    one launch per iteration) and as a loop of pso_run calls (each swarm's
    creation outside the timed regions; all three give the same results)."""
    specs = wl.batch_specs()
    with pso.Batch(specs, stream=stream) as b:
        default_shape = b.shape
        t0 = time.perf_counter()
        shape = b.autotune(probe_iters=16)
        tune_s = time.perf_counter() - t0
        b.launch()
        torch.cuda.synchronize()
        ms = timed_events(torch, stream, b.launch)
        res = b.results()
        # the streamed kernel on the same batch, for comparison
        b.set_shape(128, 0, 1 << 17)
        b.launch()
        torch.cuda.synchronize()
        ms_streamed = timed_events(torch, stream, b.launch)
        res_streamed = b.results(positions=False)
    same_streamed = all(a["gbest_fit"] == c["gbest_fit"] and a["iters"] == c["iters"]
                        for a, c in zip(res, res_streamed))
    updates = sum(sp.N * sp.D * r["iters"] for sp, r in zip(specs, res))
    # every swarm alone, in one reused workspace on the same stream
    ws = torch.empty(max(pso.pso_workspace_bytes(sp.N, sp.D) for sp in specs), dtype=torch.uint8, device="cuda")
    s_plain = s_run = 0.0
    same = True
    for sp, r in zip(specs, res):
        with pso.Swarm(sp.fitness, sp.N, sp.D, sp.box, sp.w, sp.c1, sp.c2, sp.vmax, sp.seed, shift=sp.shift,
                       workspace=ws, stream=stream) as sw:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sw.step(sp.T)
            sw.sync()
            s_plain += time.perf_counter() - t0
            a = sw.best()
            sw.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c = sw.run(sp.T)
            s_run += time.perf_counter() - t0
        same = same and a["gbest_fit"] == c["gbest_fit"] == r["gbest_fit"] and \
            (a["gbest_pos"] == r["gbest_pos"]).all() and (c["gbest_pos"] == r["gbest_pos"]).all()
    return dict(swarms=len(specs), iterations=500, ms=ms, value=updates / (ms / 1e3), unit="particle·dim updates/s",
                autotuned_shape=shape, autotune_s=tune_s, default_shape=default_shape,
                streamed_ms=ms_streamed, streamed_shape=dict(lanes=128, grid=0, part_work=1 << 17, stage_kib=0),
                streamed_equal_results=bool(same_streamed),
                plain_loop_ms=s_plain * 1e3, batched_vs_plain_speedup=s_plain * 1e3 / ms,
                pso_run_loop_ms=s_run * 1e3, batched_vs_pso_run_loop_speedup=s_run * 1e3 / ms,
                equal_results=bool(same))


def f64_leg(pso, wl, reps=3):
    """The large Rastrigin workload (D=32, N=2^20, 200 iterations) through the
    binary64 path, the paper's precision: updates/s and the share of the HBM
    roofline on its algorithmic bytes, at least 40 per update (read x, v, p;
    write x, v, 8 bytes each) plus the pbest fitness read once per particle
    -- a lower bound, since the pbest writes (8 bytes per improved
    element) are not counted."""
    spec = wl.large_rastrigin(seed=0)
    with pso.Swarm64(spec.fitness, spec.N, spec.D, spec.box, spec.w, spec.c1, spec.c2, spec.vmax, spec.seed) as g:
        g.run(spec.T)
        secs = []
        for _ in range(reps):
            g.reset()
            t0 = time.perf_counter()
            r = g.run(spec.T)
            secs.append(time.perf_counter() - t0)
    s = sorted(secs)[reps // 2]
    us = s * 1e6 / spec.T
    alg = spec.N * spec.D * 40.0 + spec.N * 8.0
    return dict(workload="Rastrigin D=32, N=2^20, 200 iterations, binary64", s_per_solve=s,
                us_per_iteration=us, value=spec.N * spec.D * spec.T / s, unit="particle·dim updates/s",
                alg_bytes_per_iteration_lower_bound=alg, hbm_frac_lower_bound=alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                gbest=float(r["gbest_fit"]))


def serving_leg(pso, wl, rates=(2000, 10000, 50000), count=20000, budget=32 << 30, chunk=0):
    """Poisson arrivals of solve requests (N lognormal median 512, D in
    [2, 64], stop at |gbest| < 1e-4 or 1000 iterations) submitted at their
    arrival times; latency is submit-to-completion inside the server.  The
    percentiles leave out the first tenth of the requests (warm-up); the
    server's own percentiles over all of them are reported beside."""
    import ctypes
    out = {}
    for rate in rates:
        specs = wl.serving_specs(count, seed=rate)
        arr, keep = pso._descs(specs)
        times = wl.poisson_arrivals(count, rate, seed=rate)
        with pso.Server(budget, chunk_updates=chunk) as srv:
            L = pso.lib()
            tk = ctypes.c_uint64()
            tickets = []
            t0 = time.perf_counter()
            for k in range(count):
                while time.perf_counter() - t0 < times[k]:
                    pass
                pso._check(L.pso_server_submit(srv.h, ctypes.byref(arr[k]), ctypes.byref(tk)), "submit")
                tickets.append(tk.value)
            submit_s = time.perf_counter() - t0
            pending = set(tickets)
            res, lat_ms = {}, {}
            r = pso._native.PsoResult()
            lat = ctypes.c_double()
            while pending:
                for t in list(pending):
                    rc = L.pso_server_poll(srv.h, t, ctypes.byref(r), ctypes.byref(lat))
                    if rc != pso.PSO_EAGAIN:
                        pso._check(rc, "poll")
                        res[t] = r.iters
                        lat_ms[t] = lat.value
                        pending.discard(t)
                if time.perf_counter() - t0 > 240:
                    break
            wall = time.perf_counter() - t0
            st = srv.stats()
        upd = sum(sp.N * sp.D * res.get(t, 0) for sp, t in zip(specs, tickets))
        import numpy as np
        warm = count // 10
        steady = np.array([lat_ms[t] for t in tickets[warm:] if t in lat_ms])
        q = (lambda f: float(np.percentile(steady, f))) if steady.size else (lambda f: None)
        # a queue that grows through the run shows as a later half slower
        # than the earlier one (requests in arrival order)
        h = steady.size // 2
        p99_halves = [float(np.percentile(x, 99)) if x.size else None for x in (steady[:h], steady[h:])]
        out[str(rate)] = dict(offered_per_s=rate, requests=count, warmup_requests=warm,
                              completed=int(st["completed"]), p50_ms=q(50), p99_ms=q(99),
                              p99_first_half_ms=p99_halves[0], p99_second_half_ms=p99_halves[1],
                              max_ms=float(steady.max()) if steady.size else None,
                              all_requests_p50_ms=st["p50_ms"], all_requests_p99_ms=st["p99_ms"],
                              throughput_per_s=st["completed"] / wall, updates_per_s=upd / wall,
                              submit_s=submit_s, wall_s=wall, launches=int(st["launches"]),
                              mem_peak_bytes=int(st["mem_peak"]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--variant", choices=["sync", "async"], default="sync")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=200)
    ap.add_argument("--legs", default="main,async,small,deep,f64,latency,paper,batched,serving",
                    help="comma list of legs beyond the main line: async, small, deep, f64, latency, paper, "
                         "batched, serving")
    ap.add_argument("--pmc-probe", nargs="?", const="step",
                    choices=["step", "batch", "deep_rosenbrock", "deep_ackley"],
                    help="for rocprofv3 counter runs: 'step' (default) = init + 20 step launches, then a 256 MiB "
                         "torch copy (calibration kernel of known size); 'batch' = one untimed and one timed launch "
                         "of the 4096-swarm batch (1024 lanes, 158 KiB staged); 'deep_rosenbrock' / 'deep_ackley' "
                         "= the D=128, N=65536 workload: init, 100 untimed and 200 timed step launches (the split "
                         "step), then the same copies; prints one line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the path is single-GPU (--gpus {args.gpus} is not supported)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2205_01313_amd as pso
    from paper_2205_01313_amd import workloads as wl

    spec = wl.large_rastrigin(seed=0)
    variant = pso.PSO_SYNC if args.variant == "sync" else pso.PSO_ASYNC
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # every kernel of the benchmark runs on this stream, so the HIP events
    # recorded on it time exactly that work
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    nbytes = pso.pso_workspace_bytes(spec.N, spec.D)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    sw = pso.Swarm(spec.fitness, spec.N, spec.D, spec.box, spec.w, spec.c1, spec.c2, spec.vmax, spec.seed,
                   variant=variant, workspace=ws, stream=stream)

    if args.pmc_probe == "batch":
        sw.close()
        specs = wl.batch_specs()
        with pso.Batch(specs, stream=stream) as b:
            b.set_shape(1024, 0, 0, stage_kib=158)
            b.launch()
            torch.cuda.synchronize()
            ms = timed_events(torch, stream, b.launch)
            res = b.results(positions=False)
        print(json.dumps({"pmc_probe": "batch", "ms": ms,
                          "updates": int(sum(sp.N * sp.D * r["iters"] for sp, r in zip(specs, res)))}), flush=True)
        return
    if args.pmc_probe in ("deep_rosenbrock", "deep_ackley"):
        sw.close()
        dspec = wl.deep_rosenbrock(0) if args.pmc_probe == "deep_rosenbrock" else wl.deep_ackley(0)
        dws = torch.empty(pso.pso_workspace_bytes(dspec.N, dspec.D), dtype=torch.uint8, device=dev)
        with pso.Swarm(dspec.fitness, dspec.N, dspec.D, dspec.box, dspec.w, dspec.c1, dspec.c2, dspec.vmax,
                       dspec.seed, shift=dspec.shift, workspace=dws, stream=stream) as g:
            for _ in range(100):
                pso.pso_step(g.h)
            torch.cuda.synchronize()
            n0 = g.counters()["pbest_improvements"]
            ms = timed_events(torch, stream, lambda: [pso.pso_step(g.h) for _ in range(200)])
            rho = (g.counters()["pbest_improvements"] - n0) / (dspec.N * 200)
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        alg = dspec.N * dspec.D * (20.0 + 4.0 * rho) + dspec.N * (4.0 + 4.0 * rho)
        print(json.dumps({"pmc_probe": args.pmc_probe, "step_launches": 300, "timed_launches": 200,
                          "us_per_launch": ms * 1e3 / 200, "pbest_improvement_rate": rho,
                          "alg_bytes_per_launch": alg, "copy_bytes": COPY_BYTES,
                          "source_digest": source_digest()}), flush=True)
        return
    if args.pmc_probe == "step":
        sw.reset()
        for _ in range(20):
            pso.pso_step(sw.h)
        torch.cuda.synchronize()
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        sw.close()
        print(json.dumps({"pmc_probe": True, "step_launches": 20, "copy_bytes": COPY_BYTES,
                          "source_digest": source_digest()}), flush=True)
        return

    def one_step(ev_a=None, ev_b=None):
        sw.reset()
        if ev_a is not None:
            ev_a.record(stream)
        for _ in range(spec.T):
            pso.pso_step(sw.h)
        if ev_b is not None:
            ev_b.record(stream)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record(stream)
    for k in range(args.steps):
        one_step(*evs[k])
    end.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    total_ms = start.elapsed_time(end)
    step_ms = sum(a.elapsed_time(b) for a, b in evs)
    best = sw.best()
    # pbest improvements of the last timed solve (counted inside the step kernel)
    rho = sw.counters()["pbest_improvements"] / (spec.N * spec.T)
    # the last timed solve, for the comparison with the oracle (outside the
    # timed region)
    gpu_run = None
    if not args.no_cpu_baseline and args.cpu_iters == spec.T:
        st = sw.state()
        gpu_run = dict(hist=sw.history(0, spec.T + 1), gkey=st["gkey"], giter=st["giter"], gpos=st["gpos"],
                       x=st["x"], v=st["v"], p=st["p"], pf=st["pf"])
        del st
    sw.close()

    ms_per_step = total_ms / args.steps
    solve_ms = sorted(a.elapsed_time(b) for a, b in evs)
    trimmed = solve_ms[1:-1] if len(solve_ms) >= 3 else solve_ms
    updates = spec.N * spec.D * spec.T
    value = updates * args.steps / (total_ms / 1e3)
    launch_us = step_ms * 1e3 / (args.steps * spec.T)

    alg_bytes = spec.N * spec.D * (20.0 + 4.0 * rho) + spec.N * (4.0 + 4.0 * rho)
    achieved = alg_bytes / (launch_us * 1e-6) / 1e9
    kernel = f"k_step<{spec.fitness}, D={spec.D}, {args.variant}>"
    counters = counters_from_profiles(kernel)
    traffic = counters["hbm_bytes_per_launch"] if counters else None
    # share of SIMD cycles issuing VALU work: a wave64 VALU instruction
    # occupies its SIMD for 4 cycles; 1024 SIMDs at 2.4 GHz
    valu_busy = (counters["valu_insts_per_dispatch"] * 4 / SIMDS / (launch_us * CLOCK_MHZ)
                 if counters and "valu_insts_per_dispatch" in counters else None)

    ceiling = copy_ceiling(torch, stream)
    out = {
        "metric": "particle·dim updates/s incl. fitness",
        "value": value,
        "unit": "particle·dim updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single swarm, Rastrigin D=32, N=2^20, 200 iterations (init + 200 per step)",
                   "fitness": spec.fitness, "N": spec.N, "D": spec.D, "iterations": spec.T,
                   "variant": args.variant, "seed": spec.seed},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel, "avg_launch_us": launch_us, "alg_bytes_per_launch": alg_bytes,
                     "pbest_improvement_rate": rho, "valu_busy_frac": valu_busy,
                     "measured_copy_ceiling": ceiling, "frac_of_measured_copy": achieved / ceiling["gbs"]},
        "gbest": {"value": float(best["gbest_fit"]), "iteration": int(best["gbest_iter"])},
        "solve_ms": {"median": solve_ms[len(solve_ms) // 2], "trimmed_mean": sum(trimmed) / len(trimmed),
                     "min": solve_ms[0], "max": solve_ms[-1]},
        "wall_s_timed": t_wall,
        "source_digest": source_digest(),
    }
    legs = set(args.legs.split(","))
    if "async" in legs:
        out["async"] = async_leg(pso, torch, wl, spec, ws, stream)
    if "small" in legs:
        out["small"] = small_leg(pso, torch, wl, stream)
    if "deep" in legs:
        out["deep"] = deep_leg(pso, torch, wl, stream)
    if "f64" in legs:
        out["f64"] = f64_leg(pso, wl)
    if "latency" in legs:
        out["latency"] = latency_leg(pso)
    if "paper" in legs:
        out["paper"] = paper_leg(pso)
    if "batched" in legs:
        out["batched"] = batched_leg(pso, torch, wl, stream)
    if "serving" in legs:
        out["serving"] = serving_leg(pso, wl)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, args.cpu_iters, gpu_run)
        if "oracle_equal" in out["cpu_baseline"]:
            out["oracle_equal"] = out["cpu_baseline"]["oracle_equal"]
        del gpu_run
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
