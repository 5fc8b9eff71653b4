"""Benchmark of the global-best PSO step on one MI355X.

Workload: one synthetic swarm, Rastrigin, D = 32, N = 2^20 particles,
200 iterations, x0 ~ U[-5.12, 5.12], vmax = 1.024, w = 0.729,
c1 = c2 = 1.49445, Philox seed 0.  One benchmark step is one whole solve:
Step 1 (initialisation) plus 200 iterations, with all state resident in HBM.

Prints one JSON line: throughput in particle-dimension updates per second
(fitness included), the step kernel's roofline figures measured with HIP
events on the stream the kernels run on, and the CPU oracle's rate on a
bounded sample of the same workload.
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


def source_digest() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2205_01313_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel: str, launches_bytes_alg: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    ent = rec.get(kernel)
    if not ent or ent.get("source_digest") != source_digest():
        return None
    return ent["hbm_bytes_per_launch"]


def cpu_baseline(spec, iters: int):
    """The oracle (binary32 mode, OpenMP over particles) on the first `iters`
    iterations of the same swarm; rate excludes initialisation."""
    import oracle

    threads = min(16, os.cpu_count() or 1)
    sw = oracle.Swarm(spec.fitness, spec.N, spec.D, spec.lo, spec.hi, spec.w, spec.c1, spec.c2, spec.vmax,
                      spec.seed, nthreads=threads)
    st = sw.init_f32()
    t0 = time.perf_counter()
    for t in range(1, iters + 1):
        sw.step_f32(st, t)
    dt = time.perf_counter() - t0
    return dict(value=spec.N * spec.D * iters / dt, unit="particle·dim updates/s", cores=threads, kind="oracle",
                sample=f"first {iters} iterations of the same swarm (N={spec.N}, D={spec.D}), init excluded, "
                       f"{dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--variant", choices=["sync", "async"], default="sync")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=200)
    ap.add_argument("--pmc-probe", action="store_true",
                    help="for rocprofv3 counter runs: init + 20 step launches, then a 256 MiB torch copy "
                         "(calibration kernel of known size); prints nothing else")
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
    stream = torch.cuda.current_stream()
    nbytes = pso.pso_workspace_bytes(spec.N, spec.D)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    sw = pso.Swarm(spec.fitness, spec.N, spec.D, spec.box, spec.w, spec.c1, spec.c2, spec.vmax, spec.seed,
                   variant=variant, workspace=ws, stream=stream)

    if args.pmc_probe:
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
    sw.close()

    ms_per_step = total_ms / args.steps
    updates = spec.N * spec.D * spec.T
    value = updates * args.steps / (total_ms / 1e3)
    launch_us = step_ms * 1e3 / (args.steps * spec.T)

    alg_bytes = spec.N * spec.D * (20.0 + 4.0 * rho) + spec.N * (4.0 + 4.0 * rho)
    achieved = alg_bytes / (launch_us * 1e-6) / 1e9
    kernel = f"k_step<{spec.fitness}, D={spec.D}, {args.variant}>"
    traffic = traffic_from_profiles(kernel, alg_bytes)

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
                     "pbest_improvement_rate": rho},
        "gbest": {"value": float(best["gbest_fit"]), "iteration": int(best["gbest_iter"])},
        "wall_s_timed": t_wall,
        "source_digest": source_digest(),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, args.cpu_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
