"""Writes the oracle regression fixtures in this folder.  Calls only oracle/.

sphere_d2_n1024_t1000_seed0.txt: Sphere, D=2, N=1024, 1000 iterations,
bounds [-100, 100], vmax 20, w=0.729, c1=c2=1.49445, seed 0 (the small
single-swarm workload); one line per iteration t = 0..1000 with the gbest
key (hex: order-mapped binary32 fitness << 32 | particle index).
rastrigin_d32_n4096_t50_seed1.txt: Rastrigin, D=32, N=4096, 50 iterations,
bounds [-5.12, 5.12], vmax 1.024, seed 1, same coefficients.
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

CASES = {
    "sphere_d2_n1024_t1000_seed0.txt": dict(fitness="sphere", N=1024, D=2, lo=-100.0, hi=100.0, vmax=20.0,
                                            seed=0, T=1000),
    "rastrigin_d32_n4096_t50_seed1.txt": dict(fitness="rastrigin", N=4096, D=32, lo=-5.12, hi=5.12,
                                              vmax=1.024, seed=1, T=50),
}


def run(case):
    c = dict(case)
    T = c.pop("T")
    sw = oracle.Swarm(c["fitness"], c["N"], c["D"], c["lo"], c["hi"], 0.729, 1.49445, 1.49445, c["vmax"],
                      c["seed"])
    return sw.run_f32(T)


def main():
    for name, case in CASES.items():
        r = run(case)
        with open(os.path.join(HERE, name), "w") as f:
            f.write(f"# {case}\n# giter {r['giter']}\n")
            for k in r["hist"]:
                f.write(f"{int(k):016x}\n")


if __name__ == "__main__":
    main()
