"""Seeded synthetic workloads (swarm parameters and shift vectors).

Holds none of the PSO arithmetic: it only chooses problem parameters, shared
by the tests, the benchmark and the examples.  The coefficients w = 0.729,
c1 = c2 = 1.49445 and vmax = 0.1 (max_pos - min_pos) are the common
constriction setting; the paper's own experiments use w = 1, c1 = c2 = 2 and
its Cubic function on [-100, 100] (Sec. 5.1, Eq. 3).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

W, C1, C2 = 0.729, 1.49445, 1.49445

# Standard search boxes.
BOX = {"sphere": (-100.0, 100.0), "rastrigin": (-5.12, 5.12), "rosenbrock": (-30.0, 30.0),
       "ackley": (-32.768, 32.768), "cubic": (-100.0, 100.0)}
FITNESS_NAMES = ["sphere", "rastrigin", "rosenbrock", "ackley", "cubic"]


def vmax_of(box) -> float:
    return float(np.float32(0.1 * (box[1] - box[0])))


def shift_vector(seed: int, D: int, amplitude: float) -> np.ndarray:
    """Shift s ~ U[-amplitude, amplitude]^D from PCG64(seed), as float32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-amplitude, amplitude, D).astype(np.float32)


@dataclass
class SwarmSpec:
    fitness: str
    N: int
    D: int
    T: int
    seed: int = 0
    box: tuple = None
    vmax: float = None
    w: float = W
    c1: float = C1
    c2: float = C2
    shift_amplitude: float = 0.0
    shift: np.ndarray = field(default=None, repr=False)

    def __post_init__(self):
        if self.box is None:
            self.box = BOX[self.fitness]
        if self.vmax is None:
            self.vmax = vmax_of(self.box)
        if self.shift is None and self.shift_amplitude > 0:
            self.shift = shift_vector(self.seed, self.D, self.shift_amplitude)

    @property
    def lo(self):
        return self.box[0]

    @property
    def hi(self):
        return self.box[1]

    def updates(self) -> int:
        return self.N * self.D * self.T


# The single-swarm workloads.
def small_sphere(seed=0):
    """Sphere, D=2, N=1024, 1000 iterations, x0 ~ U[-100,100], |v| <= 20."""
    return SwarmSpec("sphere", 1024, 2, 1000, seed=seed, box=(-100.0, 100.0), vmax=20.0)


def large_rastrigin(seed=0):
    """Rastrigin, D=32, N=2^20, 200 iterations, x0 ~ U[-5.12,5.12], vmax 1.024."""
    return SwarmSpec("rastrigin", 1 << 20, 32, 200, seed=seed, box=(-5.12, 5.12), vmax=1.024)


def deep_rosenbrock(seed=0):
    """Rosenbrock, D=128, N=65536, 2000 iterations, x0 ~ U[-30,30], vmax 6."""
    return SwarmSpec("rosenbrock", 65536, 128, 2000, seed=seed, box=(-30.0, 30.0), vmax=6.0)


def deep_ackley(seed=0):
    """Ackley, D=128, N=65536, 2000 iterations, box [-32.768, 32.768],
    vmax 6.5536, shift U[-10,10] per seed."""
    return SwarmSpec("ackley", 65536, 128, 2000, seed=seed, box=(-32.768, 32.768), vmax=6.5536,
                     shift_amplitude=10.0)


# Many independent swarms.
def batch_specs(count=4096, seed=0, T=500, shift_amplitude=5.0):
    """Swarms with N = round(exp(U[ln 32, ln 8192])), D uniform in
    {2, 4, ..., 64}, fitness uniform over Sphere/Rastrigin/Rosenbrock/Ackley
    on their standard boxes, shift U[-5, 5]^D, T iterations; swarm k uses
    Philox seed k.  Drawn from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    specs = []
    for k in range(count):
        N = int(round(np.exp(rng.uniform(np.log(32), np.log(8192)))))
        D = 2 * (1 + int(rng.integers(0, 32)))
        fit = FITNESS_NAMES[int(rng.integers(0, 4))]
        shift = rng.uniform(-shift_amplitude, shift_amplitude, D).astype(np.float32)
        specs.append(SwarmSpec(fit, N, D, T, seed=k, shift=shift))
    return specs


def serving_specs(count, seed=0, max_iter=1000, tol=1e-4):
    """Solve requests: N = lognormal(median 512, sigma 1) clipped to
    [32, 16384], D uniform in [2, 64], fitness and shift as batch_specs, stop
    at |gbest - 0| < tol or max_iter iterations.  Drawn from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    specs = []
    for k in range(count):
        N = int(np.clip(round(np.exp(rng.normal(np.log(512), 1.0))), 32, 16384))
        D = int(rng.integers(2, 65))
        fit = FITNESS_NAMES[int(rng.integers(0, 4))]
        shift = rng.uniform(-5.0, 5.0, D).astype(np.float32)
        sp = SwarmSpec(fit, N, D, max_iter, seed=k, shift=shift)
        sp.tol, sp.f_star = tol, 0.0
        specs.append(sp)
    return specs


def poisson_arrivals(count, rate, seed=0):
    """Arrival times (s) of a Poisson process of the given rate (1/s)."""
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    return np.cumsum(rng.exponential(1.0 / rate, count))
