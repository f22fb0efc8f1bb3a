"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle runs.

This module holds NO arithmetic of the method: it only names workloads (grid,
spacing, mass, time step, stopping rule, initial-data description) and draws
workload parameters (job mixes, arrival times) from seeds.  Both the HIP path
and the oracle turn an initial-data description into a field with their own
code.

Initial-data descriptions are dicts:
  {"kind": "hedgehog", "prof_lambda": 1.0}                       B = 1, R(z) = z
  {"kind": "cube_b4", "prof_lambda": 1.5}                        B = 4, O_h rational map
  {"kind": "random_product", "B": 10, "seed": 1, "radius": 3.0, "prof_lambda": 1.0}
All profiles are f(r) = pi exp(-r / prof_lambda).
"""
from __future__ import annotations

import math

MASK64 = 0xFFFFFFFFFFFFFFFF


class SplitMix64:
    """SplitMix64 (Steele, Lea, Flood, OOPSLA 2014), used here only to draw
    workload parameters (job mixes, arrivals), never the method's own draws."""

    def __init__(self, seed: int):
        self.state = int(seed) & MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next() >> 11) * 2.0 ** -53

    def choice(self, seq):
        return seq[min(int(self.uniform() * len(seq)), len(seq) - 1)]

    def randint(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi]."""
        return lo + min(int(self.uniform() * (hi - lo + 1)), hi - lo)


# ----------------------------------------------------------------- workloads
# The five workloads of the method's evaluation (sizes, spacings and stopping
# rules as specified for this implementation; the paper itself times a B = 4
# relaxation on 151^3, 127^3 and 65^3 lattices).

HEDGEHOG_40 = dict(name="hedgehog-40", n=40, h=0.2, m=1.0, dt=0.1, tol=0.0, steps=300, precision="f64",
                   init={"kind": "hedgehog", "prof_lambda": 1.0})
# the same with a smaller time step (the flow at dt = 0.1, h = 0.2 sits near
# the leapfrog stability edge in the soliton core)
HEDGEHOG_40_SMALLDT = dict(HEDGEHOG_40, name="hedgehog-40-dt0.025", dt=0.025)

CUBE_B4_128 = dict(name="cube-b4-128", n=128, h=0.15, m=1.0, dt=0.015, tol=1e-4, steps=5000, precision="f64",
                   init={"kind": "cube_b4", "prof_lambda": 1.5})

RANDOM_B10_256 = dict(name="random-b10-256", n=256, h=0.1, m=1.0, dt=0.01, tol=1e-4, steps=20000,
                      precision="f32", init={"kind": "random_product", "B": 10, "seed": 1, "radius": 3.0,
                                             "prof_lambda": 1.0})

WORKLOADS = {w["name"]: w for w in (HEDGEHOG_40, HEDGEHOG_40_SMALLDT, CUBE_B4_128, RANDOM_B10_256)}

# Single-precision force floor: max |F| of a converged FP64 field rounded to FP32,
# evaluated in FP32, measured at h = 0.1 ... 0.2 and fitted as FLOOR32_COEF / h^2.
FLOOR32_COEF = 1.3e-6


def f32_tolerance(tol: float, h: float) -> float:
    """Stopping tolerance of an FP32-bulk relaxation: the requested one, but no
    less than twice the single-precision force floor at spacing h."""
    return max(tol, 2.0 * FLOOR32_COEF / (h * h))


def batch_jobs(master_seed: int = 4, count: int = 64) -> list[dict]:
    """The batched workload: `count` independent relaxations with B ~ U{1..8},
    n ~ U{48, 64, 96, 128}, m ~ U{0, 1}, h = 0.15, dt = 0.015, FP32 bulk
    with the power arrest rule, random product-ansatz initial data with a
    per-job seed."""
    g = SplitMix64(master_seed)
    jobs = []
    for j in range(count):
        B = g.randint(1, 8)
        n = g.choice([48, 64, 96, 128])
        m = float(g.randint(0, 1))
        seed = g.next()
        jobs.append(dict(name=f"batch-{master_seed}-{j}", n=n, h=0.15, m=m, dt=0.015, tol=f32_tolerance(1e-4, 0.15),
                         steps=20000, precision="f32", flow="power",
                         init={"kind": "random_product", "B": B, "seed": seed, "radius": 3.0, "prof_lambda": 1.0}))
    return jobs


def served_stream(master_seed: int = 5, count: int = 256, rate: float = 1.0) -> list[dict]:
    """The served workload: Poisson arrivals (exponential gaps of mean 1/rate
    seconds) of relaxations with B ~ U{1..12}, n log-uniform on [48, 192]
    rounded to even, h ~ U[0.1, 0.2], precision FP32 or FP64 with p = 1/2,
    dt = 0.1 h, tolerance 1e-4, cap 20000 steps.  FP64 jobs use the energy
    arrest rule; FP32-bulk jobs the power rule and f32_tolerance(1e-4, h)."""
    g = SplitMix64(master_seed)
    t = 0.0
    jobs = []
    for j in range(count):
        t += -math.log(1.0 - g.uniform()) / rate
        B = g.randint(1, 12)
        n = int(round(math.exp(math.log(48) + g.uniform() * (math.log(192) - math.log(48))) / 2.0)) * 2
        h = 0.1 + 0.1 * g.uniform()
        prec = "f32" if g.uniform() < 0.5 else "f64"
        seed = g.next()
        jobs.append(dict(name=f"serve-{master_seed}-{j}", arrival=t, n=n, h=h, m=1.0, dt=0.1 * h,
                         tol=f32_tolerance(1e-4, h) if prec == "f32" else 1e-4, steps=20000, precision=prec,
                         flow="power" if prec == "f32" else "energy",
                         init={"kind": "random_product", "B": B, "seed": seed, "radius": 3.0, "prof_lambda": 1.0}))
    return jobs


def random_unit_field(shape, seed: int, spread: float = 0.6):
    """A smooth-ish random S^3-valued field for gradient tests: vacuum plus
    seeded noise of the given spread, normalised, frozen vacuum layers.
    Returns a float64 numpy array of shape (4, *shape)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    phi = np.zeros((4,) + tuple(shape))
    phi[0] = 1.0
    phi += spread * rng.standard_normal(phi.shape)
    phi /= np.sqrt((phi ** 2).sum(axis=0, keepdims=True))
    interior = np.zeros(tuple(shape), dtype=bool)
    interior[2:-2, 2:-2, 2:-2] = True
    phi[:, ~interior] = 0.0
    phi[0, ~interior] = 1.0
    return phi
