"""Seeded synthetic input generators shared by tests, the benchmark and the serving loop.

This module draws random numbers only; it holds none of the discretisation's arithmetic.
Every generator takes an explicit seed (numpy PCG64) so that the CPU oracle and the GPU
library can be fed the very same inputs.
"""
import numpy as np


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def primitive_perturbation(n_nodes, seed, amp=(0.05, 0.1, 0.05)):
    """Independent uniform draws in [-1, 1] for a density, velocity and pressure perturbation
    field, scaled by amp = (density, velocity, pressure) relative amplitudes.  Returns
    (drho[n], dv[3, n], dp[n])."""
    g = rng(seed)
    drho = amp[0] * g.uniform(-1.0, 1.0, n_nodes)
    dv = amp[1] * g.uniform(-1.0, 1.0, (3, n_nodes))
    dp = amp[2] * g.uniform(-1.0, 1.0, n_nodes)
    return drho, dv, dp


def state_pairs(n, seed, rho=(0.5, 2.0), vel=1.0, p=(0.5, 3.0)):
    """n random primitive state pairs (rho, v1, v2, v3, p) for point-flux checks."""
    g = rng(seed)
    out = np.empty((2, n, 5))
    for s in range(2):
        out[s, :, 0] = g.uniform(*rho, n)
        out[s, :, 1:4] = g.uniform(-vel, vel, (n, 3))
        out[s, :, 4] = g.uniform(*p, n)
    return out


def unit_vectors(n, seed):
    g = rng(seed)
    v = g.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def mixed_orders(n_elements, seed=0, lo=2, hi=6):
    """Per-element anisotropic orders (N1, N2, N3), each uniform in {lo..hi}."""
    return rng(seed).integers(lo, hi + 1, size=(n_elements, 3)).astype(np.int32)


def poisson_arrivals(n, rate, seed=0):
    """Arrival times of a Poisson process of the given rate (requests per second)."""
    return np.cumsum(rng(seed).exponential(1.0 / rate, n))


def serving_requests(n=256, seed=0):
    """Independent solve requests: E^3 periodic boxes, E in {8..24}, N in {3,4,5},
    Mach in [0.1, 0.8], half Navier-Stokes with Re in [400, 3200], half Euler (Re = 0)."""
    g = rng(seed)
    reqs = []
    for i in range(n):
        E = int(g.integers(8, 25))
        N = int(g.integers(3, 6))
        Ma = float(g.uniform(0.1, 0.8))
        viscous = bool(g.integers(0, 2))
        Re = float(g.uniform(400.0, 3200.0)) if viscous else 0.0
        reqs.append(dict(id=i, E=E, N=N, Ma=Ma, Re=Re))
    return reqs
