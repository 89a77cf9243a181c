"""Seeded synthetic inputs shared by the tests, the bench and the oracle leg.

Holds no arithmetic of the method: only workload shapes, parameter draws and
initial-condition sampling with numpy's PCG64 generator.  The paper uses no
dataset; these are the workload recipes, with the sizes, densities and
velocities of its set-ups.
"""
from __future__ import annotations

import math

import numpy as np

# Workloads (sizes as named; seeds fixed per workload)
PLAIN_SMALL = dict(name="d1q3_L256_rho10_u0", L=256, rho=10.0, u0=0.0, steps=1000, seed=1)
PLAIN_LARGE = dict(name="d1q3_L16M_rho50_u0.1", L=1 << 24, rho=50.0, u0=0.1, steps=10_000, seed=2)
DENSITY_WAVE = dict(name="d1q3_L4M_wave_rho40", L=1 << 22, rho=40.0, amp=0.05, steps=5000,
                    log_every=10, seed=3)
BATCHED = dict(name="d1q3_1024_replicas", n=1024, L_lo=1 << 10, L_hi=1 << 18, rho_lo=5,
               rho_hi=100, u_lo=-0.2, u_hi=0.2, steps=2000, seed=4)
SERVED = dict(name="d1q3_served_200_per_s", rate=200.0, L_lo=1 << 12, L_hi=1 << 24,
              steps_lo=100, steps_hi=5000, rho_lo=5, rho_hi=100, budget=200 * 10**9, seed=5)

DEFAULT_C = 10
DEFAULT_LAMBDA = (1, 1)
DEFAULT_NMAX = 255


def replica_manifest(n=None, seed=None, L_lo=None, L_hi=None):
    """Independent replicas: L uniform integer, rho uniform integer, u0 uniform."""
    cfg = BATCHED
    n = cfg["n"] if n is None else n
    g = np.random.Generator(np.random.PCG64(cfg["seed"] if seed is None else seed))
    L = g.integers(cfg["L_lo"] if L_lo is None else L_lo,
                   (cfg["L_hi"] if L_hi is None else L_hi) + 1, size=n).astype(np.uint64)
    rho = g.integers(cfg["rho_lo"], cfg["rho_hi"] + 1, size=n).astype(np.float64)
    u0 = g.uniform(cfg["u_lo"], cfg["u_hi"], size=n)
    rid = np.arange(n, dtype=np.uint64)
    return dict(L=L, rho=rho, u0=u0, replica_id=rid)


def job_trace(duration_s: float, seed=None, rate=None, L_hi=None):
    """Poisson arrivals of jobs: L log-uniform, steps and rho uniform, u0 = 0."""
    cfg = SERVED
    g = np.random.Generator(np.random.PCG64(cfg["seed"] if seed is None else seed))
    rate = cfg["rate"] if rate is None else rate
    hi = cfg["L_hi"] if L_hi is None else L_hi
    jobs = []
    t = 0.0
    jid = 0
    while True:
        t += g.exponential(1.0 / rate)
        if t > duration_s:
            break
        L = int(round(math.exp(g.uniform(math.log(cfg["L_lo"]), math.log(hi)))))
        steps = int(g.integers(cfg["steps_lo"], cfg["steps_hi"] + 1))
        rho = float(g.integers(cfg["rho_lo"], cfg["rho_hi"] + 1))
        jobs.append(dict(job_id=jid, arrival=t, L=L, steps=steps, rho=rho, u0=0.0))
        jid += 1
    return jobs


def density_wave_counts(L=None, rho=None, amp=None, seed=None) -> np.ndarray:
    """Initial counts [3][L] uint16: n_i(x) ~ Poisson(rho(x) w_i) with
    rho(x) = rho (1 + amp sin(2 pi x / L)) and D1Q3 weights (1/6, 2/3, 1/6)."""
    cfg = DENSITY_WAVE
    L = cfg["L"] if L is None else L
    rho = cfg["rho"] if rho is None else rho
    amp = cfg["amp"] if amp is None else amp
    g = np.random.Generator(np.random.PCG64(cfg["seed"] if seed is None else seed))
    x = np.arange(L, dtype=np.float64)
    r = rho * (1.0 + amp * np.sin(2.0 * np.pi * x / L))
    w = np.array([1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0])
    return g.poisson(w[:, None] * r[None, :]).astype(np.uint16)


def twiddles(L: int, n_modes: int, scale_bits: int = 24) -> np.ndarray:
    """int32 [2 n_modes][L]: round(2^24 cos(2 pi m x / L)), round(2^24 sin(...)),
    m = 1..n_modes (the projections of Eq. (A) and of S(k))."""
    x = np.arange(L, dtype=np.float64)
    out = np.empty((2 * n_modes, L), dtype=np.int32)
    s = float(1 << scale_bits)
    for m in range(1, n_modes + 1):
        ph = 2.0 * np.pi * ((m * np.arange(L, dtype=np.int64)) % L) / L
        out[2 * (m - 1)] = np.rint(s * np.cos(ph)).astype(np.int32)
        out[2 * (m - 1) + 1] = np.rint(s * np.sin(ph)).astype(np.int32)
    return out


def random_counts(L: int, means=(3.0, 12.0, 5.0), seed: int = 0) -> np.ndarray:
    g = np.random.Generator(np.random.PCG64(seed))
    return g.poisson(np.asarray(means)[:, None], size=(3, L)).astype(np.uint16)
