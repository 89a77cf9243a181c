"""The paper's D1Q3 experiments, run on the batched GPU engine.

* ``parity_histograms`` -- Fig. 1 of the D1Q3 section: occupation-number
  distributions when every site starts with an even number of rest
  particles (a parity that collisions never change).
* ``equilibrium_means`` -- Fig. 3: time-averaged site means <n_i> against
  the velocity u, beside Eq. (D1Q3equil) and the lattice Boltzmann
  equilibrium of Eq. (LBequil).
* ``pi_decay`` -- Fig. 5: decay of the ensemble mean of the pi moment from a
  uniform initial state, with streaming and, as the figure's variant,
  without it; beside Eq. (D1Q3relax) and its linearisation Eq. (D1Q3relax2).
* ``correlations`` -- the normalised correlator of Eq. (corr) and the error
  function E(u) of Eq. (error), here for D1Q3.

Every simulated number comes from the library's kernels (``mclg.Lattice``);
this module only sets up the inputs, calls the engine and turns its exact
integer sums into the figures' statistics.  The predictions it prints are the
paper's closed forms, evaluated here in double precision.

* ``galilean`` (command line) -- the relaxation rate of pi~ against u with
  the constant and the Galilean-invariant acceptance.
* ``d2q9_statistics`` -- D2Q9: the equilibrium means against u_x at
  u_y = 0.25 (Eq. (D2Q9eqdist) against Eq. (LBequil)) and the correlator of
  Eq. (corr) / Table 1 with E(u) of Eq. (error).

Run ``python -m paper_1706_01094_amd.figures fig1|fig3|fig5|corr|galilean|d2q9eq|table1
[--quick]``.
"""
from __future__ import annotations

import argparse
import math
import time
from typing import Sequence

import numpy as np

from . import mclg

SQRT2 = math.sqrt(2.0)


# ---- closed forms ---------------------------------------------------------
def feq(rho: float, u: float) -> np.ndarray:
    """Eq. (D1Q3equil): the entropic D1Q3 equilibrium (f_-1, f_0, f_+1)."""
    s = math.sqrt(1.0 + 3.0 * u * u)
    return np.array([rho * (-1.0 - 3.0 * u + 2.0 * s) / 6.0,
                     rho * (2.0 - s) * 2.0 / 3.0,
                     rho * (-1.0 + 3.0 * u + 2.0 * s) / 6.0])


def f_lb(rho: float, u: float) -> np.ndarray:
    """Eq. (LBequil) for D1Q3: weights (1/6, 2/3, 1/6), theta = 1/3."""
    w = np.array([1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0])
    v = np.array([-1.0, 0.0, 1.0])
    return rho * w * (1.0 + 3.0 * v * u + 4.5 * (v * u) ** 2 - 1.5 * u * u)


def parity_sector_means(rho: float):
    """(f_+-1, f_0) of the product measure restricted to even rest counts at
    u = 0: n_+-1 ~ Poisson(f_1), n_0 ~ Poisson(f_0) conditioned on even, with
    f_0 = 4 f_1 (the equilibrium relation f_0^2 = 16 f_-1 f_+1 of the D1Q3
    section) and total mean density 2 f_1 + f_0 tanh(f_0) = rho."""
    lo, hi = 0.0, rho / 2.0
    for _ in range(200):
        f1 = 0.5 * (lo + hi)
        if 2.0 * f1 + 4.0 * f1 * math.tanh(4.0 * f1) < rho:
            lo = f1
        else:
            hi = f1
    f1 = 0.5 * (lo + hi)
    return f1, 4.0 * f1


def poisson_pmf(mu: float, n: int) -> np.ndarray:
    k = np.arange(n)
    lg = np.array([math.lgamma(i + 1.0) for i in k])
    return np.exp(k * math.log(mu) - mu - lg) if mu > 0 else (k == 0).astype(float)


def even_poisson_pmf(mu: float, n: int) -> np.ndarray:
    p = poisson_pmf(mu, n)
    p[1::2] = 0.0
    return p * 2.0 / (1.0 + math.exp(-2.0 * mu))


def pi_moment(n) -> np.ndarray:
    """pi = sqrt(2) (n_-1 - n_0 / 2 + n_+1), the non-conserved D1Q3 moment."""
    n = np.asarray(n, dtype=np.float64)
    return SQRT2 * (n[..., 0] - n[..., 1] / 2.0 + n[..., 2])


def pi_relax(pi0: float, n_coll, rho: float, u: float = 0.0, lam: float = 1.0,
             coef: float = math.sqrt(8.0)) -> np.ndarray:
    """Eq. (D1Q3relax): pi~ after n_coll collisions.  The printed equation
    carries 2 sqrt(6) as ``coef``; expanding Eq. (1Ddecay) about pi^eq gives
    sqrt(8), the default here."""
    s = math.sqrt(1.0 + 3.0 * u * u)
    k = coef * rho * s
    n_coll = np.asarray(n_coll, dtype=np.float64)
    return k * pi0 / (np.exp(n_coll * lam * s / rho) * (k + pi0) - pi0)


def pi_relax_linear(pi0: float, n_coll, rho: float, lam: float = 1.0) -> np.ndarray:
    """Eq. (D1Q3relax2): exp(-C lambda / rho) pi~(0)."""
    return pi0 * np.exp(-np.asarray(n_coll, dtype=np.float64) * lam / rho)


def _decay_rate(pit: np.ndarray, C: int) -> np.ndarray:
    """Per-collision decay rate -ln(pi~(t) / pi~(0)) / (C t) for t >= 1 (nan
    at t = 0 or once pi~ has crossed zero)."""
    out = np.full(len(pit), np.nan)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = pit[1:] / pit[0]
        out[1:] = np.where(r > 0, -np.log(r) / (C * np.arange(1, len(pit))), np.nan)
    return out


# ---- experiments ----------------------------------------------------------
def uniform_counts(init: Sequence[int], L: int, replicas: int) -> np.ndarray:
    """Counts for Lattice(counts=...): every site of every replica in state
    init = (n_-1, n_0, n_+1)."""
    one = np.asarray(init, dtype=np.uint16)[:, None].repeat(L, 1)
    return np.ascontiguousarray(np.broadcast_to(one, (replicas, 3, L))).reshape(-1)


def parity_histograms(L: int = 100, C: int = 10, rho: int = 12, equil: int = 20000,
                      steps: int = 80000, replicas: int = 1, every: int = 1, seed: int = 1,
                      n_bins: int = 64, init=None) -> dict:
    """Fig. 1 set-up: every site starts as (a, b, a) with b even (by default
    b = 2 round(rho / 3), a = (rho - b) / 2, i.e. (2, 8, 2) at rho = 12); the
    histograms of n_i are accumulated every ``every`` steps over ``steps``
    steps after ``equil`` steps, over all sites of ``replicas`` independent
    lattices."""
    if init is None:
        b = 2 * round(rho / 3)
        if (rho - b) % 2:
            raise ValueError("rho must be even for the (a, b, a) initial state")
        init = ((rho - b) // 2, b, (rho - b) // 2)
    if init[1] % 2:
        raise ValueError("the parity experiment starts from an even rest count")
    lat = mclg.Lattice([L] * replicas, seed, C=C, counts=uniform_counts(init, L, replicas))
    torch = lat.torch
    try:
        t0 = time.time()
        lat.step(equil)
        h = torch.zeros((replicas, 3, n_bins), dtype=torch.int64, device=lat.device)
        for _ in range(steps // every):
            lat.step(every)
            lat.histogram(n_bins, out=h)
        torch.cuda.synchronize(lat.device)
        wall = time.time() - t0
        rc = lat.check()
        mom = lat.moments()
    finally:
        lat.close()
    hist = h.sum(0).cpu().numpy()
    P = hist / hist.sum(1, keepdims=True)
    f1, f0 = parity_sector_means(float(sum(init)))
    return {"init": tuple(init), "L": L, "replicas": replicas, "C": C, "equil": equil,
            "steps": steps, "every": every, "hist": hist, "P": P,
            "pred_moving": poisson_pmf(f1, n_bins), "pred_rest": even_poisson_pmf(f0, n_bins),
            "pred_rest_unconstrained": poisson_pmf(f0 * math.tanh(f0), n_bins),
            "f1": f1, "f0": f0, "sum_N": [m["sum_N"] for m in mom],
            "sum_J": [m["sum_J"] for m in mom], "n0_odd": sum(m["n0_odd"] for m in mom),
            "check": rc, "wall_s": wall}


def equilibrium_means(us: Sequence[float], rho: float = 36.0, L: int = 100, C: int = 10,
                      equil: int = 15000, steps: int = 15000, every: int = 10, seed: int = 1,
                      blocks: int = 10) -> dict:
    """Fig. 3 set-up: one lattice per velocity u, all in one batched context,
    each started from the product-Poisson state at f^eq(rho, u); the site
    means are averaged every ``every`` steps over ``steps`` steps after
    ``equil`` steps.  The standard error comes from ``blocks`` batch means.
    Predictions use each lattice's own conserved rho^ = sum N / L and
    u^ = sum J / sum N."""
    us = np.asarray(us, dtype=np.float64)
    R = len(us)
    lat = mclg.Lattice([L] * R, seed, C=C, rho=np.full(R, rho), u0=us)
    try:
        t0 = time.time()
        lat.step(equil)
        n_samp = steps // every
        samples = np.zeros((n_samp, R, 3))
        for k in range(n_samp):
            lat.step(every)
            m = lat.moments()
            samples[k] = [[v / L for v in mr["sum_n"]] for mr in m]
        wall = time.time() - t0
        mom = lat.moments()
    finally:
        lat.close()
    mean = samples.mean(0)
    nb = max(2, min(blocks, n_samp))
    bm = np.array([b.mean(0) for b in np.array_split(samples, nb)])
    se = bm.std(0, ddof=1) / math.sqrt(nb)
    rho_hat = np.array([m["sum_N"] / L for m in mom])
    u_hat = np.array([m["sum_J"] / m["sum_N"] if m["sum_N"] else 0.0 for m in mom])
    return {"u0": us, "rho_hat": rho_hat, "u_hat": u_hat, "mean": mean, "se": se,
            "feq": np.array([feq(r, u) for r, u in zip(rho_hat, u_hat)]),
            "f_lb": np.array([f_lb(r, u) for r, u in zip(rho_hat, u_hat)]),
            "L": L, "C": C, "equil": equil, "steps": steps, "every": every, "wall_s": wall}


def pi_decay(init: Sequence[int] = (100, 100, 100), L: int = 1000, replicas: int = 1000,
             C: int = 10, steps: int = 100, stream: bool = True, seed: int = 1,
             n_max: int = 300, lam=(1, 1), galilean: bool = False) -> dict:
    """Fig. 5 set-up: ``replicas`` lattices of L sites, every site in state
    ``init``; records the ensemble mean of pi after every step (C collisions
    each) with or without streaming, and with the constant acceptance lambda
    or the Galilean-invariant one, lambda / sqrt(1 + 3 U^2).  The per-step
    mean is exact (integer sums); its standard error comes from the spread of
    the replica means."""
    flags = (0 if stream else mclg.FLAG_NO_STREAM) | (mclg.FLAG_GALILEAN if galilean else 0)
    lat = mclg.Lattice([L] * replicas, seed, C=C, lam=lam, n_max=n_max, flags=flags,
                       counts=uniform_counts(init, L, replicas))
    try:
        t0 = time.time()
        mean = np.zeros(steps + 1)
        se = np.zeros(steps + 1)
        for t in range(steps + 1):
            if t:
                lat.step(1)
            m = lat.moments()
            per = pi_moment(np.array([mr["sum_n"] for mr in m], dtype=np.float64)) / L
            mean[t] = per.mean()
            se[t] = per.std(ddof=1) / math.sqrt(replicas) if replicas > 1 else float("nan")
        wall = time.time() - t0
        rc = lat.check()
        sum_N = sum(mr["sum_N"] for mr in m)
    finally:
        lat.close()
    rho = float(sum(init))
    u = (init[2] - init[0]) / rho if rho else 0.0
    lam_f = lam[0] / lam[1] / (math.sqrt(1.0 + 3.0 * u * u) if galilean else 1.0)
    pi_eq = float(pi_moment(feq(rho, u)))
    n_coll = C * np.arange(steps + 1)
    pi0 = float(pi_moment(np.asarray(init))) - pi_eq
    return {"init": tuple(init), "L": L, "replicas": replicas, "C": C, "stream": stream,
            "galilean": galilean, "u": u, "rate": _decay_rate(mean - pi_eq, C),
            "mean": mean, "se": se, "pi_eq": pi_eq, "n_coll": n_coll,
            "pred_sqrt8": pi_eq + pi_relax(pi0, n_coll, rho, u, lam_f),
            "pred_printed": pi_eq + pi_relax(pi0, n_coll, rho, u, lam_f, coef=2 * math.sqrt(6)),
            "pred_linear": pi_eq + pi_relax_linear(pi0, n_coll, rho, lam_f),
            "sum_N": sum_N, "check": rc, "wall_s": wall}


def correlations(us: Sequence[float], rho: float = 36.0, L: int = 4096, C: int = 10,
                 equil: int = 1000, steps: int = 5000, every: int = 10, seed: int = 1,
                 blocks: int = 10, n_max: int = 255) -> dict:
    """Eq. (corr) and Eq. (error) for D1Q3: one lattice per velocity u, each
    started from the product-Poisson state at f^eq(rho, u); <n_i n_j> is the
    average over sites and over samples every ``every`` steps (after
    ``equil`` steps) of the exact sums of n_i n_j, normalised as
    K_ij = (<n_i n_j> - f_i f_j) / sqrt(f_i f_j) with f = f^eq(rho^, u^) from
    each lattice's conserved sums, and E(u) = sum_ij (K_ij - delta_ij)^2.
    The standard error of K comes from ``blocks`` batch means."""
    us = np.asarray(us, dtype=np.float64)
    R = len(us)
    lat = mclg.Lattice([L] * R, seed, C=C, n_max=n_max, rho=np.full(R, rho), u0=us)
    pairs = ((0, 1), (1, 2), (0, 2))  # order of sum_nn
    try:
        t0 = time.time()
        lat.step(equil)
        n_samp = steps // every
        samples = np.zeros((n_samp, R, 3, 3))
        for k in range(n_samp):
            lat.step(every)
            for r, m in enumerate(lat.moments()):
                for i in range(3):
                    samples[k, r, i, i] = m["sum_n2"][i] / L
                for (i, j), v in zip(pairs, m["sum_nn"]):
                    samples[k, r, i, j] = samples[k, r, j, i] = v / L
        wall = time.time() - t0
        mom = lat.moments()
        rc = lat.check()
    finally:
        lat.close()
    rho_hat = np.array([m["sum_N"] / L for m in mom])
    u_hat = np.array([m["sum_J"] / m["sum_N"] if m["sum_N"] else 0.0 for m in mom])
    f = np.array([feq(a, b) for a, b in zip(rho_hat, u_hat)])
    ff = np.sqrt(f[:, :, None] * f[:, None, :])
    norm = lambda nn: (nn - f[:, :, None] * f[:, None, :]) / ff  # noqa: E731
    K = norm(samples.mean(0))
    nb = max(2, min(blocks, n_samp))
    bK = np.array([norm(b.mean(0)) for b in np.array_split(samples, nb)])
    se = bK.std(0, ddof=1) / math.sqrt(nb)
    E = ((K - np.eye(3)) ** 2).sum((1, 2))
    return {"u0": us, "rho_hat": rho_hat, "u_hat": u_hat, "K": K, "se": se, "E": E,
            "L": L, "C": C, "equil": equil, "steps": steps, "every": every, "check": rc,
            "wall_s": wall}


# ---- D2Q9 -------------------------------------------------------------------
V9 = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]


def feq9(rho: float, ux: float, uy: float) -> np.ndarray:
    """Eq. (D2Q9eqdist): rho times the product of the unit-density D1Q3
    equilibria of the two velocity components."""
    fx, fy = feq(1.0, ux), feq(1.0, uy)
    return np.array([rho * fx[vx + 1] * fy[vy + 1] for vx, vy in V9])


def d2q9_statistics(us: Sequence[Sequence[float]], rho: float, Lx: int, Ly: int, C: int = 10,
                    equil: int = 20000, steps: int = 10000, every: int = 10, seed: int = 1,
                    blocks: int = 10, lams=None) -> dict:
    """One D2Q9 lattice per velocity (ux, uy), all in one context, each
    started from the product-Poisson state at Eq. (D2Q9eqdist); time averages
    every ``every`` steps over ``steps`` steps after ``equil`` of the site
    means <n_i> and of <n_i n_j>.  Returns the means, the normalised
    correlator K_ij = (<n_i n_j> - f_i f_j) / sqrt(f_i f_j) of Eq. (corr) at
    f = f^eq(rho^, u^) from each lattice's conserved sums, E(u) of
    Eq. (error), and batch-means standard errors."""
    us = np.asarray(us, dtype=np.float64).reshape(-1, 2)
    R = len(us)
    kw = {} if lams is None else {"lams": lams}
    lat = mclg.Lattice9([Lx] * R, Ly, seed, C=C, rho=np.full(R, rho), ux=us[:, 0], uy=us[:, 1], **kw)
    S = Lx * Ly
    iu = np.triu_indices(9)
    try:
        t0 = time.time()
        lat.step(equil)
        n_samp = steps // every
        mean_s = np.zeros((n_samp, R, 9))
        nn_s = np.zeros((n_samp, R, 9, 9))
        for k in range(n_samp):
            lat.step(every)
            for r, m in enumerate(lat.moments()):
                mean_s[k, r] = np.asarray(m["sum_n"], dtype=np.float64) / S
                up = np.zeros((9, 9))
                up[iu] = np.asarray(m["sum_nn"], dtype=np.float64) / S
                nn_s[k, r] = up + np.triu(up, 1).T
        wall = time.time() - t0
        mom = lat.moments()
        rc = lat.check()
    finally:
        lat.close()
    Vx = np.array([v[0] for v in V9])
    Vy = np.array([v[1] for v in V9])
    rho_hat = np.array([m["sum_N"] / S for m in mom])
    u_hat = np.array([[m["sum_Jx"] / m["sum_N"], m["sum_Jy"] / m["sum_N"]] for m in mom])
    f = np.array([feq9(a, *b) for a, b in zip(rho_hat, u_hat)])
    ff = np.sqrt(f[:, :, None] * f[:, None, :])
    norm = lambda nn: (nn - f[:, :, None] * f[:, None, :]) / ff  # noqa: E731
    nb = max(2, min(blocks, n_samp))
    mean = mean_s.mean(0)
    se = np.array([b.mean(0) for b in np.array_split(mean_s, nb)]).std(0, ddof=1) / math.sqrt(nb)
    K = norm(nn_s.mean(0))
    bK = np.array([norm(b.mean(0)) for b in np.array_split(nn_s, nb)])
    Kse = bK.std(0, ddof=1) / math.sqrt(nb)
    E = ((K - np.eye(9)) ** 2).sum((1, 2))
    assert np.allclose(Vx @ f.T, rho_hat * u_hat[:, 0]) and np.allclose(Vy @ f.T, rho_hat * u_hat[:, 1])
    return {"u0": us, "rho_hat": rho_hat, "u_hat": u_hat, "mean": mean, "se": se, "feq": f,
            "f_lb": np.array([f_lb9(a, *b) for a, b in zip(rho_hat, u_hat)]),
            "K": K, "K_se": Kse, "E": E, "Lx": Lx, "Ly": Ly, "C": C, "equil": equil,
            "steps": steps, "every": every, "check": rc, "wall_s": wall}


# Table 1 of the paper (the correlator of Eq. (corr) at its worst outlier,
# u_x = -0.68), rows and columns in the velocity numbering of Eq. (MomD2Q9)
TABLE1_PAPER = np.array([
    [0.998863, -0.000028, -0.000482, -0.000170, -0.000343, 0.000001, -0.000114, -0.000082, 0.000010],
    [-0.000028, 0.999171, 0.000001, 0.000143, -0.000072, -0.000127, -0.000047, 0.000013, 0.000057],
    [-0.000482, 0.000001, 0.999809, -0.000112, 0.000177, -0.000515, -0.000110, -0.000022, 0.000482],
    [-0.000170, 0.000143, -0.000112, 1.000230, -0.000079, 0.000014, 0.000008, -0.000048, -0.000067],
    [-0.000343, -0.000072, 0.000177, -0.000079, 0.999648, 0.000492, -0.000023, -0.000103, -0.000480],
    [0.000001, -0.000127, -0.000515, 0.000014, 0.000492, 0.999567, -0.000065, -0.000046, 0.000593],
    [-0.000114, -0.000047, -0.000110, 0.000008, -0.000023, -0.000065, 0.999801, -0.000085, 0.000086],
    [-0.000082, 0.000013, -0.000022, -0.000048, -0.000103, -0.000046, -0.000022, 0.999687, -0.000117],
    [0.000010, 0.000057, 0.000482, -0.000067, -0.000480, 0.000593, 0.000086, -0.000117, 0.999215]])
# (the n_5 diagonal is printed -0.999567; Eq. (corr) makes it +0.999567)


def finite_size_correlator(f: np.ndarray, S: int) -> np.ndarray:
    """The correlator of Eq. (corr) that exact conservation predicts on a
    lattice of S sites: the stationary law is the product-Poisson measure
    conditioned on the totals of N, Jx, Jy, whose single-site covariance is
    D - D M^T (M D M^T)^-1 M D / S to leading order (D = diag f, M the rows
    1, v_x, v_y), while the mean stays f^eq at the conserved (rho, u); hence
    K = 1 - P / S with P = D^1/2 M^T (M D M^T)^-1 M D^1/2, a projector of
    rank 3 (the sum of its diagonal is 3)."""
    M = np.array([[1.0] * 9, [float(v[0]) for v in V9], [float(v[1]) for v in V9]])
    D = np.diag(f)
    sq = np.diag(np.sqrt(f))
    P = sq @ M.T @ np.linalg.inv(M @ D @ M.T) @ M @ sq
    return np.eye(9) - P / S


def table1_correlator(ux: float = -0.68, uy: float = 0.0, rho: float = 360.0, Lx: int = 100,
                      Ly: int = 10, C: int = 10, replicas: int = 4096, equil: int = 2000,
                      steps: int = 300_000, every: int = 25, seed: int = 360) -> dict:
    """The paper's Table 1 set-up (rho = 360, 100 x 10, C = 10, the lambda_c
    of its D2Q9 runs) as `replicas` independent lattices in one context,
    Poisson-started at Eq. (D2Q9eqdist), sampled every `every` steps.  Per
    replica: the correlator of Eq. (corr) with f = f^eq at the replica's
    conserved (rho^, u^) ("K"), the same with the replica's measured means
    ("K_cov"), and the finite-size prediction; the replicas are independent,
    so the standard errors come from their scatter."""
    iu = np.triu_indices(9)
    S = Lx * Ly
    lat = mclg.Lattice9([Lx] * replicas, Ly, seed, C=C, rho=np.full(replicas, rho),
                        ux=np.full(replicas, ux), uy=np.full(replicas, uy))
    t0 = time.time()
    try:
        lat.step(equil)
        n_samp = steps // every
        sn = np.zeros((replicas, 9))
        snn = np.zeros((replicas, 45))
        for _ in range(n_samp):
            lat.step(every)
            a = lat.moments_array()
            sn += a[:, 2:11]
            snn += a[:, 11:56]
        a = lat.moments_array()
        rc = lat.check()
    finally:
        lat.close()
    wall = time.time() - t0
    N, Jx, Jy = a[:, 56].astype(np.float64), a[:, 57].astype(np.float64), a[:, 58].astype(np.float64)
    rho_hat, u_hat = N / S, np.stack([Jx / N, Jy / N], 1)
    mean = sn / (n_samp * S)
    nn = np.zeros((replicas, 9, 9))
    nn[:, iu[0], iu[1]] = snn / (n_samp * S)
    nn = nn + np.triu(nn, 1).transpose(0, 2, 1)
    f = np.array([feq9(r, *u) for r, u in zip(rho_hat, u_hat)])
    K_r = (nn - f[:, :, None] * f[:, None, :]) / np.sqrt(f[:, :, None] * f[:, None, :])
    Kc_r = (nn - mean[:, :, None] * mean[:, None, :]) / np.sqrt(mean[:, :, None] * mean[:, None, :])
    pred_r = np.array([finite_size_correlator(x, S) for x in f])
    se = lambda x: x.std(0, ddof=1) / np.sqrt(replicas)  # noqa: E731
    K, Kc, pred = K_r.mean(0), Kc_r.mean(0), pred_r.mean(0)
    return {"ux": ux, "uy": uy, "rho": rho, "Lx": Lx, "Ly": Ly, "C": C, "replicas": replicas,
            "equil": equil, "steps": steps, "every": every, "wall_s": wall, "check": rc,
            "rho_hat": float(rho_hat.mean()), "u_hat": u_hat.mean(0),
            "K": K, "K_se": se(K_r), "K_cov": Kc, "K_cov_se": se(Kc_r), "pred": pred,
            "E": float(((K - np.eye(9)) ** 2).sum()), "E_pred": float(((pred - np.eye(9)) ** 2).sum()),
            "paper": TABLE1_PAPER * np.where(np.eye(9, dtype=bool) & (TABLE1_PAPER < 0), -1, 1)}


def d2q9_histograms(ux: float = -0.25, uy: float = 0.25, rho: float = 18.0, Lx: int = 512,
                    Ly: int = 512, C: int = 10, equil: int = 200, n_bins: int = 48,
                    seed: int = 1) -> dict:
    """The Poisson-histogram figure of the D2Q9 section: occupation-number
    distributions of every velocity after ``equil`` steps from the
    product-Poisson start at (rho, ux, uy) (one snapshot of Lx * Ly
    independent sites), beside Poisson(f_i^eq) of Eq. (D2Q9eqdist)."""
    lat = mclg.Lattice9(Lx, Ly, seed, C=C, rho=rho, ux=ux, uy=uy)
    try:
        lat.step(equil)
        h = lat.histogram(n_bins).cpu().numpy()[0]
        rc = lat.check()
        m = lat.moments()[0]
    finally:
        lat.close()
    S = Lx * Ly
    f = feq9(m["sum_N"] / S, m["sum_Jx"] / m["sum_N"], m["sum_Jy"] / m["sum_N"])
    return {"hist": h, "P": h / S, "pred": np.array([poisson_pmf(fi, n_bins) for fi in f]),
            "f": f, "check": rc, "sites": S}


def f_lb9(rho: float, ux: float, uy: float) -> np.ndarray:
    """Eq. (LBequil) for D2Q9 (weights 4/9, 1/9, 1/36, theta = 1/3)."""
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    vu = np.array([vx * ux + vy * uy for vx, vy in V9])
    return rho * w * (1 + 3 * vu + 4.5 * vu ** 2 - 1.5 * (ux * ux + uy * uy))


# ---- command line -----------------------------------------------------------
def _fig1(quick: bool):
    kw = dict(equil=2000, steps=8000, replicas=8) if quick else {}
    r = parity_histograms(**kw)
    print(f"Fig. 1  init {r['init']}  L={r['L']} x {r['replicas']}  C={r['C']}  "
          f"{r['equil']} + {r['steps']} steps  ({r['wall_s']:.1f} s)")
    print(f"  closed form: f_1 = {r['f1']:.6f}, f_0 = {r['f0']:.6f}; "
          f"odd rest counts at the end: {r['n0_odd']}")
    print("   n   P(n_-1)   P(n_+1)  Poisson(f1)   P(n_0)  even-Poisson(f0)  Poisson(<n0>)")
    for n in range(0, 21):
        print(f"  {n:2d}  {r['P'][0, n]:.5f}   {r['P'][2, n]:.5f}   {r['pred_moving'][n]:.5f}"
              f"     {r['P'][1, n]:.5f}   {r['pred_rest'][n]:.5f}           "
              f"{r['pred_rest_unconstrained'][n]:.5f}")


def _fig3(quick: bool):
    us = np.round(np.linspace(-0.9, 0.9, 19), 6)
    kw = dict(equil=1500, steps=1500) if quick else {}
    r = equilibrium_means(us, **kw)
    print(f"Fig. 3  rho=36  L={r['L']}  C={r['C']}  {r['equil']} + {r['steps']} steps, "
          f"every {r['every']}  ({r['wall_s']:.1f} s)")
    print("      u^   <n_-1>  f^eq_-1     <n_0>   f^eq_0    <n_+1>  f^eq_+1   |  f^LB (-1, 0, +1)")
    for k in range(len(us)):
        m, f, g = r["mean"][k], r["feq"][k], r["f_lb"][k]
        print(f"  {r['u_hat'][k]:+.4f}  {m[0]:7.3f}  {f[0]:7.3f}   {m[1]:7.3f}  {f[1]:7.3f}   "
              f"{m[2]:7.3f}  {f[2]:7.3f}   | {g[0]:7.3f} {g[1]:7.3f} {g[2]:7.3f}")


def _fig5(quick: bool):
    kw = dict(replicas=100, steps=60) if quick else dict(steps=150)
    for init in ((100, 100, 100), (0, 300, 0), (150, 0, 150)):
        for stream in (True, False):
            r = pi_decay(init, stream=stream, **kw)
            print(f"Fig. 5  init {init}  {'streaming' if stream else 'no streaming'}  "
                  f"L={r['L']} x {r['replicas']}  C={r['C']}  ({r['wall_s']:.1f} s)")
            print("   collisions   <pi>      se     Eq.relax(sqrt8)  Eq.relax(printed)  linear")
            for t in sorted(set([0, 1, 2, 5, 10, 20, 50, 100, len(r['mean']) - 1])):
                if t < len(r["mean"]):
                    print(f"   {r['n_coll'][t]:9d}  {r['mean'][t]:9.3f}  {r['se'][t]:6.3f}  "
                          f"{r['pred_sqrt8'][t]:12.3f}  {r['pred_printed'][t]:14.3f}  "
                          f"{r['pred_linear'][t]:9.3f}")


def _corr(quick: bool):
    us = np.round(np.linspace(-0.8, 0.8, 9), 6)
    kw = dict(equil=200, steps=1000) if quick else dict(L=1 << 16, steps=20000)
    r = correlations(us, **kw)
    print(f"Eq. (corr), Eq. (error)  rho=36  L={r['L']}  C={r['C']}  {r['equil']} + "
          f"{r['steps']} steps, every {r['every']}  ({r['wall_s']:.1f} s)")
    print("      u^    K_-1-1   K_00     K_11     K_-10     K_01     K_-11      E(u)")
    for k in range(len(us)):
        K = r["K"][k]
        print(f"  {r['u_hat'][k]:+.4f}  {K[0, 0]:.5f}  {K[1, 1]:.5f}  {K[2, 2]:.5f}  "
              f"{K[0, 1]:+.5f}  {K[1, 2]:+.5f}  {K[0, 2]:+.5f}  {r['E'][k]:.2e}")


def linear_rate(mean: np.ndarray, C: int, t1: int = 5) -> float:
    """Per-collision linear relaxation rate from successive differences,
    -ln(((pi(t1 + 1) - pi(t1)) / (pi(1) - pi(0)))^(1 / t1)) / C, which does
    not need the value pi relaxes to."""
    r = (mean[t1 + 1] - mean[t1]) / (mean[1] - mean[0])
    return -math.log(r) / (C * t1) if r > 0 else float("nan")


def galilean_rates(us: Sequence[float] = (0.0, 0.25, 0.5, 0.75), N: int = 240, C: int = 10,
                   L: int = 1000, replicas: int = 500, seed: int = 1) -> dict:
    """Linear relaxation rate of pi without streaming at N particles per site
    and site velocity U = J / N, with the constant acceptance (lambda = 1)
    and the Galilean-invariant one.  Every site starts 8 rest particles below
    the even count nearest f_0^eq(N, U); the prediction of Eq. (D1Q3relax)
    for small deviations is lambda sqrt(1 + 3 U^2) / N per collision, i.e.
    1 / N for the Galilean-invariant lambda at every U."""
    rows = []
    for u in us:
        J = int(round(u * N))
        f = feq(float(N), J / N)
        b = 2 * int(round(f[1] / 2)) - 8
        a = (N - b - J) // 2
        init = (a, N - 2 * a - J, a + J)
        r = []
        for gal in (False, True):
            d = pi_decay(init, L=L, replicas=replicas, C=C, steps=6, stream=False, n_max=N,
                         seed=seed, galilean=gal)
            r.append(linear_rate(d["mean"], C))
        rows.append({"u": J / N, "init": init, "rate": r[0], "rate_galilean": r[1],
                     "pred": math.sqrt(1 + 3 * (J / N) ** 2) / N, "pred_galilean": 1.0 / N})
    return {"N": N, "C": C, "L": L, "replicas": replicas, "rows": rows}


def _galilean(quick: bool):
    r = galilean_rates(replicas=50 if quick else 500)
    print(f"Galilean-invariant acceptance: N = {r['N']} per site, C = {r['C']}, no streaming, "
          f"L = {r['L']} x {r['replicas']}")
    print("     U    init              rate      lambda s / N   rate Galilean  lambda / N")
    for w in r["rows"]:
        print(f"  {w['u']:4.2f}  {str(w['init']):16s}  {w['rate']:.6f}  {w['pred']:.6f}       "
              f"{w['rate_galilean']:.6f}       {w['pred_galilean']:.6f}")


def _d2q9eq(quick: bool):
    uxs = np.round(np.linspace(-0.6, 0.6, 13), 6)
    kw = dict(equil=2000, steps=1000) if quick else {}
    r = d2q9_statistics([(u, 0.25) for u in uxs], 36.0, 100, 10, **kw)
    print(f"D2Q9 equilibrium (Fig. of Eq. (D2Q9eqdist)): rho=36, uy=0.25, 100x10, C={r['C']}, "
          f"{r['equil']} + {r['steps']} steps, every {r['every']} ({r['wall_s']:.1f} s)")
    print("   ux^     " + "  ".join(f"<n{i}>/f{i}".rjust(11) for i in range(9)))
    for k in range(len(uxs)):
        cells = "  ".join(f"{r['mean'][k, i]:5.2f}/{r['feq'][k, i]:5.2f}" for i in range(9))
        print(f"  {r['u_hat'][k, 0]:+.3f}  {cells}")


def _d2q9hist(quick: bool):
    r = d2q9_histograms(Lx=128 if quick else 512, Ly=128 if quick else 512)
    print(f"D2Q9 occupation numbers at U = (-0.25, 0.25), rho = 18, {r['sites']} sites "
          f"(one snapshot after 200 steps)")
    print("   n   " + "   ".join(f"P(n{i}) Poisson".rjust(15) for i in (0, 1, 2, 7)))
    for n in range(0, 16):
        print(f"  {n:2d}  " + "   ".join(f"{r['P'][i, n]:.5f} {r['pred'][i, n]:.5f}" for i in (0, 1, 2, 7)))


def _table1(quick: bool):
    kw = dict(replicas=1024, steps=20_000) if quick else {}
    r = table1_correlator(**kw)
    print(f"Table 1 set-up (Eq. (corr)): rho={r['rho']}, ux={r['ux']}, uy={r['uy']}, "
          f"{r['Lx']}x{r['Ly']}, C={r['C']}, {r['replicas']} replicas, {r['equil']} + "
          f"{r['steps']} steps sampled every {r['every']} ({r['wall_s']:.1f} s, check {r['check']})")
    for name, key in (("measured K (f = f^eq at the conserved rho, u)", "K"),
                      ("measured K with the replicas' own means", "K_cov"),
                      ("finite-size prediction 1 - P/S", "pred"),
                      ("paper, Table 1 (n_5 diagonal sign restored)", "paper")):
        print(f"  {name}:")
        for i in range(9):
            print("   " + " ".join(f"{v:+.6f}" for v in r[key][i]))
    print(f"  standard errors of K: {r['K_se'].min():.1e} .. {r['K_se'].max():.1e}; of K_cov: "
          f"{r['K_cov_se'].min():.1e} .. {r['K_cov_se'].max():.1e}")
    z = np.abs(r["K"] - r["pred"]) / r["K_se"]
    zc = np.abs(r["K_cov"] - r["pred"]) / r["K_cov_se"]
    print(f"  largest |K - prediction| / se {z.max():.2f}, |K_cov - prediction| / se {zc.max():.2f}")
    print(f"  E(u) measured {r['E']:.3e}, predicted {r['E_pred']:.3e}, paper "
          f"{((r['paper'] - np.eye(9)) ** 2).sum():.3e}")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("figure", choices=["fig1", "fig3", "fig5", "corr", "galilean", "d2q9eq",
                                       "d2q9hist", "table1"])
    ap.add_argument("--quick", action="store_true", help="reduced step counts")
    a = ap.parse_args(argv)
    {"fig1": _fig1, "fig3": _fig3, "fig5": _fig5, "corr": _corr,
     "galilean": _galilean, "d2q9eq": _d2q9eq, "d2q9hist": _d2q9hist,
     "table1": _table1}[a.figure](a.quick)


if __name__ == "__main__":
    main()
