"""Exact law of the paper's sub-collision loop, by brute-force enumeration.

Written from the paper's description of one sub-collision (Eq. (select),
Eq. (omega), the D1Q3 transition table of Sec. "A D1Q3 implementation"):
pick an ordered pair of two distinct particles uniformly, identify their
velocities by cumulative sums in the order -1, 0, +1, then apply an outgoing
pair with the tabulated probability.  Everything is exact (``Fraction``) and
enumerates particles one by one, so it shares nothing with the oracle's
tridiagonal integer weights: it is a pin for them.
"""
import math
from fractions import Fraction
from functools import lru_cache

import numpy as np

# D1Q3 transition probabilities, "A D1Q3 implementation" (lambda symbolic).
def transition_table(lam: Fraction):
    return {
        (-1, 1): {(0, 0): lam, (-1, 1): 1 - lam, (1, -1): Fraction(0)},
        (1, -1): {(0, 0): lam, (1, -1): 1 - lam, (-1, 1): Fraction(0)},
        (0, 0): {(0, 0): 1 - lam / 8, (-1, 1): lam / 16, (1, -1): lam / 16},
    }


def one_subcollision(state, lam: Fraction):
    """Exact distribution of the state (a, b, c) after one sub-collision."""
    a, b, c = state
    N = a + b + c
    if N < 2:
        return {state: Fraction(1)}
    vel = [-1] * a + [0] * b + [1] * c  # particle r has velocity vel[r]
    table = transition_table(lam)
    out = {}
    npairs = N * (N - 1)
    for r1 in range(N):
        for r2 in range(N):
            if r1 == r2:
                continue
            s1, s2 = vel[r1], vel[r2]
            outs = table.get((s1, s2), {(s1, s2): Fraction(1)})
            for (s3, s4), p in outs.items():
                if p == 0:
                    continue
                n = {-1: a, 0: b, 1: c}
                n[s1] -= 1; n[s2] -= 1; n[s3] += 1; n[s4] += 1  # Eq. (omega)
                key = (n[-1], n[0], n[1])
                out[key] = out.get(key, Fraction(0)) + p / npairs
    return out


def c_step_law(state, C: int, lam: Fraction):
    dist = {tuple(state): Fraction(1)}
    cache = {}
    for _ in range(C):
        nd = {}
        for s, p in dist.items():
            if s not in cache:
                cache[s] = one_subcollision(s, lam)
            for s2, q in cache[s].items():
                nd[s2] = nd.get(s2, Fraction(0)) + p * q
        dist = nd
    return dist


def rest_marginal(dist, N: int, absJ: int):
    """Probabilities of n0' over the fiber's states in ascending n0'."""
    par = (N - absJ) % 2
    m = (N - absJ) // 2 + 1
    probs = [Fraction(0)] * m
    for (a, b, c), p in dist.items():
        probs[(b - par) // 2] += p
    return probs


def quantise(probs):
    """floor(2^32 * cumulative) for all but the last outcome."""
    out, cum = [], Fraction(0)
    for p in probs[:-1]:
        cum += p
        out.append((cum.numerator << 32) // cum.denominator)
    return out


def fiber_stationary(N: int, J: int, lam: Fraction):
    """Stationary law on the (N, J) fiber of the one-sub-collision chain,
    found by power-free exact linear algebra on the enumerated kernel."""
    absJ = abs(J)
    par = (N - absJ) % 2
    m = (N - absJ) // 2 + 1
    states = []
    for k in range(m):
        b = par + 2 * k
        a = (N - b - J) // 2
        c = (N - b + J) // 2
        states.append((a, b, c))
    idx = {s: i for i, s in enumerate(states)}
    T = [[Fraction(0)] * m for _ in range(m)]
    for s in states:
        for s2, p in one_subcollision(s, lam).items():
            T[idx[s]][idx[s2]] += p
    # birth-death chain: detailed balance pi_{k+1} T[k+1][k] = pi_k T[k][k+1]
    pi = [Fraction(1)]
    for k in range(m - 1):
        pi.append(pi[-1] * T[k][k + 1] / T[k + 1][k])
    Z = sum(pi)
    return [p / Z for p in pi]


def one_subcollision_counted(state, lam: Fraction):
    """Same law as ``one_subcollision`` with the ordered distinct pairs of
    velocities (s1, s2) counted as n_s1 (n_s2 - [s1 == s2]) instead of
    enumerated particle by particle (fast for large N)."""
    a, b, c = state
    N = a + b + c
    if N < 2:
        return {state: Fraction(1)}
    n = {-1: a, 0: b, 1: c}
    table = transition_table(lam)
    out = {}
    npairs = N * (N - 1)
    for s1 in (-1, 0, 1):
        for s2 in (-1, 0, 1):
            mult = n[s1] * (n[s2] - (1 if s1 == s2 else 0))
            if mult <= 0:
                continue
            outs = table.get((s1, s2), {(s1, s2): Fraction(1)})
            for (s3, s4), p in outs.items():
                if p == 0:
                    continue
                m = dict(n)
                m[s1] -= 1; m[s2] -= 1; m[s3] += 1; m[s4] += 1
                key = (m[-1], m[0], m[1])
                out[key] = out.get(key, Fraction(0)) + p * Fraction(mult, npairs)
    return out


def no_stream_pi_moments(abc, C, steps, lam: Fraction = Fraction(1)):
    """(E[pi], E[pi^2]) after ``steps`` steps of C sub-collisions at one site
    that never streams, started in state abc, with pi = sqrt(2) (n_-1 - n_0/2
    + n_+1): the fiber chain of ``one_subcollision_counted`` at acceptance
    ``lam`` (exact probabilities, propagated in float64)."""
    N = sum(abc)
    J = abc[2] - abc[0]
    absJ = abs(J)
    par = (N - absJ) % 2
    m = (N - absJ) // 2 + 1
    T = np.zeros((m, m))
    for k in range(m):
        b = par + 2 * k
        a, c = (N - b - J) // 2, (N - b + J) // 2
        for s2, p in one_subcollision_counted((a, b, c), lam).items():
            T[k, (s2[1] - par) // 2] += float(p)
    v = np.zeros(m)
    v[(abc[1] - par) // 2] = 1.0
    TC = np.linalg.matrix_power(T, C * steps)
    v = v @ TC
    b = par + 2 * np.arange(m)
    pi = math.sqrt(2) * ((N - b) - b / 2)
    return float(v @ pi), float(v @ pi**2)
