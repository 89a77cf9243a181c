"""Pins of the oracle against what the paper and the mathematics fix.

Every test here runs on the CPU.  None of them compares the oracle with
itself: the exact laws come from brute-force enumeration of the paper's
literal sub-collision loop (tests/exact_law.py), from the paper's printed
values (tests/golden/), from closed forms, invariants, and library routines
(scipy's Poisson law, rocRAND's Philox).
"""
import json
import math
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle as O
from tests import exact_law as X

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# RNG
# --------------------------------------------------------------------------
def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(w, 16) for w in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(ctr, key, expect):
    assert list(O.philox(ctr, key)) == expect


ROCRAND_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned int v[][6] = {
    {0u, 0u, 0u, 0u, 1u, 0u}, {12345u, 7u, 99u, 0u, 0xdeadbeefu, 42u},
    {4294967295u, 1u, 2u, 3u, 5u, 6u}, {17u, 1000u, 3u, 1u, 2u, 0u}};
  for (auto &r : v) {
    unsigned long long seed = (unsigned long long)r[4] | ((unsigned long long)r[5] << 32);
    unsigned long long subseq = (unsigned long long)r[2] | ((unsigned long long)r[3] << 32);
    unsigned long long offset = 4ull * ((unsigned long long)r[0] | ((unsigned long long)r[1] << 32));
    rocrand_device::philox4x32_10_engine e(seed, subseq, offset);
    unsigned int a = e.next(), b = e.next(), c = e.next(), d = e.next();
    printf("%u %u %u %u %u %u %u %u %u %u\n", r[0], r[1], r[2], r[3], r[4], r[5], a, b, c, d);
  }
}
"""


def test_philox_matches_rocrand(tmp_path):
    """rocRAND's open-source Philox engine, called (not copied), as a second
    independent source of Philox4x32-10 values."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = tmp_path / "probe.cpp"
    src.write_text(ROCRAND_PROBE)
    exe = tmp_path / "probe"
    subprocess.run([hipcc, "-O1", "--offload-arch=gfx950", str(src), "-o", str(exe)], check=True,
                   capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    for line in out.strip().splitlines():
        v = [int(w) for w in line.split()]
        assert list(O.philox(v[0:4], v[4:6])) == v[6:10]


# --------------------------------------------------------------------------
# Collision law
# --------------------------------------------------------------------------
def _states(N):
    for a in range(N + 1):
        for b in range(N + 1 - a):
            yield a, b, N - a - b


@pytest.mark.parametrize("C", [1, 2, 3])
@pytest.mark.parametrize("lam", [(1, 1), (1, 2), (3, 4)])
def test_rows_equal_brute_force_small(C, lam):
    """Exact quantised rows equal the enumerated law of the literal loop."""
    lf = Fraction(*lam)
    for N in range(0, 6):
        for a, b, c in _states(N):
            J = c - a
            dist = X.c_step_law((a, b, c), C, lf)
            want = X.quantise(X.rest_marginal(dist, N, abs(J)))
            got = O.row_thresholds(C, lam, N, abs(J), b)
            assert [int(v) for v in got] == want, (a, b, c)


@pytest.mark.parametrize("N", [6, 8])
def test_rows_equal_brute_force_c10(N):
    lam = (1, 1)
    for a, b, c in _states(N):
        if c < a:
            continue
        dist = X.c_step_law((a, b, c), 10, Fraction(1))
        want = X.quantise(X.rest_marginal(dist, N, c - a))
        got = O.row_thresholds(10, lam, N, c - a, b)
        assert [int(v) for v in got] == want, (a, b, c)


def test_paper_transition_table():
    """The printed D1Q3 table: from (1,0,1) one sub-collision brings the pair
    to rest with probability lambda; from (0,2,0) the rest pair leaves with
    lambda/16 + lambda/16."""
    g = json.load(open(os.path.join(GOLDEN, "paper_d1q3.json")))
    tp = g["transition_probabilities"]
    for lam in [(1, 1), (1, 2), (3, 4)]:
        lf = lam[0] / lam[1]
        p_rest = tp["P_-11_to_00"][0] * lf + tp["P_-11_to_00"][1]
        p_leave = (tp["P_00_to_-11"][0] + tp["P_00_to_1-1"][0]) * lf
        thr = O.row_thresholds(1, lam, 2, 0, 0)  # outcomes n0' = 0, 2
        assert int(thr[0]) == math.floor((1 - p_rest) * 2**32)
        thr = O.row_thresholds(1, lam, 2, 0, 2)
        assert int(thr[0]) == math.floor(p_leave * 2**32)
    r = g["detailed_balance_ratio"]["value"]
    assert Fraction(tp["P_00_to_-11"][0]).limit_denominator() / Fraction(tp["P_-11_to_00"][0]) == Fraction(*r)
    w = g["weights"]
    assert Fraction(*w["w_m1"]) * Fraction(*w["w_p1"]) / Fraction(*w["w_0"]) ** 2 == Fraction(*r)


def test_counted_pairs_equal_enumerated_pairs():
    for N in range(0, 7):
        for st in _states(N):
            for lam in (Fraction(1), Fraction(2, 3)):
                assert X.one_subcollision_counted(st, lam) == X.one_subcollision(st, lam)


def test_local_equilibrium_rows():
    """C = infinity rows equal the exact stationary law of the enumerated
    one-sub-collision chain (detailed balance, Eq. (transprob))."""
    g = json.load(open(os.path.join(GOLDEN, "paper_d1q3.json")))
    # N = 2, J = 0: outcomes n0' = 0 -> (1,0,1), n0' = 2 -> (0,2,0)
    pi = X.fiber_stationary(2, 0, Fraction(1))
    want = g["local_equilibrium_N2_printed"]["distinct_pair_reading"]
    assert pi[1] == Fraction(*want[0]) and pi[0] == Fraction(*want[1])
    for N in range(2, 9):
        for J in range(0, N + 1):
            if (N - J) // 2 + 1 < 2:
                continue
            want_thr = X.quantise(X.fiber_stationary(N, J, Fraction(1)))
            for b in range((N - J) % 2, N - J + 1, 2):
                got = O.row_thresholds(O.C_EQUILIBRIUM, (1, 1), N, J, b)
                assert [int(v) for v in got] == want_thr, (N, J, b)


def test_local_equilibrium_pi_moment():
    """Eq. (local): N = 1 has pi = -sqrt(1/2); N = 2 under the distinct-pair
    reading has E[pi] = -(4/3) sqrt(1/2) (the printed -28/17 sqrt(1/2)
    follows from 16/17 : 1/17)."""
    g = json.load(open(os.path.join(GOLDEN, "paper_d1q3.json")))

    def pi(a, b, c):  # pi = sqrt(2) (n_-1 - n_0 / 2 + n_1), Sec. D1Q3 results
        return math.sqrt(2) * (a - b / 2 + c)

    assert pi(0, 1, 0) == pytest.approx(g["local_equilibrium_N1"]["pi"], abs=1e-15)
    thr = O.row_thresholds(O.C_EQUILIBRIUM, (1, 1), 2, 0, 0)
    p101 = int(thr[0]) / 2**32
    e_pi = p101 * pi(1, 0, 1) + (1 - p101) * pi(0, 2, 0)
    assert e_pi == pytest.approx(-(4 / 3) * math.sqrt(0.5), abs=1e-8)


def test_mean_subcollision_matches_paper_mean_field():
    """Eq. (collmatD1Q3): the mean change of n0 in one sub-collision tends to
    lambda/rho^2 (4 f_-1 f_1 - f_0^2 / 4) for large N."""
    for (a, b, c) in [(300, 1200, 500), (700, 400, 900)]:
        N, J = a + b + c, c - a
        thr = O.row_thresholds(1, (1, 1), N, abs(J), b)
        edges = np.concatenate([[0], thr.astype(np.float64), [2.0**32]])
        p = np.diff(edges) / 2**32
        par = (N - abs(J)) % 2
        n0p = par + 2 * np.arange(len(p))
        mean_delta = float((p * (n0p - b)).sum())
        paper = (4 * a * c - b * b / 4) / N**2
        assert mean_delta == pytest.approx(paper, rel=10.0 / N, abs=2e-6)


def _chi2_pvalue(counts, probs, n):
    exp = np.asarray(probs, dtype=np.float64) * n
    obs = np.asarray(counts, dtype=np.float64)
    # merge bins until each expected count is >= 5
    e_m, o_m, ea, oa = [], [], 0.0, 0.0
    for e, o in zip(exp, obs):
        ea += e; oa += o
        if ea >= 5:
            e_m.append(ea); o_m.append(oa); ea = oa = 0.0
    if ea > 0:
        e_m[-1] += ea; o_m[-1] += oa
    assert abs(sum(o_m) - n) < 0.5
    chi2 = sum((o - e) ** 2 / e for o, e in zip(o_m, e_m))
    return stats.chi2.sf(chi2, len(e_m) - 1)


@pytest.mark.parametrize("abc,C", [((1, 2, 1), 1), ((1, 2, 2), 10), ((0, 8, 0), 10), ((2, 2, 2), 3)])
@pytest.mark.parametrize("direct", [False, True])
def test_sampler_chi_squared(abc, C, direct):
    """Table sampler and literal direct sampler both follow the exact law
    (Bonferroni over 8 cases: p > 1e-3 each)."""
    n = 1_000_000
    h = O.histogram(C, (1, 1), abc, n, seed=7, t=3, direct=direct)
    N = sum(abc)
    J = abc[2] - abc[0]
    probs = X.rest_marginal(X.c_step_law(abc, C, Fraction(1)), N, abs(J))
    par = (N - abs(J)) % 2
    counts = [int(h[par + 2 * k]) for k in range(len(probs))]
    assert sum(counts) == n  # nothing outside the fiber
    assert _chi2_pvalue(counts, [float(p) for p in probs], n) > 1e-3


# lambda = (3 2^25 + 1) / (3 2^26): the literal loop's uniform integers below
# q = 3 2^26 and 8 q reject 1/64 and 1/4 of their 32-bit words (2^32 mod q =
# 2^26, 2^32 mod 8q = 2^30), so Lemire's rejection step runs often
LAMBDA_REJECT = (3 * 2**25 + 1, 3 * 2**26)


@pytest.mark.parametrize("abc,C", [((1, 2, 1), 1), ((2, 6, 3), 10), ((0, 8, 0), 3)])
@pytest.mark.parametrize("direct", [False, True])
def test_sampler_chi_squared_with_rejections(abc, C, direct):
    """With a lambda whose Bernoulli draws reject often, the table sampler
    and the literal loop still follow the exact law (p > 1e-3 each)."""
    n = 1_000_000
    h = O.histogram(C, LAMBDA_REJECT, abc, n, seed=13, t=5, direct=direct)
    N = sum(abc)
    J = abc[2] - abc[0]
    lam = Fraction(*LAMBDA_REJECT)
    probs = X.rest_marginal(X.c_step_law(abc, C, lam), N, abs(J))
    par = (N - abs(J)) % 2
    counts = [int(h[par + 2 * k]) for k in range(len(probs))]
    assert sum(counts) == n
    assert _chi2_pvalue(counts, [float(p) for p in probs], n) > 1e-3


def test_direct_and_table_have_equal_law_large_n():
    """At N = 40 the direct loop and the table draw agree in distribution
    (two-sample chi-squared)."""
    abc = (6, 25, 9)
    n = 400_000
    h1 = O.histogram(10, (1, 1), abc, n, seed=11, t=0, direct=False).astype(np.float64)
    h2 = O.histogram(10, (1, 1), abc, n, seed=12, t=0, direct=True).astype(np.float64)
    keep = (h1 + h2) >= 10
    tab = np.vstack([h1[keep], h2[keep]])
    _, p, _, _ = stats.chi2_contingency(tab)
    assert p > 1e-3


# --------------------------------------------------------------------------
# Streaming, conservation, invariants
# --------------------------------------------------------------------------
def test_pure_streaming_is_a_shift():
    """With C = 0 the evolution equation is n_i(x + v_i, t + 1) = n_i(x, t)."""
    rng = np.random.default_rng(0)
    L = 37
    c0 = rng.integers(0, 50, size=(3, L), dtype=np.uint16)
    s = O.OracleSim([L], seed=3, C=0)
    s.init_counts(0, c0)
    s.step(5)
    got = s.counts(0)
    assert np.array_equal(got[0], np.roll(c0[0], -5))
    assert np.array_equal(got[1], c0[1])
    assert np.array_equal(got[2], np.roll(c0[2], 5))


def test_collision_conserves_mass_and_momentum_per_site():
    rng = np.random.default_rng(1)
    L = 4096
    c0 = rng.poisson([[3.0], [12.0], [5.0]], size=(3, L)).astype(np.uint16)
    s = O.OracleSim([L], seed=5, C=10, flags=O.FLAG_NO_STREAM)
    s.init_counts(0, c0)
    for _ in range(5):
        s.step(1)
        c = s.counts(0).astype(np.int64)
        assert np.array_equal(c.sum(0), c0.astype(np.int64).sum(0))
        assert np.array_equal(c[2] - c[0], c0[2].astype(np.int64) - c0[0])
        assert np.array_equal(c[1] & 1, c0[1].astype(np.int64) & 1)
    assert not np.array_equal(s.counts(0), c0)


def test_global_conservation_and_rest_parity_with_streaming():
    s = O.OracleSim([1000], seed=9, C=10)
    s.init_poisson(0, 30.0, 0.05)
    c0 = s.counts(0).astype(np.int64)
    m0 = s.moments(0)
    s.step(50)
    m1 = s.moments(0)
    c1 = s.counts(0).astype(np.int64)
    assert m1["sum_N"] == m0["sum_N"] and m1["sum_J"] == m0["sum_J"]
    # rest particles never move and change only in pairs (Fig. 1 discussion)
    assert np.array_equal(c1[1] & 1, c0[1] & 1)
    assert m1["n0_odd"] == m0["n0_odd"]


def test_moments_are_the_plain_sums():
    rng = np.random.default_rng(2)
    L = 300
    c0 = rng.integers(0, 200, size=(3, L), dtype=np.uint16)
    s = O.OracleSim([L], seed=1, C=0)
    s.init_counts(0, c0)
    tw = rng.integers(-(1 << 24), 1 << 24, size=(4, L), dtype=np.int32)
    m = s.moments(0, tw)
    c = c0.astype(np.int64)
    N = c.sum(0)
    assert m["sum_n"] == list(c.sum(1))
    assert m["sum_n2"] == list((c * c).sum(1))
    assert m["sum_nn"] == [int((c[0] * c[1]).sum()), int((c[1] * c[2]).sum()), int((c[0] * c[2]).sum())]
    assert m["sum_N2"] == int((N * N).sum()) and m["max_N"] == int(N.max())
    assert m["n0_odd"] == int((c[1] & 1).sum())
    assert m["fourier"][0] == [int((N * tw[0]).sum()), int((N * tw[1]).sum())]
    assert m["fourier"][1] == [int((N * tw[2]).sum()), int((N * tw[3]).sum())]


# --------------------------------------------------------------------------
# Equilibrium and fluctuations
# --------------------------------------------------------------------------
def test_feq_closed_form_properties():
    """Eq. (D1Q3equil): mass and momentum moments, the equilibrium condition
    f_0^2 = 16 f_-1 f_1 of Eq. (1Ddecay), f = rho w at u = 0 and
    f_{+-1} = rho at u = +-1."""
    g = json.load(open(os.path.join(GOLDEN, "paper_d1q3.json")))
    w = [Fraction(*g["weights"][k]) for k in ("w_m1", "w_0", "w_p1")]
    for rho in [1.0, 10.0, 50.0]:
        for u in np.linspace(-0.9, 0.9, 13):
            f = O.feq(rho, u)
            assert f.sum() == pytest.approx(rho, rel=1e-14)
            assert f[2] - f[0] == pytest.approx(rho * u, rel=1e-12, abs=1e-12)
            assert f[1] ** 2 == pytest.approx(16 * f[0] * f[2], rel=1e-12)
        assert list(O.feq(rho, 0.0)) == pytest.approx([rho * float(x) for x in w], rel=1e-15)
    for u in g["extreme_velocity"]["u"]:
        f = O.feq(7.0, u)
        assert f[1 + int(u)] == pytest.approx(7.0, rel=1e-15)


def test_temperature_closed_form():
    """Second moment about u divided by rho: (2 sqrt(1+3u^2) - 1)/3 - u^2
    (derived from Eq. (D1Q3equil)); 1/3 at u = 0 and 0 at |u| = 1 (Fig. 4)."""
    for u in [0.0, 0.1, 0.5, 1.0]:
        f = O.feq(1.0, u)
        th = sum(fi * (v - u) ** 2 for fi, v in zip(f, (-1, 0, 1)))
        assert th == pytest.approx((2 * math.sqrt(1 + 3 * u * u) - 1) / 3 - u * u, abs=1e-14)
    assert sum(fi * v * v for fi, v in zip(O.feq(1.0, 0.0), (-1, 0, 1))) == pytest.approx(1 / 3)


@pytest.mark.parametrize("mu", [0.3, 1.6666666666666667, 6.081485941, 32.83702812, 100.0])
def test_poisson_thresholds_match_poisson_law(mu):
    k_lo, thr = O.poisson_thresholds(mu)
    ks = k_lo + np.arange(len(thr))
    cdf = stats.poisson.cdf(ks, mu)
    assert np.max(np.abs(thr.astype(np.float64) / 2**32 - cdf)) < 1e-9
    assert stats.poisson.cdf(k_lo - 1, mu) < 1e-15 if k_lo > 0 else True
    assert stats.poisson.sf(k_lo + len(thr), mu) < 1e-15


def _site_stats(c):
    c = c.astype(np.float64)
    mean = c.mean(1)
    var = c.var(1)
    return mean, var


@pytest.mark.slow
@pytest.mark.parametrize("init,rho_u", [((0, 30, 0), (30.0, 0.0)), ((0, 20, 10), (30.0, 1 / 3))])
def test_relaxation_to_entropic_equilibrium(init, rho_u):
    """From a far-from-equilibrium state the site means relax to
    Eq. (D1Q3equil) at the conserved (rho, u), within 3 standard errors."""
    L = 1 << 15
    c0 = np.array(init, dtype=np.uint16)[:, None].repeat(L, 1)
    s = O.OracleSim([L], seed=21, C=10)
    s.init_counts(0, c0)
    s.step(150)
    f = O.feq(*rho_u)
    acc = np.zeros(3)
    n_snap = 6
    for _ in range(n_snap):
        s.step(10)
        acc += s.counts(0).astype(np.float64).mean(1)
    mean = acc / n_snap
    se = np.sqrt(f / L)  # Poisson variance per site; snapshots are not independent
    assert np.all(np.abs(mean - f) < 3 * se + 1e-9), (mean, f)


@pytest.mark.slow
@pytest.mark.parametrize("u0", [0.0, 0.1])
def test_poisson_fluctuations(u0):
    """Eq. (poisson): var(n_i)/mean(n_i) = 1 within 0.01, also at u != 0."""
    L = 1 << 17
    s = O.OracleSim([L], seed=31, C=10)
    s.init_poisson(0, 50.0, u0)
    s.step(40)
    mean, var = _site_stats(s.counts(0))
    f = O.feq(50.0, u0)
    assert np.all(np.abs(var / mean - 1) < 0.01), var / mean
    assert np.all(np.abs(mean - f) < 4 * np.sqrt(f / L))
    # correlator of Eq. (corr) between different velocities at one site
    c = s.counts(0).astype(np.float64)
    for i, j in [(0, 1), (1, 2), (0, 2)]:
        corr = ((c[i] * c[j]).mean() - mean[i] * mean[j]) / math.sqrt(mean[i] * mean[j])
        assert abs(corr) < 0.02


@pytest.mark.slow
def test_rest_parity_sector_histogram():
    """Fig. 1 set-up (rho = 12, all n0 even): n0 follows the Poisson law
    restricted to even values, n_{+-1} the plain Poisson law, with
    2 f_1 + f_0 tanh f_0 = 12 and f_0 = 4 f_1 (so f_0 ~ 8, f_1 ~ 2)."""
    rng = np.random.default_rng(4)
    L = 1 << 14
    f1 = 2.0
    f0 = 8.0
    n0 = rng.poisson(f0, size=L)
    odd = n0 % 2 == 1
    while odd.any():
        n0[odd] = rng.poisson(f0, size=odd.sum())
        odd = n0 % 2 == 1
    c0 = np.vstack([rng.poisson(f1, L), n0, rng.poisson(f1, L)]).astype(np.uint16)
    s = O.OracleSim([L], seed=41, C=10)
    s.init_counts(0, c0)
    s.step(100)
    c = s.counts(0)
    assert not (c[1] % 2).any()
    h = np.bincount(c[1], minlength=40)[:40]
    k = np.arange(0, 40, 2)
    p = stats.poisson.pmf(k, f0) * 2 / (1 + math.exp(-2 * f0))
    assert _chi2_pvalue(h[k], p / p.sum(), h[k].sum()) > 1e-3
    hm = np.bincount(c[0], minlength=20)[:20]
    pm = stats.poisson.pmf(np.arange(20), f1)
    assert _chi2_pvalue(hm, pm / pm.sum(), hm.sum()) > 1e-3


@pytest.mark.slow
def test_pi_relaxation_without_streaming():
    """Relaxation of the pi moment toward local equilibrium when collisions
    act without streaming (Fig. 5 variant): ensemble mean equals the exact
    chain expectation within 3 standard errors."""
    abc = (100, 100, 100)
    L = 20000
    s = O.OracleSim([L], seed=51, C=10, n_max=300, flags=O.FLAG_NO_STREAM)
    s.init_counts(0, np.array(abc, dtype=np.uint16)[:, None].repeat(L, 1))
    for steps in (1, 3, 10):
        s.step(steps - s.t(0))
        c = s.counts(0).astype(np.float64)
        pi = math.sqrt(2) * (c[0] - c[1] / 2 + c[2])
        mean_exact, m2 = X.no_stream_pi_moments(abc, 10, steps)
        sd = math.sqrt(max(m2 - mean_exact**2, 1e-12))
        assert abs(pi.mean() - mean_exact) < 3 * sd / math.sqrt(L) + 1e-9, (steps, pi.mean(), mean_exact)


# --------------------------------------------------------------------------
# Galilean-invariant acceptance (the remedy proposed after Eq. (D1Q3relax))
# --------------------------------------------------------------------------
def _galilean_exact(num, den, N, J):
    """floor(floor(2^32 N / sqrt(N^2 + 3 J^2)) num / den) with Python's exact
    integer square root: floor(sqrt(floor(y))) = floor(sqrt(y))."""
    g = math.isqrt((2**64 * N * N) // (N * N + 3 * J * J)) if N else 2**32
    return g * num // den


def test_galilean_lambda_is_the_exact_rounding():
    """The oracle's per-fiber acceptance numerator equals the exact integer
    rounding, is within 2^-31 of lambda~ / sqrt(1 + 3 (J/N)^2), is
    floor(2^32 lambda~) at J = 0, and never grows with |J|."""
    rng = np.random.default_rng(3)
    cases = [(1, 1, 0, 0), (1, 1, 1, 1), (1, 1, 65535, 65535), (3, 4, 65535, 1),
             (2, 3, 300, 150), ((1 << 28) - 1, (1 << 28) - 1, 1000, 999)]
    for _ in range(3000):
        den = int(rng.integers(1, 1 << 28))
        num = int(rng.integers(1, den + 1))
        N = int(rng.integers(0, 65536))
        cases.append((num, den, N, int(rng.integers(0, N + 1))))
    for num, den, N, J in cases:
        got = O.galilean_lambda((num, den), N, J)
        assert got == _galilean_exact(num, den, N, J), (num, den, N, J)
        lam = num / den / math.sqrt(1 + 3 * (J / N) ** 2) if N else num / den
        assert abs(got / 2**32 - lam) < 2**-31
    for N in (2, 17, 255, 4000):
        seq = [O.galilean_lambda((1, 1), N, J) for J in range(N + 1)]
        assert seq[0] == 2**32 and all(x >= y for x, y in zip(seq, seq[1:]))


@pytest.mark.parametrize("C", [1, 3])
@pytest.mark.parametrize("lam", [(1, 1), (3, 4)])
def test_galilean_rows_equal_brute_force(C, lam):
    """With the flag, each fiber's quantised rows equal the enumerated law of
    the literal loop at lambda = (its rounded numerator) / 2^32."""
    for N in range(0, 7):
        for a, b, c in _states(N):
            J = abs(c - a)
            lf = Fraction(_galilean_exact(lam[0], lam[1], N, J), 2**32)
            want = X.quantise(X.rest_marginal(X.c_step_law((a, b, c), C, lf), N, J))
            got = O.row_thresholds(C, lam, N, J, b, flags=O.FLAG_GALILEAN)
            assert [int(v) for v in got] == want, (a, b, c)


@pytest.mark.parametrize("abc", [(1, 2, 5), (30, 10, 5), (0, 40, 12)])
def test_galilean_direct_sampler_follows_rows(abc):
    """The literal loop with the Galilean acceptance (one word against the
    numerator for a moving pair, a 35-bit uniform for a rest pair) draws from
    the exact law of the flagged rows (chi-squared, p > 1e-3)."""
    n = 400_000
    C = 10
    h = O.histogram(C, (1, 1), abc, n, seed=9, t=2, direct=True, flags=O.FLAG_GALILEAN)
    N, J = sum(abc), abs(abc[2] - abc[0])
    lf = Fraction(_galilean_exact(1, 1, N, J), 2**32)
    if N <= 12:
        probs = [float(p) for p in X.rest_marginal(X.c_step_law(abc, C, lf), N, J)]
    else:
        thr = O.row_thresholds(C, (1, 1), N, J, abc[1], flags=O.FLAG_GALILEAN).astype(np.float64)
        cum = np.concatenate([[0.0], thr / 2**32, [1.0]])
        probs = list(np.diff(cum))
    par = (N - J) % 2
    counts = [int(h[par + 2 * k]) for k in range(len(probs))]
    assert sum(counts) == n
    assert _chi2_pvalue(counts, probs, n) > 1e-3


def _fiber_gap(N, J, lam):
    par, m = (N - J) % 2, (N - J) // 2 + 1
    T = np.zeros((m, m))
    for k in range(m):
        b = par + 2 * k
        for s2, p in X.one_subcollision_counted(((N - b - J) // 2, b, (N - b + J) // 2), lam).items():
            T[k, (s2[1] - par) // 2] += float(p)
    ev = np.sort(np.real(np.linalg.eigvals(T)))[::-1]
    return 1.0 - ev[1]


def test_galilean_acceptance_removes_velocity_dependence_of_relaxation():
    """Relaxation rate of one fiber (spectral gap of the one-sub-collision
    chain, N = 240): with a constant lambda it grows as sqrt(1 + 3 U^2)
    (the velocity dependence of Eq. (D1Q3relax)), with the Galilean
    acceptance it stays at the U = 0 value within 1%."""
    N = 240
    g0 = _fiber_gap(N, 0, Fraction(1))
    for J in (60, 120, 180):
        U = J / N
        plain = _fiber_gap(N, J, Fraction(1)) / g0
        assert plain == pytest.approx(math.sqrt(1 + 3 * U * U), rel=0.01)
        gal = _fiber_gap(N, J, Fraction(_galilean_exact(1, 1, N, J), 2**32)) / g0
        assert gal == pytest.approx(1.0, abs=0.01)
