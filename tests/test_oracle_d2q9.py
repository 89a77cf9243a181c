"""Pins of the D2Q9 oracle against what the paper and the mathematics fix.

The D2Q9 collision rules are not printed (the figure of the nine classes is
missing); the oracle reconstructs them (every momentum-conserving swap of two
unordered velocity pairs, detailed balance with respect to the product
weights, classes numbered as the lambda_c of Eq. (D2Q9MOmega)).  These tests
pin that reading to what is printed: the moment matrix Eq. (MomD2Q9) and the
linearised collision term Eq. (D2Q9MOmega) (tests/golden/paper_d2q9.json),
the equilibrium Eq. (D2Q9eqdist) as an exactly stationary product measure,
the paper's lambda values satisfying its own decoupling and isotropy
conditions, and the literal loop's law against enumeration.
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle as O

G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_d2q9.json")))
W = np.array(G["weights_1296"], dtype=np.float64) / 1296.0
M = np.array([[a / b * math.sqrt(c) for a, b, c in r] for r in G["moment_matrix"]["rows"]])
NAMES = G["moment_matrix"]["names"]
V = np.array(O.V9)


def _single_class(c, value=(1, 8)):
    lam = [(0, 1)] * 9
    lam[c - 1] = value
    return lam


def _rule_probabilities(lams):
    """P[i][j] = [(k, l, probability)] of the oracle's rule table."""
    P = {}
    for i in range(9):
        for j in range(9):
            tg, D = O.targets9(lams, i, j)
            P[i, j] = [(k, l, w / D) for k, l, _, w in tg]
    return P


def test_velocities_follow_the_moment_matrix():
    """The momentum rows of Eq. (MomD2Q9) are sqrt(3) v_x and sqrt(3) v_y of
    the oracle's numbering, M is orthonormal under the weights, and one
    streaming step moves a particle of velocity i by v_i."""
    assert np.allclose(M[1], math.sqrt(3) * V[:, 0]) and np.allclose(M[2], math.sqrt(3) * V[:, 1])
    assert np.allclose(M @ np.diag(W) @ M.T, np.eye(9), atol=1e-14)
    Lx, Ly = 5, 4
    for i in range(9):
        s = O.OracleSim9([Lx], [Ly], 1, C=0)
        c = np.zeros((9, Ly, Lx), dtype=np.uint16)
        c[i, 1, 2] = 1
        s.init_counts(0, c)
        s.step(1)
        got = np.argwhere(s.counts(0))
        assert got.tolist() == [[i, (1 + V[i, 1]) % Ly, (2 + V[i, 0]) % Lx]]


def _mean_field_matrix(lams):
    """d(Delta M^b) / d(dM^a) per sub-collision at rho = 1, u = 0, times
    rho / 2: the Boltzmann average of the oracle's rules (ordered pairs drawn
    with probability f_i f_j / rho^2), linearised about f = rho w."""
    P = _rule_probabilities(lams)
    out = np.zeros((9, 9))
    for a in range(9):
        df = W * M[a]  # f = w (rho + eps m^a): derivative in eps
        f0 = W.copy()
        dn = np.zeros(9)
        for (i, j), tg in P.items():
            dpair = df[i] * f0[j] + f0[i] * df[j]
            for k, l, p in tg:
                e = np.zeros(9)
                e[i] -= 1
                e[j] -= 1
                e[k] += 1
                e[l] += 1
                dn += dpair * p * e
        out[:, a] = M @ dn / 2.0
    return out


@pytest.mark.parametrize("c", range(1, 10))
def test_linearised_collision_equals_paper(c):
    """Each class alone (lambda_c = 1/8, the others 0): the linearised
    Boltzmann-averaged change of every non-conserved moment equals the
    coefficients of lambda_c in Eq. (D2Q9MOmega); mass and momentum are
    unchanged."""
    K = _mean_field_matrix(_single_class(c)) * 8
    want = np.zeros((9, 9))
    for row, per in G["omega_linear"].items():
        if not row.startswith("_") and str(c) in per:
            for src, (num, den) in per[str(c)].items():
                want[NAMES.index(row), NAMES.index(src)] = num / den
    assert np.allclose(K[3:, 3:], want[3:, 3:], atol=1e-12), (c, K[3:, 3:], want[3:, 3:])
    assert np.allclose(K[:3], 0, atol=1e-12)


def test_paper_lambdas_decouple_and_are_isotropic():
    """With the lambda values of the paper's D2Q9 equilibrium run, the
    oracle's linearised collision decouples sigma_+ from t (Eq. (decouple))
    and relaxes sigma_xy and sigma_- at one rate (Eq. (rotational))."""
    lams = [tuple(v) for v in G["lambda_equilibrium_run"]]
    K = _mean_field_matrix(lams)
    sp, t, sm, sxy = NAMES.index("sigma_plus"), NAMES.index("t"), NAMES.index("sigma_minus"), NAMES.index("sigma_xy")
    assert abs(K[sp, t]) < 1e-14 and abs(K[t, sp]) < 1e-14
    assert K[sm, sm] == pytest.approx(K[sxy, sxy], abs=1e-14)
    # Eq. (tausigma): the sigma_xy rate per collision is (8 l1 + l3 + 2 (l4 + l6 + 2 l7 + 4 l8)) / (9 rho)
    l = [Fraction(*v) for v in lams]
    rate = (8 * l[0] + l[2] + 2 * (l[3] + l[5] + 2 * l[6] + 4 * l[7])) / 9
    assert -2 * K[sxy, sxy] == pytest.approx(float(rate), abs=1e-14)


def _states(N):
    for comp in itertools.combinations_with_replacement(range(9), N):
        n = [0] * 9
        for v in comp:
            n[v] += 1
        yield tuple(n)


def _exact_step(n, P):
    """Law of one sub-collision of the literal loop from state n (ordered
    pair of distinct particles, then the rule table)."""
    N = sum(n)
    out = {}
    if N < 2:
        return {n: 1.0}
    for i in range(9):
        for j in range(9):
            mult = n[i] * (n[j] - (i == j))
            if mult <= 0:
                continue
            pij = mult / (N * (N - 1))
            rest = 1.0
            for k, l, p in P[i, j]:
                m = list(n)
                m[i] -= 1; m[j] -= 1; m[k] += 1; m[l] += 1
                out[tuple(m)] = out.get(tuple(m), 0.0) + pij * p
                rest -= p
            out[n] = out.get(n, 0.0) + pij * rest
    return out


@pytest.mark.parametrize("u", [(0.0, 0.0), (0.3, -0.2), (-0.6, 0.45)])
def test_product_equilibrium_is_stationary(u):
    """Eq. (D2Q9eqdist): the product of Poisson laws at f^eq(rho, u) is
    stationary under one sub-collision, i.e. every fiber's law prop. to
    prod f_i^n_i / n_i! is invariant (all states with N <= 4)."""
    f = O.feq9(7.0, *u)
    P = _rule_probabilities(O.LAMBDA9_PAPER)
    for N in range(2, 5):
        states = list(_states(N))
        pi = {s: np.prod([f[i] ** s[i] / math.factorial(s[i]) for i in range(9)]) for s in states}
        new = {s: 0.0 for s in states}
        for s in states:
            for s2, p in _exact_step(s, P).items():
                new[s2] += pi[s] * p
        for s in states:
            assert new[s] == pytest.approx(pi[s], rel=1e-12, abs=1e-300)


def test_feq_is_the_product_of_the_d1q3_equilibria():
    """Eq. (D2Q9eqdist) equals rho prod_a w_a [1 + 3 v u + (3 v^2 - 1)(sqrt(1 + 3 u^2) - 1)]
    and reduces to rho w_i at u = 0; its first moments are rho and rho u."""
    for rho, ux, uy in [(36.0, 0.0, 0.0), (36.0, 0.25, 0.25), (360.0, -0.7, 0.1)]:
        f = O.feq9(rho, ux, uy)
        w1 = {-1: 1 / 6, 0: 2 / 3, 1: 1 / 6}
        g = lambda v, u: w1[v] * (1 + 3 * v * u + (3 * v * v - 1) * (math.sqrt(1 + 3 * u * u) - 1))  # noqa: E731
        want = [rho * g(vx, ux) * g(vy, uy) for vx, vy in O.V9]
        assert np.allclose(f, want, rtol=1e-15)
        assert f.sum() == pytest.approx(rho, rel=1e-14)
        assert (f * V[:, 0]).sum() == pytest.approx(rho * ux, abs=1e-12)
        assert (f * V[:, 1]).sum() == pytest.approx(rho * uy, abs=1e-12)
    assert np.allclose(O.feq9(9.0, 0.0, 0.0), 9.0 * W, rtol=1e-15)


@pytest.mark.parametrize("n", [(1, 1, 0, 0, 0, 1, 0, 0, 0), (2, 1, 0, 1, 0, 0, 1, 0, 1), (0, 2, 0, 0, 0, 0, 1, 0, 1)])
def test_literal_loop_follows_enumerated_law(n):
    """One sub-collision (C = 1) of the oracle's literal loop at 300000
    sites: outcome frequencies match the enumerated law (chi-squared,
    p > 1e-3)."""
    P = _rule_probabilities(O.LAMBDA9_PAPER)
    law = _exact_step(tuple(n), P)
    keys = sorted(law)
    idx = {k: q for q, k in enumerate(keys)}
    cnt = np.zeros(len(keys))
    draws = 300_000
    for s in range(draws):
        out = tuple(int(v) for v in O.collide_site9(1, O.LAMBDA9_PAPER, 5, 0, 3, s, n))
        cnt[idx[out]] += 1
    exp = np.array([law[k] for k in keys]) * draws
    keep = exp >= 5
    obs, e = cnt[keep], exp[keep]
    assert cnt[~keep].sum() <= max(5.0, 3 * exp[~keep].sum() + 5)
    e *= obs.sum() / e.sum()
    assert stats.chisquare(obs, e).pvalue > 1e-3


def test_conservation_and_streaming():
    """Per site, collisions conserve N, Jx, Jy exactly; globally the sums
    stay constant under streaming; C = 0 is a pure shift."""
    rng = np.random.default_rng(2)
    for s in range(200):
        n = rng.integers(0, 7, size=9)
        out = O.collide_site9(10, O.LAMBDA9_PAPER, 9, 1, 4, s, n)
        assert out.sum() == n.sum()
        assert (out * V[:, 0]).sum() == (n * V[:, 0]).sum()
        assert (out * V[:, 1]).sum() == (n * V[:, 1]).sum()
    sim = O.OracleSim9([12, 7], [5, 9], 3)
    sim.init_poisson(0, 20.0, 0.2, -0.1)
    sim.init_poisson(1, 5.0, 0.0, 0.3)
    m0 = [sim.moments(r) for r in range(2)]
    assert sim.step(25) == 0
    for r in range(2):
        m = sim.moments(r)
        assert (m["sum_N"], m["sum_Jx"], m["sum_Jy"]) == (m0[r]["sum_N"], m0[r]["sum_Jx"], m0[r]["sum_Jy"])
    free = O.OracleSim9([6], [5], 3, C=0)
    c = np.random.default_rng(1).integers(0, 9, size=(9, 5, 6)).astype(np.uint16)
    free.init_counts(0, c)
    free.step(3)
    got = free.counts(0)
    for i in range(9):
        assert np.array_equal(got[i], np.roll(c[i], (3 * V[i, 1], 3 * V[i, 0]), axis=(0, 1)))


def test_moments_are_the_plain_sums():
    """Every moment of the D2Q9 oracle equals numpy's sums over the same
    counts: per velocity, all 45 products n_i n_j (i <= j, row-major upper
    triangle), N, Jx, Jy, max N -- on counts large enough that any wrong
    index or transposed pair shows."""
    rng = np.random.default_rng(5)
    Lx, Ly = 11, 7
    c = rng.integers(0, 3000, size=(9, Ly, Lx)).astype(np.uint16)
    sim = O.OracleSim9([Lx], [Ly], 3, C=0)
    sim.init_counts(0, c)
    m = sim.moments(0)
    n = c.reshape(9, -1).astype(np.int64)
    assert m["t"] == 0 and m["sites"] == Lx * Ly
    assert m["sum_n"] == [int(v) for v in n.sum(1)]
    want = [int((n[i] * n[j]).sum()) for i in range(9) for j in range(i, 9)]
    assert m["sum_nn"] == want
    N = n.sum(0)
    assert m["sum_N"] == int(N.sum()) and m["max_N"] == int(N.max())
    assert m["sum_Jx"] == int((V[:, 0][:, None] * n).sum())
    assert m["sum_Jy"] == int((V[:, 1][:, None] * n).sum())
    # the sums follow the logical sites through streaming: after five steps
    # of a pure shift they are those of the shifted arrays
    sim.step(5)
    r = np.stack([np.roll(c[i], (5 * V[i, 1], 5 * V[i, 0]), axis=(0, 1)) for i in range(9)])
    r = r.reshape(9, -1).astype(np.int64)
    m5 = sim.moments(0)
    assert m5["sum_nn"] == [int((r[i] * r[j]).sum()) for i in range(9) for j in range(i, 9)]
    assert m5["sum_nn"] != want and m5["max_N"] == int(r.sum(0).max())


def test_poisson_start_means():
    """Poisson start at (rho, u): site means within 4 standard errors of
    Eq. (D2Q9eqdist), per velocity, on 2^15 sites."""
    sim = O.OracleSim9([256], [128], 4)
    sim.init_poisson(0, 36.0, 0.25, 0.25)
    c = sim.counts(0).reshape(9, -1).astype(np.float64)
    f = O.feq9(36.0, 0.25, 0.25)
    assert np.all(np.abs(c.mean(1) - f) < 4 * np.sqrt(f / c.shape[1]))
