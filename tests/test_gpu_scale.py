"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times: the whole state compared with the oracle after every step
of a long prefix (L = 2^24 and the L = 2^22 density wave), the 1024-replica
batch on a sample of replicas that includes the densest, and the largest and
an HBM-resident lattice on light-cone windows the oracle recomputes.

The oracle is single-threaded C; independent replicas and windows run in a
thread pool (the ctypes calls release the interpreter lock).
"""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as O
import synth
from paper_1706_01094_amd.mclg import DRAIN_PATCH, Lattice
from tests.state_digest import digest

pytestmark = pytest.mark.gpu

WORKERS = max(1, min(16, os.cpu_count() or 1))


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def _diff(a, b, what):
    if not np.array_equal(a, b):
        bad = np.argwhere(a != b)
        raise AssertionError(f"{what}: {len(bad)} counts differ, first {bad[:5].tolist()}")


def test_plain_large_every_step_100():
    """L = 2^24, rho = 50, u0 = 0.1, seed 2 (the benchmark's workload and
    schedule): the whole state equals the oracle's after each of 100 steps,
    and the device digest equals the host digest of the oracle's state."""
    w = synth.PLAIN_LARGE
    L = w["L"]
    say("plain", L)
    g = Lattice(L, w["seed"], rho=w["rho"], u0=w["u0"])
    o = O.OracleSim([L], w["seed"], C=10)
    o.init_poisson(0, w["rho"], w["u0"])
    _diff(g.counts(0), o.counts(0), "t=0")
    for t in range(1, 101):
        g.step(1)
        o.step(1)
        want = o.counts(0)
        _diff(g.counts(0), want, f"t={t}")
        if t % 25 == 0:
            say("t", t)
            assert g.moments(digest=True)[0]["digest"] == digest(want)
    g.close()
    o.close()


def test_density_wave_every_step_100():
    """L = 2^22 density wave from synthetic counts: whole state every step for
    100 steps, the int64 Fourier projection of Eq. (A) every 10 steps."""
    import torch
    w = synth.DENSITY_WAVE
    L = w["L"]
    counts = synth.density_wave_counts()
    say("density wave", L)
    g = Lattice(L, w["seed"], counts=counts)
    o = O.OracleSim([L], w["seed"], C=10)
    o.init_counts(0, counts)
    tw = synth.twiddles(L, 1)
    twd = torch.as_tensor(tw).to("cuda:0")
    for t in range(1, 101):
        g.step(1)
        o.step(1)
        _diff(g.counts(0), o.counts(0), f"t={t}")
        if t % 10 == 0:
            m, mo = g.moments(twd, 1)[0], o.moments(0, tw)
            assert m["fourier"][0] == mo["fourier"][0], t
            assert m["sum_N"] == mo["sum_N"] and m["sum_N2"] == mo["sum_N2"]
    g.close()
    o.close()


def _oracle_replica(man, seed, r, T, every):
    """Counts of replica r after every `every` steps up to T."""
    o = O.OracleSim([int(man["L"][r])], seed, C=10, replica_id=[int(man["replica_id"][r])])
    o.init_poisson(0, float(man["rho"][r]), float(man["u0"][r]))
    out = []
    for _ in range(T // every):
        o.step(every)
        out.append(o.counts(0))
    o.close()
    return out


def test_batched_replicas_50_steps():
    """All 1024 replicas of the batched workload (826 MB, so the launches
    resolve each chunk's undecided draws before its store), one launch per
    step: 64 replicas -- the 8 densest, the 4 largest, the 4 smallest and 48
    drawn at random -- equal the oracle's runs every 5 steps up to t = 50."""
    man = synth.replica_manifest()
    seed = synth.BATCHED["seed"]
    n = len(man["L"])
    dense = list(np.argsort(-man["rho"], kind="stable")[:8])
    big = list(np.argsort(-man["L"].astype(np.int64), kind="stable")[:4])
    small = list(np.argsort(man["L"].astype(np.int64), kind="stable")[:4])
    rng = np.random.default_rng(1)
    pick = sorted(set(int(r) for r in dense + big + small))
    rest = [r for r in rng.permutation(n) if r not in pick]
    pick = sorted(pick + [int(r) for r in rest[: 64 - len(pick)]])
    assert len(pick) == 64
    say("batched", n, int(man["L"].sum()), "checking", len(pick))
    T, every = 50, 5
    with ThreadPoolExecutor(WORKERS) as ex:
        futs = {r: ex.submit(_oracle_replica, man, seed, r, T, every) for r in pick}
        g = Lattice(man["L"], seed, rho=man["rho"], u0=man["u0"], replica_id=man["replica_id"])
        got = {r: [] for r in pick}
        for _ in range(T // every):
            g.step(every)
            for r in pick:
                got[r].append(g.counts(r))
        g.close()
        for r in pick:
            want = futs[r].result()
            for k in range(T // every):
                _diff(got[r][k], want[k], f"replica {r} t={(k + 1) * every}")


def _oracle_window(L, seed, rho, u0, T, x0, W, counts=None, rid=None):
    """Counts of sites x0 .. x0 + W - 1 after T steps, from the oracle run on
    their light cone x0 - T .. x0 + W + T - 1 alone (its own ends are wrong
    after t steps only within t sites of them).  The sites keep their
    logical positions (and the replica its id) for the random numbers; the
    start is the Poisson draw or the given counts."""
    lo = x0 - T
    o = O.OracleSim([W + 2 * T], seed, C=10, replica_id=None if rid is None else [rid])
    o.set_site_offset(0, lo, 0)
    if counts is None:
        o.init_poisson(0, rho, u0)
    else:
        o.init_counts(0, counts[:, lo:lo + W + 2 * T])
    o.step(T)
    out = o.counts(0)[:, T:T + W]
    o.close()
    return out


def _windows(g, L, seed, rho, u0, T, x0s, W=1500):
    full = g.counts(0)
    with ThreadPoolExecutor(WORKERS) as ex:
        futs = [(x0, ex.submit(_oracle_window, L, seed, rho, u0, T, x0, W)) for x0 in x0s]
        for x0, f in futs:
            _diff(full[:, x0:x0 + W], f.result(), f"window at {x0}")


@pytest.mark.parametrize("policy", [None, DRAIN_PATCH], ids=["auto", "patch"])
def test_hbm_resident_lattice_windows(policy):
    """L = 2^27 (768 MiB of state, larger than the Infinity Cache; the
    default policy resolves each chunk's draws before its store): exact
    conservation over the whole lattice and 16 oracle windows after 24
    steps."""
    w = synth.PLAIN_LARGE
    L = 1 << 27
    say("hbm-resident", L, policy)
    g = Lattice(L, w["seed"], rho=w["rho"], u0=w["u0"])
    if policy is not None:
        g.set_drain(policy)
    m0 = g.moments()[0]
    T = 24
    g.step(T)
    m1 = g.moments()[0]
    assert (m1["sum_N"], m1["sum_J"], m1["n0_odd"]) == (m0["sum_N"], m0["sum_J"], m0["n0_odd"])
    rng = np.random.default_rng(2)
    x0s = [T, L // 2, L - 1500 - T] + [int(v) for v in rng.integers(T, L - 1500 - T, size=13)]
    _windows(g, L, w["seed"], w["rho"], w["u0"], T, x0s)
    g.close()


def test_largest_lattice_windows():
    """L = 2^29, the largest lattice (the step kernel's 32-bit byte offsets
    reach their top): conservation and oracle windows at both ends and in
    the middle after a few steps."""
    L = 1 << 29
    say("largest lattice", L)
    g = Lattice(L, 41, rho=8.0, u0=0.05)
    m0 = g.moments()[0]
    T = 3
    g.step(T)
    m1 = g.moments()[0]
    assert m1["sum_N"] == m0["sum_N"] and m1["sum_J"] == m0["sum_J"]
    _windows(g, L, 41, 8.0, 0.05, T, [T, L // 2 + 12345, L - 1500 - T])
    g.close()


def _full_run_windows(g, L, seed, rho, u0, steps, every, per, W=256, counts=None, pick_seed=7):
    """Steps the one-lattice g to `steps` and compares `per` oracle
    light-cone windows with its counts at every multiple of `every`."""
    rng = np.random.default_rng(pick_seed)
    marks = list(range(every, steps + 1, every))
    with ThreadPoolExecutor(WORKERS) as ex:
        futs = {}
        for T in marks:
            x0s = [int(v) for v in rng.integers(T, L - W - T, size=per)]
            futs[T] = [(x0, ex.submit(_oracle_window, L, seed, rho, u0, T, x0, W, counts))
                       for x0 in x0s]
        t = 0
        for T in marks:
            g.step(T - t)
            t = T
            full = g.counts(0)
            for x0, f in futs[T]:
                _diff(full[:, x0:x0 + W], f.result(), f"t={T} window at {x0}")
            say("t", T, "windows equal")


def test_plain_large_full_run_windows():
    """The whole 10^4-step run of the L = 2^24 workload: three oracle
    light-cone windows of 256 sites equal the GPU's counts after every 1000
    steps (the oracle recomputes each window from the Poisson start)."""
    w = synth.PLAIN_LARGE
    L = w["L"]
    say("plain full run", L)
    g = Lattice(L, w["seed"], rho=w["rho"], u0=w["u0"])
    _full_run_windows(g, L, w["seed"], w["rho"], w["u0"], steps=10_000, every=1000, per=3)
    g.close()


def test_density_wave_full_run_windows():
    """The whole 5000-step density-wave run: three oracle windows from the
    synthetic counts after every 1000 steps."""
    w = synth.DENSITY_WAVE
    L = w["L"]
    counts = synth.density_wave_counts()
    say("density wave full run", L)
    g = Lattice(L, w["seed"], counts=counts)
    _full_run_windows(g, L, w["seed"], None, None, steps=5000, every=1000, per=3, counts=counts)
    g.close()


def test_batched_full_run():
    """The whole 2000-step batched run: the 12 smallest replicas equal the
    oracle's whole runs at t = 1000 and 2000, and two oracle windows in each
    of the 8 densest and 4 largest replicas equal the GPU's there."""
    man = synth.replica_manifest()
    seed = synth.BATCHED["seed"]
    Ls = man["L"].astype(np.int64)
    small = [int(r) for r in np.argsort(Ls, kind="stable")[:12]]
    dense = [int(r) for r in np.argsort(-man["rho"], kind="stable")[:8]]
    big = [int(r) for r in np.argsort(-Ls, kind="stable")[:4]]
    T, every, W = 2000, 1000, 256
    rng = np.random.default_rng(11)
    say("batched full run", len(Ls))
    with ThreadPoolExecutor(WORKERS) as ex:
        whole = {r: ex.submit(_oracle_replica, man, seed, r, T, every) for r in small}
        wins = {}
        for r in dense + big:
            if r in whole:
                continue
            L = int(Ls[r])
            if L < W + 2 * T + 1:  # too short for a window: the whole replica
                whole[r] = ex.submit(_oracle_replica, man, seed, r, T, every)
                continue
            for t in range(every, T + 1, every):
                for x0 in (int(v) for v in rng.integers(t, L - W - t, size=2)):
                    wins.setdefault((r, t), []).append(
                        (x0, ex.submit(_oracle_window, L, seed, float(man["rho"][r]),
                                       float(man["u0"][r]), t, x0, W, None,
                                       int(man["replica_id"][r]))))
        g = Lattice(man["L"], seed, rho=man["rho"], u0=man["u0"], replica_id=man["replica_id"])
        for k, t in enumerate(range(every, T + 1, every)):
            g.step(every)
            for r, f in whole.items():
                _diff(g.counts(r), f.result()[k], f"replica {r} t={t}")
            for (r, tt), lst in wins.items():
                if tt != t:
                    continue
                full = g.counts(r)
                for x0, f in lst:
                    _diff(full[:, x0:x0 + W], f.result(), f"replica {r} t={t} window at {x0}")
            say("t", t, "replicas and windows equal")
        g.close()
