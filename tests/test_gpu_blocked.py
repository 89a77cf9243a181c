"""Several steps per launch (temporal blocking, mclg_set_blocked): every
count equals the oracle's, and the state equals the one-step-per-launch
state, for group sizes from 2 to 256, calls that are not multiples of the
group, the flags and collision parameters, and the full-size workloads."""
import sys

import numpy as np
import pytest

import oracle as O
import synth
from paper_1706_01094_amd.mclg import DRAIN_PATCH, FLAG_GALILEAN, FLAG_NO_STREAM, Lattice, MclgError
from tests.state_digest import digest

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def pair(L, seed, K, C=10, lam=(1, 1), n_max=255, rho=20.0, u0=0.1, flags=0):
    say("case", dict(L=L, seed=seed, K=K, C=C, lam=lam, n_max=n_max, rho=rho, u0=u0, flags=flags))
    g = Lattice(L, seed, C=C, lam=lam, n_max=n_max, rho=rho, u0=u0, flags=flags)
    g.set_blocked(K)
    o = O.OracleSim([L], seed, C=C, lam=lam, n_max=n_max, flags=flags)
    o.init_poisson(0, rho, u0)
    return g, o


def same(g, o, what):
    a, b = g.counts(0), o.counts(0)
    if not np.array_equal(a, b):
        bad = np.argwhere(a != b)
        raise AssertionError(f"{what}: {len(bad)} counts differ, first {bad[:5].tolist()}")


@pytest.mark.parametrize("L,K", [(1 << 17, 2), (1 << 17, 8), (3 * (1 << 16) + 8 * 37, 5),
                                 (1 << 18, 16), (1 << 20, 64), (1 << 20, 256)])
def test_blocked_equals_oracle(L, K):
    g, o = pair(L, 71, K)
    t = 0
    for n in (K, 2 * K + 3, 1, K - 1 if K > 1 else 1, 3 * K):
        g.step(n)
        o.step(n)
        t += n
        same(g, o, f"L={L} K={K} t={t}")
    g.close()


@pytest.mark.parametrize("C,lam,n_max,flags", [
    (0, (1, 1), 255, 0),
    (3, (1, 2), 255, 0),
    (-1, (1, 1), 255, 0),
    (10, (1, 1), 24, 0),
    (10, (1, 1), 255, FLAG_NO_STREAM),
    (10, (3, 4), 255, FLAG_GALILEAN),
    (10, (1, 1), 16, FLAG_GALILEAN),
])
def test_blocked_flags_and_parameters(C, lam, n_max, flags):
    """The literal loop for N > n_max (n_max = 24 and 16: its random numbers
    are keyed by the lattice site, not the site of the block's copy), C = 0,
    C = infinity, no streaming and the Galilean acceptance, 8 steps per
    launch."""
    L = 1 << 17
    g, o = pair(L, 73, 8, C=C, lam=lam, n_max=n_max, rho=30.0, u0=0.15, flags=flags)
    for n in (8, 11, 16):
        g.step(n)
        o.step(n)
        same(g, o, f"C={C} n_max={n_max} flags={flags}")
    g.close()


def test_blocked_equals_single_steps_full_size():
    """L = 2^24 (the benchmark's workload): 10 steps per launch give the same
    state as one step per launch after 100 and 205 steps."""
    w = synth.PLAIN_LARGE
    L = w["L"]
    a = Lattice(L, w["seed"], rho=w["rho"], u0=w["u0"])
    b = Lattice(L, w["seed"], rho=w["rho"], u0=w["u0"])
    b.set_blocked(10)
    for n in (100, 105):
        a.step(n)
        b.step(n)
        ma, mb = a.moments(digest=True)[0], b.moments(digest=True)[0]
        assert ma == mb
    assert digest(a.counts(0)) == digest(b.counts(0))
    a.close()
    b.close()


def test_blocked_density_wave_windows():
    """The L = 2^22 density wave, 10 steps per launch: oracle light-cone
    windows after 500 steps."""
    from concurrent.futures import ThreadPoolExecutor
    w = synth.DENSITY_WAVE
    L = w["L"]
    counts = synth.density_wave_counts()
    g = Lattice(L, w["seed"], counts=counts)
    g.set_blocked(10)
    T, W = 500, 512

    def window(x0):
        lo = x0 - T
        o = O.OracleSim([W + 2 * T], w["seed"], C=10)
        o.set_site_offset(0, lo, 0)
        o.init_counts(0, counts[:, lo:lo + W + 2 * T])
        o.step(T)
        out = o.counts(0)[:, T:T + W]
        o.close()
        return out

    x0s = [T, L // 3, L - W - T]
    with ThreadPoolExecutor(3) as ex:
        futs = [(x0, ex.submit(window, x0)) for x0 in x0s]
        g.step(T)
        full = g.counts(0)
        for x0, f in futs:
            assert np.array_equal(full[:, x0:x0 + W], f.result()), x0
    g.close()


def test_blocked_refused_where_it_does_not_apply():
    g = Lattice([4096, 4096], 3, rho=5.0, u0=0.0)
    with pytest.raises(MclgError):
        g.set_blocked(4, 1024)  # replicas are copied whole, not in tiles
    g.set_blocked(4)
    g.close()
    g = Lattice(1 << 17, 3, rho=5.0, u0=0.0)
    with pytest.raises(MclgError):
        g.set_blocked(257)  # more than 256 steps
    g.set_blocked(1)  # off
    g.step(3)
    g.close()


def test_blocked_full_size_256_steps_per_launch_windows():
    """The benchmark's launch shape, L = 2^24 with 256 steps per launch: oracle
    light-cone windows after 528 steps (two launches and 16 single steps)."""
    from concurrent.futures import ThreadPoolExecutor
    w = synth.PLAIN_LARGE
    L = w["L"]
    g = Lattice(L, w["seed"], rho=w["rho"], u0=w["u0"])
    g.set_blocked(256)
    T, W = 528, 256

    def window(x0):
        lo = x0 - T
        o = O.OracleSim([W + 2 * T], w["seed"], C=10)
        o.set_site_offset(0, lo, 0)
        o.init_poisson(0, w["rho"], w["u0"])
        o.step(T)
        out = o.counts(0)[:, T:T + W]
        o.close()
        return out

    # the first block's extra sites wrap around the lattice's start; others
    # sit at block boundaries (65536 sites per block) and in the middle
    x0s = [T, 65536 - W // 2, L // 2 + 12345, L - W - T]
    with ThreadPoolExecutor(4) as ex:
        futs = [(x0, ex.submit(window, x0)) for x0 in x0s]
        g.step(T)
        full = g.counts(0)
        for x0, f in futs:
            assert np.array_equal(full[:, x0:x0 + W], f.result()), x0
    g.close()


# ---- tiles: each block goes through its range in tiles of `tile` sites ----

def pair_tiled(L, seed, K, tile, **kw):
    g, o = pair(L, seed, K, **kw)
    g.set_blocked(K, tile)
    return g, o


@pytest.mark.parametrize("L,K,tile", [
    (1 << 20, 8, 2048),             # two full tiles per block, carries between them
    (1 << 20, 16, 1024),            # five tiles per block, the last one short
    (1 << 20, 2, 4096 + 16),        # a tile longer than the block's range
    (3 * (1 << 16) + 8 * 37, 5, 256),  # a ragged lattice: the last block's range is short
    ((1 << 17) + 8, 64, 192),       # blocks that own no sites; side areas wider than a range
    (1 << 18, 16, 48),              # tiles of kh sites (shorter than the carry)
    (1 << 18, 16, 40),              # tiles of 8 sites
])
def test_tiled_equals_oracle(L, K, tile):
    g, o = pair_tiled(L, 91, K, tile)
    t = 0
    for n in (K, 2 * K + 3, 1, 3 * K):
        g.step(n)
        o.step(n)
        t += n
        same(g, o, f"tiles L={L} K={K} tile={tile} t={t}")
    g.close()


@pytest.mark.parametrize("C,lam,n_max,flags", [
    (0, (1, 1), 255, 0),
    (10, (1, 1), 24, 0),
    (10, (1, 1), 255, FLAG_NO_STREAM),
    (10, (3, 4), 255, FLAG_GALILEAN),
])
def test_tiled_flags_and_parameters(C, lam, n_max, flags):
    L = 1 << 18
    g, o = pair_tiled(L, 93, 8, 512, C=C, lam=lam, n_max=n_max, rho=30.0, u0=0.15, flags=flags)
    for n in (8, 11, 16):
        g.step(n)
        o.step(n)
        same(g, o, f"tiles C={C} n_max={n_max} flags={flags}")
    g.close()


def test_tiled_refuses_bad_tiles():
    g = Lattice(1 << 18, 3, rho=5.0, u0=0.0)
    for tile in (2000 + 4, 32, 1 << 21):  # not a multiple of 8, no own sites, too long
        with pytest.raises(MclgError):
            g.set_blocked(16, tile)
    g.close()


def test_tiled_full_size_hbm_resident_windows():
    """L = 2^27 (more than the caches hold: tiles of 65536 sites by default),
    16 steps per launch: oracle light-cone windows after 37 steps (two
    launches and 5 single steps) at a tile boundary, a block boundary, the
    lattice's wrap and inside a tile."""
    from concurrent.futures import ThreadPoolExecutor
    w = synth.PLAIN_LARGE
    L = 1 << 27
    g = Lattice(L, w["seed"], rho=w["rho"], u0=w["u0"])
    g.set_blocked(16)
    T, W = 37, 256
    R = L // 256
    tile_body = 65536 - 32

    def window(x0):
        lo = x0 - T
        o = O.OracleSim([W + 2 * T], w["seed"], C=10)
        o.set_site_offset(0, lo, 0)
        o.init_poisson(0, w["rho"], w["u0"])
        o.step(T)
        out = o.counts(0)[:, T:T + W]
        o.close()
        return out

    x0s = [T, tile_body - W // 2, R - W // 2, 5 * R + 3 * tile_body + 1000, L - W - T]
    with ThreadPoolExecutor(5) as ex:
        futs = [(x0, ex.submit(window, x0)) for x0 in x0s]
        g.step(T)
        full = g.counts(0)
        for x0, f in futs:
            assert np.array_equal(full[:, x0:x0 + W], f.result()), x0
    g.close()


# ---- several replicas: each block advances whole replicas ----

REPS = dict(L=[100, 2048, 3000, 777, 5, 4096, 1, 70001, 12345],
            rid=[10, 11, 12, 13, 14, 99, 3, 7, 8],
            rho=[5.0, 10.0, 50.0, 80.0, 20.0, 33.0, 4.0, 45.0, 100.0],
            u0=[0.0, 0.1, -0.2, 0.05, 0.0, 0.15, 0.0, -0.1, 0.2])


def pair_reps(seed, K, C=10, lam=(1, 1), n_max=255, flags=0, drain=None):
    say("replicas", dict(seed=seed, K=K, C=C, lam=lam, n_max=n_max, flags=flags, drain=drain))
    g = Lattice(REPS["L"], seed, C=C, lam=lam, n_max=n_max, rho=REPS["rho"], u0=REPS["u0"],
                flags=flags, replica_id=REPS["rid"])
    if drain is not None:
        g.set_drain(drain)
    g.set_blocked(K)
    o = O.OracleSim(REPS["L"], seed, C=C, lam=lam, n_max=n_max, flags=flags,
                    replica_id=REPS["rid"])
    for r in range(len(REPS["L"])):
        o.init_poisson(r, REPS["rho"][r], REPS["u0"][r])
    return g, o


def same_all(g, o, what):
    for r in range(len(REPS["L"])):
        a, b = g.counts(r), o.counts(r)
        if not np.array_equal(a, b):
            bad = np.argwhere(a != b)
            raise AssertionError(f"{what} replica {r}: {len(bad)} counts differ, "
                                 f"first {bad[:5].tolist()}")


@pytest.mark.parametrize("K,drain", [(2, None), (7, None), (32, None), (7, DRAIN_PATCH),
                                     (32, DRAIN_PATCH)])
def test_replicas_equal_oracle(K, drain):
    """Replicas of 1 to 70001 sites (lengths not multiples of 8, shorter than
    a lane's eight sites), each with its own density, velocity and collision
    image, blocks holding several of them; misses resolved at the end of each
    step or per chunk (patched)."""
    g, o = pair_reps(97, K, drain=drain)
    t = 0
    for n in (K, 2 * K + 3, 1, 3 * K):
        g.step(n)
        for r in range(len(REPS["L"])):
            o.step(n, rep=r)
        t += n
        same_all(g, o, f"K={K} t={t}")
    g.close()


@pytest.mark.parametrize("C,lam,n_max,flags,drain", [
    (0, (1, 1), 255, 0, None),
    (10, (1, 1), 24, 0, None),
    (10, (1, 1), 255, FLAG_NO_STREAM, None),
    (10, (3, 4), 255, FLAG_GALILEAN, None),
    (10, (1, 1), 24, 0, DRAIN_PATCH),
    (10, (3, 4), 255, FLAG_GALILEAN, DRAIN_PATCH),
])
def test_replicas_flags_and_parameters(C, lam, n_max, flags, drain):
    g, o = pair_reps(99, 8, C=C, lam=lam, n_max=n_max, flags=flags, drain=drain)
    for n in (8, 11, 16):
        g.step(n)
        for r in range(len(REPS["L"])):
            o.step(n, rep=r)
        same_all(g, o, f"C={C} n_max={n_max} flags={flags}")
    g.close()


def test_replicas_full_size_batched_sampled():
    """The 1024-replica batched workload (826 MB: misses resolved per chunk)
    with 16 steps per launch: 64
    replicas (the 8 densest, the 4 largest, the 4 smallest and 48 drawn at
    random) equal the oracle's runs after every launch up to t = 48, and every
    replica's state digest equals one launch per step's."""
    from concurrent.futures import ThreadPoolExecutor
    from tests.test_gpu_scale import WORKERS, _oracle_replica
    man = synth.replica_manifest()
    seed = synth.BATCHED["seed"]
    n = len(man["L"])
    dense = list(np.argsort(-man["rho"], kind="stable")[:8])
    big = list(np.argsort(-man["L"].astype(np.int64), kind="stable")[:4])
    small = list(np.argsort(man["L"].astype(np.int64), kind="stable")[:4])
    rng = np.random.default_rng(2)
    pick = sorted(set(int(r) for r in dense + big + small))
    rest = [r for r in rng.permutation(n) if r not in pick]
    pick = sorted(pick + [int(r) for r in rest[: 64 - len(pick)]])
    T, every = 48, 16
    say("replicas full size", n, "checking", len(pick))
    with ThreadPoolExecutor(WORKERS) as ex:
        futs = {r: ex.submit(_oracle_replica, man, seed, r, T, every) for r in pick}
        g = Lattice(man["L"], seed, rho=man["rho"], u0=man["u0"], replica_id=man["replica_id"])
        g.set_blocked(every)
        got = {r: [] for r in pick}
        for _ in range(T // every):
            g.step(every)
            for r in pick:
                got[r].append(g.counts(r))
        dg = g.moments(digest=True)
        g.close()
        for r in pick:
            want = futs[r].result()
            for k in range(T // every):
                a, b = got[r][k], want[k]
                assert np.array_equal(a, b), (r, (k + 1) * every)
    h = Lattice(man["L"], seed, rho=man["rho"], u0=man["u0"], replica_id=man["replica_id"])
    h.step(T)
    dh = h.moments(digest=True)
    h.close()
    assert [m["digest"] for m in dg] == [m["digest"] for m in dh]
