"""GPU parity: the HIP path through the C ABI against the oracle, bit for bit.

The state is integer counts, so the bar is exact equality of every count
after every compared step.  Inputs are seeded (synth/); the oracle computes
its own initial state from the same rule or takes the same synthetic counts.
Every small case runs under each policy by which the step kernel resolves
the draws its LDS image cannot decide (deferred, after each chunk, before
each chunk's store), since the library picks between them by state size.
The largest lattice is checked on light-cone windows the oracle recomputes
independently, and by exact conservation; the full-size workloads are in
test_gpu_scale.py.
"""
import sys

import numpy as np
import pytest

import oracle as O
import synth
from paper_1706_01094_amd.mclg import (DRAIN_CHUNK, DRAIN_DEFERRED, DRAIN_PATCH, E_RANGE,
                                      FLAG_GALILEAN, FLAG_NO_STREAM, Lattice, MclgError)
from tests.state_digest import digest

pytestmark = pytest.mark.gpu

DRAINS = [DRAIN_DEFERRED, DRAIN_CHUNK, DRAIN_PATCH]
drains = pytest.mark.parametrize("drain", DRAINS, ids=["deferred", "chunk", "patch"])


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def pair(L, seed, C=10, lam=(1, 1), n_max=255, rho=10.0, u0=0.0, counts=None, flags=0,
         replica_id=None, drain=None):
    say("case", dict(L=L, seed=seed, C=C, lam=lam, n_max=n_max, rho=rho, u0=u0, flags=flags,
                     drain=drain))
    g = Lattice(L, seed, C=C, lam=lam, n_max=n_max, rho=rho, u0=u0, counts=counts, flags=flags,
                replica_id=replica_id)
    if drain is not None:
        g.set_drain(drain)
    o = O.OracleSim(L, seed, C=C, lam=lam, n_max=n_max, flags=flags, replica_id=replica_id)
    Ls = np.atleast_1d(L)
    rhos = np.broadcast_to(np.asarray(rho, dtype=float), (len(Ls),))
    u0s = np.broadcast_to(np.asarray(u0, dtype=float), (len(Ls),))
    off = 0
    for r in range(len(Ls)):
        if counts is None:
            o.init_poisson(r, float(rhos[r]), float(u0s[r]))
        else:
            n = int(Ls[r])
            o.init_counts(r, np.asarray(counts).reshape(-1)[3 * off: 3 * (off + n)].reshape(3, n))
            off += n
    return g, o


def same(g, o, r=0, allow_range=False):
    a = g.counts(r, allow_range=allow_range)
    b = o.counts(r)
    if not np.array_equal(a, b):
        bad = np.argwhere(a != b)
        raise AssertionError(f"replica {r} t={o.t(r)}: {len(bad)} counts differ, first {bad[:5].tolist()}")


def test_plain_small_every_step():
    """L = 256, rho = 10, u = 0, seed 1, C = 10, lambda = 1: 1000 steps, the
    full state compared after every step."""
    w = synth.PLAIN_SMALL
    g, o = pair(w["L"], w["seed"], rho=w["rho"], u0=w["u0"])
    same(g, o)
    for _ in range(w["steps"]):
        g.step(1)
        o.step(1)
        same(g, o)
    m = g.moments()[0]
    mo = o.moments(0)
    for k in ("t", "sum_n", "sum_n2", "sum_nn", "sum_N", "sum_J", "sum_N2", "n0_odd", "max_N"):
        assert m[k] == mo[k], k


@pytest.mark.parametrize("groups,threads,lds", [(1, 64, 96 << 10), (1, 256, 0), (1, 128, 4096),
                                                (1, 1024, 112 << 10), (1, 512, 32 << 10),
                                                (1, 1024, 0), (1, 64, 128 << 10)])
@drains
def test_ragged_tiles_and_schedules(groups, threads, lds, drain):
    """Several tiles plus a ragged tail, at u != 0; every schedule and LDS
    image size (0 = every draw from the global rows) gives the oracle's bits."""
    L = 3 * 2048 + 37
    g, o = pair(L, 7, rho=30.0, u0=0.15, drain=drain)
    g.set_schedule(groups, threads, lds)
    say("lds coverage", g.lds_coverage())
    for _ in range(12):
        g.step(5)
        o.step(5)
        same(g, o)


@pytest.mark.parametrize("threads,blocks,lds", [(64, 1, 112 << 10), (256, 2, 96 << 10),
                                                (1024, 1, 112 << 10), (512, 3, 0),
                                                (768, 2, 96 << 10), (832, 3, 64 << 10),
                                                (576, 1, 0)])
@drains
def test_long_runs_per_wave(threads, blocks, lds, drain):
    """A capped grid gives each wave long runs of contiguous chunks: the
    boundary vectors passed from chunk to chunk, drains between chunks and the
    chunks that wrap around the lattice end, over shifts t = 0..23 (every
    misalignment of the shifted windows).  Block sizes of 8, 9, 12, 13 and 16
    waves cover every rule by which a block's young waves stop claiming its
    last chunks (every chunk must still be taken)."""
    L = 3 * 2 ** 14 + 37
    g, o = pair(L, 31, rho=30.0, u0=0.1, drain=drain)
    g.set_schedule(1, threads, lds)
    g.set_grid_limit(blocks)
    for _ in range(8):
        g.step(3)
        o.step(3)
        same(g, o)


@pytest.mark.parametrize("L", [1, 2, 3, 4, 5, 7, 129])
@drains
def test_tiny_lattices(L, drain):
    counts = synth.random_counts(L, seed=L)
    g, o = pair(L, 3, counts=counts, drain=drain)
    for _ in range(20):
        g.step(1)
        o.step(1)
        same(g, o)


@drains
def test_direct_path_above_n_max(drain):
    """Sites with N > n_max take the paper's literal sub-collision loop."""
    g, o = pair(3000, 11, n_max=24, rho=30.0, u0=-0.05, drain=drain)
    m = g.moments()[0]
    assert m["max_N"] > 24
    for _ in range(10):
        g.step(3)
        o.step(3)
        same(g, o)


# lambda with denominator q = 3 * 2^26: the literal loop's uniform integer
# below q rejects 1/64 of its 32-bit words (2^32 mod q = 2^26) and the one
# below 8 q a quarter (2^32 mod 8q = 2^30), so both rejection branches run
LAMBDA_REJECT = (3 * 2**25 + 1, 3 * 2**26)


@drains
@pytest.mark.parametrize("C", [1, 10])
def test_literal_loop_with_rejected_draws(C, drain):
    """n_max = 24 sends most sites (rho = 30) to the literal loop, whose
    Bernoulli draws with lambda = (3 2^25 + 1) / (3 2^26) take Lemire's
    rejection step often; every count equals the oracle's after every step."""
    g, o = pair(3000, 43, C=C, lam=LAMBDA_REJECT, n_max=24, rho=30.0, u0=0.1, drain=drain)
    for _ in range(10):
        g.step(1)
        o.step(1)
        same(g, o)


def test_state_digest_equals_host_digest():
    """The digest the moments kernel sums equals the host-side definition,
    for the GPU's own counts and the oracle's, over ragged replicas."""
    L = [1, 7, 513, 2048, 5000]
    g, o = pair(L, 47, rho=[3.0, 20.0, 40.0, 8.0, 60.0], u0=[0.0, 0.1, -0.2, 0.05, 0.3])
    for _ in range(3):
        g.step(5)
        o.step(5)
        m = g.moments(digest=True)
        for r in range(len(L)):
            assert m[r]["digest"] == digest(g.counts(r)) == digest(o.counts(r)), r
    assert g.moments()[0]["digest"] == 0


@pytest.mark.parametrize("C,lam", [(0, (1, 1)), (1, (1, 1)), (3, (1, 2)), (10, (3, 4)), (-1, (1, 1))])
@drains
def test_collision_parameters(C, lam, drain):
    g, o = pair(2500, 13, C=C, lam=lam, rho=20.0, u0=0.1, drain=drain)
    for _ in range(8):
        g.step(4)
        o.step(4)
        same(g, o)


@drains
def test_no_stream_flag(drain):
    g, o = pair(2000, 17, rho=40.0, flags=1, drain=drain)
    for _ in range(10):
        g.step(2)
        o.step(2)
        same(g, o)


@pytest.mark.parametrize("n_max,rho,u0,lam,flags", [
    (255, 12.0, 0.4, (3, 4), FLAG_GALILEAN),
    (16, 20.0, -0.5, (1, 1), FLAG_GALILEAN),
    (16, 20.0, 0.3, (2, 3), FLAG_GALILEAN | FLAG_NO_STREAM)])
@drains
def test_galilean_acceptance(n_max, rho, u0, lam, flags, drain):
    """Galilean-invariant acceptance: L = 3000, C = 10, the per-fiber tables
    (n_max = 255) and the device's own per-site numerator in the literal loop
    (n_max = 16, where most sites have N > n_max); every count equal to the
    oracle's after each of 12 steps."""
    g, o = pair(3000, 21, C=10, lam=lam, n_max=n_max, rho=rho, u0=u0, flags=flags, drain=drain)
    for _ in range(12):
        g.step(1)
        o.step(1)
        same(g, o)


def test_moments_with_fourier_modes():
    import torch
    L = 5000
    g, o = pair(L, 19, rho=25.0, u0=0.05)
    tw = synth.twiddles(L, 3)
    twd = torch.as_tensor(tw).to("cuda:0")
    for _ in range(3):
        g.step(7)
        o.step(7)
        m = g.moments(twd, 3)[0]
        mo = o.moments(0, tw)
        assert m["fourier"][:3] == mo["fourier"][:3]
        for k in ("t", "sum_n", "sum_n2", "sum_nn", "sum_N", "sum_J", "sum_N2", "n0_odd", "max_N"):
            assert m[k] == mo[k], k


@drains
def test_overflow_is_flagged_and_site_kept(drain):
    """A site with N > 65535 is not collided and raises the sticky range
    error on both sides."""
    L = 64
    counts = synth.random_counts(L, seed=5)
    counts[:, 10] = 30000
    g, o = pair(L, 23, counts=counts, drain=drain)
    g.step(1)
    rc = o.step(1)
    assert rc == -2
    assert g.check() == E_RANGE
    same(g, o, allow_range=True)
    with pytest.raises(MclgError):
        g.counts(0)


@drains
def test_batched_replicas_step_replica_and_graph(drain):
    """Uneven replicas in one launch, single-replica launches and a captured
    HIP graph all reproduce the oracle; graph replays are checked one by one
    with eager work in between."""
    L = [100, 2048, 3000, 777, 5, 4096]
    rid = [10, 11, 12, 13, 14, 99]
    rho = [5.0, 10.0, 50.0, 80.0, 20.0, 33.0]
    u0 = [0.0, 0.1, -0.2, 0.05, 0.0, 0.15]
    g, o = pair(L, 29, rho=rho, u0=u0, replica_id=rid, drain=drain)
    for r in range(len(L)):
        same(g, o, r)
    g.step(10)
    o.step(10)
    for r in range(len(L)):
        same(g, o, r)
    g.step_replica(2, 5)
    o.step(5, rep=2)
    g.step(3)
    o.step(3)
    for r in range(len(L)):
        same(g, o, r)
    for _ in range(3):
        g.step_graph(4)
        o.step(4)
        for r in range(len(L)):
            same(g, o, r)
        g.step(1)
        o.step(1)
    for r in range(len(L)):
        same(g, o, r)
