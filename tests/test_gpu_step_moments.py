"""The logging loop in one call (mclg_step_log): n_logs times `every` steps
and the moments of the state they reach.  With several steps per launch each
launch sums the logs that fall in it from the blocks' copies (the last one as
it writes the sites back).  Every record equals plain numpy sums of the
oracle's counts at the same step (and the state digest), and the state stays
equal to the oracle's; logs between a launch's steps, at its end, several per
launch, one per several launches, launches cut at the logs (digest, Galilean
acceptance) and the fallback to the separate moment kernels (two modes with
the digest, no blocking, tiles, whole replicas) are all covered."""
import ctypes as ct
import sys

import numpy as np
import pytest

import oracle as O
import synth
from paper_1706_01094_amd import mclg as M
from paper_1706_01094_amd.mclg import FLAG_GALILEAN, Lattice
from tests.state_digest import digest
from tests.test_gpu_moments import plain_moments

pytestmark = pytest.mark.gpu

FIELDS = ("sites", "sum_n", "sum_n2", "sum_nn", "sum_N", "sum_J", "sum_N2", "n0_odd", "max_N")
WORDS = ct.sizeof(M.mclg_moments_t) // 8


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def records(lat, out, n):
    lat.stream.synchronize()
    host = np.ascontiguousarray(out.cpu().numpy()).reshape(-1, WORDS)
    return [M.mclg_moments_t.from_buffer_copy(host[k].tobytes()).as_dict() for k in range(n)]


def new_out(lat, n_logs):
    import torch
    return torch.full((n_logs * lat.n, WORDS), -1, dtype=torch.int64, device=lat.device)


def expect(have, c, tw, n_modes, dig, t, what):
    want = plain_moments(c, tw, n_modes)
    for f in FIELDS:
        assert have[f] == want[f], (what, f, have[f], want[f])
    assert have["fourier"][:n_modes] == want["fourier"], (what, "fourier")
    assert all(v == [0, 0] for v in have["fourier"][n_modes:]), (what, "fourier beyond")
    assert have["digest"] == (digest(c) if dig else 0), (what, "digest")
    assert have["t"] == t, (what, "t", have["t"], t)


def run_against_oracle(L, K, calls, seed=83, flags=0, lam=(1, 1)):
    import torch
    say("case", dict(L=L, K=K, calls=calls, flags=flags))
    g = Lattice(L, seed, C=10, lam=lam, rho=20.0, u0=0.1, flags=flags)
    g.set_blocked(K)
    o = O.OracleSim([L], seed, C=10, lam=lam, flags=flags)
    o.init_poisson(0, 20.0, 0.1)
    tw = synth.twiddles(L, 2)
    twd = torch.as_tensor(np.ascontiguousarray(tw.reshape(-1))).to(g.device)
    g.stream.wait_stream(torch.cuda.current_stream(g.device))
    t = 0
    for every, n_logs, n_modes, dig in calls:
        out = new_out(g, n_logs)
        g.step_log(every, n_logs, out, twd[: 2 * n_modes * L] if n_modes else None, n_modes,
                   digest=dig)
        recs = records(g, out, n_logs)
        for j in range(n_logs):
            o.step(every)
            t += every
            expect(recs[j], o.counts(0), tw, n_modes, dig, t, (L, K, every, n_logs, n_modes, dig, j))
        assert np.array_equal(g.counts(0), o.counts(0)), ("state", t)
    g.close()
    o.close()


@pytest.mark.parametrize("L,K", [(1 << 17, 8), ((1 << 17) + 8, 12), (3 * (1 << 16) + 8 * 37, 5)])
def test_step_log_blocked_equal_oracle(L, K):
    """Logs between a launch's steps (every < K), at its end (every = K), not
    aligned with launches (every not dividing K), one per several launches
    (every > K), with 0, 1 and 2 modes; the digest (launches cut at the
    logs) and two modes with the digest (the separate moment kernels); at
    lattices where every block owns sites and where the last blocks own none
    (2^17 + 8 sites)."""
    run_against_oracle(L, K, [(2, 5, 1, False), (K, 2, 0, False), (3, 7, 2, False),
                              (K + 3, 2, 1, False), (1, 3, 0, False), (3, 4, 1, True),
                              (K, 1, 0, True), (2, 3, 2, True)])


def test_step_log_galilean_cuts_launches_at_logs():
    run_against_oracle(1 << 17, 8, [(3, 5, 1, False), (8, 2, 0, False)], seed=85,
                       flags=FLAG_GALILEAN, lam=(3, 4))


def test_step_log_without_blocking_and_several_replicas():
    """The fallback path: several replicas without blocking, three modes,
    against numpy's sums of the counts read back after each call."""
    import torch
    Ls = [4099, 33000, 7]
    g = Lattice(Ls, 5, rho=[10.0, 40.0, 3.0], u0=[0.0, 0.1, -0.2])
    tw = [synth.twiddles(L, 3) for L in Ls]
    twd = torch.as_tensor(np.concatenate([w.reshape(-1) for w in tw])).to(g.device)
    g.stream.wait_stream(torch.cuda.current_stream(g.device))
    t = 0
    for every, dig in ((3, False), (5, True)):
        out = new_out(g, 1)
        g.step_log(every, 1, out, twd, 3, digest=dig)
        t += every
        recs = records(g, out, len(Ls))
        for r, L in enumerate(Ls):
            expect(recs[r], g.counts(r), tw[r], 3, dig, t, (r, every, dig))
    g.close()


def test_step_log_density_wave_full_size():
    """The L = 2^22 density wave, 100 steps per launch (ten logs in each),
    one mode every 10 steps for 300 steps: every record equals the separate
    moments call on a second lattice stepped 10 steps at a time, and the last
    one equals numpy's sums of the counts."""
    import torch
    w = synth.DENSITY_WAVE
    L = w["L"]
    counts = synth.density_wave_counts()
    tw = synth.twiddles(L, 1)
    a = Lattice(L, w["seed"], counts=counts)
    b = Lattice(L, w["seed"], counts=counts)
    a.set_blocked(100)
    b.set_blocked(10)
    twd = torch.as_tensor(np.ascontiguousarray(tw.reshape(-1))).to(a.device)
    a.stream.wait_stream(torch.cuda.current_stream(a.device))
    b.stream.wait_stream(torch.cuda.current_stream(b.device))
    n = 30
    la = new_out(a, n)
    lb = torch.zeros((n, WORDS), dtype=torch.int64, device=b.device)
    a.step_log(10, n, la, twd, 1)
    for k in range(n):
        b.step(10)
        b.moments_to_device(lb[k], twd, 1)
    a.stream.synchronize()
    b.stream.synchronize()
    assert torch.equal(la.cpu(), lb.cpu())
    rec = records(a, la, n)[-1]
    expect(rec, a.counts(0), tw, 1, False, 10 * n, "wave")
    a.close()
    b.close()


def test_step_log_refuses_bad_arguments():
    g = Lattice(1 << 17, 3, rho=5.0, u0=0.0)
    g.set_blocked(4)
    out = new_out(g, 2)
    f = M.lib().mclg_step_log
    for every, n_modes, flags in ((4, 1, 0), (4, 9, 0), (4, 0, 2), (0, 0, 0)):
        # no twiddles, 9 modes, an unknown flag, every = 0
        assert f(g.ctx, every, 2, 0, n_modes, flags, out.data_ptr()) == M.E_INVAL
    assert f(g.ctx, 4, 2, 0, 0, 0, 0) == M.E_INVAL
    assert f(g.ctx, 1 << 40, 1 << 40, 0, 0, 0, out.data_ptr()) == M.E_INVAL
    g.close()


@pytest.mark.parametrize("Ls,tile", [([1 << 20], 1024), ([4099, 33000, 7, 70001], 0)])
def test_step_log_with_tiles_and_replicas(Ls, tile):
    """Blocking in tiles (one lattice) or on whole replicas (several) takes
    the moment kernels after each interval: records equal numpy's sums of
    the oracle's counts at every log."""
    import torch
    K = 8
    say("step_log blocked", dict(L=Ls, tile=tile))
    rho, u0 = 25.0, 0.05
    g = Lattice(Ls, 87, C=10, rho=rho, u0=u0)
    g.set_blocked(K, tile)
    o = O.OracleSim(Ls, 87, C=10)
    for r in range(len(Ls)):
        o.init_poisson(r, rho, u0)
    tw = [synth.twiddles(L, 1) for L in Ls]
    twd = torch.as_tensor(np.concatenate([w.reshape(-1) for w in tw])).to(g.device)
    g.stream.wait_stream(torch.cuda.current_stream(g.device))
    n_logs, every = 3, 12
    out = new_out(g, n_logs)
    g.step_log(every, n_logs, out, twd, 1)
    recs = records(g, out, n_logs * len(Ls))
    for j in range(n_logs):
        o.step(every)
        for r in range(len(Ls)):
            expect(recs[j * len(Ls) + r], o.counts(r), tw[r], 1, False, every * (j + 1),
                   (Ls, tile, j, r))
    g.close()
    o.close()
