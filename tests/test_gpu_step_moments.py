"""Steps followed by the moments of the state they reach, in one call
(mclg_step_moments): with several steps per launch the last launch sums the
moments of the sites it writes back.  Every record equals plain numpy sums of
the counts read back at the same step (and the state digest), and the state
stays equal to the oracle's; calls that fall back to the separate moment
kernels (steps not a multiple of the group, two modes with the digest, no
blocking, several replicas) give the same records."""
import ctypes as ct
import sys

import numpy as np
import pytest

import oracle as O
import synth
from paper_1706_01094_amd import mclg as M
from paper_1706_01094_amd.mclg import Lattice
from tests.state_digest import digest
from tests.test_gpu_moments import plain_moments

pytestmark = pytest.mark.gpu

FIELDS = ("sites", "sum_n", "sum_n2", "sum_nn", "sum_N", "sum_J", "sum_N2", "n0_odd", "max_N")


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def records(lat, out):
    lat.stream.synchronize()
    host = np.ascontiguousarray(out.cpu().numpy())
    return [M.mclg_moments_t.from_buffer_copy(host[r].tobytes()).as_dict() for r in range(lat.n)]


def new_out(lat):
    import torch
    words = ct.sizeof(M.mclg_moments_t) // 8
    return torch.full((lat.n, words), -1, dtype=torch.int64, device=lat.device)


def expect(have, c, tw, n_modes, dig, t, what):
    want = plain_moments(c, tw, n_modes)
    for f in FIELDS:
        assert have[f] == want[f], (what, f, have[f], want[f])
    assert have["fourier"][:n_modes] == want["fourier"], (what, "fourier")
    assert all(v == [0, 0] for v in have["fourier"][n_modes:]), (what, "fourier beyond")
    assert have["digest"] == (digest(c) if dig else 0), (what, "digest")
    assert have["t"] == t, (what, "t", have["t"], t)


@pytest.mark.parametrize("L,K", [(1 << 17, 4), ((1 << 17) + 8, 8), (3 * (1 << 16) + 8 * 37, 5)])
def test_step_moments_blocked_equal_plain_sums_and_oracle(L, K):
    """Every mode count and digest flag, at lattices where every block owns
    sites and where the last blocks own none (2^17 + 8 sites); calls of one
    group, of several groups, and one not a multiple of the group."""
    import torch
    say("case", dict(L=L, K=K))
    g = Lattice(L, 83, C=10, rho=20.0, u0=0.1)
    g.set_blocked(K)
    o = O.OracleSim([L], 83, C=10)
    o.init_poisson(0, 20.0, 0.1)
    tw = synth.twiddles(L, 2)
    twd = torch.as_tensor(np.ascontiguousarray(tw.reshape(-1))).to(g.device)
    g.stream.wait_stream(torch.cuda.current_stream(g.device))
    t = 0
    for n, n_modes, dig in ((K, 0, False), (2 * K, 1, False), (K, 2, False), (K, 0, True),
                            (3 * K, 1, True), (K, 2, True), (K + 1, 1, False), (K, 1, False)):
        out = new_out(g)
        g.step_moments(n, out, twd[: 2 * n_modes * L] if n_modes else None, n_modes, digest=dig)
        t += n
        rec = records(g, out)[0]
        o.step(n)
        c = g.counts(0)
        assert np.array_equal(c, o.counts(0)), ("state", t)
        expect(rec, c, tw, n_modes, dig, t, (L, K, n, n_modes, dig))
    g.close()
    o.close()


def test_step_moments_without_blocking_and_several_replicas():
    """The fallback path: several replicas (no blocking possible), three
    modes."""
    import torch
    Ls = [4099, 33000, 7]
    g = Lattice(Ls, 5, rho=[10.0, 40.0, 3.0], u0=[0.0, 0.1, -0.2])
    tw = [synth.twiddles(L, 3) for L in Ls]
    twd = torch.as_tensor(np.concatenate([w.reshape(-1) for w in tw])).to(g.device)
    g.stream.wait_stream(torch.cuda.current_stream(g.device))
    t = 0
    for n, dig in ((3, False), (5, True)):
        out = new_out(g)
        g.step_moments(n, out, twd, 3, digest=dig)
        t += n
        recs = records(g, out)
        for r, L in enumerate(Ls):
            expect(recs[r], g.counts(r), tw[r], 3, dig, t, (r, n, dig))
    g.close()


def test_step_moments_density_wave_full_size():
    """The L = 2^22 density wave, 10 steps per launch, one mode logged every
    10 steps for 300 steps: every record equals the separate moments call on
    a second lattice stepped alongside, and the last one equals numpy's sums
    of the counts."""
    import torch
    w = synth.DENSITY_WAVE
    L = w["L"]
    counts = synth.density_wave_counts()
    tw = synth.twiddles(L, 1)
    a = Lattice(L, w["seed"], counts=counts)
    b = Lattice(L, w["seed"], counts=counts)
    a.set_blocked(10)
    b.set_blocked(10)
    twd = torch.as_tensor(np.ascontiguousarray(tw.reshape(-1))).to(a.device)
    a.stream.wait_stream(torch.cuda.current_stream(a.device))
    b.stream.wait_stream(torch.cuda.current_stream(b.device))
    n = 30
    ra, rb = new_out(a), new_out(b)
    words = ra.shape[1]
    la = torch.zeros((n, words), dtype=torch.int64, device=a.device)
    lb = torch.zeros((n, words), dtype=torch.int64, device=b.device)
    for k in range(n):
        a.step_moments(10, la[k], twd, 1)
        b.step(10)
        b.moments_to_device(lb[k], twd, 1)
    a.stream.synchronize()
    b.stream.synchronize()
    assert torch.equal(la.cpu(), lb.cpu())
    rec = M.mclg_moments_t.from_buffer_copy(np.ascontiguousarray(la[-1].cpu().numpy()).tobytes())
    expect(rec.as_dict(), a.counts(0), tw, 1, False, 10 * n, "wave")
    a.close()
    b.close()


def test_step_moments_refuses_bad_arguments():
    g = Lattice(1 << 17, 3, rho=5.0, u0=0.0)
    g.set_blocked(4)
    out = new_out(g)
    for args in ((4, 0, 1, 0), (4, 0, 9, 0), (4, 0, 0, 2)):  # no twiddles, 9 modes, bad flag
        rc = M.lib().mclg_step_moments(g.ctx, args[0], args[1], args[2], args[3], out.data_ptr())
        assert rc == M.E_INVAL, args
    rc = M.lib().mclg_step_moments(g.ctx, 4, 0, 0, 0, 0)
    assert rc == M.E_INVAL
    g.close()
