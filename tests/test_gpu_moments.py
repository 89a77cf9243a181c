"""The moment kernels against plain numpy sums of the same counts (read back
in logical order), at lattice sizes where segments hold several pipelined
batches of passes and the shifted windows wrap inside them: every field of
mclg_moments_t, with 0 to 3 Fourier modes and the state digest, over several
step counts (so the shift t mod L moves the wrap points around)."""
import sys

import numpy as np
import pytest

import synth
from paper_1706_01094_amd.mclg import Lattice
from tests.state_digest import digest

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def plain_moments(c: np.ndarray, tw: np.ndarray, n_modes: int) -> dict:
    """The sums of one replica's counts c [3][L] (v = -1, 0, +1), int64."""
    a, b, d = (c[i].astype(np.int64) for i in range(3))
    N = a + b + d
    out = {"sites": c.shape[1], "sum_n": [int(a.sum()), int(b.sum()), int(d.sum())],
           "sum_n2": [int((a * a).sum()), int((b * b).sum()), int((d * d).sum())],
           "sum_nn": [int((a * b).sum()), int((b * d).sum()), int((a * d).sum())],
           "sum_N": int(N.sum()), "sum_J": int((d - a).sum()), "sum_N2": int((N * N).sum()),
           "n0_odd": int((b & 1).sum()), "max_N": int(N.max()) if N.size else 0}
    out["fourier"] = [[int((N * tw[2 * m].astype(np.int64)).sum()),
                       int((N * tw[2 * m + 1].astype(np.int64)).sum())] for m in range(n_modes)]
    return out


def twiddle_rows(Ls, n_modes):
    """The twiddle input of a lattice of replicas Ls: per replica its
    [2 n_modes][L] block, concatenated."""
    blocks = [synth.twiddles(int(L), n_modes) for L in Ls]
    return blocks, np.concatenate([b.reshape(-1) for b in blocks])


CASES = [
    # L per replica, rho, u0, C: two and six full 16384-site segments with
    # ragged ends; several replicas in one call; counts of 256 and more
    ([2 * 16384 + 37], 20.0, 0.1, 10),
    ([3 * 65536 + 5], 50.0, -0.15, 10),
    ([33000, 50001, 7, 16384], [5.0, 80.0, 30.0, 12.0], [0.0, 0.2, -0.1, 0.05], 10),
    ([100003], 330.0, 0.0, 0),
]


@pytest.mark.parametrize("Ls,rho,u0,C", CASES)
def test_moments_equal_numpy_sums(Ls, rho, u0, C):
    import torch
    say("case", dict(L=Ls, rho=rho, u0=u0, C=C))
    g = Lattice(Ls, 61, C=C, rho=rho, u0=u0)
    modes = (0, 1, 2, 3)
    tws = {m: twiddle_rows(Ls, m) for m in modes if m}
    twd = {m: torch.as_tensor(tws[m][1]).to("cuda:0") for m in tws}
    for k in (0, 1, 16387, 2507):
        if k:
            g.step(k)
        counts = [g.counts(r) for r in range(len(Ls))]
        for m in modes:
            for dig in (False, True):
                got = g.moments(twd[m], m, digest=dig) if m else g.moments(digest=dig)
                for r, c in enumerate(counts):
                    want = plain_moments(c, tws[m][0][r] if m else None, m)
                    have = got[r]
                    for f in ("sites", "sum_n", "sum_n2", "sum_nn", "sum_N", "sum_J", "sum_N2",
                              "n0_odd", "max_N"):
                        assert have[f] == want[f], (k, m, dig, r, f)
                    assert have["fourier"][:m] == want["fourier"], (k, m, dig, r)
                    assert all(v == [0, 0] for v in have["fourier"][m:]), (k, m, dig, r)
                    assert have["digest"] == (digest(c) if dig else 0), (k, m, dig, r)
    g.close()


def test_fourier_sums_on_a_lattice_past_2_28_sites():
    """L = 2^28 + 4097 (twiddle rows past 2^31 bytes, where the moments
    kernel takes its unpipelined path with 64-bit row addressing): the
    Fourier sums of one and two modes, and the plain sums, equal numpy's,
    summed in slices of the read-back counts."""
    import torch
    L = (1 << 28) + 4097
    say("large fourier", L)
    g = Lattice(L, 67, C=0, rho=6.0, u0=0.1)
    g.step(3)
    c = g.counts(0)
    tw = synth.twiddles(L, 2)
    twd = torch.as_tensor(tw.reshape(-1)).to("cuda:0")
    for m in (1, 2):
        got = g.moments(twd[: 2 * m * L], m)[0]
        f = np.zeros((m, 2), dtype=np.int64)
        sN = 0
        step = 1 << 24
        for lo in range(0, L, step):
            N = c[:, lo:lo + step].astype(np.int64).sum(0)
            sN += int(N.sum())
            for k in range(m):
                f[k, 0] += int((N * tw[2 * k, lo:lo + step].astype(np.int64)).sum())
                f[k, 1] += int((N * tw[2 * k + 1, lo:lo + step].astype(np.int64)).sum())
        assert got["sum_N"] == sN, m
        assert got["fourier"][:m] == f.tolist(), m
    g.close()
