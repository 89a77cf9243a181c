"""GPU parity of the D2Q9 path: the HIP kernels through the C ABI against the
oracle, count for count, after every compared step; exact moments equal the
oracle's sums; D2Q9-only entry points refuse D1Q3 work and vice versa."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1706_01094_amd.mclg import (E_UNSUPPORTED, FLAG_NO_STREAM, LAMBDA9_PAPER, Lattice9,
                                       MclgError)

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def pair9(Lx, Ly, seed, C=10, lams=LAMBDA9_PAPER, flags=0, rho=12.0, ux=0.0, uy=0.0,
          counts=None):
    say("d2q9 case", dict(Lx=Lx, Ly=Ly, seed=seed, C=C, flags=flags, rho=rho, ux=ux, uy=uy))
    g = Lattice9(Lx, Ly, seed, C=C, lams=lams, flags=flags, rho=rho, ux=ux, uy=uy, counts=counts)
    o = O.OracleSim9(Lx, Ly, seed, C=C, lams=lams, flags=flags)
    Lxs = np.atleast_1d(Lx)
    Lys = np.broadcast_to(np.asarray(Ly), Lxs.shape)
    par = [np.broadcast_to(np.asarray(v, dtype=float), Lxs.shape) for v in (rho, ux, uy)]
    off = 0
    for r in range(len(Lxs)):
        S = int(Lxs[r]) * int(Lys[r])
        if counts is None:
            o.init_poisson(r, float(par[0][r]), float(par[1][r]), float(par[2][r]))
        else:
            o.init_counts(r, np.asarray(counts).reshape(-1)[9 * off: 9 * (off + S)])
            off += S
    return g, o


def same9(g, o, n):
    for r in range(n):
        a, b = g.counts(r), o.counts(r)
        if not np.array_equal(a, b):
            bad = np.argwhere(a != b)
            raise AssertionError(f"replica {r} t={o.t(r)}: {len(bad)} counts differ, first {bad[:5].tolist()}")


def test_d2q9_ragged_replicas_every_step():
    """Four replicas (37x5, 64x64, 1x3, 130x2), Poisson starts at different
    (rho, ux, uy): every count equal after the start and after each of 12
    steps, and the exact moments equal the oracle's."""
    Lx, Ly = [37, 64, 1, 130], [5, 64, 3, 2]
    g, o = pair9(Lx, Ly, 3, rho=[12.0, 36.0, 5.0, 20.0], ux=[0.0, 0.25, -0.3, 0.1],
                 uy=[0.0, 0.25, 0.6, -0.2])
    same9(g, o, 4)
    for _ in range(12):
        g.step(1)
        assert o.step(1) == 0
        same9(g, o, 4)
    mg = g.moments()
    for r in range(4):
        mo = o.moments(r)
        for k in ("t", "sites", "sum_n", "sum_nn", "sum_N", "sum_Jx", "sum_Jy", "max_N"):
            assert mg[r][k] == mo[k], (r, k)
    assert g.check() == 0
    g.close()


@pytest.mark.parametrize("C,lams,flags", [(1, [(1, 8)] * 9, 0), (3, LAMBDA9_PAPER, FLAG_NO_STREAM),
                                          (0, LAMBDA9_PAPER, 0)])
def test_d2q9_parameters(C, lams, flags):
    """C = 1, 3 and 0 (pure streaming), all lambda 1/8, no-stream flag: 50 x
    17 sites at rho = 30, every count equal after each of 8 steps."""
    g, o = pair9(50, 17, 8, C=C, lams=lams, flags=flags, rho=30.0, ux=-0.1, uy=0.2)
    for _ in range(8):
        g.step(1)
        o.step(1)
        same9(g, o, 1)
    g.close()


def test_d2q9_counts_start_and_larger_lattice():
    """Given counts (uniform random 0..40 per velocity, N up to 360) on
    256 x 96: equal after 6 steps; the step counter and conservation hold."""
    rng = np.random.default_rng(5)
    c = rng.integers(0, 41, size=(9, 96, 256)).astype(np.uint16)
    g, o = pair9(256, 96, 11, counts=c.reshape(-1))
    m0 = g.moments()[0]
    g.step(6)
    o.step(6)
    same9(g, o, 1)
    m = g.moments()[0]
    assert m["t"] == 6 and (m["sum_N"], m["sum_Jx"], m["sum_Jy"]) == (m0["sum_N"], m0["sum_Jx"], m0["sum_Jy"])
    with pytest.raises(MclgError) as e:
        from paper_1706_01094_amd import mclg as M
        M.mclg_step_graph(g.ctx, 2)
    assert e.value.code == E_UNSUPPORTED
    g.close()


def test_d2q9_histogram_equals_oracle_bincount():
    """mclg_histogram on D2Q9 replicas (37x5, 64x64, 1x3): after 5 steps every
    velocity's histogram equals np.bincount of the oracle's counts (last bin
    clipped); a second call adds the same again."""
    Lx, Ly = [37, 64, 1], [5, 64, 3]
    g, o = pair9(Lx, Ly, 4, rho=[18.0, 36.0, 5.0], ux=[-0.25, 0.1, 0.0], uy=[0.25, 0.0, 0.3])
    g.step(5)
    o.step(5)
    for n_bins in (1, 12, 40):
        h = g.histogram(n_bins).cpu().numpy()
        for r in range(3):
            c = o.counts(r).reshape(9, -1)
            for i in range(9):
                want = np.bincount(np.minimum(c[i], n_bins - 1), minlength=n_bins)
                assert np.array_equal(h[r, i], want), (n_bins, r, i)
        h2 = g.histogram(n_bins, out=g.histogram(n_bins)).cpu().numpy()
        assert np.array_equal(h2, 2 * h)
    g.close()


def test_d2q9_overflow_is_flagged_and_site_kept():
    """A D2Q9 site with N > 65535 (8000 per velocity) is not collided, only
    streamed, and raises the sticky range error on both sides."""
    rng = np.random.default_rng(8)
    c = rng.integers(0, 6, size=(9, 6, 10)).astype(np.uint16)
    c[:, 2, 3] = 8000
    g, o = pair9(10, 6, 12, counts=c.reshape(-1))
    g.step(1)
    assert o.step(1) == -2
    from paper_1706_01094_amd.mclg import E_RANGE
    assert g.check() == E_RANGE
    a = g.counts(0, allow_range=True)
    assert np.array_equal(a, o.counts(0))
    g.close()


@pytest.mark.parametrize("Lx,Ly", [(1, 7), (7, 1), (2, 2), (1, 1)])
def test_d2q9_thin_lattices(Lx, Ly):
    """Degenerate tori (a single row or column, 2 x 2, one site): every count
    equal after each of 10 steps at rho = 20."""
    g, o = pair9(Lx, Ly, 13, rho=20.0, ux=0.2, uy=-0.3)
    for _ in range(10):
        g.step(1)
        o.step(1)
        same9(g, o, 1)
    g.close()
