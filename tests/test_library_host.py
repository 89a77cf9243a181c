"""Host-side checks of the HIP library (no GPU): it loads, exports every
entry point its header declares, validates arguments, and its independently
built exact tables equal the oracle's byte for byte."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_1706_01094_amd import mclg as M

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "mclg.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(mclg_\w+)\s*\(", txt, re.M)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 20
    lib = M.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(M.exported_symbols())


@pytest.mark.parametrize("C,lam", [(10, (1, 1)), (1, (1, 1)), (3, (1, 2)), (10, (3, 4)), (-1, (1, 1))])
def test_table_rows_equal_oracle(C, lam):
    rng = np.random.default_rng(abs(C) * 7 + lam[1])
    cases = [(2, 0, 0), (2, 0, 2), (5, 1, 2), (8, 0, 0), (37, 3, 20), (60, 0, 30), (255, 0, 171),
             (255, 255, 0), (100, 98, 0), (3, 1, 0)]
    for _ in range(30):
        N = int(rng.integers(2, 256))
        J = int(rng.integers(0, N + 1))
        k = int(rng.integers(0, (N - J) // 2 + 1))
        cases.append((N, J, (N - J) % 2 + 2 * k))
    for N, J, n0 in cases:
        a = M.mclg_table_row(C, lam, N, J, n0)
        b = O.row_thresholds(C, lam, N, J, n0)
        assert np.array_equal(a, b), (N, J, n0)


@pytest.mark.parametrize("C,lam", [(10, (1, 1)), (3, (3, 4))])
def test_galilean_rows_and_lambda_equal_oracle(C, lam):
    """Galilean-invariant acceptance: the library's per-fiber numerators
    (estimate and integer correction) and flagged rows equal the oracle's
    (bisection) for random fibers up to N = 65535 and rows up to N = 255."""
    rng = np.random.default_rng(C + lam[0])
    for _ in range(2000):
        N = int(rng.integers(0, 65536))
        J = int(rng.integers(0, N + 1))
        assert M.mclg_galilean_lambda(lam, N, J) == O.galilean_lambda(lam, N, J), (N, J)
    cases = [(2, 0, 0), (2, 2, 0), (37, 3, 20), (255, 0, 171), (255, 200, 1), (120, 60, 30)]
    for _ in range(20):
        N = int(rng.integers(2, 256))
        J = int(rng.integers(0, N + 1))
        k = int(rng.integers(0, (N - J) // 2 + 1))
        cases.append((N, J, (N - J) % 2 + 2 * k))
    for N, J, n0 in cases:
        a = M.mclg_table_row(C, lam, N, J, n0, flags=M.FLAG_GALILEAN)
        b = O.row_thresholds(C, lam, N, J, n0, flags=O.FLAG_GALILEAN)
        assert np.array_equal(a, b), (N, J, n0)
    with pytest.raises(M.MclgError):
        M.mclg_table_row(C, lam, 4, 0, 0, flags=M.FLAG_NO_STREAM)


@pytest.mark.parametrize("lams", [O.LAMBDA9_PAPER, [(1, 8)] * 9, [(3, 7), (0, 1), (1, 5), (2, 9), (1, 3), (0, 1), (1, 6), (1, 11), (1, 13)]])
def test_d2q9_rules_equal_oracle(lams):
    """The library's D2Q9 rule table (targets in order, cumulative integer
    weights, denominator D) equals the oracle's, built independently."""
    rules, D = M.mclg_d2q9_rules(lams)

    def change(word):
        return [((int(word) >> (3 * v)) & 7) - 2 for v in range(9)]

    for i in range(9):
        for j in range(9):
            tg, D2 = O.targets9(lams, i, j)
            assert D == D2
            e = rules[i * 9 + j]
            cum = 0
            for q in range(4):
                if q < len(tg):
                    k, l, _, w = tg[q]
                    cum += w
                    want = [0] * 9
                    want[i] -= 1
                    want[j] -= 1
                    want[k] += 1
                    want[l] += 1
                    assert e[q] == cum and change(e[4 + q]) == want, (i, j, q)
                else:
                    assert e[q] == D
            assert change(e[4 + len(tg)]) == [0] * 9
    with pytest.raises(M.MclgError):
        M.mclg_d2q9_rules([(1, 1)] * 9)  # targets of one source would exceed probability one


@pytest.mark.parametrize("mu", [0.0, 1e-3, 0.5, 1.6666666666666667, 6.081485941486, 32.83702811702, 88.0, 612.5])
def test_poisson_thresholds_equal_oracle(mu):
    k1, t1 = M.mclg_poisson_thresholds(mu)
    k2, t2 = O.poisson_thresholds(mu)
    assert k1 == k2 and np.array_equal(t1, t2)


def test_feq_means_equal_oracle_through_poisson_rule():
    # the library's equilibrium means feed its Poisson rule; equal thresholds
    # for the means of a few (rho, u) pairs pin the evaluation order
    for rho, u in [(10.0, 0.0), (50.0, 0.1), (37.0, -0.173), (5.0, 0.2)]:
        for mu in O.feq(rho, u):
            assert M.mclg_poisson_thresholds(float(mu))[1].tobytes() == O.poisson_thresholds(float(mu))[1].tobytes()


def _cfg(L, C=10, lam=(1, 1), n_max=255, lattice=M.D1Q3, abi=M.ABI_VERSION, flags=0):
    arr = (ct.c_uint64 * len(L))(*L)
    c = M.mclg_config()
    c.abi_version = abi
    c.lattice = lattice
    c.n_replicas = len(L)
    c.flags = flags
    c.L = arr
    c.seed = 1
    c.C = C
    c.lambda_num, c.lambda_den = lam
    c.n_max = n_max
    c._keep = arr
    return c


def test_sizes_and_validation():
    sb, wb = M.mclg_sizes(_cfg([256]))
    assert sb == 3 * 256 * 2 and wb > 0
    sb2, _ = M.mclg_sizes(_cfg([300, 5]))
    assert sb2 == 3 * (384 + 128) * 2
    lib = M.lib()
    s, w = ct.c_uint64(), ct.c_uint64()
    # D2Q9 needs Ly and lambda9; nine arrays of Lx Ly (padded to 128) per replica
    assert lib.mclg_sizes(ct.byref(_cfg([256], lattice=M.D2Q9)), ct.byref(s), ct.byref(w)) == M.E_INVAL
    c9 = _cfg([100, 7], lattice=M.D2Q9)
    Ly = np.array([10, 3], dtype=np.uint64)
    lam9 = np.asarray(M.LAMBDA9_PAPER, dtype=np.uint32).reshape(18)
    c9.Ly = Ly.ctypes.data_as(ct.POINTER(ct.c_uint64))
    c9.lambda9 = lam9.ctypes.data_as(ct.POINTER(ct.c_uint32))
    assert lib.mclg_sizes(ct.byref(c9), ct.byref(s), ct.byref(w)) == M.OK
    assert s.value == 9 * (1024 + 128) * 2
    Ly[1] = 1 << 26  # 7 x 2^26 sites > 2^28
    assert lib.mclg_sizes(ct.byref(c9), ct.byref(s), ct.byref(w)) == M.E_INVAL
    # largest lattice: 2^29 sites (32-bit byte offsets into a slot's three arrays)
    sb3, _ = M.mclg_sizes(_cfg([1 << 29]))
    assert sb3 == 3 * (1 << 29) * 2
    for bad in [_cfg([0]), _cfg([(1 << 29) + 1]), _cfg([256], C=-2), _cfg([256], lam=(2, 1)),
                _cfg([256], lam=(0, 1)),
                _cfg([256], n_max=2000), _cfg([256], abi=99), _cfg([256], flags=8)]:
        assert lib.mclg_sizes(ct.byref(bad), ct.byref(s), ct.byref(w)) == M.E_INVAL
    assert lib.mclg_init(None, None, None) == M.E_INVAL
    assert lib.mclg_step(None, 1) == M.E_INVAL
    assert M.mclg_strerror(M.E_RANGE) == "site occupation out of range"


def test_gpu_entry_points_fail_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(RuntimeError):
        M.Lattice([256], seed=1, rho=10.0)
