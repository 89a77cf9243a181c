"""ctypes binding of the MCLG oracle (plain single-threaded C).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product path
(the HIP library and its binding) never does.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

from . import build_oracle

C_EQUILIBRIUM = -1
FLAG_NO_STREAM = 1
FLAG_GALILEAN = 2
MAX_MODES = 8


class Moments(ct.Structure):
    _fields_ = [
        ("t", ct.c_int64), ("sites", ct.c_int64),
        ("sum_n", ct.c_int64 * 3), ("sum_n2", ct.c_int64 * 3), ("sum_nn", ct.c_int64 * 3),
        ("sum_N", ct.c_int64), ("sum_J", ct.c_int64), ("sum_N2", ct.c_int64),
        ("n0_odd", ct.c_int64), ("max_N", ct.c_int64),
        ("fourier", (ct.c_int64 * 2) * MAX_MODES),
    ]

    def as_dict(self) -> dict:
        return {
            "t": self.t, "sites": self.sites,
            "sum_n": list(self.sum_n), "sum_n2": list(self.sum_n2), "sum_nn": list(self.sum_nn),
            "sum_N": self.sum_N, "sum_J": self.sum_J, "sum_N2": self.sum_N2,
            "n0_odd": self.n0_odd, "max_N": self.max_N,
            "fourier": [list(self.fourier[m]) for m in range(MAX_MODES)],
        }


_lib = None


def lib() -> ct.CDLL:
    global _lib
    if _lib is None:
        path = build_oracle.build(force=False)
        L = ct.CDLL(path)
        u32, u64, i32, i64 = ct.c_uint32, ct.c_uint64, ct.c_int32, ct.c_int64
        P = ct.POINTER
        L.mco_create.argtypes = [u32, P(u64), P(u64), u64, i32, u32, u32, u32, u32, P(ct.c_void_p)]
        L.mco_destroy.argtypes = [ct.c_void_p]
        L.mco_destroy.restype = None
        L.mco_init_counts.argtypes = [ct.c_void_p, u32, P(ct.c_uint16)]
        L.mco_init_poisson.argtypes = [ct.c_void_p, u32, ct.c_double, ct.c_double]
        L.mco_step_replica.argtypes = [ct.c_void_p, u32, u64]
        L.mco_step.argtypes = [ct.c_void_p, u64]
        L.mco_get_counts.argtypes = [ct.c_void_p, u32, P(ct.c_uint16)]
        L.mco_get_t.argtypes = [ct.c_void_p, u32]
        L.mco_get_t.restype = i64
        L.mco_set_site_offset.argtypes = [ct.c_void_p, u32, u64, i64]
        L.mco_moments.argtypes = [ct.c_void_p, u32, P(ct.c_int32), u32, P(Moments)]
        L.mco_philox4x32_10.argtypes = [P(u32), P(u32), P(u32)]
        L.mco_philox4x32_10.restype = None
        L.mco_row_thresholds.argtypes = [i32, u32, u32, u32, u32, u32, u32, P(u64), P(u32)]
        L.mco_galilean_lambda.argtypes = [u32, u32, u64, u64]
        L.mco_galilean_lambda.restype = u64
        L.mco_poisson_thresholds.argtypes = [ct.c_double, P(u32), P(u32), P(u64), u32]
        L.mco_feq.argtypes = [ct.c_double, ct.c_double, P(ct.c_double)]
        L.mco_feq.restype = None
        L.mco_collide_site.argtypes = [i32, u32, u32, u32, u32, u64, u64, u64, u64, P(u32)]
        L.mco_collide_site_direct.argtypes = [i32, u32, u32, u32, u64, u64, u64, u64, P(u32)]
        L.mco_histogram.argtypes = [i32, u32, u32, u32, ct.c_int, u64, u64, u64, P(u32), P(u64)]
        L.mco9_create.argtypes = [u32, P(u64), P(u64), P(u64), u64, i32, P(u32), u32,
                                  P(ct.c_void_p)]
        L.mco9_destroy.argtypes = [ct.c_void_p]
        L.mco9_destroy.restype = None
        L.mco9_init_counts.argtypes = [ct.c_void_p, u32, P(ct.c_uint16)]
        L.mco9_init_poisson.argtypes = [ct.c_void_p, u32, ct.c_double, ct.c_double, ct.c_double]
        L.mco9_step.argtypes = [ct.c_void_p, u64]
        L.mco9_get_counts.argtypes = [ct.c_void_p, u32, P(ct.c_uint16)]
        L.mco9_get_t.argtypes = [ct.c_void_p, u32]
        L.mco9_get_t.restype = i64
        L.mco9_moments.argtypes = [ct.c_void_p, u32, P(Moments9)]
        L.mco9_feq.argtypes = [ct.c_double, ct.c_double, ct.c_double, P(ct.c_double)]
        L.mco9_feq.restype = None
        L.mco9_targets.argtypes = [P(u32), u32, u32, P(u32), P(u32), P(u32), P(u32), P(u64),
                                   P(u64)]
        L.mco9_collide_site.argtypes = [i32, P(u32), u64, u64, u64, u64, P(u32)]
        _lib = L
    return _lib


class Moments9(ct.Structure):
    _fields_ = [("t", ct.c_int64), ("sites", ct.c_int64), ("sum_n", ct.c_int64 * 9),
                ("sum_nn", ct.c_int64 * 45), ("sum_N", ct.c_int64), ("sum_Jx", ct.c_int64),
                ("sum_Jy", ct.c_int64), ("max_N", ct.c_int64)]

    def as_dict(self) -> dict:
        return {"t": self.t, "sites": self.sites, "sum_n": list(self.sum_n),
                "sum_nn": list(self.sum_nn), "sum_N": self.sum_N, "sum_Jx": self.sum_Jx,
                "sum_Jy": self.sum_Jy, "max_N": self.max_N}


def _ptr(arr: np.ndarray, ctype):
    return arr.ctypes.data_as(ct.POINTER(ctype))


def _check(rc: int, what: str) -> int:
    if rc not in (0, -2):
        raise RuntimeError(f"oracle {what} failed with code {rc}")
    return rc


class OracleError(RuntimeError):
    pass


def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().mco_philox4x32_10(_ptr(c, ct.c_uint32), _ptr(k, ct.c_uint32), _ptr(out, ct.c_uint32))
    return out


def row_thresholds(C: int, lam: tuple, N: int, absJ: int, n0: int, flags: int = 0) -> np.ndarray:
    m = (N - absJ) // 2 + 1
    thr = np.zeros(max(m - 1, 1), dtype=np.uint64)
    mo = ct.c_uint32(0)
    rc = lib().mco_row_thresholds(C, lam[0], lam[1], flags, N, absJ, n0, _ptr(thr, ct.c_uint64),
                                  ct.byref(mo))
    if rc != 0:
        raise OracleError(f"row_thresholds rc={rc}")
    return thr[: mo.value - 1]


def poisson_thresholds(mu: float):
    cap = 1 << 16
    thr = np.zeros(cap, dtype=np.uint64)
    k_lo, cnt = ct.c_uint32(0), ct.c_uint32(0)
    rc = lib().mco_poisson_thresholds(mu, ct.byref(k_lo), ct.byref(cnt), _ptr(thr, ct.c_uint64), cap)
    if rc != 0:
        raise OracleError(f"poisson_thresholds rc={rc}")
    return k_lo.value, thr[: cnt.value - 1].copy()


def feq(rho: float, u: float) -> np.ndarray:
    out = np.zeros(3, dtype=np.float64)
    lib().mco_feq(rho, u, _ptr(out, ct.c_double))
    return out


def galilean_lambda(lam: tuple, N: int, absJ: int) -> int:
    """Numerator over 2^32 of the Galilean-invariant acceptance (R7)."""
    return int(lib().mco_galilean_lambda(lam[0], lam[1], N, absJ))


def collide_site(C, lam, n_max, seed, replica, t, x, abc, direct=False, flags=0):
    s = np.asarray(abc, dtype=np.uint32).copy()
    if direct:
        rc = lib().mco_collide_site_direct(C, lam[0], lam[1], flags, seed, replica, t, x,
                                           _ptr(s, ct.c_uint32))
    else:
        rc = lib().mco_collide_site(C, lam[0], lam[1], flags, n_max, seed, replica, t, x,
                                    _ptr(s, ct.c_uint32))
    return rc, s


def histogram(C, lam, abc, n_draws, seed=1, t=0, direct=False, flags=0) -> np.ndarray:
    s = np.asarray(abc, dtype=np.uint32)
    N = int(s.sum())
    h = np.zeros(N + 1, dtype=np.uint64)
    rc = lib().mco_histogram(C, lam[0], lam[1], flags, int(direct), seed, t, n_draws,
                             _ptr(s, ct.c_uint32), _ptr(h, ct.c_uint64))
    if rc != 0:
        raise OracleError(f"histogram rc={rc}")
    return h


class OracleSim:
    """n_rep independent periodic D1Q3 lattices advanced by the oracle."""

    def __init__(self, L, seed, C=10, lam=(1, 1), n_max=255, replica_id=None, flags=0):
        self.L = np.ascontiguousarray(np.atleast_1d(np.asarray(L, dtype=np.uint64)))
        self.n_rep = len(self.L)
        rid = None if replica_id is None else np.ascontiguousarray(np.asarray(replica_id, dtype=np.uint64))
        self._rid = rid
        h = ct.c_void_p()
        rc = lib().mco_create(self.n_rep, _ptr(self.L, ct.c_uint64),
                              None if rid is None else _ptr(rid, ct.c_uint64),
                              seed, C, lam[0], lam[1], n_max, flags, ct.byref(h))
        if rc != 0:
            raise OracleError(f"mco_create rc={rc}")
        self._h = h
        self.range_error = False

    def close(self):
        if self._h:
            lib().mco_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_counts(self, rep: int, counts: np.ndarray):
        c = np.ascontiguousarray(counts, dtype=np.uint16)
        assert c.shape == (3, int(self.L[rep]))
        _check(lib().mco_init_counts(self._h, rep, _ptr(c, ct.c_uint16)), "init_counts")

    def init_poisson(self, rep: int, rho: float, u0: float):
        rc = lib().mco_init_poisson(self._h, rep, rho, u0)
        if rc != 0:
            raise OracleError(f"init_poisson rc={rc}")

    def step(self, n: int = 1, rep: int | None = None) -> int:
        if rep is None:
            rc = lib().mco_step(self._h, n)
        else:
            rc = lib().mco_step_replica(self._h, rep, n)
        _check(rc, "step")
        if rc == -2:
            self.range_error = True
        return rc

    def counts(self, rep: int = 0) -> np.ndarray:
        out = np.zeros((3, int(self.L[rep])), dtype=np.uint16)
        _check(lib().mco_get_counts(self._h, rep, _ptr(out, ct.c_uint16)), "get_counts")
        return out

    def set_site_offset(self, rep: int, xoff: int, t: int = 0):
        rc = lib().mco_set_site_offset(self._h, rep, xoff, t)
        if rc != 0:
            raise OracleError(f"set_site_offset rc={rc}")

    def t(self, rep: int = 0) -> int:
        return int(lib().mco_get_t(self._h, rep))

    def moments(self, rep: int = 0, twiddle: np.ndarray | None = None) -> dict:
        m = Moments()
        if twiddle is None:
            rc = lib().mco_moments(self._h, rep, None, 0, ct.byref(m))
        else:
            tw = np.ascontiguousarray(twiddle, dtype=np.int32)
            n_modes = tw.shape[0] // 2
            rc = lib().mco_moments(self._h, rep, _ptr(tw, ct.c_int32), n_modes, ct.byref(m))
        _check(rc, "moments")
        return m.as_dict()


# ---- D2Q9 -------------------------------------------------------------------
# Velocity i of D2Q9 (columns of Eq. (MomD2Q9)).
V9 = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
# lambda_1..9 of the paper's D2Q9 equilibrium run (lambda_1 = 15/128,
# lambda_2-7 = 1/4, lambda_8 = 1/8, lambda_9 = 18/144).
LAMBDA9_PAPER = [(15, 128)] + [(1, 4)] * 6 + [(1, 8), (18, 144)]


def _lam9(lams) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(lams, dtype=np.uint32).reshape(18))


def targets9(lams, i: int, j: int):
    """[(k, l, class, weight)], D for the ordered source pair (i, j)."""
    lam = _lam9(lams)
    n = ct.c_uint32(0)
    k = (ct.c_uint32 * 8)(); l_ = (ct.c_uint32 * 8)(); c = (ct.c_uint32 * 8)()
    w = (ct.c_uint64 * 8)(); D = ct.c_uint64(0)
    _check(lib().mco9_targets(_ptr(lam, ct.c_uint32), i, j, ct.byref(n), k, l_, c, w,
                              ct.byref(D)), "targets9")
    return [(k[q], l_[q], c[q], w[q]) for q in range(n.value)], D.value


def feq9(rho: float, ux: float, uy: float) -> np.ndarray:
    out = np.zeros(9, dtype=np.float64)
    lib().mco9_feq(rho, ux, uy, _ptr(out, ct.c_double))
    return out


def collide_site9(C, lams, seed, replica, t, s, n9):
    n = np.ascontiguousarray(np.asarray(n9, dtype=np.uint32).copy())
    lam = _lam9(lams)
    _check(lib().mco9_collide_site(C, _ptr(lam, ct.c_uint32), seed, replica, t, s,
                                   _ptr(n, ct.c_uint32)), "collide_site9")
    return n


class OracleSim9:
    """n_rep independent periodic D2Q9 lattices (Lx x Ly) advanced by the oracle."""

    def __init__(self, Lx, Ly, seed, C=10, lams=LAMBDA9_PAPER, replica_id=None, flags=0):
        self.Lx = np.ascontiguousarray(np.atleast_1d(np.asarray(Lx, dtype=np.uint64)))
        self.Ly = np.ascontiguousarray(np.broadcast_to(np.asarray(Ly, dtype=np.uint64),
                                                       self.Lx.shape).copy())
        self.n_rep = len(self.Lx)
        rid = None if replica_id is None else np.ascontiguousarray(np.asarray(replica_id, dtype=np.uint64))
        lam = _lam9(lams)
        h = ct.c_void_p()
        rc = lib().mco9_create(self.n_rep, _ptr(self.Lx, ct.c_uint64), _ptr(self.Ly, ct.c_uint64),
                               None if rid is None else _ptr(rid, ct.c_uint64), seed, C,
                               _ptr(lam, ct.c_uint32), flags, ct.byref(h))
        if rc != 0:
            raise OracleError(f"mco9_create rc={rc}")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().mco9_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sites(self, rep: int = 0) -> int:
        return int(self.Lx[rep]) * int(self.Ly[rep])

    def init_counts(self, rep: int, counts: np.ndarray):
        c = np.ascontiguousarray(np.asarray(counts, dtype=np.uint16).reshape(9 * self.sites(rep)))
        _check(lib().mco9_init_counts(self._h, rep, _ptr(c, ct.c_uint16)), "init_counts9")

    def init_poisson(self, rep: int, rho: float, ux: float, uy: float):
        _check(lib().mco9_init_poisson(self._h, rep, rho, ux, uy), "init_poisson9")

    def step(self, n: int = 1) -> int:
        return lib().mco9_step(self._h, n)

    def counts(self, rep: int = 0) -> np.ndarray:
        """[9, Ly, Lx] uint16."""
        out = np.zeros(9 * self.sites(rep), dtype=np.uint16)
        _check(lib().mco9_get_counts(self._h, rep, _ptr(out, ct.c_uint16)), "get_counts9")
        return out.reshape(9, int(self.Ly[rep]), int(self.Lx[rep]))

    def t(self, rep: int = 0) -> int:
        return int(lib().mco9_get_t(self._h, rep))

    def moments(self, rep: int = 0) -> dict:
        m = Moments9()
        _check(lib().mco9_moments(self._h, rep, ct.byref(m)), "moments9")
        return m.as_dict()
