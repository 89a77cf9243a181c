"""Python binding of libmclg.so (the MI355X MCLG library).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides device memory (caller-owned tensors) and the
stream.  The functions keep the C names; ``Lattice`` and ``Server`` are thin
owners of the tensors a context needs.  There is no CPU fallback: without the
built library or a GPU every entry point raises.
"""
from __future__ import annotations

import ctypes as ct
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmclg.so")

ABI_VERSION = 1
D1Q3, D2Q9 = 1, 2
C_EQUILIBRIUM = -1
FLAG_NO_STREAM = 1
FLAG_GALILEAN = 2
INIT_COUNTS, INIT_POISSON = 1, 2
MAX_MODES = 8
MAX_HIST_BINS = 4096
MOMENTS_DIGEST = 1
DRAIN_AUTO, DRAIN_DEFERRED, DRAIN_CHUNK, DRAIN_PATCH = 0, 1, 2, 3
OK, E_INVAL, E_RANGE, E_HIP, E_NOMEM, E_UNSUPPORTED, E_FULL, E_INTERNAL = 0, -1, -2, -3, -4, -5, -6, -7
E_TOO_LARGE = -8

u32, u64, i32, i64, dbl, vp = ct.c_uint32, ct.c_uint64, ct.c_int32, ct.c_int64, ct.c_double, ct.c_void_p
P = ct.POINTER


class mclg_config(ct.Structure):
    _fields_ = [("abi_version", u32), ("lattice", u32), ("n_replicas", u32), ("flags", u32),
                ("L", P(u64)), ("replica_id", P(u64)), ("seed", u64), ("C", i32),
                ("lambda_num", u32), ("lambda_den", u32), ("n_max", u32), ("stream", vp),
                ("state", vp), ("state_bytes", u64), ("workspace", vp), ("workspace_bytes", u64),
                ("Ly", P(u64)), ("lambda9", P(u32))]


class mclg_init_spec(ct.Structure):
    _fields_ = [("kind", u32), ("counts", vp), ("rho", P(dbl)), ("u0", P(dbl)), ("u0y", P(dbl))]


class mclg_moments9_t(ct.Structure):
    _fields_ = [("t", i64), ("sites", i64), ("sum_n", i64 * 9), ("sum_nn", i64 * 45),
                ("sum_N", i64), ("sum_Jx", i64), ("sum_Jy", i64), ("max_N", i64)]

    def as_dict(self) -> dict:
        return {"t": self.t, "sites": self.sites, "sum_n": list(self.sum_n),
                "sum_nn": list(self.sum_nn), "sum_N": self.sum_N, "sum_Jx": self.sum_Jx,
                "sum_Jy": self.sum_Jy, "max_N": self.max_N}


class mclg_moments_t(ct.Structure):
    _fields_ = [("t", i64), ("sites", i64), ("sum_n", i64 * 3), ("sum_n2", i64 * 3),
                ("sum_nn", i64 * 3), ("sum_N", i64), ("sum_J", i64), ("sum_N2", i64),
                ("n0_odd", i64), ("max_N", i64), ("fourier", (i64 * 2) * MAX_MODES),
                ("digest", i64)]

    def as_dict(self) -> dict:
        return {"t": self.t, "sites": self.sites, "sum_n": list(self.sum_n),
                "sum_n2": list(self.sum_n2), "sum_nn": list(self.sum_nn), "sum_N": self.sum_N,
                "sum_J": self.sum_J, "sum_N2": self.sum_N2, "n0_odd": self.n0_odd,
                "max_N": self.max_N, "fourier": [list(self.fourier[m]) for m in range(MAX_MODES)],
                "digest": self.digest & 0xFFFFFFFFFFFFFFFF}


class mclg_server_config(ct.Structure):
    _fields_ = [("abi_version", u32), ("max_slots", u32), ("seed", u64), ("C", i32),
                ("lambda_num", u32), ("lambda_den", u32), ("n_max", u32), ("stream", vp),
                ("arena", vp), ("arena_bytes", u64), ("workspace", vp), ("workspace_bytes", u64)]


class mclg_job(ct.Structure):
    _fields_ = [("job_id", u64), ("L", u64), ("steps", u64), ("rho", dbl), ("u0", dbl)]


class mclg_job_result(ct.Structure):
    _fields_ = [("job_id", u64), ("moments", mclg_moments_t)]


class MclgError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what} failed: {mclg_strerror(code)} ({code})")
        self.code = code


_lib: Optional[ct.CDLL] = None

_SIGS = {
    "mclg_sizes": [P(mclg_config), P(u64), P(u64)],
    "mclg_init": [P(mclg_config), P(mclg_init_spec), P(vp)],
    "mclg_step": [vp, u64],
    "mclg_step_replica": [vp, u32, u64],
    "mclg_step_graph": [vp, u64],
    "mclg_moments": [vp, vp, u32, u32, P(mclg_moments_t)],
    "mclg_moments_noalloc": [vp, vp, u32, u32, vp],
    "mclg_step_log": [vp, u64, u64, vp, u32, u32, vp],
    "mclg_histogram": [vp, u32, vp],
    "mclg_moments9": [vp, P(mclg_moments9_t)],
    "mclg_d2q9_rules": [P(u32), P(u32), P(u32)],
    "mclg_get_counts": [vp, u32, P(ct.c_uint16)],
    "mclg_check": [vp],
    "mclg_set_schedule": [vp, u32, u32, u32],
    "mclg_set_grid_limit": [vp, u32],
    "mclg_set_drain": [vp, u32],
    "mclg_blocked_bytes": [vp, u32, u32, P(u64)],
    "mclg_set_blocked": [vp, u32, u32, vp, u64],
    "mclg_lds_coverage": [vp, P(dbl), P(u32)],
    "mclg_destroy": [vp],
    "mclg_strerror": [ct.c_int],
    "mclg_last_hip_error": [vp],
    "mclg_table_row": [i32, u32, u32, u32, u32, u32, u32, P(u64), u32, P(u32)],
    "mclg_galilean_lambda": [u32, u32, u32, u32, P(u64)],
    "mclg_poisson_thresholds": [dbl, P(u32), P(u32), P(u64), u32],
    "mclg_server_sizes": [P(mclg_server_config), P(u64)],
    "mclg_server_create": [P(mclg_server_config), P(vp)],
    "mclg_server_submit": [vp, P(mclg_job)],
    "mclg_server_tick": [vp, u32],
    "mclg_server_poll": [vp, P(mclg_job_result), u32, P(u32)],
    "mclg_server_stats": [vp, P(u64), P(u64), P(u64)],
    "mclg_server_destroy": [vp],
}


def lib() -> ct.CDLL:
    """Load libmclg.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1706_01094_amd.build")
        L = ct.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ct.c_char_p if name == "mclg_strerror" else ct.c_int
        _lib = L
    return _lib


def exported_symbols() -> list:
    return list(_SIGS)


def mclg_strerror(code: int) -> str:
    return lib().mclg_strerror(code).decode()


def _check(rc: int, what: str) -> int:
    if rc != OK:
        raise MclgError(rc, what)
    return rc


# ---- host-only inspection -------------------------------------------------
def mclg_table_row(C: int, lam: Sequence[int], N: int, absJ: int, n0: int,
                   flags: int = 0) -> np.ndarray:
    m = (N - absJ) // 2 + 1
    thr = np.zeros(max(m - 1, 1), dtype=np.uint64)
    mo = u32(0)
    _check(lib().mclg_table_row(C, lam[0], lam[1], flags, N, absJ, n0,
                                thr.ctypes.data_as(P(u64)), len(thr), ct.byref(mo)), "mclg_table_row")
    return thr[: mo.value - 1]


def mclg_d2q9_rules(lams):
    """(rules [81, 12] uint32, D) of the D2Q9 rule table (host only)."""
    lam = np.ascontiguousarray(np.asarray(lams, dtype=np.uint32).reshape(18))
    out = np.zeros(81 * 12, dtype=np.uint32)
    D = u32(0)
    _check(lib().mclg_d2q9_rules(lam.ctypes.data_as(P(u32)), out.ctypes.data_as(P(u32)),
                                 ct.byref(D)), "mclg_d2q9_rules")
    return out.reshape(81, 12), D.value


def mclg_galilean_lambda(lam: Sequence[int], N: int, absJ: int) -> int:
    out = u64(0)
    _check(lib().mclg_galilean_lambda(lam[0], lam[1], N, absJ, ct.byref(out)),
           "mclg_galilean_lambda")
    return out.value


def mclg_poisson_thresholds(mu: float):
    cap = 1 << 16
    thr = np.zeros(cap, dtype=np.uint64)
    k_lo, cnt = u32(0), u32(0)
    _check(lib().mclg_poisson_thresholds(mu, ct.byref(k_lo), ct.byref(cnt),
                                         thr.ctypes.data_as(P(u64)), cap), "mclg_poisson_thresholds")
    return k_lo.value, thr[: cnt.value - 1].copy()


def _require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the MCLG library needs a ROCm GPU; none is visible")
    return torch


def _stream_ptr(stream) -> int:
    return int(stream.cuda_stream)


# ---- simulation contexts --------------------------------------------------
def mclg_sizes(cfg: mclg_config):
    sb, wb = u64(0), u64(0)
    _check(lib().mclg_sizes(ct.byref(cfg), ct.byref(sb), ct.byref(wb)), "mclg_sizes")
    return sb.value, wb.value


def mclg_init(cfg: mclg_config, spec: mclg_init_spec) -> int:
    h = vp()
    rc = lib().mclg_init(ct.byref(cfg), ct.byref(spec), ct.byref(h))
    _check(rc, "mclg_init")
    return h.value


def mclg_step(ctx: int, n: int):
    _check(lib().mclg_step(ctx, n), "mclg_step")


def mclg_step_replica(ctx: int, replica: int, n: int):
    _check(lib().mclg_step_replica(ctx, replica, n), "mclg_step_replica")


def mclg_step_graph(ctx: int, n: int):
    _check(lib().mclg_step_graph(ctx, n), "mclg_step_graph")


def mclg_set_schedule(ctx: int, groups: int, threads: int, lds_budget: int = 96 * 1024):
    _check(lib().mclg_set_schedule(ctx, groups, threads, lds_budget), "mclg_set_schedule")


def mclg_set_grid_limit(ctx: int, max_blocks: int):
    _check(lib().mclg_set_grid_limit(ctx, max_blocks), "mclg_set_grid_limit")


def mclg_set_drain(ctx: int, policy: int):
    _check(lib().mclg_set_drain(ctx, policy), "mclg_set_drain")


def mclg_lds_coverage(ctx: int):
    f, b = dbl(0), u32(0)
    _check(lib().mclg_lds_coverage(ctx, ct.byref(f), ct.byref(b)), "mclg_lds_coverage")
    return f.value, b.value


def mclg_histogram(ctx: int, n_bins: int, dev_hist: int):
    _check(lib().mclg_histogram(ctx, n_bins, dev_hist), "mclg_histogram")


def mclg_check(ctx: int) -> int:
    return lib().mclg_check(ctx)


def mclg_destroy(ctx: int):
    lib().mclg_destroy(ctx)


class Lattice:
    """n_replicas periodic D1Q3 lattices resident on the GPU."""

    def __init__(self, L, seed: int, C: int = 10, lam=(1, 1), n_max: int = 255,
                 replica_id=None, flags: int = 0, rho=None, u0=None, counts=None,
                 stream=None, device: str = "cuda:0"):
        torch = _require_gpu()
        self.torch = torch
        self.L = np.ascontiguousarray(np.atleast_1d(np.asarray(L, dtype=np.uint64)))
        self.n = len(self.L)
        self._rid = None if replica_id is None else np.ascontiguousarray(
            np.asarray(replica_id, dtype=np.uint64))
        self.device = torch.device(device)
        # A stream of its own (default priority): graph capture needs a
        # non-null stream.
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        cfg = mclg_config()
        cfg.abi_version = ABI_VERSION
        cfg.lattice = D1Q3
        cfg.n_replicas = self.n
        cfg.flags = flags
        cfg.L = self.L.ctypes.data_as(P(u64))
        cfg.replica_id = None if self._rid is None else self._rid.ctypes.data_as(P(u64))
        cfg.seed = seed
        cfg.C = C
        cfg.lambda_num, cfg.lambda_den = lam
        cfg.n_max = n_max
        cfg.stream = _stream_ptr(self.stream)
        sb, wb = mclg_sizes(cfg)
        self.state = torch.empty(sb // 2 + 64, dtype=torch.int16, device=self.device)
        self.workspace = torch.empty(wb // 8 + 32, dtype=torch.int64, device=self.device)
        cfg.state = self.state.data_ptr()
        cfg.state_bytes = sb
        cfg.workspace = self.workspace.data_ptr()
        cfg.workspace_bytes = wb
        self.state_bytes, self.workspace_bytes = sb, wb
        spec = mclg_init_spec()
        keep = []
        if counts is not None:
            ct_ = counts if isinstance(counts, torch.Tensor) else torch.as_tensor(
                np.ascontiguousarray(counts).view(np.int16))
            ct_ = ct_.to(self.device).contiguous()
            if ct_.numel() != 3 * int(self.L.sum()) or ct_.element_size() != 2:
                raise ValueError("counts must hold 3 * sum(L) uint16 values")
            keep.append(ct_)
            spec.kind = INIT_COUNTS
            spec.counts = ct_.data_ptr()
        else:
            r = np.ascontiguousarray(np.broadcast_to(np.asarray(rho, dtype=np.float64), (self.n,)))
            u = np.ascontiguousarray(np.broadcast_to(np.asarray(0.0 if u0 is None else u0,
                                                                dtype=np.float64), (self.n,)))
            keep += [r, u]
            spec.kind = INIT_POISSON
            spec.rho = r.ctypes.data_as(P(dbl))
            spec.u0 = u.ctypes.data_as(P(dbl))
        self._cfg = cfg
        # tensors written on torch's stream must be ready for the library's
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self.ctx = mclg_init(cfg, spec)

    def close(self):
        if getattr(self, "ctx", None):
            mclg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        mclg_step(self.ctx, n)

    def step_replica(self, replica: int, n: int = 1):
        mclg_step_replica(self.ctx, replica, n)

    def step_graph(self, n: int):
        mclg_step_graph(self.ctx, n)

    def set_schedule(self, groups: int, threads: int, lds_budget: int = 96 * 1024):
        mclg_set_schedule(self.ctx, groups, threads, lds_budget)

    def set_grid_limit(self, max_blocks: int):
        mclg_set_grid_limit(self.ctx, max_blocks)

    def set_drain(self, policy: int):
        mclg_set_drain(self.ctx, policy)

    def set_blocked(self, steps: int, tile: int = 0):
        """mclg_set_blocked: `steps` steps per launch (temporal blocking) on
        whole block ranges (tile = 1) or in tiles of `tile` sites (>= 2;
        0 picks), with a scratch tensor of this lattice's device owned here;
        steps <= 1 switches it off."""
        if steps <= 1:
            _check(lib().mclg_set_blocked(self.ctx, 0, 0, None, 0), "mclg_set_blocked")
            self._tb = None
            return
        n = u64(0)
        _check(lib().mclg_blocked_bytes(self.ctx, steps, tile, ct.byref(n)), "mclg_blocked_bytes")
        buf = self.torch.empty(int(n.value), dtype=self.torch.uint8, device=self.device)
        _check(lib().mclg_set_blocked(self.ctx, steps, tile, buf.data_ptr(), int(n.value)),
               "mclg_set_blocked")
        self._tb = buf

    def lds_coverage(self):
        return mclg_lds_coverage(self.ctx)

    def check(self) -> int:
        return mclg_check(self.ctx)

    def moments(self, twiddle=None, n_modes: int = 0, allow_range=False, digest=False):
        """Exact moments of every replica; with digest=True also the state
        digest (see state_digest)."""
        out = (mclg_moments_t * self.n)()
        tw = 0
        if twiddle is not None:
            if twiddle.numel() < 2 * n_modes * int(self.L.sum()) or twiddle.element_size() != 4:
                raise ValueError("twiddle must hold 2 * n_modes * sum(L) int32 values")
            self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
            tw = twiddle.data_ptr()
        rc = lib().mclg_moments(self.ctx, tw, n_modes, MOMENTS_DIGEST if digest else 0, out)
        if rc != OK and not (allow_range and rc == E_RANGE):
            raise MclgError(rc, "mclg_moments")
        return [o.as_dict() for o in out]

    def moments_to_device(self, out, twiddle=None, n_modes: int = 0, digest=False):
        """mclg_moments_noalloc: the moments of every replica written, in the
        stream order of this lattice's stream and without allocating or
        synchronising, into ``out`` (a contiguous int64 tensor of at least
        n_replicas * 33 elements on the device, one mclg_moments_t per
        replica); t is the device's step counter."""
        tw = self._device_out(out, twiddle, n_modes)
        _check(lib().mclg_moments_noalloc(self.ctx, tw, n_modes, MOMENTS_DIGEST if digest else 0,
                                          out.data_ptr()), "mclg_moments_noalloc")
        return out

    def step_log(self, every: int, n_logs: int, out, twiddle=None, n_modes: int = 0,
                 digest=False):
        """mclg_step_log: n_logs times `every` steps and the moments of every
        replica after them, written into ``out`` (a contiguous int64 tensor of
        at least n_logs * n_replicas * 33 values on the device; log j of
        replica r is row j * n_replicas + r) in stream order, without
        synchronising; with blocking on, each launch sums the logs that fall
        in it."""
        tw = self._device_out(out, twiddle, n_modes, n_logs)
        _check(lib().mclg_step_log(self.ctx, every, n_logs, tw, n_modes,
                                   MOMENTS_DIGEST if digest else 0, out.data_ptr()),
               "mclg_step_log")
        return out

    def _device_out(self, out, twiddle, n_modes, n_records=1):
        """Checks of a device result tensor (n_records records per replica)
        and twiddle input; the twiddle pointer (0 without)."""
        words = ct.sizeof(mclg_moments_t) // 8
        if out.dtype != self.torch.int64 or out.numel() < words * self.n * n_records or \
                not out.is_contiguous():
            raise ValueError("out must be a contiguous int64 tensor of records * n_replicas * 33 "
                             "values")
        if twiddle is None:
            return 0
        if twiddle.numel() < 2 * n_modes * int(self.L.sum()) or twiddle.element_size() != 4:
            raise ValueError("twiddle must hold 2 * n_modes * sum(L) int32 values")
        return twiddle.data_ptr()

    def histogram(self, n_bins: int, out=None):
        """Add this state's occupation-number histograms to ``out`` (an int64
        tensor [n_replicas, 3, n_bins] on the device, zeros if None) and
        return it; the last bin counts every n >= n_bins - 1."""
        torch = self.torch
        if out is None:
            out = torch.zeros((self.n, 3, n_bins), dtype=torch.int64, device=self.device)
        if out.dtype != torch.int64 or out.numel() != 3 * self.n * n_bins or not out.is_contiguous():
            raise ValueError("out must be a contiguous int64 tensor of n_replicas * 3 * n_bins")
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        mclg_histogram(self.ctx, n_bins, out.data_ptr())
        cur.wait_stream(self.stream)
        return out

    def counts(self, replica: int = 0, allow_range=False) -> np.ndarray:
        L = int(self.L[replica])
        out = np.zeros((3, L), dtype=np.uint16)
        rc = lib().mclg_get_counts(self.ctx, replica, out.ctypes.data_as(P(ct.c_uint16)))
        if rc != OK and not (allow_range and rc == E_RANGE):
            raise MclgError(rc, "mclg_get_counts")
        return out


# lambda_1..9 of the paper's D2Q9 equilibrium run: 15/128, 1/4 (x6), 1/8, 18/144
LAMBDA9_PAPER = [(15, 128)] + [(1, 4)] * 6 + [(1, 8), (18, 144)]


class Lattice9:
    """n_replicas periodic D2Q9 lattices (Lx[r] x Ly[r]) resident on the GPU."""

    def __init__(self, Lx, Ly, seed: int, C: int = 10, lams=LAMBDA9_PAPER, replica_id=None,
                 flags: int = 0, rho=None, ux=None, uy=None, counts=None, stream=None,
                 device: str = "cuda:0"):
        torch = _require_gpu()
        self.torch = torch
        self.Lx = np.ascontiguousarray(np.atleast_1d(np.asarray(Lx, dtype=np.uint64)))
        self.n = len(self.Lx)
        self.Ly = np.ascontiguousarray(np.broadcast_to(np.asarray(Ly, dtype=np.uint64),
                                                       (self.n,)).copy())
        self._lam = np.ascontiguousarray(np.asarray(lams, dtype=np.uint32).reshape(18))
        self._rid = None if replica_id is None else np.ascontiguousarray(
            np.asarray(replica_id, dtype=np.uint64))
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        cfg = mclg_config()
        cfg.abi_version = ABI_VERSION
        cfg.lattice = D2Q9
        cfg.n_replicas = self.n
        cfg.flags = flags
        cfg.L = self.Lx.ctypes.data_as(P(u64))
        cfg.Ly = self.Ly.ctypes.data_as(P(u64))
        cfg.lambda9 = self._lam.ctypes.data_as(P(u32))
        cfg.replica_id = None if self._rid is None else self._rid.ctypes.data_as(P(u64))
        cfg.seed = seed
        cfg.C = C
        cfg.lambda_num, cfg.lambda_den = 1, 1
        cfg.stream = _stream_ptr(self.stream)
        sb, wb = mclg_sizes(cfg)
        self.state = torch.empty(sb // 2 + 64, dtype=torch.int16, device=self.device)
        self.workspace = torch.empty(wb // 8 + 32, dtype=torch.int64, device=self.device)
        cfg.state = self.state.data_ptr()
        cfg.state_bytes = sb
        cfg.workspace = self.workspace.data_ptr()
        cfg.workspace_bytes = wb
        spec = mclg_init_spec()
        keep = []
        sites = int((self.Lx * self.Ly).sum())
        if counts is not None:
            ct_ = counts if isinstance(counts, torch.Tensor) else torch.as_tensor(
                np.ascontiguousarray(counts).reshape(-1).view(np.int16))
            ct_ = ct_.to(self.device).contiguous()
            if ct_.numel() != 9 * sites or ct_.element_size() != 2:
                raise ValueError("counts must hold 9 * sum(Lx * Ly) uint16 values")
            keep.append(ct_)
            spec.kind = INIT_COUNTS
            spec.counts = ct_.data_ptr()
        else:
            vals = [np.ascontiguousarray(np.broadcast_to(np.asarray(0.0 if v is None else v,
                                                                    dtype=np.float64), (self.n,)))
                    for v in (rho, ux, uy)]
            keep += vals
            spec.kind = INIT_POISSON
            spec.rho, spec.u0, spec.u0y = (v.ctypes.data_as(P(dbl)) for v in vals)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self.ctx = mclg_init(cfg, spec)

    def close(self):
        if getattr(self, "ctx", None):
            mclg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        mclg_step(self.ctx, n)

    def check(self) -> int:
        return mclg_check(self.ctx)

    def counts(self, replica: int = 0, allow_range=False) -> np.ndarray:
        """[9, Ly, Lx] uint16 in logical order."""
        Lx, Ly = int(self.Lx[replica]), int(self.Ly[replica])
        out = np.zeros((9, Ly, Lx), dtype=np.uint16)
        rc = lib().mclg_get_counts(self.ctx, replica, out.ctypes.data_as(P(ct.c_uint16)))
        if rc != OK and not (allow_range and rc == E_RANGE):
            raise MclgError(rc, "mclg_get_counts")
        return out

    def histogram(self, n_bins: int, out=None):
        """Add the occupation-number histograms to ``out`` (int64 [n_replicas,
        9, n_bins] on the device, zeros if None) and return it; the last bin
        counts every n >= n_bins - 1."""
        torch = self.torch
        if out is None:
            out = torch.zeros((self.n, 9, n_bins), dtype=torch.int64, device=self.device)
        if out.dtype != torch.int64 or out.numel() != 9 * self.n * n_bins or not out.is_contiguous():
            raise ValueError("out must be a contiguous int64 tensor of n_replicas * 9 * n_bins")
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        mclg_histogram(self.ctx, n_bins, out.data_ptr())
        cur.wait_stream(self.stream)
        return out

    def moments(self, allow_range=False):
        return [o.as_dict() for o in self._moments9(allow_range)]

    def moments_array(self, allow_range=False) -> np.ndarray:
        """The same sums as an int64 array [n_replicas, 60] in the field
        order of mclg_moments9_t (t, sites, sum_n[9], sum_nn[45], sum_N,
        sum_Jx, sum_Jy, max_N)."""
        out = self._moments9(allow_range)
        return np.frombuffer(out, dtype=np.int64).reshape(self.n, -1).copy()

    def _moments9(self, allow_range):
        out = (mclg_moments9_t * self.n)()
        rc = lib().mclg_moments9(self.ctx, out)
        if rc != OK and not (allow_range and rc == E_RANGE):
            raise MclgError(rc, "mclg_moments9")
        return out


class Server:
    """Continuous-batching server of D1Q3 jobs with state resident in an arena."""

    def __init__(self, arena_bytes: int, max_slots: int, seed: int, C: int = 10, lam=(1, 1),
                 n_max: int = 255, stream=None, device: str = "cuda:0"):
        torch = _require_gpu()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        cfg = mclg_server_config()
        cfg.abi_version = ABI_VERSION
        cfg.max_slots = max_slots
        cfg.seed = seed
        cfg.C = C
        cfg.lambda_num, cfg.lambda_den = lam
        cfg.n_max = n_max
        cfg.stream = _stream_ptr(self.stream)
        cfg.arena_bytes = arena_bytes
        wb = u64(0)
        _check(lib().mclg_server_sizes(ct.byref(cfg), ct.byref(wb)), "mclg_server_sizes")
        self.arena = torch.empty(arena_bytes // 8 + 32, dtype=torch.int64, device=self.device)
        self.workspace = torch.empty(wb.value // 8 + 32, dtype=torch.int64, device=self.device)
        cfg.arena = self.arena.data_ptr()
        cfg.workspace = self.workspace.data_ptr()
        cfg.workspace_bytes = wb.value
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        h = vp()
        _check(lib().mclg_server_create(ct.byref(cfg), ct.byref(h)), "mclg_server_create")
        self.h = h.value
        self._cfg = cfg

    def submit(self, job_id: int, L: int, steps: int, rho: float, u0: float = 0.0):
        j = mclg_job(job_id, L, steps, rho, u0)
        _check(lib().mclg_server_submit(self.h, ct.byref(j)), "mclg_server_submit")

    def tick(self, k: int):
        _check(lib().mclg_server_tick(self.h, k), "mclg_server_tick")

    def poll(self, cap: int = 4096):
        out = (mclg_job_result * cap)()
        n = u32(0)
        _check(lib().mclg_server_poll(self.h, out, cap, ct.byref(n)), "mclg_server_poll")
        return [(out[i].job_id, out[i].moments.as_dict()) for i in range(n.value)]

    def stats(self):
        q, r, a = u64(0), u64(0), u64(0)
        _check(lib().mclg_server_stats(self.h, ct.byref(q), ct.byref(r), ct.byref(a)), "mclg_server_stats")
        return q.value, r.value, a.value

    def close(self):
        if getattr(self, "h", None):
            lib().mclg_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
