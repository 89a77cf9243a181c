"""The allocation-free moments entry point (mclg_moments_noalloc) through the
C ABI: its device-side results equal mclg_moments's on two calls in a row,
the second with a smaller input (the static scratch area keeps the first
call's contents), and a context too large for the area is refused."""
import ctypes as ct
import sys

import numpy as np
import pytest

import synth
from paper_1706_01094_amd import mclg as M
from paper_1706_01094_amd.mclg import Lattice

pytestmark = pytest.mark.gpu

KEYS = ("t", "sites", "sum_n", "sum_n2", "sum_nn", "sum_N", "sum_J", "sum_N2", "n0_odd",
        "max_N", "fourier", "digest")


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def noalloc(lat, twiddle=None, n_modes=0, flags=0):
    import torch
    words = ct.sizeof(M.mclg_moments_t) // 8
    out = torch.full((lat.n, words), -1, dtype=torch.int64, device=lat.device)
    lat.stream.wait_stream(torch.cuda.current_stream(lat.device))
    tw = 0 if twiddle is None else twiddle.data_ptr()
    rc = M.lib().mclg_moments_noalloc(lat.ctx, tw, n_modes, flags, out.data_ptr())
    assert rc == M.OK, M.mclg_strerror(rc)
    lat.stream.synchronize()
    host = np.ascontiguousarray(out.cpu().numpy())
    return [M.mclg_moments_t.from_buffer_copy(host[r].tobytes()).as_dict() for r in range(lat.n)]


def check(lat, tw=None, n_modes=0):
    for flags, digest in ((0, False), (M.MOMENTS_DIGEST, True)):
        got = noalloc(lat, tw, n_modes, flags)
        want = lat.moments(tw, n_modes, digest=digest)
        for r in range(lat.n):
            for k in KEYS:
                assert got[r][k] == want[r][k], (r, k, flags)


def test_noalloc_equals_moments_on_two_calls():
    import torch
    # first call: 24 replicas (ragged, up to 2^20 sites) with three Fourier modes
    man = synth.replica_manifest(n=24, seed=11, L_lo=1, L_hi=1 << 20)
    say("first", len(man["L"]), int(man["L"].sum()))
    big = Lattice(man["L"], 3, rho=man["rho"], u0=man["u0"], replica_id=man["replica_id"])
    # replica r's block is [6][L[r]], blocks packed in replica order
    tw = np.concatenate([synth.twiddles(int(L), 3).ravel() for L in man["L"]])
    twd = torch.as_tensor(np.ascontiguousarray(tw)).to("cuda:0")
    big.step(7)
    check(big, twd, 3)
    big.close()
    # second call: a smaller context, no modes; the area still holds the
    # first call's records
    say("second")
    small = Lattice([1, 1000, 4097], 5, rho=[2.0, 30.0, 90.0], u0=[0.0, 0.1, -0.2])
    small.step(3)
    check(small)
    small.step(2)
    check(small)
    small.close()


def test_too_large_for_the_scratch_area_is_refused():
    # one 256-byte partial record per replica of one site: 32769 records
    # exceed the 8 MiB area
    n = (8 << 20) // 256 + 1
    say("too large", n)
    lat = Lattice(np.ones(n, dtype=np.uint64), 1, rho=3.0, u0=0.0)
    import torch
    out = torch.zeros((n, ct.sizeof(M.mclg_moments_t) // 8), dtype=torch.int64, device=lat.device)
    rc = M.lib().mclg_moments_noalloc(lat.ctx, 0, 0, 0, out.data_ptr())
    assert rc == M.E_TOO_LARGE
    assert lat.moments()[n - 1]["sites"] == 1  # the workspace path still serves it
    lat.close()
