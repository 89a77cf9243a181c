"""The state digest of the moments call, computed on the host from counts.

The digest is a checksum, not part of the method: for a D1Q3 state in
logical order (counts[i][x], i = 0, 1, 2 for v = -1, 0, +1) it is the sum
over sites and velocities of fmix32(fmix32(4 x + i + 1) ^ n_i(x)) modulo
2^64, with fmix32 the 32-bit finaliser of MurmurHash3.  Tests use it to
compare whole states (GPU against the oracle, a job alone against the same
job among others) without moving them.
"""
import numpy as np


def fmix32(k: np.ndarray) -> np.ndarray:
    k = k.astype(np.uint32, copy=True)
    k ^= k >> np.uint32(16)
    k *= np.uint32(0x85EBCA6B)
    k ^= k >> np.uint32(13)
    k *= np.uint32(0xC2B2AE35)
    k ^= k >> np.uint32(16)
    return k


def digest(counts: np.ndarray) -> int:
    counts = np.asarray(counts)
    L = counts.shape[1]
    x4 = np.arange(L, dtype=np.uint32) * np.uint32(4)
    total = 0
    for i in range(3):
        h = fmix32(fmix32(x4 + np.uint32(i + 1)) ^ counts[i].astype(np.uint32))
        total += int(h.astype(np.uint64).sum(dtype=np.uint64))
    return total % (1 << 64)
