"""Philox4x32-10 counter-based generator (oracle side).

Written from the published definition (Salmon, Moraes, Dror, Shaw,
"Parallel Random Numbers: As Easy as 1, 2, 3", SC'11): four 32-bit counter
words and a two-word key; each of ten rounds multiplies counter words 0 and
2 by two fixed odd constants, exchanges the high and low halves across the
words and XORs in the key, and the key advances by two Weyl constants between
rounds.  Pinned by the generator's published known-answer vectors
(tests/golden/philox_kat.txt).
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_SH = np.uint64(32)


def philox4x32_10(ctr, key):
    """ctr: uint [..., 4], key: uint [..., 2] -> uint32 [..., 4] (broadcasting)."""
    ctr = np.asarray(ctr, dtype=np.uint64) & _MASK
    key = np.asarray(key, dtype=np.uint64) & _MASK
    c0, c1, c2, c3 = (ctr[..., i] for i in range(4))
    k0, k1 = key[..., 0], key[..., 1]
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0          # < 2^64: exact in uint64
        p1 = _M1 * c2
        hi0, lo0 = p0 >> _SH, p0 & _MASK
        hi1, lo1 = p1 >> _SH, p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return np.stack(np.broadcast_arrays(c0, c1, c2, c3), -1).astype(np.uint32)


def uniform01(x):
    """Top 24 bits of a 32-bit word as a float in [0, 1) (exact in fp32 and fp64)."""
    return (np.asarray(x, dtype=np.uint32) >> np.uint32(8)).astype(np.float64) * (1.0 / 16777216.0)
