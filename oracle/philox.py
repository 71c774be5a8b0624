"""Philox4x64-10 counter-based RNG and the Z4 noise drawn from it (oracle).

Philox4x64-10 follows its published definition (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11): a 4-word counter and a
2-word key; each of the 10 rounds multiplies counter words 0 and 2 by the two
Philox multipliers (full 128-bit products), then outputs
    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))
and the key is bumped by the two Weyl constants between rounds.

Z4 noise (paper Introduction, eq. test: entries drawn uniformly from
{1, -1, i, -i}).  Reading used by this build: the component index is
c = (site*4 + spin)*3 + colour; component c takes 2 bits from the Philox block
with counter (c // 128, sample, level, instance) and key (seed, 0): word
(c % 128) // 32, bits 2*(c % 32) and up (low bits first).  The 2-bit value k
maps to z = i**k (0 -> 1, 1 -> i, 2 -> -1, 3 -> -i).

Parity: pinned against numpy.random.Philox raw output (a separate
implementation of the same generator) and by the uniformity of k.
"""

import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
MASK64 = (1 << 64) - 1


def philox4x64_scalar(ctr, key, rounds=10):
    """Reference Philox4x64 on Python integers (one block)."""
    c = [int(v) & MASK64 for v in ctr]
    k0, k1 = int(key[0]) & MASK64, int(key[1]) & MASK64
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + W0) & MASK64
            k1 = (k1 + W1) & MASK64
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a, b):
    """Full 64x64 -> 128 product of uint64 arrays, as (hi, lo)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a_lo, a_hi = a & _LO32, a >> _S32
    b_lo, b_hi = b & _LO32, b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    cross = (ll >> _S32) + (lh & _LO32) + (hl & _LO32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (cross >> _S32)
    lo = a * b
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0, k1, rounds=10):
    """Vectorised Philox4x64 over uint64 arrays (broadcast); returns 4 arrays."""
    with np.errstate(over='ignore'):
        c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) for v in (c0, c1, c2, c3))
        c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
        k0 = np.uint64(int(k0) & MASK64)
        k1 = np.uint64(int(k1) & MASK64)
        for r in range(rounds):
            if r > 0:
                k0 = np.uint64((int(k0) + W0) & MASK64)
                k1 = np.uint64((int(k1) + W1) & MASK64)
            hi0, lo0 = _mulhilo(np.uint64(M0), c0)
            hi1, lo1 = _mulhilo(np.uint64(M1), c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


Z4_VALUES = np.array([1.0, 1.0j, -1.0, -1.0j], dtype=np.complex128)


def z4_codes(V, seed, instance, level, sample):
    """The 2-bit codes k (uint8, shape (V,4,3)) of one Z4 noise vector."""
    n = 12 * V
    nblk = (n + 127) // 128
    b = np.arange(nblk, dtype=np.uint64)
    words = philox4x64(b, np.uint64(sample), np.uint64(level), np.uint64(instance),
                       seed, 0)
    words = np.stack(words, axis=1)  # (nblk, 4)
    c = np.arange(n, dtype=np.int64)
    w = words[c // 128, (c % 128) // 32]
    k = (w >> (2 * (c % 32)).astype(np.uint64)) & np.uint64(3)
    return k.astype(np.uint8).reshape(V, 4, 3)


def z4_noise(V, seed, instance, level, sample):
    """One Z4 noise vector in canonical layout (V, 4, 3) complex128."""
    return Z4_VALUES[z4_codes(V, seed, instance, level, sample)]
