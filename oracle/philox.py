"""Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC'11) -- oracle side.

The paper fixes no random number generator (its experiments average ten
runs, Sections 3 and 5).  The reading taken here, shared by contract with the
HIP side (which implements the same published generator independently), is
a counter-based generator so that every draw is a pure function of
(seed, index, iteration, phase, system):

    block = Philox4x64_10(counter=(j >> 2, it, phase, sys), key=(seed, key1))
    word  = block[j & 3]

One round maps (c0, c1, c2, c3) with key (k0, k1) to
    (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0))
and the key is bumped by the Weyl constants between rounds; ten rounds.

Test infrastructure only (see the package docstring).
"""
import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
MASK64 = (1 << 64) - 1
ROUNDS = 10


def philox4x64_10_int(ctr, key):
    """Scalar reference with Python integers (exact 128-bit products).

    ctr: 4 ints < 2**64, key: 2 ints < 2**64.  Returns a tuple of 4 ints."""
    c0, c1, c2, c3 = (int(v) & MASK64 for v in ctr)
    k0, k1 = (int(v) & MASK64 for v in key)
    for r in range(ROUNDS):
        if r:
            k0 = (k0 + W0) & MASK64
            k1 = (k1 + W1) & MASK64
        p0 = M0 * c0
        p1 = M1 * c2
        c0, c1, c2, c3 = ((p1 >> 64) ^ c1 ^ k0, p1 & MASK64,
                          (p0 >> 64) ^ c3 ^ k1, p0 & MASK64)
    return c0, c1, c2, c3


_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a, b):
    """128-bit product of uint64 arrays a*b as (hi, lo), via 32-bit limbs."""
    a_lo = a & _LO32
    a_hi = a >> _S32
    b_lo = b & _LO32
    b_hi = b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _S32) + (lh & _LO32) + (hl & _LO32)
    lo = (mid << _S32) | (ll & _LO32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x64-10 over uint64 numpy arrays (broadcasting).

    Returns four uint64 arrays (the output block words 0..3)."""
    with np.errstate(over="ignore"):
        c0 = np.asarray(c0, dtype=np.uint64)
        c1 = np.asarray(c1, dtype=np.uint64)
        c2 = np.asarray(c2, dtype=np.uint64)
        c3 = np.asarray(c3, dtype=np.uint64)
        c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
        k0 = np.uint64(int(k0) & MASK64)
        k1 = np.uint64(int(k1) & MASK64)
        m0 = np.full(c0.shape, M0, dtype=np.uint64)
        m1 = np.full(c0.shape, M1, dtype=np.uint64)
        for r in range(ROUNDS):
            if r:
                k0 = np.uint64((int(k0) + W0) & MASK64)
                k1 = np.uint64((int(k1) + W1) & MASK64)
            hi0, lo0 = _mulhilo(m0, c0)
            hi1, lo1 = _mulhilo(m1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def index_words(idx, seed, it, phase, sys=0, key1=0):
    """The 64-bit random word assigned to each index in ``idx``.

    Counter (idx >> 2, it, phase, sys), key (seed, key1); word idx & 3."""
    idx = np.asarray(idx, dtype=np.int64)
    g = (idx >> 2).astype(np.uint64)
    o0, o1, o2, o3 = philox4x64_10(g, np.uint64(it), np.uint64(phase),
                                   np.uint64(sys), seed, key1)
    lane = idx & 3
    return np.choose(lane, [o0, o1, o2, o3]).astype(np.uint64)


def words_to_unit(w):
    """Map 64-bit words to doubles in the open interval (0, 1).

    u = (2*(w >> 12) + 1) * 2**-53: the odd integer is below 2**53, so the
    conversion and the power-of-two scaling are exact."""
    w = np.asarray(w, dtype=np.uint64)
    odd = (w >> np.uint64(12)) * np.uint64(2) + np.uint64(1)
    return odd.astype(np.float64) * (2.0 ** -53)
