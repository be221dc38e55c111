"""Block selection of RGDBEK -- oracle side.

Section 2 (the column/row set probabilities and Algorithm 1): compute the
residual weights eps_j, form P(j) = eps_j / sum_l eps_l, and select a block of
k indices "using P".  The paper does not say with or without replacement nor
how ties, zero weights or too few nonzero weights are handled.  Readings:

* Without replacement, by successive weighted sampling: the block equals
  what drawing one index at a time with probability proportional to eps
  among those not yet drawn would give.  Realised through exponential clocks
  (Efraimidis & Spirakis, Inf. Proc. Letters 97(5), 2006): with E_j an
  independent Exp(1) variable, the k indices with the smallest keys
  E_j / eps_j are distributed exactly as successive sampling.  P is never
  normalised: the keys need eps only.
* Indices with eps_j = 0 have probability zero and are never drawn.  A
  weight that is zero only up to rounding -- the columns (rows) a projection
  has just annihilated keep residuals of order u * ||A_(j)|| ||z|| -- is
  treated as zero too: only eps_j > floor * max_l eps_l counts as positive
  (floor = 1e-20 for FP64 weights; floor = 0 keeps the exact test
  eps_j > 0).  Without this, a block larger than the number of genuinely
  positive weights would be filled from rounding noise.  When at most k
  weights pass the test, all of them are taken.
* Equal keys are ordered by index; the result is returned in ascending
  index order.
* A NaN, negative or infinite weight is a numeric error.

E_j = -ln(u_j), u_j from the Philox word of index j (see ``philox``).

Test infrastructure only (see the package docstring).
"""
import numpy as np

from .philox import index_words, words_to_unit
from .lnfun import ln_own


class NumericError(ValueError):
    """A weight was NaN, negative or infinite."""


def block_size(eta, d):
    """k = min(d, max(1, floor(eta*d + 0.5))) -- the reading of "select
    n*eta columns / m*eta rows" (Algorithm 1) when eta*d is not an integer."""
    if d <= 0:
        return 0
    k = int(np.floor(eta * d + 0.5))
    return min(d, max(1, k))


def exp_keys(idx, eps_idx, seed, it, phase, sys=0, key1=0):
    """Exponential-clock keys E_j / eps_j for the indices ``idx`` whose
    weights are ``eps_idx`` (all positive)."""
    u = words_to_unit(index_words(idx, seed, it, phase, sys, key1))
    e = -ln_own(u)
    return e / eps_idx


FLOOR_FP64 = 1e-20


def select(eps, k, seed, it, phase, sys=0, key1=0, floor=FLOOR_FP64):
    """Indices (ascending, int64) of the block drawn from weights ``eps``.

    eps: 1-D FP64 weights; k: block size; (seed, it, phase, sys, key1): the
    generator coordinates (phase 0 = column block, 1 = row block); floor:
    relative weight floor (see the module docstring)."""
    eps = np.asarray(eps, dtype=np.float64)
    if eps.ndim != 1:
        raise ValueError("eps must be one-dimensional")
    if not np.all(np.isfinite(eps)) or np.any(eps < 0):
        raise NumericError("selection weights must be finite and >= 0")
    if k < 0:
        raise ValueError("k must be >= 0")
    mx = eps.max() if eps.size else 0.0
    cut = floor * mx if floor > 0 else 0.0
    cand = np.flatnonzero(eps > cut)
    if cand.size <= k:
        return cand.astype(np.int64)
    keys = exp_keys(cand, eps[cand], seed, it, phase, sys, key1)
    order = np.lexsort((cand, keys))        # by key, then by index
    chosen = cand[order[:k]]
    return np.sort(chosen).astype(np.int64)


def select_threshold(eps, eta):
    """GDBEK's greedy set {j : eps_j >= eta * max eps} (Section 2), in
    ascending index order; empty when every weight is zero."""
    eps = np.asarray(eps, dtype=np.float64)
    if not np.all(np.isfinite(eps)) or np.any(eps < 0):
        raise NumericError("selection weights must be finite and >= 0")
    mx = eps.max() if eps.size else 0.0
    if mx <= 0:
        return np.zeros(0, dtype=np.int64)
    return np.flatnonzero(eps >= eta * mx).astype(np.int64)


def select_block_law(eps, s, seed, it, phase, sys=0, key1=0, floor=FLOOR_FP64):
    """A block of size s from the law of Lemma 2.1 (Section 2):
    P(B) proportional to sum_{j in B} w_j^2 over all s-subsets, with the
    weights w_j^2 = eps_j.  Since every index lies in C(d-1, s-1) blocks,
    this law is: one index j* drawn with probability eps_j / sum eps, then
    a uniform (s-1)-subset of the other d-1 indices.

    j* is the one-index draw of ``select`` (k = 1, same generator
    coordinates and weight floor); the subset takes the s-1 smallest keys
    -ln(u'_j) over j != j* (ties by index), u'_j from the Philox stream of
    phase + 2.  Every weight zero (after the floor): the empty block, as
    for the other rules.  Ascending indices."""
    eps = np.asarray(eps, dtype=np.float64)
    d = eps.size
    first = select(eps, 1, seed, it, phase, sys, key1, floor)
    if first.size == 0 or s <= 0:
        return np.zeros(0, dtype=np.int64)
    j0 = int(first[0])
    if s >= d:
        return np.arange(d, dtype=np.int64)
    idx = np.delete(np.arange(d, dtype=np.int64), j0)
    u = words_to_unit(index_words(idx, seed, it, phase + 2, sys, key1))
    keys = -ln_own(u)
    order = np.lexsort((idx, keys))
    chosen = idx[order[:s - 1]]
    return np.sort(np.concatenate([chosen, [j0]])).astype(np.int64)


def iid_shift(d):
    """sh = 63 - ceil(log2 d): integer weights up to 2^sh sum below 2^63."""
    return 63 - (int(d) - 1).bit_length()


def iid_weights(eps, floor=FLOOR_FP64):
    """Integer weights w_j = floor(eps_j / max eps * 2^sh), zero where
    eps_j <= floor * max eps; (w, sh).  The quotient is one correctly
    rounded FP64 division, the scaling by 2^sh is exact."""
    eps = np.asarray(eps, dtype=np.float64)
    d = eps.size
    sh = iid_shift(max(d, 1))
    mx = eps.max() if d else 0.0
    if not mx > 0:
        return np.zeros(d, dtype=np.uint64), sh
    q = np.floor((eps / mx) * (2.0 ** sh))
    q[~(eps > floor * mx)] = 0.0
    return q.astype(np.uint64), sh


def select_iid(eps, k, seed, it, phase, sys=0, key1=0, floor=FLOOR_FP64):
    """k independent draws with replacement from P(j) = eps_j / sum eps
    (Section 2, Algorithm 1), the distinct indices kept, ascending.

    The probabilities are the integer weights of ``iid_weights`` over their
    total W (relative resolution 2^-sh of the largest weight).  Draw t takes
    the Philox word u_t of index t in the stream of phase + 4, r_t =
    floor(u_t W / 2^64), and the index j whose cumulative-weight interval
    [P_(j-1), P_j) holds r_t (exact integer arithmetic, so any summation
    order gives the same P).  Every weight zero: the empty block."""
    eps = np.asarray(eps, dtype=np.float64)
    if not np.all(np.isfinite(eps)) or np.any(eps < 0):
        raise NumericError("selection weights must be finite and >= 0")
    if eps.size == 0 or k <= 0:
        return np.zeros(0, dtype=np.int64)
    w, _ = iid_weights(eps, floor)
    P = np.cumsum(w, dtype=np.uint64)
    W = int(P[-1])
    if W == 0:
        return np.zeros(0, dtype=np.int64)
    u = index_words(np.arange(k, dtype=np.int64), seed, it, phase + 4, sys, key1)
    r = np.array([(int(v) * W) >> 64 for v in u], dtype=np.uint64)
    j = np.searchsorted(P, r, side="right")
    return np.unique(j).astype(np.int64)
