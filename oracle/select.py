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
