"""Natural logarithm for the exponential selection keys -- oracle side.

Why a hand-rolled logarithm: block selection must agree bit for bit between
the CPU and the GPU on identical residual inputs, and library ``log``
implementations differ in their last bits.  The function below uses only
correctly rounded IEEE-754 operations (+, -, *, /, frexp, comparisons) in a
fixed order with no fused multiply-add, so any implementation that follows
the same recipe gets the same bits.  Accuracy needed is "a few ulp": the
value only shapes the sampling distribution.

Recipe (the classical atanh series, Abramowitz & Stegun 4.1.27):
  u = f * 2**e with f in [sqrt(1/2), sqrt(2));
  s = (f - 1) / (f + 1), t = s*s;
  ln f = 2s + 2s * t * P(t),  P(t) = sum_{i=1..11} t**(i-1) / (2i + 1)
  (Horner from the top coefficient down);
  ln u = e * LN2 + ln f, LN2 the double nearest ln 2.

Test infrastructure only (see the package docstring).
"""
import numpy as np

SQRT_HALF = 0.7071067811865476
LN2 = 0.6931471805599453
NCOEF = 11
# c_i = 1/(2i+1), i = 1..11, each the correctly rounded double quotient.
COEF = [1.0 / (2 * i + 1) for i in range(1, NCOEF + 1)]


def ln_own(u):
    """ln(u) for positive finite doubles (vectorised, FP64, fixed order)."""
    u = np.asarray(u, dtype=np.float64)
    f, e = np.frexp(u)
    small = f < SQRT_HALF
    f = np.where(small, f * 2.0, f)
    e = np.where(small, e - 1, e).astype(np.float64)
    s = (f - 1.0) / (f + 1.0)
    t = s * s
    p = np.full_like(t, COEF[NCOEF - 1])
    for i in range(NCOEF - 2, -1, -1):
        p = p * t
        p = p + COEF[i]
    s2 = s + s
    lnf = s2 + s2 * (t * p)
    return e * LN2 + lnf
