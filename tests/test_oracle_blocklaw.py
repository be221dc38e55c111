"""The block law of Lemma 2.1 (Section 2) and a Monte-Carlo check of the
lemma's inequality.  CPU only.

Law: P(B) = sum_{j in B} w_j^2 / (C(d-1, s-1) T), T = sum_j w_j^2, over the
s-subsets B of {0..d-1}; the sampler (oracle/select.py select_block_law)
draws j* with probability w_j^2 / T and a uniform (s-1)-subset of the rest.

Inequality: the lemma states E ||P_B v||^2 >= mu^{-1} ||U v||^2 / ||U||_2^2
with mu = max_B ||U_B^T U_B||_2 / ||U_B||_2^2 -- which is 1 for every
matrix (||X^T X||_2 = ||X||_2^2).  Counting the blocks that hold a pair
j != k gives C(d-2, s-2), not C(d-1, s-1), so the proof's double count is
off; the exact identity is
    E ||U_B v||^2 = ((s-1)/(d-1)) ||U v||^2
                    + (1 - (s-1)/(d-1)) sum_j w_j^4 ||u_j||^2 / T,
and E ||P_B v||^2 >= E ||U_B v||^2 / ||U||_2^2 (||U_B v|| <= ||U_B|| ||P_B v||
and ||U_B|| <= ||U||).  The stated bound fails for orthonormal U with s < d
(the check below shows a counterexample); the corrected one holds.
"""
import itertools
import math

import numpy as np
import pytest

from oracle.select import select_block_law


def exact_law(w2, s):
    d = len(w2)
    T = w2.sum()
    c = math.comb(d - 1, s - 1)
    return {B: w2[list(B)].sum() / (c * T)
            for B in itertools.combinations(range(d), s)}


@pytest.mark.parametrize("s", [2, 3])
def test_block_law_frequencies(s):
    # chi-square of 12000 draws (generator iteration counter 0..11999)
    # against the exact law on d = 5
    w2 = np.array([0.1, 0.5, 1.0, 2.0, 0.4])
    law = exact_law(w2, s)
    counts = dict.fromkeys(law, 0)
    n = 12000
    for it in range(n):
        B = tuple(int(j) for j in select_block_law(w2, s, 7, it, 0))
        counts[B] += 1
    chi2 = sum((counts[B] - n * p) ** 2 / (n * p) for B, p in law.items())
    dof = len(law) - 1
    # 1e-4 upper tail of chi-square(dof) is below dof + 6 sqrt(2 dof) + 10
    assert chi2 < dof + 6 * math.sqrt(2 * dof) + 10, (chi2, counts)


def test_block_law_inclusion_probability():
    # P(j in B) = w_j^2/T + (1 - w_j^2/T)(s-1)/(d-1)
    rng = np.random.default_rng(3)
    d, s, n = 40, 6, 6000
    w2 = rng.random(d) ** 3
    inc = np.zeros(d)
    for it in range(n):
        B = select_block_law(w2, s, 11, it, 1)
        assert B.size == s and np.all(np.diff(B) > 0)
        inc[B] += 1
    p = w2 / w2.sum()
    want = p + (1 - p) * (s - 1) / (d - 1)
    sd = np.sqrt(want * (1 - want) / n)
    assert np.all(np.abs(inc / n - want) <= 5 * sd + 1e-3)


def test_block_law_edge_cases():
    assert select_block_law(np.zeros(7), 3, 0, 0, 0).size == 0
    assert list(select_block_law(np.ones(4), 9, 0, 0, 0)) == [0, 1, 2, 3]
    # one positive weight: that index is always in the block
    w2 = np.zeros(10)
    w2[6] = 1.0
    for it in range(50):
        assert 6 in select_block_law(w2, 3, 1, it, 0)


def moments(U, v, s):
    """Exact E ||U_B v||^2 and E ||P_B v||^2 under the law (enumeration)."""
    d = U.shape[0]
    w2 = (U @ v) ** 2 / (U * U).sum(axis=1)
    e_ub, e_pb = 0.0, 0.0
    for B, p in exact_law(w2, s).items():
        UB = U[list(B)]
        e_ub += p * np.sum((UB @ v) ** 2)
        q, _ = np.linalg.qr(UB.T)
        rk = np.linalg.matrix_rank(UB)
        e_pb += p * np.sum((q[:, :rk].T @ v) ** 2)
    return w2, e_ub, e_pb


@pytest.mark.parametrize("d,p,s,seed", [(6, 4, 2, 0), (6, 4, 4, 1), (7, 3, 3, 2),
                                        (6, 6, 5, 3)])
def test_expectation_identity_and_corrected_bound(d, p, s, seed):
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((d, p))
    v = rng.standard_normal(p)
    w2, e_ub, e_pb = moments(U, v, s)
    T = w2.sum()
    rn2 = (U * U).sum(axis=1)
    f = (s - 1) / (d - 1)
    ident = f * np.sum((U @ v) ** 2) + (1 - f) * np.sum(w2 ** 2 * rn2) / T
    assert abs(e_ub - ident) <= 1e-12 * ident
    assert e_pb >= ident / np.linalg.norm(U, 2) ** 2 * (1 - 1e-12)


def test_stated_bound_fails_for_orthonormal_rows():
    # U = I_4, v = (1,1,1,1)/2, s = 2: every block has probability 1/6 and
    # ||P_B v||^2 = 1/2, while ||U v||^2 / ||U||^2 = 1 (mu = 1)
    U = np.eye(4)
    v = np.full(4, 0.5)
    w2, e_ub, e_pb = moments(U, v, 2)
    assert abs(e_pb - 0.5) < 1e-14
    stated = np.sum((U @ v) ** 2) / np.linalg.norm(U, 2) ** 2
    assert e_pb < stated
    T = w2.sum()
    corrected = (1 / 3) * 1.0 + (2 / 3) * np.sum(w2 ** 2) / T
    assert abs(e_pb - corrected) < 1e-14


def test_monte_carlo_identity_with_the_sampler():
    # the sampler's empirical mean of ||U_B v||^2 matches the identity
    rng = np.random.default_rng(9)
    d, p, s, n = 30, 10, 6, 5000
    U = rng.standard_normal((d, p))
    v = rng.standard_normal(p)
    w2 = (U @ v) ** 2 / (U * U).sum(axis=1)
    vals = np.empty(n)
    for it in range(n):
        B = select_block_law(w2, s, 5, it, 0)
        vals[it] = np.sum((U[B] @ v) ** 2)
    f = (s - 1) / (d - 1)
    ident = f * np.sum((U @ v) ** 2) + (1 - f) * np.sum(w2 ** 2 * (U * U).sum(axis=1)) / w2.sum()
    assert abs(vals.mean() - ident) <= 5 * vals.std() / np.sqrt(n)
