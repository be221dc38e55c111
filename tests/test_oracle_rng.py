"""Pins of the oracle's generator, logarithm and block selection against
things other than itself: numpy's independent Philox implementation, the
library logarithm, brute-force probabilities of successive sampling, and the
Efraimidis-Spirakis equivalence."""
import itertools
import math

import numpy as np
import pytest

from oracle import philox, lnfun
from oracle.select import select, block_size, NumericError, select_threshold


def numpy_philox_block(ctr, key):
    """Block for counter ctr via numpy.random.Philox, which increments its
    256-bit counter before producing a block."""
    c = sum(int(v) << (64 * i) for i, v in enumerate(ctr))
    bg = np.random.Philox(key=int(key[0]) | (int(key[1]) << 64),
                          counter=(c - 1) % (1 << 256))
    return tuple(int(v) for v in bg.random_raw(4))


def test_philox_zero_known_answer():
    # Known-answer vector of Philox4x64-10 for zero counter and key.
    want = (0x16554d9eca36314c, 0xdb20fe9d672d0fdc, 0xd7e772cee186176b,
            0x7e68b68aec7ba23b)
    assert philox.philox4x64_10_int((0, 0, 0, 0), (0, 0)) == want
    assert numpy_philox_block((0, 0, 0, 0), (0, 0)) == want


def test_philox_matches_numpy_random_blocks():
    rng = np.random.default_rng(7)
    M = (1 << 64) - 1
    cases = [((M, M, M, M), (M, M)), ((1, 0, 0, 0), (0, 0)),
             ((0, 0, 0, 1), (1, 0))]
    for _ in range(300):
        ctr = tuple(int(v) * 2 + 1 for v in rng.integers(0, 1 << 63, 4, dtype=np.int64))
        key = tuple(int(v) * 2 for v in rng.integers(0, 1 << 63, 2, dtype=np.int64))
        cases.append((ctr, key))
    for ctr, key in cases:
        want = numpy_philox_block(ctr, key)
        assert philox.philox4x64_10_int(ctr, key) == want
        vec = philox.philox4x64_10(*[np.array([c], np.uint64) for c in ctr],
                                   key[0], key[1])
        assert tuple(int(v[0]) for v in vec) == want


def test_index_words_layout():
    # word j&3 of block (j>>2, it, phase, sys) under key (seed, key1)
    idx = np.arange(37)
    w = philox.index_words(idx, seed=123, it=5, phase=1, sys=9, key1=1)
    for j in idx:
        blk = numpy_philox_block((j >> 2, 5, 1, 9), (123, 1))
        assert int(w[j]) == blk[j & 3]


def test_words_to_unit_exact_open_interval():
    w = np.array([0, (1 << 64) - 1, 1 << 12, (1 << 63)], dtype=np.uint64)
    u = philox.words_to_unit(w)
    assert u[0] == 2.0 ** -53
    assert u[1] == 1.0 - 2.0 ** -53
    assert u[2] == 3 * 2.0 ** -53
    assert u[3] == 0.5 + 2.0 ** -53
    assert np.all((u > 0) & (u < 1))


def test_ln_own_within_4_ulp():
    rng = np.random.default_rng(0)
    u = np.concatenate([
        rng.random(1_000_000),
        np.exp(-rng.random(200_000) * 700.0),
        [2.0 ** -53, 1 - 2.0 ** -53, 0.5, lnfun.SQRT_HALF,
         np.nextafter(lnfun.SQRT_HALF, 0), np.nextafter(lnfun.SQRT_HALF, 1),
         5e-324, 1e-300, 1.0, 0.75, 2.0 ** -1022]])
    u = u[u > 0]
    got = lnfun.ln_own(u)
    ref = np.log(u)
    ulp = np.spacing(np.abs(ref))
    ulp[ref == 0] = np.spacing(0.0)
    assert np.max(np.abs(got - ref) / ulp) <= 4.0
    assert lnfun.ln_own(np.array([1.0]))[0] == 0.0
    for v in [2.0 ** -53, 0.3, 0.999]:
        assert abs(lnfun.ln_own(np.array([v]))[0] - math.log(v)) <= 4 * np.spacing(abs(math.log(v)))


def test_block_size_rounding():
    assert block_size(0.5, 250) == 125
    assert block_size(0.5, 5) == 3          # 2.5 rounds half up
    assert block_size(0.1, 25) == 3         # 2.5 -> 3
    assert block_size(0.001, 10) == 1       # never below one
    assert block_size(1.0, 10) == 10
    assert block_size(0.5, 0) == 0


def test_select_basic_properties():
    rng = np.random.default_rng(3)
    eps = rng.random(1000) ** 3
    eps[rng.random(1000) < 0.2] = 0.0
    for k in [1, 7, 100, 500]:
        s = select(eps, k, seed=1, it=4, phase=0)
        assert s.size == k
        assert np.all(np.diff(s) > 0)
        assert np.all(eps[s] > 0)
    # at most k positive weights: all of them
    e2 = np.zeros(50)
    e2[[3, 17, 40]] = [1.0, 2.0, 0.5]
    assert list(select(e2, 5, 0, 0, 1)) == [3, 17, 40]
    assert list(select(e2, 3, 0, 0, 1)) == [3, 17, 40]
    assert select(np.zeros(10), 4, 0, 0, 0).size == 0
    with pytest.raises(NumericError):
        select(np.array([1.0, np.nan]), 1, 0, 0, 0)
    with pytest.raises(NumericError):
        select(np.array([1.0, -1.0]), 1, 0, 0, 0)
    with pytest.raises(NumericError):
        select(np.array([1.0, np.inf]), 1, 0, 0, 0)


def test_select_equal_weights_takes_largest_uniforms():
    # With equal weights the keys order like E_j = -ln u_j, so the block is
    # the k indices with the largest u_j; u_j recomputed via numpy's Philox.
    d, k = 64, 9
    eps = np.full(d, 2.5)
    s = select(eps, k, seed=11, it=2, phase=1, sys=3)
    w = np.array([numpy_philox_block((j >> 2, 2, 1, 3), (11, 0))[j & 3]
                  for j in range(d)], dtype=np.uint64)
    u = ((w >> np.uint64(12)).astype(np.float64) * 2 + 1) * 2.0 ** -53
    want = np.sort(np.argsort(-u, kind="stable")[:k])
    assert list(s) == list(want)


def test_select_k1_is_categorical():
    # k = 1: P(j) = eps_j / sum eps (chi-square over 15000 draws).
    eps = np.array([0.05, 0.1, 0.15, 0.2, 0.5, 0.0, 1.0])
    p = eps / eps.sum()
    n = 15000
    counts = np.zeros(eps.size)
    for it in range(n):
        counts[select(eps, 1, seed=5, it=it, phase=0)[0]] += 1
    nz = p > 0
    assert counts[~nz].sum() == 0
    chi2 = np.sum((counts[nz] - n * p[nz]) ** 2 / (n * p[nz]))
    assert chi2 < 22.5      # 99.9% quantile of chi^2 with 5 dof is 20.5


def successive_inclusion(eps, k):
    """Brute-force inclusion probabilities of successive weighted sampling
    without replacement: enumerate every ordered draw sequence."""
    d = eps.size
    incl = np.zeros(d)
    for seq in itertools.permutations(range(d), k):
        pr = 1.0
        rest = eps.sum()
        for j in seq:
            pr *= eps[j] / rest
            rest -= eps[j]
        for j in seq:
            incl[j] += pr
    return incl


@pytest.mark.parametrize("k", [2, 3])
def test_select_matches_successive_sampling_law(k):
    eps = np.array([0.1, 0.4, 0.2, 1.3, 0.05, 0.7])
    want = successive_inclusion(eps, k)
    n = 12000
    counts = np.zeros(eps.size)
    for it in range(n):
        counts[select(eps, k, seed=9, it=it, phase=1, sys=2)] += 1
    freq = counts / n
    sd = np.sqrt(want * (1 - want) / n)
    assert np.all(np.abs(freq - want) <= 5 * sd + 1e-12)
    assert abs(counts.sum() - n * k) == 0


def test_select_streams_differ_by_coordinates():
    eps = np.random.default_rng(1).random(400)
    base = select(eps, 40, seed=0, it=0, phase=0)
    for kw in [dict(seed=1, it=0, phase=0), dict(seed=0, it=1, phase=0),
               dict(seed=0, it=0, phase=1), dict(seed=0, it=0, phase=0, sys=1),
               dict(seed=0, it=0, phase=0, key1=1)]:
        assert not np.array_equal(select(eps, 40, **kw), base)
    assert np.array_equal(select(eps, 40, seed=0, it=0, phase=0), base)


def test_threshold_set():
    eps = np.array([0.1, 0.9, 0.45, 0.0, 1.0])
    assert list(select_threshold(eps, 0.5)) == [1, 4]
    assert list(select_threshold(eps, 0.45)) == [1, 2, 4]
    assert select_threshold(np.zeros(3), 0.5).size == 0


def test_select_weight_floor():
    # weights at rounding level relative to the largest are not drawn
    eps = np.array([1.0, 0.5, 1e-25, 3e-30, 0.25, 0.0])
    assert list(select(eps, 5, 0, 0, 0)) == [0, 1, 4]
    assert list(select(eps, 5, 0, 0, 0, floor=0.0)) == [0, 1, 2, 3, 4]
    assert list(select(eps, 5, 0, 0, 0, floor=1e-26)) == [0, 1, 2, 4]
    # the floor is relative: scaling all weights changes nothing
    e = np.random.default_rng(4).random(300) ** 8
    assert np.array_equal(select(e, 40, 1, 2, 1), select(e * 1e-200, 40, 1, 2, 1))
