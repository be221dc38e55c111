"""The allocation-free block draw (rgdbek_select_noalloc) against the
allocating one (rgdbek_select) on the same weights: identical index sets,
bit for bit, on two calls in a row (the second on a smaller input, so stale
contents of the shared static work space would show), across the one-
workgroup, persistent and large-d forms of the draw, and the size limit."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rg():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2509_19267_amd as rg
    rg.load()
    return rg


def _weights(d, seed, zero_frac=0.0):
    rng = np.random.default_rng(seed)
    e = rng.random(d) ** 3
    if zero_frac:
        e[rng.random(d) < zero_frac] = 0.0
    return torch.as_tensor(e).cuda()


# (d, k) pairs: first a larger draw, then a smaller one
PAIRS = [
    ((1_048_576, 100_000), (600_000, 50_000)),   # persistent, then persistent
    ((300_000, 30_000), (5_000, 700)),           # persistent, then one workgroup
    ((60_000, 60_000), (20_000, 1)),             # k = d, then k = 1
    ((8_192, 4_000), (8_193, 8_000)),            # both sides of the LDS bound
]


@pytest.mark.parametrize("pair", PAIRS, ids=lambda p: f"{p[0][0]}-{p[1][0]}")
def test_noalloc_matches_select_twice(rg, pair):
    for call, (d, k) in enumerate(pair):
        eps = _weights(d, 10 * call + d % 97, zero_frac=0.3 if call else 0.0)
        for floor in (1e-20, 0.0):
            want = rg.select(eps, k, seed=5, it=3 + call, phase=call, sys=1,
                             floor=floor)
            got = rg.select_noalloc(eps, k, seed=5, it=3 + call, phase=call,
                                    sys=1, floor=floor)
            torch.cuda.synchronize()
            assert got.numel() == want.numel(), (d, k, floor)
            assert torch.equal(got, want), (d, k, floor)


def test_noalloc_reuses_caller_output(rg):
    eps = _weights(50_000, 7)
    out = torch.full((2_000,), -1, dtype=torch.int32, device="cuda")
    got = rg.select_noalloc(eps, 2_000, seed=1, it=2, out=out)
    want = rg.select(eps, 2_000, seed=1, it=2)
    assert got.data_ptr() == out.data_ptr()
    assert torch.equal(got, want)


def test_noalloc_size_limit_and_errors(rg):
    from paper_2509_19267_amd import RgdbekError
    big = torch.ones(1_048_577, dtype=torch.float64, device="cuda")
    with pytest.raises(RgdbekError, match="static work space"):
        rg.select_noalloc(big, 10)
    bad = torch.ones(1000, dtype=torch.float64, device="cuda")
    bad[17] = float("nan")
    with pytest.raises(RgdbekError):
        rg.select_noalloc(bad, 10)
    # the call after an error still matches the allocating draw
    eps = _weights(123_457, 3)
    assert torch.equal(rg.select_noalloc(eps, 999, seed=2),
                       rg.select(eps, 999, seed=2))
