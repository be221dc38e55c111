"""Pins of the oracle's Algorithm 1 against the mathematics: pseudoinverse
limits, the REK and Kaczmarz special cases, per-update invariants, the
Pythagoras identity of the convergence proof, planted solutions, resume,
the paper's iteration counts (loose band), gradients by finite differences,
and the generators' structure."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.rgdbek import rgdbek
from oracle.blockls import column_projection, row_projection
from oracle.refsol import pinv_solution, grad_reference, grad_via_solves
from oracle.select import block_size
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rank_deficient(m, n, r, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, r)) @ rng.standard_normal((r, n))


def test_full_blocks_one_iteration_is_pinv():
    # k_col = n and k_row = m: z_1 = (I - A A^+) b and x_1 = A^+ b.
    rng = np.random.default_rng(0)
    a = rng.standard_normal((14, 9))
    b = rng.standard_normal(14)
    x, z, info = rgdbek(a, b, k_col=9, k_row=14, max_iter=1)
    xs, rs = pinv_solution(a)(b)
    assert np.linalg.norm(x - xs) <= 1e-13 * np.linalg.norm(xs)
    assert np.linalg.norm(z - rs) <= 1e-13 * np.linalg.norm(b)
    assert np.allclose(x, np.linalg.lstsq(a, b, rcond=None)[0], atol=1e-13)


def test_rek_special_case():
    # k_col = k_row = 1 reproduces the REK update formulas (Section 1) for
    # the drawn column j and row i.
    rng = np.random.default_rng(1)
    a = rng.standard_normal((12, 7))
    b = rng.standard_normal(12)
    x, z, info = rgdbek(a, b, k_col=1, k_row=1, max_iter=6, record=True)
    for t in info.trace:
        j = int(t["U"][0])
        i = int(t["J"][0])
        aj = a[:, j]
        zprev = t["z_prev"]
        z_rek = zprev - (aj @ zprev) / (aj @ aj) * aj
        assert np.allclose(t["z"], z_rek, rtol=0, atol=1e-13)
        ai = a[i, :]
        xprev = t["x_prev"]
        x_rek = xprev + (b[i] - z_rek[i] - ai @ xprev) / (ai @ ai) * ai
        assert np.allclose(t["x"], x_rek, rtol=0, atol=1e-12)


def test_kaczmarz_special_case_consistent():
    # b in range(A) and z frozen at r = 0 -> the row update is the Kaczmarz
    # projection onto the hyperplane of row i (Section 1).
    rng = np.random.default_rng(2)
    a = rng.standard_normal((10, 6))
    b = a @ rng.standard_normal(6)
    x0 = rng.standard_normal(6)
    x, z, info = rgdbek(a, b, k_col=1, k_row=1, max_iter=1, record=True,
                        x0=x0, z0=np.zeros(10))
    t = info.trace[0]
    assert np.allclose(t["z"], 0.0)
    i = int(t["J"][0])
    ai = a[i]
    want = x0 + (b[i] - ai @ x0) / (ai @ ai) * ai
    assert np.allclose(x, want, atol=1e-13)


@pytest.mark.parametrize("shape,rank", [((12, 8), 8), ((8, 12), 8),
                                        ((10, 10), 6)])
def test_limits_are_pinv(shape, rank):
    # x_inf = A^+ b (min norm, x stays in range(A^T)) and z_inf = (I-AA^+) b.
    m, n = shape
    a = rank_deficient(m, n, rank, seed=4)
    b = np.random.default_rng(5).standard_normal(m)
    x, z, info = rgdbek(a, b, k_col=max(1, n // 2), k_row=max(1, m // 2),
                        max_iter=20000, stop="res_ext", tol=1e-13)
    xs, rs = pinv_solution(a)(b)
    assert info.converged
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)
    assert np.linalg.norm(z - rs) <= 1e-9 * np.linalg.norm(b)


def test_invariants_and_pythagoras():
    # After the column update A_U^T z_{k+1} = 0; after the row update the
    # selected equations hold exactly (full row rank blocks) and the
    # correction lies in range((A^J)^T); ||z_k - r||^2 drops by exactly
    # ||P_U (z_k - r)||^2 (Theorem 2.3, proof).
    p = workloads.dense_least_squares(120, 40, seed=3)
    a, b = p.a, p.b
    r = p.r_perp
    x, z, info = rgdbek(a, b, k_col=10, k_row=15, max_iter=25, record=True)
    prev = np.linalg.norm(b - r)
    for t in info.trace:
        au = a[:, t["U"]]
        zn = t["z"]
        scale = np.linalg.norm(au) * np.linalg.norm(t["z_prev"])
        assert np.linalg.norm(au.T @ zn) <= 1e-13 * scale
        aj = a[t["J"], :]
        lhs = aj @ t["x"]
        rhs = b[t["J"]] - zn[t["J"]]
        assert np.linalg.norm(lhs - rhs) <= 1e-12 * (
            np.linalg.norm(aj) * np.linalg.norm(t["x"]) + np.linalg.norm(rhs))
        d = t["x"] - t["x_prev"]
        coef = np.linalg.lstsq(aj.T, d, rcond=None)[0]
        assert np.linalg.norm(aj.T @ coef - d) <= 1e-12 * np.linalg.norm(d)
        e_prev = t["z_prev"] - r
        pu = au @ np.linalg.lstsq(au, e_prev, rcond=None)[0]
        e_next = zn - r
        assert abs(e_next @ e_next - (e_prev @ e_prev - pu @ pu)) <= 1e-10 * (e_prev @ e_prev)
        cur = np.linalg.norm(e_next)
        assert cur <= prev * (1 + 1e-12)
        prev = cur


def test_planted_consistent_dense():
    p = workloads.dense_consistent(500, 250, seed=0)
    x, z, info = rgdbek(p.a, p.b, eta=0.5, max_iter=300, stop="err_ref",
                        tol=1e-10, x_ref=p.x_star)
    assert info.converged and info.metric <= 1e-10
    assert np.linalg.norm(z) <= 1e-8 * np.linalg.norm(p.b)


def test_planted_least_squares_dense():
    p = workloads.dense_least_squares(400, 100, seed=1)
    x, z, info = rgdbek(p.a, p.b, k_col=30, k_row=40, max_iter=2000,
                        stop="err_ref", tol=1e-10, x_ref=p.x_star)
    assert info.converged
    assert np.linalg.norm(z - p.r_perp) <= 1e-8 * np.linalg.norm(p.r_perp)


def test_sparse_path_matches_dense_path():
    p = workloads.sparse_uniform(300, 120, density=0.05, seed=2)
    xd, zd, _ = rgdbek(p.a.toarray(), p.b, k_col=20, k_row=40, max_iter=15)
    xs, zs, _ = rgdbek(p.a, p.b, k_col=20, k_row=40, max_iter=15)
    assert np.linalg.norm(xd - xs) <= 1e-11 * np.linalg.norm(xd)
    assert np.linalg.norm(zd - zs) <= 1e-11 * np.linalg.norm(zd)


def test_resume_is_bitwise():
    p = workloads.dense_least_squares(150, 60, seed=4)
    x2, z2, _ = rgdbek(p.a, p.b, k_col=12, k_row=20, max_iter=10, seed=3)
    x1, z1, _ = rgdbek(p.a, p.b, k_col=12, k_row=20, max_iter=5, seed=3)
    xr, zr, _ = rgdbek(p.a, p.b, k_col=12, k_row=20, max_iter=5, seed=3,
                       x0=x1, z0=z1, it0=5)
    assert np.array_equal(xr, x2) and np.array_equal(zr, z2)


def test_stop_rules_return_the_tested_iterate():
    p = workloads.dense_consistent(60, 30, seed=6)
    x, z, info = rgdbek(p.a, p.b, k_col=10, k_row=20, max_iter=500,
                        stop="rse", tol=1e-12)
    assert info.converged
    assert np.linalg.norm(p.a @ x - p.b) ** 2 <= 1e-12 * np.linalg.norm(p.b) ** 2
    x3, _, i3 = rgdbek(p.a, p.b, k_col=10, k_row=20, max_iter=info.iterations)
    assert np.array_equal(x3, x)
    x4, _, i4 = rgdbek(p.a, p.b, k_col=10, k_row=20, max_iter=3,
                       stop="err_ref", tol=1e-30, x_ref=p.x_star)
    assert not i4.converged and i4.iterations == 3


def test_zero_rows_and_columns():
    rng = np.random.default_rng(8)
    a = rng.standard_normal((20, 10))
    a[4, :] = 0.0
    a[:, 7] = 0.0
    b = rng.standard_normal(20)
    x, z, info = rgdbek(a, b, k_col=3, k_row=5, max_iter=3000,
                        stop="res_ext", tol=1e-12, record=False)
    xs, rs = pinv_solution(a)(b)
    assert x[7] == 0.0
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)
    assert abs(z[4] - b[4]) <= 1e-12


def test_paper_iteration_band_tall():
    # Table 2: 8000 x 500, sprandn 99% sparse, eta = 0.5, squared relative
    # residual <= 1e-6: 11.8 iterations on average.  Different generator and
    # exact block solves -> only a loose band (+-50%) is meaningful.
    with open(os.path.join(GOLDEN, "paper_iteration_counts.json")) as f:
        ref = json.load(f)["tall_8000_rows"]["500"]
    its = []
    for seed in range(2):
        p = workloads.sparse_uniform(8000, 500, density=0.01, seed=seed)
        x, z, info = rgdbek(p.a, p.b, eta=0.5, max_iter=200, stop="rse",
                            tol=1e-6, seed=seed)
        assert info.converged
        its.append(info.iterations)
    assert 0.5 * ref <= np.mean(its) <= 1.5 * ref


def test_gradient_reference_matches_finite_differences():
    rng = np.random.default_rng(10)
    m, n = 9, 5
    a = rng.standard_normal((m, n))
    b = rng.standard_normal(m)
    c = rng.standard_normal(n)          # L = c . x(A, b)
    da, db = grad_reference(a, b, c)
    h = 1e-6

    def loss(aa, bb):
        return c @ np.linalg.lstsq(aa, bb, rcond=None)[0]
    fd_b = np.array([(loss(a, b + h * e) - loss(a, b - h * e)) / (2 * h)
                     for e in np.eye(m)])
    assert np.allclose(db, fd_b, rtol=1e-6, atol=1e-8)
    fd_a = np.zeros_like(a)
    for i in range(m):
        for j in range(n):
            e = np.zeros_like(a)
            e[i, j] = h
            fd_a[i, j] = (loss(a + e, b) - loss(a - e, b)) / (2 * h)
    assert np.allclose(da, fd_a, rtol=1e-6, atol=1e-8)


def test_gradient_via_rgdbek_solves_matches_reference():
    p = workloads.dense_least_squares(40, 12, seed=11)
    c = np.random.default_rng(12).standard_normal(12)
    x = np.linalg.lstsq(p.a, p.b, rcond=None)[0]
    da, w, lam = grad_via_solves(p.a, p.b, c, x, k_col=4, k_row=8,
                                 max_iter=5000, tol=1e-14)
    da_ref, w_ref = grad_reference(p.a, p.b, c)
    assert np.linalg.norm(w - w_ref) <= 1e-9 * np.linalg.norm(w_ref)
    assert np.linalg.norm(da - da_ref) <= 1e-9 * np.linalg.norm(da_ref)


def test_generator_least_squares_structure():
    p = workloads.dense_least_squares(600, 150, seed=0)
    a, r = p.a, p.r_perp
    assert np.linalg.norm(a.T @ r) <= 1e-14 * np.linalg.norm(a, 2) * np.linalg.norm(r)
    assert abs(np.linalg.norm(r) / np.linalg.norm(a @ p.x_star) - 0.1) <= 1e-12
    assert np.allclose(np.linalg.lstsq(a, p.b, rcond=None)[0], p.x_star, atol=1e-10)


def test_generator_powerlaw_structure():
    p = workloads.sparse_powerlaw(20000, 8000, mean_len=10, max_len=400, seed=0)
    a = p.a
    lens = np.diff(a.indptr)
    assert lens[0] == 400 and lens.max() == 400 and lens.min() >= 1
    assert 8.5 <= lens.mean() <= 11.5
    norms = np.sqrt(np.asarray(a.multiply(a).sum(axis=1)).ravel())
    assert np.allclose(norms, 1.0, atol=1e-14)
    for i in [0, 5, 19999]:
        cols = a.indices[a.indptr[i]:a.indptr[i + 1]]
        assert np.all(np.diff(cols) > 0)
    assert np.allclose(a @ p.x_star, p.b)


def test_generator_blur_structure():
    a = workloads.blur_operator(npix=40, dtype=np.float64)
    # nnz of T kron T with T banded (half-width 7) of order 40
    t_nnz = 40 * 15 - 2 * sum(range(1, 8))
    assert a.nnz == t_nnz ** 2
    assert abs(a - a.T).max() == 0.0
    from workloads.generators import gaussian_psf_1d
    w = gaussian_psf_1d()
    assert abs(w.sum() - 0.9998) < 2e-4
    full = workloads.blur_operator.__defaults__[0]
    assert full == 512


def test_generator_laplacian_batch_structure():
    ps = workloads.laplacian_batch(count=6, n_min=100, n_max=2000, seed=0)
    for p in ps:
        m, n = p.a.shape
        nx, ny = p.meta["nx"], p.meta["ny"]
        assert n == nx * ny and m == n + int(round(0.2 * n))
        assert 100 * 0.8 <= n <= 2000 * 1.2
        assert np.allclose(p.a @ p.x_star, p.b)
        lap = p.a[:n].toarray()
        assert np.allclose(np.diag(lap), 4 + p.meta["shift"])
        ext = p.a[n:]
        assert np.all(np.diff(ext.indptr) == 8)


def test_block_size_reading_matches_configs():
    assert block_size(0.5, 250) == 125 and block_size(0.5, 500) == 250
    assert block_size(0.1, 500_000) == 50_000
    assert block_size(0.1, 1_000_000) == 100_000


# ------------------------------------------------------------ GDBEK (greedy)
def test_greedy_eta_one_is_greedy_rek():
    # threshold 1 keeps only the largest weight: with distinct weights one
    # iteration is the REK step (Section 1) on the column of largest
    # |A_(j)^T z|^2/||A_(j)||^2 and then the row of largest residual weight
    # -- computed here from scratch, by argmax.
    rng = np.random.default_rng(11)
    a = rng.standard_normal((12, 7))
    b = rng.standard_normal(12)
    x, z, info = rgdbek(a, b, greedy=1.0, max_iter=1, record=True)
    t = info.trace[0]
    cn = (a * a).sum(axis=0)
    j = int(np.argmax((a.T @ b) ** 2 / cn))
    assert list(t["U"]) == [j]
    aj = a[:, j]
    z_rek = b - (aj @ b) / (aj @ aj) * aj
    assert np.allclose(z, z_rek, atol=1e-13)
    rn = (a * a).sum(axis=1)
    i = int(np.argmax((b - z_rek) ** 2 / rn))
    assert list(t["J"]) == [i]
    ai = a[i]
    assert np.allclose(x, (b[i] - z_rek[i]) / (ai @ ai) * ai, atol=1e-13)


def test_greedy_tiny_threshold_takes_every_positive_weight():
    # a threshold below every positive weight ratio selects all columns and
    # rows: one iteration gives A^+ b and (I - A A^+) b (full-rank A)
    rng = np.random.default_rng(12)
    a = rng.standard_normal((14, 9))
    b = rng.standard_normal(14)
    x, z, info = rgdbek(a, b, greedy=1e-300, max_iter=1, record=True)
    assert info.trace[0]["U"].size == 9 and info.trace[0]["J"].size == 14
    xs, rs = pinv_solution(a)(b)
    assert np.linalg.norm(x - xs) <= 1e-13 * np.linalg.norm(xs)
    assert np.linalg.norm(z - rs) <= 1e-13 * np.linalg.norm(b)


def test_greedy_converges_to_planted_solutions():
    # GDBEK with the paper's sequential threshold converges on a consistent
    # system and on a least-squares one (b with a null(A^T) part)
    p = workloads.dense_consistent(60, 30, seed=13)
    x, z, info = rgdbek(p.a, p.b, greedy=0.5, max_iter=3000, stop="err_ref",
                        tol=1e-10, x_ref=p.x_star)
    assert info.converged
    q = workloads.dense_least_squares(80, 20, seed=14)
    x, z, info = rgdbek(q.a, q.b, greedy=0.5, max_iter=3000, stop="err_ref",
                        tol=1e-10, x_ref=q.x_star)
    assert info.converged


def test_greedy_all_zero_weights_skip():
    # zero residuals: empty greedy sets (R7), x and z stay put
    a = np.eye(4)
    x, z, info = rgdbek(a, np.zeros(4), greedy=0.5, max_iter=2, record=True)
    assert all(t["U"].size == 0 and t["J"].size == 0 for t in info.trace)
    assert np.all(x == 0) and np.all(z == 0)


def test_table2_gdbek_iterations_loose():
    # GDBEK (threshold 0.5) on 8000x500 sprandn-like matrices: the paper's
    # Table 2 reports 35.1 iterations on average to RSE <= 1e-6; our
    # synthetic stand-in must land within 15% of it, and above RGDBEK's
    # count on the same matrices (the table's ordering)
    with open(os.path.join(GOLDEN, "paper_iteration_counts.json")) as f:
        gold = json.load(f)
    ref = gold["gdbek_tall_8000_rows"]["500"]
    its_g, its_r = [], []
    for seed in range(2):
        p = workloads.sparse_uniform(8000, 500, density=0.01, seed=seed)
        x, z, info = rgdbek(p.a, p.b, greedy=0.5, max_iter=400, stop="rse",
                            tol=1e-6)
        assert info.converged
        its_g.append(info.iterations)
        x, z, info = rgdbek(p.a, p.b, eta=0.5, max_iter=200, stop="rse",
                            tol=1e-6, seed=seed)
        its_r.append(info.iterations)
    assert abs(np.mean(its_g) - ref) <= 0.15 * ref, its_g
    assert np.mean(its_g) > np.mean(its_r)
