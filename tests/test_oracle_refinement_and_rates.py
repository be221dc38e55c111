"""Pins of three oracle parts that the other CPU tests do not reach:

* the correction system of the extended-residual refinement (the
  ``col_offset`` argument of ``oracle.rgdbek.rgdbek``), against the
  pseudoinverse solution it must reach;
* the LSQR branch of ``oracle.blockls.pinv_apply`` (sparse blocks with a
  dimension above the dense limit), against dense LAPACK least squares on
  the same block;
* the residual decay of Theorem 2.3 (Section 2), statistically, over many
  generator seeds on a tiny system.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.blockls import DENSE_LIMIT, pinv_apply
from oracle.refsol import pinv_solution
from oracle.rgdbek import rgdbek


def ls_system(m, n, seed, resid=0.3):
    """Dense A with b = A x* + r, r in null(A^T) scaled to resid*||A x*||."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((m, n))
    xs = rng.standard_normal(n)
    g = rng.standard_normal(m)
    q, _ = np.linalg.qr(a)
    r = g - q @ (q.T @ g)
    r *= resid * np.linalg.norm(a @ xs) / np.linalg.norm(r)
    return a, a @ xs + r, xs, r


# ------------------------------------------------------------ correction system
@pytest.mark.parametrize("sparse", [False, True])
def test_correction_system_reaches_pinv(sparse):
    # From any x, the refinement pass runs Algorithm 1 on the correction
    # (dx, dz) with right-hand side 0, z_0 = 0 and column residual
    # A^T dz + t, t = A^T (b - A x).  Its fixed point is x + dx = A^+ b and
    # (b - A x) + dz = (I - A A^+) b (Theorem 2.3's limits).
    a, b, xs, r = ls_system(40, 15, seed=3)
    xs_p, r_p = pinv_solution(a)(b)
    assert np.linalg.norm(xs_p - xs) <= 1e-12 * np.linalg.norm(xs)
    x = np.random.default_rng(4).standard_normal(15)
    s = b - a @ x
    t = a.T @ s
    mat = sp.csr_matrix(a) if sparse else a
    dx, dz, info = rgdbek(mat, np.zeros(40), k_col=6, k_row=14, max_iter=300,
                          col_offset=t, seed=1)
    assert np.linalg.norm(x + dx - xs) <= 1e-12 * np.linalg.norm(xs)
    assert np.linalg.norm(s + dz - r) <= 1e-12 * np.linalg.norm(b)


def test_correction_system_two_passes():
    # Two refinement passes, each a few correction iterations from the
    # current x, land on A^+ b: the second pass starts where the first one
    # stopped, with a fresh z = b - A x.
    a, b, xs, r = ls_system(60, 20, seed=5)
    x = np.zeros(20)
    for it0, iters in [(0, 4), (4, 300)]:
        t = a.T @ (b - a @ x)
        dx, _, _ = rgdbek(a, np.zeros(60), k_col=8, k_row=20,
                          max_iter=iters, col_offset=t, it0=it0, seed=2)
        x = x + dx
    assert np.linalg.norm(x - xs) <= 1e-12 * np.linalg.norm(xs)


def test_zero_offset_is_algorithm_one():
    # t = 0 and b = the right-hand side leave Algorithm 1 unchanged.
    a, b, _, _ = ls_system(30, 10, seed=6)
    x1, z1, _ = rgdbek(a, b, k_col=4, k_row=9, max_iter=5, seed=3)
    x2, z2, _ = rgdbek(a, b, k_col=4, k_row=9, max_iter=5, seed=3,
                       col_offset=np.zeros(10))
    assert np.array_equal(x1, x2) and np.array_equal(z1, z2)


# ------------------------------------------------------------ LSQR branch
def sparse_block(m, n, density, seed, dup_cols=0):
    rng = np.random.default_rng(seed)
    a = sp.random(m, n, density=density, format="csc", random_state=rng,
                  data_rvs=rng.standard_normal)
    if dup_cols:   # repeated columns: rank deficient
        a = sp.hstack([a, a[:, :dup_cols]], format="csc")
    return a.tocsr()


@pytest.mark.parametrize("shape,dup", [((6000, 300), 0), ((300, 6000), 0),
                                       ((5000, 200), 20)],
                         ids=["tall", "fat", "rank_deficient"])
def test_lsqr_branch_matches_dense_lstsq(shape, dup):
    # Blocks with a dimension above DENSE_LIMIT take scipy's LSQR from
    # zero, which converges to the minimum-norm least-squares solution;
    # the same block through LAPACK's SVD solver must agree.
    m, n = shape
    assert max(m, n) > DENSE_LIMIT
    blk = sparse_block(m, n, 0.03 if m > n else 0.05, seed=m + n, dup_cols=dup)
    rhs = np.random.default_rng(7).standard_normal(blk.shape[0])
    y, nr = pinv_apply(blk, rhs)
    want = np.linalg.lstsq(blk.toarray(), rhs, rcond=None)[0]
    assert np.linalg.norm(y - want) <= 1e-12 * np.linalg.norm(want)
    assert nr <= 1e-13


# ------------------------------------------------------------ Theorem 2.3
def test_theorem_2_3_residual_decay_over_seeds():
    # Theorem 2.3 a): E ||z_k - r||^2 <= gamma^k ||z_0 - r||^2 with
    # gamma = 1 - sigma_min^2(A) / (mu ||A||_2^2).  mu_col, the largest
    # ||A_U^T A_U||_2 / ||A_U||_2^2 over column blocks, is enumerated (it is
    # 1: the two norms coincide).  The expectation is estimated by the mean
    # over 200 generator seeds; it must sit below the bound at every k and
    # keep falling geometrically.  A second, weaker bound that holds for
    # this sampling rule (the block always holds the one-index draw j* with
    # P(j*) proportional to eps^z, so E||P_U e||^2 >= sum eps^2 / sum eps
    # >= sigma_min^2 ||e||^2 / (n max_j ||A_(j)||^2)) is checked as well.
    a, b, xs, r = ls_system(10, 6, seed=11, resid=0.5)
    n, kc = 6, 3
    mu = max(np.linalg.norm(a[:, list(u)].T @ a[:, list(u)], 2) /
             np.linalg.norm(a[:, list(u)], 2) ** 2
             for u in itertools.combinations(range(n), kc))
    assert abs(mu - 1.0) <= 1e-12
    sv = np.linalg.svd(a, compute_uv=False)
    gamma = 1.0 - sv[-1] ** 2 / (mu * sv[0] ** 2)
    gamma_rule = 1.0 - sv[-1] ** 2 / (n * np.max(np.sum(a * a, axis=0)))
    K = 8
    errs = np.zeros(K + 1)
    seeds = 200
    for seed in range(seeds):
        z = b.copy()
        x = np.zeros(n)
        errs[0] += np.linalg.norm(z - r) ** 2
        for k in range(K):
            x, z, _ = rgdbek(a, b, k_col=kc, k_row=5, max_iter=1, seed=seed,
                             x0=x, z0=z, it0=k)
            errs[k + 1] += np.linalg.norm(z - r) ** 2
    errs /= seeds
    e0 = errs[0]
    for k in range(1, K + 1):
        assert errs[k] <= gamma ** k * e0, (k, errs[k], gamma ** k * e0)
        assert errs[k] <= gamma_rule ** k * e0
        assert errs[k] < errs[k - 1]
    # geometric: the log-mean falls at a steady rate (least-squares slope)
    slope = np.polyfit(np.arange(K + 1), np.log(errs), 1)[0]
    assert slope < np.log(gamma)


def test_tikhonov_kron_closed_form_against_lstsq():
    """The Kronecker closed form of the regularised deblurring solution
    against a dense least-squares solve of the stacked system [A; s I]
    (8 x 8 image), on the exact-in-FP32 operator the workload builds."""
    import workloads
    from oracle.refsol import tikhonov_kron
    aug, t, s = workloads.blur_tikhonov(npix=8, mu=1e-2)
    n = 64
    a = aug[:n].toarray()
    assert np.allclose(a, np.kron(t, t), rtol=0, atol=0)
    rng = np.random.default_rng(3)
    b = rng.standard_normal((n, 3))
    want = np.linalg.lstsq(aug.toarray(), np.vstack([b, np.zeros((n, 3))]),
                           rcond=None)[0]
    got = tikhonov_kron(t, b, s)
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)
    # a dropped regulariser or a transposed factor fails the normal equations
    ne = a.T @ (a @ got - b) + s * s * got
    assert np.linalg.norm(ne) <= 1e-12 * np.linalg.norm(a.T @ b)
    # without the regulariser the answer moves well beyond the tolerance
    assert (np.linalg.norm(tikhonov_kron(t, b[:, 0], 0.0) - want[:, 0])
            > 1e-3 * np.linalg.norm(want[:, 0]))


def test_tikhonov_kron_lam_against_pinv_gradient():
    """The closed-form adjoint of the deblurring layer: lam and, from it,
    w = dL/db and dL/dA = r lam^T - w x^T against the dense pinv reference
    of the implicit gradient (8 x 8 image, loss gradient dL/dx = c)."""
    import workloads
    from oracle.refsol import grad_reference, tikhonov_kron, tikhonov_kron_lam
    aug, t, s = workloads.blur_tikhonov(npix=8, mu=1e-2)
    n = 64
    ad = aug.toarray()
    rng = np.random.default_rng(4)
    b = np.concatenate([rng.standard_normal(n), np.zeros(n)])
    c = rng.standard_normal(n)
    lam = tikhonov_kron_lam(t, c, s)
    x = tikhonov_kron(t, b[:n], s)
    w = ad @ lam
    r = b - ad @ x
    da = np.outer(r, lam) - np.outer(w, x)
    da_want, w_want = grad_reference(ad, b, c)
    assert np.linalg.norm(w - w_want) <= 1e-11 * np.linalg.norm(w_want)
    assert np.linalg.norm(da - da_want) <= 1e-11 * np.linalg.norm(da_want)
    # the normal equations of lam (a missing s^2 or a transposed factor
    # fails them)
    a = ad[:n]
    ne = a.T @ (a @ lam) + s * s * lam - c
    assert np.linalg.norm(ne) <= 1e-12 * np.linalg.norm(c)
