"""Parity at the full workload sizes, through the C-ABI.

The oracle cannot run whole solves at these sizes in seconds, so each test
checks either sampled outputs the oracle computes one by one, or properties
that hold at any size:

* dense least squares 20000 x 5000 (the benchmark workload): the first
  iteration with the benchmark's block sizes and exact projections equals
  the oracle's (one oracle iteration takes about a second); the benchmark's
  own tuned configurations reach ||x - x*|| <= 1e-8 ||x*||;
* sparse power-law 1,000,000 x 500,000: sampled rows/columns of both
  residual products; after one iteration with exact projections, the
  columns the column projection annihilated (A_U^T z_1 = 0) and the rows the
  row projection satisfied are, up to near-ties, the oracle's draws on the
  same weights (Section 2);
* 256 uneven Laplacian systems: the same per-system properties on sampled
  systems after one batched iteration;
* Gaussian blur 512 x 512 (the replicated operator): sampled products
  with 64 right-hand sides, one-iteration properties with 4.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import workloads
from oracle.rgdbek import rgdbek
from oracle.select import select as oselect, block_size

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rg():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2509_19267_amd as rg
    rg.load()
    return rg


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype=dtype).cuda()


def csr_tensors(a, dtype=np.float64):
    rp, ci, v = workloads.to_csr_arrays(a, value_dtype=dtype)
    return (torch.as_tensor(rp).cuda(), torch.as_tensor(ci).cuda(),
            torch.as_tensor(v).cuda())


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


def free():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def weights(v, nrm):
    """eps = v^2 / nrm with zero for zero norms (Section 2)."""
    out = np.zeros_like(v)
    pos = nrm > 0
    out[pos] = v[pos] * v[pos] / nrm[pos]
    return out


def check_first_iteration(a, b, x1, z1, k_col, k_row, seed=0, sys=0,
                          tol_col=1e-10, tol_row=1e-10, max_off=1e-3):
    """Properties of one RGDBEK iteration from x_0 = 0, z_0 = b (sparse A).

    Draws: U is the oracle's draw on eps^z = (A^T b)^2 / kappa and J its draw
    on r^2 / rho with r = b - z_1 (A x_0 = 0) (Section 2).  The column update
    moves z only on rows that the columns of U touch, and the row update
    moves x only on columns that the rows of J touch: z_1 - b and x_1 must be
    zero outside those sets (exactly zero on the GPU; the oracle's SVD leaves
    rounding-level values), so a different draw shows up as changes outside
    them.
    Projections: ||A_U^T z_1|| <= tol_col ||A_U^T b|| and
    ||A_J^T (r_J - A_J x_1)|| <= tol_row ||A_J^T r_J|| (the normal-equation
    residuals of the two projected systems).  max_off bounds the share of
    indices that near-ties of the keys (squared norms summed in different
    orders on the two sides) may move."""
    a = sp.csr_matrix(a)
    ac = a.tocsc()
    kappa = np.asarray(a.multiply(a).sum(axis=0)).ravel()
    rho = np.asarray(a.multiply(a).sum(axis=1)).ravel()
    g0 = a.T @ b
    U = oselect(weights(g0, kappa), k_col, seed, 0, 0, sys)
    rows_u = np.zeros(a.shape[0], bool)
    rows_u[ac[:, U].indices] = True
    moved = np.abs(z1 - b) > 1e-12 * np.abs(b).max()
    assert moved.any()
    assert (moved & ~rows_u).sum() <= max_off * rows_u.sum()
    hu = ac[:, U].T @ z1
    assert np.linalg.norm(hu) <= tol_col * np.linalg.norm(g0[U])
    r = b - z1
    J = oselect(weights(r, rho), k_row, seed, 0, 1, sys)
    cols_j = np.zeros(a.shape[1], bool)
    cols_j[a[J].indices] = True
    nz = np.abs(x1) > 1e-12 * np.abs(x1).max()
    assert nz.any()
    assert (nz & ~cols_j).sum() <= max_off * cols_j.sum()
    aj = a[J]
    ne = aj.T @ (r[J] - aj @ x1)
    assert np.linalg.norm(ne) <= tol_row * np.linalg.norm(aj.T @ r[J])
    return U, J


# ------------------------------------------------------------ dense 20000x5000
def test_dense_ls_fullsize_first_iteration(rg):
    from paper_2509_19267_amd import tune
    p = workloads.dense_least_squares(20000, 5000, seed=0)
    ch = tune.lookup("dense", 20000, 5000, "fp64") or dict(k_col=1500, k_row=1500)
    kc, kr = ch["k_col"], ch["k_row"]
    s = rg.Solver(dev(p.a), k_col=kc, k_row=kr, gram_aat=True, stop="none",
                  max_iter=1, inner_max=400, inner_tol=1e-14)
    x, _ = s.solve(dev(p.b))
    z = s.get_z().cpu().numpy()
    s.close()
    xo, zo, _ = rgdbek(p.a, p.b, k_col=kc, k_row=kr, max_iter=1)
    print(f"dense 20000x5000 k={kc}/{kr}: rel_x {rel(x.cpu().numpy(), xo):.2e} "
          f"rel_z {rel(z, zo):.2e}", flush=True)
    assert rel(x.cpu().numpy(), xo) <= 1e-10
    assert rel(z, zo) <= 1e-10
    free()


def test_dense_ls_fullsize_eta_half_first_iteration(rg):
    # Section 3's eta = 0.5 on the 20000 x 5000 system: 2500-column and
    # 10000-row blocks (row blocks twice as tall as A is wide, beyond the
    # Gram limit; projected by CGLS); exact projections, one iteration
    p = workloads.dense_least_squares(20000, 5000, seed=0)
    kc, kr = 2500, 10000
    s = rg.Solver(dev(p.a), k_col=kc, k_row=kr, stop="none", max_iter=1,
                  inner_max=400, inner_tol=1e-14, graph_iters=1)
    x, _ = s.solve(dev(p.b))
    z = s.get_z().cpu().numpy()
    s.close()
    free()
    xo, zo, _ = rgdbek(p.a, p.b, k_col=kc, k_row=kr, max_iter=1)
    print(f"dense 20000x5000 eta=0.5 k={kc}/{kr}: rel_x "
          f"{rel(x.cpu().numpy(), xo):.2e} rel_z {rel(z, zo):.2e}", flush=True)
    assert rel(x.cpu().numpy(), xo) <= 1e-10
    assert rel(z, zo) <= 1e-10


@pytest.mark.parametrize("form", ["fp64", "mixed_f32"])
def test_dense_ls_fullsize_bench_config(rg, form):
    from paper_2509_19267_amd import tune
    p = workloads.dense_least_squares(20000, 5000, seed=0)
    ch = tune.lookup("dense", 20000, 5000, form)
    if ch is None:
        pytest.skip("no tuned configuration cached")
    s = rg.Solver(dev(p.a), k_col=ch["k_col"], k_row=ch["k_row"],
                  gram_aat=ch.get("gram_aat", False), stop="err_ref", tol=1e-8,
                  max_iter=20000, precision=form,
                  inner_tol=ch.get("inner_tol", 0.0),
                  inner_max=ch.get("inner_max", 0),
                  tile_rows=ch.get("tile_rows", 0))
    x, info = s.solve(dev(p.b), x_ref=dev(p.x_star))
    s.close()
    err = rel(x.cpu().numpy(), p.x_star)
    print(f"{form}: {info} err {err:.2e}", flush=True)
    assert info["converged"] == 1
    assert err <= 1e-8
    free()


# ------------------------------------------------------------ sparse 1M x 500K
@pytest.fixture(scope="module")
def powerlaw():
    return workloads.sparse_powerlaw(1_000_000, 500_000, mean_len=10,
                                     max_len=2000, seed=0)


def test_powerlaw_fullsize_products(rg, powerlaw):
    a = powerlaw.a
    m, n = a.shape
    s = rg.Solver(csr=csr_tensors(a), shape=(m, n), eta=0.1)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(n)
    z = rng.standard_normal(m)
    ax, atz = s.apply(dev(x), dev(z))
    torch.cuda.synchronize()
    rows = rng.choice(m, 5000, replace=False)
    cols = rng.choice(n, 5000, replace=False)
    want_r = a[rows] @ x
    want_c = a[:, cols].T @ z
    assert rel(ax.cpu().numpy()[rows], want_r) <= 1e-13
    assert rel(atz.cpu().numpy()[cols], want_c) <= 1e-13
    s.close()
    free()


def test_powerlaw_fullsize_first_iteration(rg, powerlaw):
    a, b = powerlaw.a, powerlaw.b
    m, n = a.shape
    kc, kr = block_size(0.1, n), block_size(0.1, m)
    s = rg.Solver(csr=csr_tensors(a), shape=(m, n), k_col=kc, k_row=kr,
                  stop="none", max_iter=1, inner_max=400, graph_iters=1)
    x, _ = s.solve(dev(b))
    z = s.get_z().cpu().numpy()
    s.close()
    # over half the rows have one nonzero, so row blocks repeat rows and
    # are (nearly) singular: CG reaches the projection only slowly (the
    # exact trajectories are checked at smaller sizes)
    U, J = check_first_iteration(a, b, x.cpu().numpy(), z, kc, kr,
                                 tol_row=1e-2)
    print(f"powerlaw 1Mx500K: |U| {len(U)} |J| {len(J)}", flush=True)
    free()


# ------------------------------------------------------------ 256-system batch
def test_batch_fullsize_first_iteration(rg):
    from paper_2509_19267_amd import block_diagonal
    ps = workloads.laplacian_batch(count=256, n_min=2000, n_max=200000, seed=0)
    rp, ci, v, ro, co = block_diagonal([q.a for q in ps])
    csr = (torch.as_tensor(rp).cuda(), torch.as_tensor(ci).cuda(),
           torch.as_tensor(v).cuda())
    b = np.concatenate([q.b for q in ps])
    s = rg.BatchSolver(csr, ro, co, eta=0.1, stop="none", max_iter=1,
                       inner_max=400, graph_iters=1)
    x, _ = s.solve(dev(b))
    z = s.get_z().cpu().numpy()
    x = x.cpu().numpy()
    s.close()
    del csr
    free()
    for i in [0, 17, 128, 255]:
        q = ps[i]
        xs, zs = x[co[i]:co[i + 1]], z[ro[i]:ro[i + 1]]
        U, J = check_first_iteration(q.a, q.b, xs, zs,
                                     block_size(0.1, q.a.shape[1]),
                                     block_size(0.1, q.a.shape[0]), sys=i)
        print(f"batch system {i}: n {q.a.shape[1]} |U| {len(U)} |J| {len(J)}",
              flush=True)


# ------------------------------------------------------------ many RHS
def test_multirhs_segments_survive_setup(rg):
    # 64 right-hand sides of a 256 x 256 deblurring operator (8.4M virtual
    # rows): the per-system descriptors are uploaded after the zero fills of
    # their allocations (a plain copy was not ordered after the fills queued
    # behind the norm replication, and lost to them at this size), so every
    # right-hand side's first iteration moves z and x
    aug, _, _ = workloads.blur_tikhonov(256, 1e-2)
    n = 256 * 256
    m = aug.shape[0]
    b_img, _ = workloads.blur_rhs(aug[:n], npix=256, nrhs=64, seed=1)
    bb = np.zeros((64, m))
    bb[:, :n] = b_img.T
    s = rg.MultiRhsSolver(csr_tensors(aug, np.float32), (m, n), 64, eta=0.1,
                          stop="none", max_iter=1, inner_tol=0.1,
                          inner_max=16)
    x, info = s.solve(dev(bb.ravel()))
    z = s.get_z().cpu().numpy().reshape(64, m)
    x = x.cpu().numpy().reshape(64, n)
    s.close()
    dz = np.linalg.norm(z - bb, axis=1) / np.linalg.norm(bb, axis=1)
    print(f"many-RHS first iteration: dz {dz.min():.3f}..{dz.max():.3f}", flush=True)
    assert dz.min() > 0.5 and np.linalg.norm(x, axis=1).min() > 0.0
    free()


# ------------------------------------------------------------ blur, 64 RHS
def test_blur_fullsize_multirhs(rg):
    # the products with all 64 right-hand sides; one exact iteration (its
    # CG steps sweep the replicated operator) with the first 4 of them
    npix, R = 512, 64
    a = workloads.blur_operator(npix=npix, dtype=np.float32).astype(np.float64)
    a = sp.csr_matrix(a)
    n = a.shape[0]
    bs = workloads.blur_rhs(a, npix=npix, nrhs=R, seed=0)[0].T   # (R, n)
    s = rg.MultiRhsSolver(csr_tensors(a), a.shape, R, eta=0.1)
    rng = np.random.default_rng(4)
    xv = rng.standard_normal(R * n)
    zv = rng.standard_normal(R * n)
    ax, atz = s.apply(dev(xv), dev(zv))
    torch.cuda.synchronize()
    ax = ax.cpu().numpy().reshape(R, n)
    atz = atz.cpu().numpy().reshape(R, n)
    for r in [0, 31, 63]:
        rows = rng.choice(n, 3000, replace=False)
        assert rel(ax[r, rows], a[rows] @ xv[r * n:(r + 1) * n]) <= 1e-13
        assert rel(atz[r, rows], a[:, rows].T @ zv[r * n:(r + 1) * n]) <= 1e-13
    s.close()
    free()
    R4 = 4
    s = rg.MultiRhsSolver(csr_tensors(a), a.shape, R4, eta=0.1, stop="none",
                          max_iter=1, inner_max=30, graph_iters=1)
    x, _ = s.solve(dev(bs[:R4].ravel()))
    z = s.get_z().cpu().numpy().reshape(R4, n)
    x = x.cpu().numpy().reshape(R4, n)
    s.close()
    free()
    k = block_size(0.1, n)
    # cond(A) ~ 1e12: 30 CG steps only start each projection; the draws and
    # the supports of the updates are exact all the same
    for r in [0, 3]:
        U, J = check_first_iteration(a, bs[r], x[r], z[r], k, k, sys=r,
                                     tol_col=0.5, tol_row=0.9)
        print(f"blur rhs {r}: |U| {len(U)} |J| {len(J)}", flush=True)
