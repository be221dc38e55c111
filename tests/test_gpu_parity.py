"""GPU parity of the HIP path against the FP64 oracle, through the C-ABI.

Selection: bit-exact index sets on identical weights.  Iterates: relative
difference <= 1e-10 in FP64 after a fixed number of iterations (trajectory
mode) and at convergence (solution mode).  Mixed precision: <= 1e-5 against
the FP64 solution before refinement, FP64 level after."""
from types import SimpleNamespace

import numpy as np
import pytest
import torch

import workloads
from oracle.rgdbek import rgdbek
from oracle.select import select as oselect
from oracle.refsol import pinv_solution

pytestmark = pytest.mark.gpu

TRAJ_TOL = 1e-10


@pytest.fixture(scope="module")
def rg():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2509_19267_amd as rg
    rg.load()
    return rg


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype=dtype).cuda()


def csr_tensors(a):
    rp, ci, v = workloads.to_csr_arrays(a)
    return (torch.as_tensor(rp).cuda(), torch.as_tensor(ci).cuda(),
            torch.as_tensor(v).cuda())


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


# ------------------------------------------------------------ selection
def sel_cases():
    rng = np.random.default_rng(0)
    yield "random", rng.random(1000) ** 4, 100
    e = rng.random(5000)
    e[rng.random(5000) < 0.9] = 0.0
    yield "zero_heavy", e, 300
    yield "ties", np.repeat([0.5, 1.0, 2.0], [300, 300, 400]), 250
    yield "k1", rng.random(777), 1
    yield "k_eq_d", rng.random(333) + 0.1, 333
    yield "k_gt_pos", np.where(rng.random(400) < 0.05, 1.0, 0.0), 50
    yield "denormal", np.full(200, 5e-324), 17
    # 1000 equal (infinite) keys: more equal keys than the one-workgroup
    # ranking holds, resolved by the ordered scan
    yield "equal_keys", np.full(1000, 5e-324), 300
    yield "one_weight", np.eye(1, 97, 13).ravel(), 5
    yield "small_max", rng.random(65536), 6553
    yield "large_min", rng.random(65537), 6554
    yield "rows_1e6", rng.random(1_000_000) ** 2, 100_000
    big = rng.random(300_000)
    big[::3] = 0.25
    yield "large_ties", big, 120_000
    yield "large_all", np.where(rng.random(200_000) < 0.01, rng.random(200_000), 0.0), 5000


@pytest.mark.parametrize("case", list(sel_cases()), ids=lambda c: c[0])
def test_select_bit_exact(rg, case):
    name, eps, k = case
    print(f"select case {name} d={eps.size} k={k}", flush=True)
    for (seed, it, phase, sys, key1) in [(0, 0, 0, 0, 0), (12345, 77, 1, 3, 1)]:
        got = rg.select(dev(eps), k, seed=seed, it=it, phase=phase, sys=sys,
                        key1=key1).cpu().numpy()
        want = oselect(eps, k, seed, it, phase, sys, key1)
        assert got.dtype == np.int32
        assert np.array_equal(got.astype(np.int64), want), name


@pytest.mark.parametrize("floor", [0.0, 1e-20, 1e-26, 1e-8])
def test_select_weight_floor_bit_exact(rg, floor):
    rng = np.random.default_rng(5)
    for d, k in [(3000, 2000), (120_000, 90_000)]:
        e = rng.random(d)
        noise = rng.random(d) < 0.5
        e[noise] = rng.random(int(noise.sum())) * 1e-28   # rounding-level weights
        got = rg.select(dev(e), k, seed=4, it=9, phase=0, floor=floor).cpu().numpy()
        want = oselect(e, k, 4, 9, 0, floor=floor)
        assert np.array_equal(got.astype(np.int64), want)


def test_select_numeric_error(rg):
    with pytest.raises(rg.RgdbekError) as ei:
        rg.select(dev(np.array([1.0, np.nan, 2.0])), 1)
    assert ei.value.status == 2
    with pytest.raises(rg.RgdbekError):
        rg.select(dev(np.array([1.0, -1.0])), 1)


# ------------------------------------------------------------ trajectories
def run_both(rg, p, k_col, k_row, iters, seed=0, sparse=False, **kw):
    if sparse:
        s = rg.Solver(csr=csr_tensors(p.a), shape=p.a.shape, k_col=k_col,
                      k_row=k_row, stop="none", max_iter=iters, seed=seed, **kw)
    else:
        s = rg.Solver(dev(p.a), k_col=k_col, k_row=k_row, stop="none",
                      max_iter=iters, seed=seed, **kw)
    x, info = s.solve(dev(p.b))
    z = s.get_z().cpu().numpy()
    xo, zo, io = rgdbek(p.a, p.b, k_col=k_col, k_row=k_row, max_iter=iters,
                        seed=seed)
    s.close()
    return x.cpu().numpy(), z, info, xo, zo


def test_trajectory_dense_consistent_c1(rg):
    # 500 x 250 N(0,1), eta = 0.5: 125 columns, 250 rows (square row blocks)
    p = workloads.dense_consistent(500, 250, seed=0)
    for iters in [1, 3, 8]:
        x, z, info, xo, zo = run_both(rg, p, 125, 250, iters)
        print(f"c1 iters={iters} rel_x={rel(x, xo):.3e} rel_z={rel(z, zo):.3e}", flush=True)
        assert info["iterations"] == iters
        assert rel(x, xo) <= TRAJ_TOL
        assert rel(z, zo) <= TRAJ_TOL


def test_solution_dense_consistent_c1(rg):
    p = workloads.dense_consistent(500, 250, seed=0)
    s = rg.Solver(dev(p.a), eta=0.5, stop="err_ref", tol=1e-10, max_iter=500)
    x, info = s.solve(dev(p.b), x_ref=dev(p.x_star))
    xo, zo, io = rgdbek(p.a, p.b, eta=0.5, max_iter=500, stop="err_ref",
                        tol=1e-10, x_ref=p.x_star)
    print("c1 solve", info, io.iterations, flush=True)
    assert info["converged"] == 1
    assert rel(x.cpu().numpy(), p.x_star) <= 1e-10
    assert rel(x.cpu().numpy(), xo) <= 2e-10
    assert abs(info["iterations"] - io.iterations) <= 1


@pytest.mark.parametrize("kc,kr,solver", [(40, 80, 0), (300, 400, 0), (120, 200, 2)])
def test_trajectory_dense_least_squares(rg, kc, kr, solver):
    p = workloads.dense_least_squares(2000, 500, seed=2)
    x, z, info, xo, zo = run_both(rg, p, kc, kr, 4, seed=5, solver=solver,
                                  inner_max=200)
    print(f"ls kc={kc} kr={kr} solver={solver} rel_x={rel(x, xo):.3e} rel_z={rel(z, zo):.3e}", flush=True)
    assert rel(x, xo) <= TRAJ_TOL
    assert rel(z, zo) <= TRAJ_TOL


@pytest.mark.parametrize("kc,kr,gram_aat", [(301, 403, False), (301, 403, True),
                                            (300, 400, True)])
def test_trajectory_dense_pcg_gram_sources(rg, kc, kr, gram_aat):
    # persistent PCG on both projections: the column block gathered from
    # A^T A inside the first CG step, the row block from A A^T likewise
    # (gram_aat) or formed from the rows; odd block sizes take the scalar
    # row loads, even ones the 16-byte loads
    p = workloads.dense_least_squares(2000, 500, seed=7)
    x, z, info, xo, zo = run_both(rg, p, kc, kr, 4, seed=3, solver=0,
                                  inner_max=200, gram_aat=gram_aat)
    print(f"pcg kc={kc} kr={kr} aat={gram_aat} rel_x={rel(x, xo):.3e} rel_z={rel(z, zo):.3e}", flush=True)
    assert info["iterations"] == 4
    assert rel(x, xo) <= TRAJ_TOL
    assert rel(z, zo) <= TRAJ_TOL


@pytest.mark.parametrize("gram_aat", [True, False])
def test_trajectory_dense_two_launch_pcg(rg, gram_aat):
    # FP64 blocks of 4097..8192 indices: beyond the persistent PCG's LDS
    # staging, so the Gram block is gathered (or formed from the rows) by its
    # own launch and every CG step takes two launches
    p = workloads.dense_least_squares(6000, 5000, seed=9)
    x, z, info, xo, zo = run_both(rg, p, 4500, 4200, 1, seed=6, solver=0,
                                  inner_max=800, graph_iters=1,
                                  gram_aat=gram_aat)
    print(f"two-launch pcg aat={gram_aat} rel_x={rel(x, xo):.3e} "
          f"rel_z={rel(z, zo):.3e}", flush=True)
    assert rel(x, xo) <= TRAJ_TOL
    assert rel(z, zo) <= TRAJ_TOL
    torch.cuda.empty_cache()


@pytest.mark.parametrize("sparse_cg", [False, True], ids=["gram", "cg"])
def test_trajectory_sparse_uniform(rg, sparse_cg):
    # small enough for the Gram projections (default) and, forced, the
    # matrix-free CG
    p = workloads.sparse_uniform(3000, 1500, density=0.01, seed=3)
    x, z, info, xo, zo = run_both(rg, p, 150, 300, 4, sparse=True,
                                  inner_max=200, sparse_cg=sparse_cg)
    print(f"sparse uniform cg={sparse_cg} rel_x={rel(x, xo):.3e} rel_z={rel(z, zo):.3e}", flush=True)
    assert rel(x, xo) <= TRAJ_TOL
    assert rel(z, zo) <= TRAJ_TOL


def test_trajectory_sparse_powerlaw(rg):
    # long rows (up to 400 nnz) take the one-workgroup-per-row kernel
    # some row blocks are rank-deficient (rows sharing their single column):
    # CG on the singular consistent Gram needs more steps
    p = workloads.sparse_powerlaw(6000, 3000, mean_len=10, max_len=400, seed=4)
    x, z, info, xo, zo = run_both(rg, p, 300, 600, 3, sparse=True,
                                  inner_max=1000, graph_iters=1)
    print(f"sparse powerlaw rel_x={rel(x, xo):.3e} rel_z={rel(z, zo):.3e}", flush=True)
    assert rel(x, xo) <= TRAJ_TOL
    assert rel(z, zo) <= TRAJ_TOL


@pytest.mark.parametrize("shape,kc,kr,mean,rows", [((6000, 3000), 300, 600, 10, 400),
                                                   ((20000, 9000), 900, 2000, 30, 2000)])
def test_sparse_block_restricted_equals_full(rg, shape, kc, kr, mean, rows):
    # the CG's wide products over the block's own entries (copied once per
    # iteration) against the products over all of A: the same sums grouped
    # differently across lanes, so both at the oracle's trajectory and at
    # rounding distance of each other; power-law rows include long ones (up
    # to `rows` entries: one workgroup each in the full passes, G lanes in
    # the block copy); with mean length 10 some row blocks are
    # rank-deficient (rows sharing their single column), and CG on the
    # singular consistent Gram needs many steps
    m, n = shape
    p = workloads.sparse_powerlaw(m, n, mean_len=mean, max_len=rows, seed=21)
    xs = []
    for full in (False, True):
        s = rg.Solver(csr=csr_tensors(p.a), shape=p.a.shape, k_col=kc,
                      k_row=kr, stop="none", max_iter=3, seed=4,
                      inner_max=1000, graph_iters=1, sparse_cg=True,
                      sparse_full=full)
        x, _ = s.solve(dev(p.b))
        xs.append((x.cpu().numpy(), s.get_z().cpu().numpy()))
        s.close()
    xo, zo, _ = rgdbek(p.a, p.b, k_col=kc, k_row=kr, max_iter=3, seed=4)
    print(f"restricted sparse {shape}: rel_x {rel(xs[0][0], xo):.3e} "
          f"full {rel(xs[1][0], xo):.3e} between {rel(xs[0][0], xs[1][0]):.3e}",
          flush=True)
    for x, z in xs:
        assert rel(x, xo) <= TRAJ_TOL
        assert rel(z, zo) <= TRAJ_TOL
    assert rel(xs[0][0], xs[1][0]) <= 1e-12


def test_solution_sparse_consistent(rg):
    p = workloads.sparse_powerlaw(6000, 3000, mean_len=10, max_len=400, seed=5)
    s = rg.Solver(csr=csr_tensors(p.a), shape=p.a.shape, eta=0.1,
                  stop="err_ref", tol=1e-10, max_iter=3000, inner_max=100)
    x, info = s.solve(dev(p.b), x_ref=dev(p.x_star))
    print("sparse solve", info, flush=True)
    assert info["converged"] == 1
    assert rel(x.cpu().numpy(), p.x_star) <= 1e-10


def test_resume_is_bitwise(rg):
    p = workloads.dense_least_squares(800, 200, seed=6)
    s = rg.Solver(dev(p.a), k_col=30, k_row=60, stop="none", max_iter=6, seed=2)
    x2, _ = s.solve(dev(p.b))
    z2 = s.get_z()
    s.close()
    s = rg.Solver(dev(p.a), k_col=30, k_row=60, stop="none", max_iter=3, seed=2)
    x1, _ = s.solve(dev(p.b))
    z1 = s.get_z()
    s.solve_resume(dev(p.b), x1, z1, 3)
    assert torch.equal(x1, x2) and torch.equal(z1, z2)
    s.close()


def test_stop_rules_and_errors(rg):
    p = workloads.dense_consistent(120, 60, seed=7)
    s = rg.Solver(dev(p.a), k_col=10, k_row=20, stop="rse", tol=1e-12,
                  max_iter=2000)
    x, info = s.solve(dev(p.b))
    xo, _, io = rgdbek(p.a, p.b, k_col=10, k_row=20, max_iter=2000,
                       stop="rse", tol=1e-12)
    assert info["converged"] == 1
    assert abs(info["iterations"] - io.iterations) <= 1
    s.close()
    s = rg.Solver(dev(p.a), k_col=10, k_row=20, stop="err_ref", tol=1e-30,
                  max_iter=3)
    x, info = s.solve(dev(p.b), x_ref=dev(p.x_star))
    assert info["converged"] == 0 and info["iterations"] == 3
    assert info["status"] == 3
    xo, _, _ = rgdbek(p.a, p.b, k_col=10, k_row=20, max_iter=3)
    assert rel(x.cpu().numpy(), xo) <= TRAJ_TOL
    bad = p.b.copy()
    bad[5] = np.nan
    with pytest.raises(rg.RgdbekError) as ei:
        s.solve(dev(bad), x_ref=dev(p.x_star))
    assert ei.value.status == 2
    s.close()
    with pytest.raises(rg.RgdbekError) as ei:
        rg.Solver(dev(p.a), k_col=61, k_row=20)
    assert ei.value.status == 1
    a = p.a.copy()
    a[3, 3] = np.inf
    with pytest.raises(rg.RgdbekError) as ei:
        rg.Solver(dev(a), k_col=10, k_row=20)
    assert ei.value.status == 2


def test_csr_structure_errors(rg):
    p = workloads.sparse_uniform(50, 40, density=0.1, seed=8)
    rp, ci, v = csr_tensors(p.a)
    ci_bad = ci.clone()
    ci_bad[0] = 40
    with pytest.raises(rg.RgdbekError) as ei:
        rg.Solver(csr=(rp, ci_bad, v), shape=(50, 40), k_col=5, k_row=5)
    assert ei.value.status == 1
    rp_bad = rp.clone()
    rp_bad[10] = rp_bad[11] + 1
    with pytest.raises(rg.RgdbekError):
        rg.Solver(csr=(rp_bad, ci, v), shape=(50, 40), k_col=5, k_row=5)


def test_zero_rows_and_columns(rg):
    rng = np.random.default_rng(8)
    a = rng.standard_normal((40, 20))
    a[4, :] = 0.0
    a[:, 7] = 0.0
    b = rng.standard_normal(40)
    s = rg.Solver(dev(a), k_col=6, k_row=10, stop="res_ext", tol=1e-11,
                  max_iter=5000)
    x, info = s.solve(dev(b))
    xs, rs = pinv_solution(a)(b)
    assert info["converged"] == 1
    assert rel(x.cpu().numpy(), xs) <= 1e-9
    assert x[7].item() == 0.0
    z = s.get_z().cpu().numpy()
    assert abs(z[4] - b[4]) <= 1e-12


# ------------------------------------------------------------ adjoint / grad
def test_adjoint_solve(rg):
    p = workloads.dense_least_squares(300, 80, seed=9)
    g = np.random.default_rng(1).standard_normal(80)
    s = rg.Solver(dev(p.a), k_col=20, k_row=40, stop="res_ext", tol=1e-13,
                  max_iter=5000)
    w, info = s.solve_adjoint(dev(g))
    w_ref = np.linalg.pinv(p.a.T) @ g
    print("adjoint", info, rel(w.cpu().numpy(), w_ref), flush=True)
    assert rel(w.cpu().numpy(), w_ref) <= 1e-10
    s.close()


def test_gradient_pattern_and_autograd_dense(rg):
    p = workloads.dense_least_squares(200, 50, seed=10)
    from oracle.refsol import grad_reference
    c = np.random.default_rng(2).standard_normal(50)
    a_t = dev(p.a).requires_grad_(True)
    b_t = dev(p.b).requires_grad_(True)
    s = rg.Solver(a_t.detach(), k_col=15, k_row=30, stop="res_ext", tol=1e-13,
                  max_iter=5000)
    x = rg.solve(s, a_t.reshape(-1), b_t, least_squares=True)
    loss = (x * dev(c)).sum()
    loss.backward()
    da_ref, db_ref = grad_reference(p.a, p.b, c)
    assert rel(b_t.grad.cpu().numpy(), db_ref) <= 1e-9
    assert rel(a_t.grad.cpu().numpy(), da_ref) <= 1e-9
    s.close()


def test_gradient_sparse_pattern(rg):
    p = workloads.sparse_uniform(400, 150, density=0.05, seed=11)
    from oracle.refsol import grad_reference
    c = np.random.default_rng(3).standard_normal(150)
    rp, ci, v = csr_tensors(p.a)
    v = v.requires_grad_(True)
    b_t = dev(p.b).requires_grad_(True)
    s = rg.Solver(csr=(rp, ci, v.detach()), shape=p.a.shape, k_col=30,
                  k_row=60, stop="res_ext", tol=1e-13, max_iter=5000,
                  inner_max=100)
    x = rg.solve(s, v, b_t, least_squares=False)
    (x * dev(c)).sum().backward()
    da_ref, db_ref = grad_reference(p.a.toarray(), p.b, c)
    a = p.a.tocsr()
    rows = np.repeat(np.arange(a.shape[0]), np.diff(a.indptr))
    want = da_ref[rows, a.indices]
    assert rel(b_t.grad.cpu().numpy(), db_ref) <= 1e-9
    assert rel(v.grad.cpu().numpy(), want) <= 1e-9
    s.close()


# ------------------------------------------------------------ mixed
def test_mixed_dense_least_squares(rg):
    p = workloads.dense_least_squares(2000, 500, seed=12)
    s = rg.Solver(dev(p.a), k_col=100, k_row=100, precision="mixed_f32",
                  stop="err_ref", tol=1e-11, max_iter=5000)
    x, info = s.solve(dev(p.b), x_ref=dev(p.x_star))
    print("mixed dense", info, rel(x.cpu().numpy(), p.x_star), flush=True)
    assert info["converged"] == 1
    assert rel(x.cpu().numpy(), p.x_star) <= 1e-10
    s.close()


def test_mixed_first_pass_within_1e5(rg):
    # the first FP32 pass alone (before any FP64 refinement update) lands
    # within 1e-5 of the FP64 solution
    p = workloads.dense_least_squares(2000, 500, seed=13)
    s = rg.Solver(dev(p.a), k_col=100, k_row=100, precision="mixed_f32",
                  stop="none", max_iter=400)
    x, info = s.solve(dev(p.b))
    assert info["outer_iterations"] == 1
    xo = np.linalg.lstsq(p.a, p.b, rcond=None)[0]
    print("mixed first pass", rel(x.cpu().numpy(), xo), flush=True)
    assert rel(x.cpu().numpy(), xo) <= 1e-5
    s.close()


def test_mixed_rse(rg):
    p = workloads.dense_consistent(400, 200, seed=15)
    s = rg.Solver(dev(p.a), k_col=50, k_row=100, precision="mixed_f32",
                  stop="rse", tol=1e-24, max_iter=5000)
    x, info = s.solve(dev(p.b))
    assert info["converged"] == 1
    assert rel(x.cpu().numpy(), p.x_star) <= 1e-10
    s.close()


@pytest.mark.parametrize("kind", ["dense_ls", "dense_consistent", "sparse"])
def test_mixed_res_ext_refines_without_reference(rg, kind):
    """The mixed form under RES_EXT: no planted solution anywhere in the
    solve (its passes end on residuals only); the refined iterate reaches
    the least-squares solution (dense, with a component of b in null(A^T))
    or the planted solution (consistent) to 1e-10."""
    if kind == "dense_ls":
        p = workloads.dense_least_squares(2000, 500, seed=31)
        s = rg.Solver(dev(p.a), k_col=100, k_row=100, precision="mixed_f32",
                      stop="res_ext", tol=1e-12, max_iter=20000)
    elif kind == "dense_consistent":
        p = workloads.dense_consistent(1500, 400, seed=32)
        s = rg.Solver(dev(p.a), k_col=200, k_row=300, precision="mixed_f32",
                      stop="res_ext", tol=1e-12, max_iter=20000)
    else:
        p = workloads.sparse_powerlaw(6000, 3000, mean_len=10, max_len=400,
                                      seed=33)
        s = rg.Solver(csr=csr_tensors(p.a), shape=p.a.shape, eta=0.1,
                      precision="mixed_f32", stop="res_ext", tol=1e-12,
                      max_iter=20000, inner_max=100)
    x, info = s.solve(dev(p.b))
    print(f"mixed res_ext {kind}", info, flush=True)
    assert info["converged"] == 1 and info["final_metric"] <= 1e-12
    assert info["outer_iterations"] >= 2
    assert rel(x.cpu().numpy(), p.x_star) <= 1e-10
    # the FP64 form under the same test agrees
    s.close()


def test_batch_mixed_res_ext(rg):
    ps = workloads.laplacian_batch(count=6, n_min=500, n_max=4000, seed=34)
    mats = [rounded_f32(p.a) for p in ps]
    csr, ro, co = batch_tensors([SimpleNamespace(a=a) for a in mats])
    b = np.concatenate([a @ p.x_star for a, p in zip(mats, ps)])
    csr32 = (csr[0], csr[1], csr[2].to(torch.float32))
    s = rg.BatchSolver(csr32, ro, co, eta=0.1, stop="res_ext", tol=1e-12,
                       max_iter=20000, inner_max=200, precision="mixed_f32")
    x, info = s.solve(dev(b))
    its, met, conv = s.batch_info()
    print("batch mixed res_ext", info, list(met), flush=True)
    assert info["converged"] == 1 and all(conv)
    assert max(met) <= 1e-12
    x = x.cpu().numpy()
    for i, p in enumerate(ps):
        assert rel(x[co[i]:co[i + 1]], p.x_star) <= 1e-9
    s.close()


def test_apply_matches_products(rg):
    p = workloads.sparse_powerlaw(5000, 2000, mean_len=10, max_len=300, seed=16)
    rng = np.random.default_rng(0)
    xv, zv = rng.standard_normal(2000), rng.standard_normal(5000)
    s = rg.Solver(csr=csr_tensors(p.a), shape=p.a.shape, k_col=10, k_row=10,
                  precision="mixed_f32")
    ax, atz = s.apply(dev(xv), dev(zv))
    torch.cuda.synchronize()
    assert rel(ax.cpu().numpy(), p.a @ xv) <= 1e-14
    assert rel(atz.cpu().numpy(), p.a.T @ zv) <= 1e-14
    ax, atz = s.apply(dev(xv, torch.float32), dev(zv, torch.float32), precision="f32")
    torch.cuda.synchronize()
    assert rel(ax.cpu().numpy(), p.a @ xv) <= 1e-5
    s.close()
    d = workloads.dense_least_squares(3000, 700, seed=17)
    s = rg.Solver(dev(d.a), k_col=10, k_row=10)
    xv, zv = rng.standard_normal(700), rng.standard_normal(3000)
    ax, atz = s.apply(dev(xv), dev(zv))
    torch.cuda.synchronize()
    assert rel(ax.cpu().numpy(), d.a @ xv) <= 1e-14
    assert rel(atz.cpu().numpy(), d.a.T @ zv) <= 1e-14
    s.close()


def test_mixed_sparse_consistent(rg):
    p = workloads.sparse_powerlaw(6000, 3000, mean_len=10, max_len=400, seed=14)
    s = rg.Solver(csr=csr_tensors(p.a), shape=p.a.shape, eta=0.1,
                  precision="mixed_f32", stop="err_ref", tol=1e-10,
                  max_iter=5000, inner_max=100)
    x, info = s.solve(dev(p.b), x_ref=dev(p.x_star))
    print("mixed sparse", info, flush=True)
    assert info["converged"] == 1
    assert rel(x.cpu().numpy(), p.x_star) <= 1e-10
    s.close()


# ------------------------------------------------------------ batches
def batch_tensors(ps):
    rp, ci, v, ro, co = rg_block_diagonal([p.a for p in ps])
    return ((torch.as_tensor(rp).cuda(), torch.as_tensor(ci).cuda(),
             torch.as_tensor(v).cuda()), ro, co)


def rg_block_diagonal(mats):
    from paper_2509_19267_amd import block_diagonal
    return block_diagonal(mats)


def test_batch_trajectory_per_system(rg):
    # each system's iterate equals the oracle run on that system alone with
    # its own block sizes and generator stream (system id s)
    ps = workloads.laplacian_batch(count=6, n_min=300, n_max=900, seed=21)
    csr, ro, co = batch_tensors(ps)
    b = np.concatenate([p.b for p in ps])
    s = rg.BatchSolver(csr, ro, co, eta=0.1, stop="none", max_iter=3,
                       inner_max=300, graph_iters=1)
    x, info = s.solve(dev(b))
    x = x.cpu().numpy()
    for i, p in enumerate(ps):
        xo, _, _ = rgdbek(p.a, p.b, eta=0.1, max_iter=3, sys=i)
        xs = x[co[i]:co[i + 1]]
        print(f"batch system {i} n={p.a.shape[1]} rel={rel(xs, xo):.2e}", flush=True)
        assert rel(xs, xo) <= TRAJ_TOL
    s.close()


def test_batch_solution_per_system(rg):
    ps = workloads.laplacian_batch(count=12, n_min=200, n_max=3000, seed=22)
    csr, ro, co = batch_tensors(ps)
    b = np.concatenate([p.b for p in ps])
    xs = np.concatenate([p.x_star for p in ps])
    s = rg.BatchSolver(csr, ro, co, eta=0.1, stop="err_ref", tol=1e-10,
                       max_iter=5000, inner_max=200)
    x, info = s.solve(dev(b), x_ref=dev(xs))
    its, met, conv = s.batch_info()
    print("batch solve", info, its, flush=True)
    assert info["converged"] == 1 and all(conv)
    x = x.cpu().numpy()
    for i, p in enumerate(ps):
        assert rel(x[co[i]:co[i + 1]], p.x_star) <= 1e-10
    # iteration counts against the oracle on the two smallest systems (the
    # oracle needs minutes for the larger ones)
    for i in sorted(range(len(ps)), key=lambda j: ps[j].a.shape[1])[:2]:
        p = ps[i]
        xo, _, io = rgdbek(p.a, p.b, eta=0.1, max_iter=5000, sys=i,
                           stop="err_ref", tol=1e-10, x_ref=p.x_star)
        print(f"system {i} n={p.a.shape[1]}: {its[i]} vs oracle {io.iterations}",
              flush=True)
        assert abs(its[i] - io.iterations) <= 1
    s.close()


def rounded_f32(a):
    """The matrix with its values rounded to FP32 (what FP32 storage holds),
    as FP64: the system the mixed form solves exactly."""
    a = a.copy()
    a.data = a.data.astype(np.float32).astype(np.float64)
    return a


def test_batch_mixed_refinement(rg):
    # FP32 storage: the planted solutions belong to the FP32-rounded values
    ps = workloads.laplacian_batch(count=8, n_min=500, n_max=5000, seed=23)
    mats = [rounded_f32(p.a) for p in ps]
    csr, ro, co = batch_tensors([SimpleNamespace(a=a) for a in mats])
    b = np.concatenate([a @ p.x_star for a, p in zip(mats, ps)])
    xs = np.concatenate([p.x_star for p in ps])
    csr32 = (csr[0], csr[1], csr[2].to(torch.float32))
    s = rg.BatchSolver(csr32, ro, co, eta=0.1, stop="err_ref", tol=1e-10,
                       max_iter=20000, inner_max=200, precision="mixed_f32")
    x, info = s.solve(dev(b), x_ref=dev(xs))
    its, met, conv = s.batch_info()
    print("batch mixed", info, flush=True)
    assert info["converged"] == 1 and all(conv)
    x = x.cpu().numpy()
    for i, p in enumerate(ps):
        assert rel(x[co[i]:co[i + 1]], p.x_star) <= 1e-10
    s.close()


def test_batch_rejects_coupled_rows(rg):
    ps = workloads.laplacian_batch(count=2, n_min=50, n_max=80, seed=24)
    (rp, ci, v), ro, co = batch_tensors(ps)
    ci = ci.clone()
    ci[0] = co[1]          # row of system 0 pointing into system 1
    ci_sorted_ok = ci      # first entry of the row: still increasing
    with pytest.raises(rg.RgdbekError) as ei:
        rg.BatchSolver((rp, ci_sorted_ok, v), ro, co, eta=0.1)
    assert ei.value.status == 1


# ------------------------------------------------------------ many RHS
# R = 6 takes the per-right-hand-side products; 20 and 70 the interleaved
# ones (one group of 64 lanes with idle lanes; a full group and a ragged
# one).  One CG runs over the block-diagonal system of all right-hand
# sides, so its spectrum is the union of theirs: the power-law matrix (some
# row blocks singular) needs about 2000 steps per row projection at 20
# right-hand sides, and the 70-RHS case takes a well-conditioned matrix.
@pytest.mark.parametrize("R", [6, 20, 70])
def test_multirhs_trajectory_per_rhs(rg, R):
    if R < 70:
        a = workloads.sparse_powerlaw(3000, 1500, mean_len=10, max_len=100,
                                      seed=31).a
    else:
        a = workloads.sparse_uniform(1200, 400, density=0.03, seed=32).a
    m, n = a.shape
    rng = np.random.default_rng(1)
    xs = rng.standard_normal((R, n))
    bs = np.stack([a @ x for x in xs])
    s = rg.MultiRhsSolver(csr_tensors(a), a.shape, R, eta=0.1,
                          stop="none", max_iter=3,
                          inner_max=1500 if R < 16 else 4096, graph_iters=1)
    x, info = s.solve(dev(bs.ravel()))
    x = x.cpu().numpy().reshape(R, n)
    for r in range(R):
        xo, _, _ = rgdbek(a, bs[r], eta=0.1, max_iter=3, sys=r)
        print(f"rhs {r} rel={rel(x[r], xo):.2e}", flush=True)
        assert rel(x[r], xo) <= TRAJ_TOL
    s.close()


def tikhonov_blur(npix, mu):
    import scipy.sparse as sp
    a = workloads.blur_operator(npix=npix, dtype=np.float64)
    n = a.shape[0]
    return sp.vstack([a, np.sqrt(mu) * sp.identity(n)]).tocsr()


@pytest.mark.parametrize("R", [8, 20])
@pytest.mark.parametrize("precision", ["fp64", "mixed_f32"])
def test_multirhs_blur_tikhonov_solution(rg, precision, R):
    npix, mu = 32, 1e-2
    aa = tikhonov_blur(npix, mu)
    if precision == "mixed_f32":
        aa = rounded_f32(aa)      # FP32 storage: solve the rounded system
    n = npix * npix
    xt = workloads.generators.smooth_fields(npix, R, seed=5, corr=3.0).T
    bs = np.stack([np.concatenate([aa[:n] @ x, np.zeros(n)]) for x in xt])
    xls = np.stack([np.linalg.lstsq(aa.toarray(), b, rcond=None)[0] for b in bs])
    rp, ci, v = csr_tensors(aa)
    if precision == "mixed_f32":
        v = v.to(torch.float32)
    s = rg.MultiRhsSolver((rp, ci, v), aa.shape, R, eta=0.1, stop="err_ref",
                          tol=1e-10, max_iter=20000, inner_max=200,
                          precision=precision)
    x, info = s.solve(dev(bs.ravel()), x_ref=dev(xls.ravel()))
    its, met, conv = s.batch_info()
    print(f"blur {precision}", info, its, flush=True)
    assert info["converged"] == 1 and all(conv)
    x = x.cpu().numpy().reshape(R, n)
    for r in range(R):
        assert rel(x[r], xls[r]) <= 1e-10
    s.close()


@pytest.mark.parametrize("R", [3, 17])
def test_multirhs_gradient_layer(rg, R):
    # differentiable deblurring layer: x_s = A^+ b_s for every right-hand
    # side, loss L = sum_s <c_s, x_s>; dL/db and dL/dA (pattern, summed over
    # right-hand sides) against the pinv reference and central differences
    from oracle.refsol import grad_reference
    npix, mu = 16, 1e-2
    aa = tikhonov_blur(npix, mu)
    m, n = aa.shape
    rng = np.random.default_rng(7)
    bs = rng.standard_normal((R, m))
    cs = rng.standard_normal((R, n))
    rp, ci, v = csr_tensors(aa)
    v = v.requires_grad_(True)
    b_t = dev(bs.ravel()).requires_grad_(True)
    s = rg.MultiRhsSolver((rp, ci, v.detach()), aa.shape, R, eta=0.2,
                          stop="res_ext", tol=1e-13, max_iter=20000,
                          inner_max=200)
    x = rg.solve(s, v, b_t, least_squares=True)
    (x * dev(cs.ravel())).sum().backward()
    ad = aa.toarray()
    rows = np.repeat(np.arange(m), np.diff(aa.indptr))
    da_want = np.zeros(aa.nnz)
    db_want = []
    for r in range(R):
        da, db = grad_reference(ad, bs[r], cs[r])
        da_want += da[rows, aa.indices]
        db_want.append(db)
    assert rel(b_t.grad.cpu().numpy(), np.concatenate(db_want)) <= 1e-9
    assert rel(v.grad.cpu().numpy(), da_want) <= 1e-9
    # central differences on three stored entries
    h = 1e-6
    for e in [0, aa.nnz // 2, aa.nnz - 1]:
        vals = []
        for sgn in (1, -1):
            a2 = aa.copy()
            a2.data[e] += sgn * h
            vals.append(sum(cs[r] @ np.linalg.lstsq(a2.toarray(), bs[r], rcond=None)[0]
                            for r in range(R)))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - v.grad[e].item()) <= 1e-6 * max(1.0, abs(fd))
    s.close()


@pytest.mark.parametrize("R", [5, 16, 20, 64, 70])
def test_multirhs_apply(rg, R):
    # (A x_s, A^T z_s) for every right-hand side in one residual pass, FP64
    # and (on a mixed handle) FP32, against the products done one by one
    p = workloads.sparse_powerlaw(2000, 900, mean_len=12, max_len=300, seed=33)
    a = p.a
    m, n = a.shape
    rng = np.random.default_rng(2)
    xs = rng.standard_normal((R, n))
    zs = rng.standard_normal((R, m))
    for prec, form, tol in (("f64", "fp64", 1e-13), ("f32", "mixed_f32", 1e-5)):
        rp, ci, v = csr_tensors(a)
        s = rg.MultiRhsSolver((rp, ci, v), (m, n), R, eta=0.1, precision=form)
        dt = torch.float64 if prec == "f64" else torch.float32
        ax, atz = s.apply(dev(xs.ravel()).to(dt), dev(zs.ravel()).to(dt),
                          precision=prec)
        torch.cuda.synchronize()
        ax = ax.double().cpu().numpy().reshape(R, m)
        atz = atz.double().cpu().numpy().reshape(R, n)
        for r in range(R):
            assert rel(ax[r], a @ xs[r]) <= tol, (prec, r)
            assert rel(atz[r], a.T @ zs[r]) <= tol, (prec, r)
        s.close()


# ------------------------------------------------------------ GDBEK sets
def threshold_cases():
    rng = np.random.default_rng(40)
    yield "random", rng.random(1000) ** 3, 0.5, None
    e = rng.random(9000)
    e[rng.random(9000) < 0.7] = 0.0
    e[::17] = 0.25 * e.max()            # ties exactly at the threshold
    yield "ties_at_threshold", e, 0.25, None
    yield "all_zero", np.zeros(300), 0.5, None
    yield "eta_one", rng.random(5000), 1.0, None
    big = rng.random(300_000) ** 8
    yield "multi_block", big, 0.01, None
    yield "capped", rng.random(20_000), 0.1, 1000


@pytest.mark.parametrize("case", list(threshold_cases()), ids=lambda c: c[0])
def test_select_threshold_bit_exact(rg, case):
    from oracle.select import select_threshold as othr
    name, eps, eta, cap = case
    got = rg.select_threshold(dev(eps), eta, cap).cpu().numpy().astype(np.int64)
    want = othr(eps, eta)
    if cap is not None:
        want = want[:cap]
    assert np.array_equal(got, want), name


@pytest.mark.parametrize("kind", ["dense_c1", "dense_ls", "sparse"])
def test_gdbek_trajectory(rg, kind):
    # GDBEK's greedy sets (Section 2) on the same kernels: iterates equal
    # the oracle's with the same threshold
    if kind == "dense_c1":
        p = workloads.dense_consistent(500, 250, seed=0)
        s = rg.Solver(dev(p.a), eta=0.5, select="greedy", stop="none",
                      max_iter=4, inner_max=500)
    elif kind == "dense_ls":
        p = workloads.dense_least_squares(1200, 300, seed=41)
        s = rg.Solver(dev(p.a), eta=0.3, select="greedy", stop="none",
                      max_iter=4, inner_max=500)
    else:
        p = workloads.sparse_uniform(3000, 1500, density=0.01, seed=42)
        s = rg.Solver(csr=csr_tensors(p.a), shape=p.a.shape, eta=0.5,
                      select="greedy", stop="none", max_iter=4, inner_max=500)
    x, _ = s.solve(dev(p.b))
    z = s.get_z().cpu().numpy()
    s.close()
    xo, zo, _ = rgdbek(p.a, p.b, greedy=0.5 if kind != "dense_ls" else 0.3,
                       max_iter=4)
    print(f"gdbek {kind}: rel_x {rel(x.cpu().numpy(), xo):.2e} rel_z {rel(z, zo):.2e}",
          flush=True)
    assert rel(x.cpu().numpy(), xo) <= TRAJ_TOL
    assert rel(z, zo) <= TRAJ_TOL


def test_gdbek_solution_and_batch_rejected(rg):
    p = workloads.dense_consistent(500, 250, seed=0)
    s = rg.Solver(dev(p.a), eta=0.5, select="greedy", stop="err_ref",
                  tol=1e-10, max_iter=2000, inner_max=500)
    x, info = s.solve(dev(p.b), x_ref=dev(p.x_star))
    s.close()
    xo, _, io = rgdbek(p.a, p.b, greedy=0.5, max_iter=2000, stop="err_ref",
                       tol=1e-10, x_ref=p.x_star)
    print("gdbek solve", info, io.iterations, flush=True)
    assert info["converged"] == 1
    assert rel(x.cpu().numpy(), p.x_star) <= 1e-10
    assert abs(info["iterations"] - io.iterations) <= 1
    ps = workloads.laplacian_batch(count=2, n_min=50, n_max=80, seed=24)
    csr, ro, co = batch_tensors(ps)
    with pytest.raises(rg.RgdbekError) as ei:
        rg.BatchSolver(csr, ro, co, eta=0.5, select="greedy")
    assert ei.value.status == 6


# ------------------------------------------------------------ Lemma 2.1 law
def block_law_cases():
    rng = np.random.default_rng(50)
    yield "random", rng.random(1000) ** 3, 100
    yield "s1", rng.random(777), 1
    yield "all_zero", np.zeros(500), 10
    yield "s_ge_d", rng.random(50) + 0.1, 80
    one = np.zeros(3000)
    one[1234] = 2.0
    yield "one_positive", one, 40
    yield "persistent", rng.random(70_000) ** 2, 5000


@pytest.mark.parametrize("case", list(block_law_cases()), ids=lambda c: c[0])
def test_select_block_law_bit_exact(rg, case):
    from oracle.select import select_block_law as obl
    name, eps, s = case
    for (seed, it, phase, sys, key1) in [(0, 0, 0, 0, 0), (99, 5, 1, 2, 1)]:
        got = rg.select_block_law(dev(eps), s, seed=seed, it=it, phase=phase,
                                  sys=sys, key1=key1).cpu().numpy()
        want = obl(eps, s, seed, it, phase, sys, key1)
        assert np.array_equal(got.astype(np.int64), want), name


def test_block_law_trajectory(rg):
    # RGDBEK iterations with the blocks drawn from the law of Lemma 2.1
    p = workloads.dense_least_squares(2000, 500, seed=51)
    s = rg.Solver(dev(p.a), k_col=100, k_row=200, select="block_law",
                  stop="none", max_iter=4, inner_max=300)
    x, _ = s.solve(dev(p.b))
    z = s.get_z().cpu().numpy()
    s.close()
    xo, zo, _ = rgdbek(p.a, p.b, k_col=100, k_row=200, max_iter=4,
                       block_law=True)
    print(f"block law: rel_x {rel(x.cpu().numpy(), xo):.2e} rel_z {rel(z, zo):.2e}",
          flush=True)
    assert rel(x.cpu().numpy(), xo) <= TRAJ_TOL
    assert rel(z, zo) <= TRAJ_TOL


# ------------------------------------------------- finite-element systems
@pytest.mark.parametrize("sparse_cg", [False, True], ids=["gram", "cg"])
@pytest.mark.parametrize("npts,k,mode", [(25, 0.0, 1), (50, 25.0, 4)],
                         ids=["poisson", "helmholtz"])
def test_fem_trajectory(rg, npts, k, mode, sparse_cg):
    # Section 6's FEM systems at eta = 0.5 (313 / 1250 of 625 / 2500
    # columns and rows): symmetric, boundary identity rows, and right-hand
    # sides that vanish on the boundary (zero weights that are never drawn)
    A, b, u, xy = workloads.fem_p1_unit_square(npts, k, mode)
    p = SimpleNamespace(a=A, b=b)
    kc = kr = int(np.floor(0.5 * A.shape[0] + 0.5))
    x, z, info, xo, zo = run_both(rg, p, kc, kr, 4, sparse=True,
                                  inner_max=2000, sparse_cg=sparse_cg)
    print(f"fem npts={npts} k={k} cg={sparse_cg} rel_x={rel(x, xo):.3e} rel_z={rel(z, zo):.3e}", flush=True)
    assert rel(x, xo) <= TRAJ_TOL
    assert rel(z, zo) <= TRAJ_TOL


# ------------------------------------------------- draws with replacement
def iid_cases():
    rng = np.random.default_rng(60)
    yield "random", rng.random(1000) ** 4, 500
    e = rng.random(5000)
    e[rng.random(5000) < 0.7] = 0.0
    yield "zero_heavy", e, 3000
    yield "ties", np.repeat([0.5, 1.0, 2.0], [300, 300, 400]), 700
    yield "k1", rng.random(777), 1
    yield "k_gt_d", rng.random(300) + 0.1, 2000
    yield "one_weight", np.eye(1, 97, 13).ravel(), 5
    yield "all_zero", np.zeros(400), 30
    yield "denormal", np.full(200, 5e-324), 17
    yield "chunk_edge", rng.random(4097), 4097
    yield "multi_chunk", rng.random(300_000) ** 3, 100_000
    big = rng.random(1_000_000)
    big[rng.random(1_000_000) < 0.5] = 0.0
    yield "rows_1e6", big, 250_000


@pytest.mark.parametrize("case", list(iid_cases()), ids=lambda c: c[0])
def test_select_iid_bit_exact(rg, case):
    from oracle.select import select_iid as oiid
    name, eps, k = case
    print(f"iid case {name} d={eps.size} k={k}", flush=True)
    for (seed, it, phase, sys, key1, floor) in [(0, 0, 0, 0, 0, 1e-20),
                                                (77, 9, 1, 3, 1, 0.0)]:
        got = rg.select_iid(dev(eps), k, seed=seed, it=it, phase=phase,
                            sys=sys, key1=key1, floor=floor).cpu().numpy()
        want = oiid(eps, k, seed, it, phase, sys, key1, floor)
        assert np.array_equal(got.astype(np.int64), want), name


def test_select_iid_size_limit(rg):
    # the largest supported dimension (4096 chunks of 4096 weights) draws
    # bit-exactly; one more weight is rejected
    from oracle.select import select_iid as oiid
    d = 4096 * 4096
    eps = np.random.default_rng(63).random(d) ** 2
    got = rg.select_iid(dev(eps), 100_000, seed=5, it=2).cpu().numpy()
    assert np.array_equal(got.astype(np.int64), oiid(eps, 100_000, 5, 2, 0))
    with pytest.raises(rg.RgdbekError) as ei:
        rg.select_iid(torch.zeros(d + 1, dtype=torch.float64, device="cuda"), 10)
    assert ei.value.status == 1


def test_iid_trajectories(rg):
    # dense least squares and sparse uniform, blocks drawn with replacement
    p = workloads.dense_least_squares(2000, 500, seed=61)
    s = rg.Solver(dev(p.a), k_col=120, k_row=300, select="iid", stop="none",
                  max_iter=4, inner_max=300)
    x, _ = s.solve(dev(p.b))
    z = s.get_z().cpu().numpy()
    s.close()
    xo, zo, _ = rgdbek(p.a, p.b, k_col=120, k_row=300, max_iter=4, iid=True)
    print(f"iid dense: rel_x {rel(x.cpu().numpy(), xo):.2e} rel_z {rel(z, zo):.2e}", flush=True)
    assert rel(x.cpu().numpy(), xo) <= TRAJ_TOL
    assert rel(z, zo) <= TRAJ_TOL
    p = workloads.sparse_uniform(3000, 1500, density=0.01, seed=62)
    s = rg.Solver(csr=csr_tensors(p.a), shape=p.a.shape, k_col=150, k_row=300,
                  select="iid", stop="none", max_iter=4, inner_max=300)
    x, _ = s.solve(dev(p.b))
    z = s.get_z().cpu().numpy()
    s.close()
    xo, zo, _ = rgdbek(p.a, p.b, k_col=150, k_row=300, max_iter=4, iid=True)
    print(f"iid sparse: rel_x {rel(x.cpu().numpy(), xo):.2e} rel_z {rel(z, zo):.2e}", flush=True)
    assert rel(x.cpu().numpy(), xo) <= TRAJ_TOL
    assert rel(z, zo) <= TRAJ_TOL


def test_iid_table_iteration_counts(rg):
    # Tables 1 and 2 (sparse 1% random, eta = 0.5, RSE <= 1e-6): with draws
    # with replacement the GPU solver needs the paper's iteration counts
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden",
                           "paper_iteration_counts.json")) as f:
        gold = json.load(f)
    for m, n, ref in ((8000, 500, gold["tall_8000_rows"]["500"]),
                      (8000, 1000, gold["tall_8000_rows"]["1000"]),
                      (500, 8000, gold["fat_8000_columns"]["500"]),
                      (1000, 8000, gold["fat_8000_columns"]["1000"])):
        its = []
        for seed in range(3):
            p = workloads.sparse_uniform(m, n, density=0.01, seed=seed)
            s = rg.Solver(csr=csr_tensors(p.a), shape=(m, n), eta=0.5,
                          select="iid", stop="rse", tol=1e-6, max_iter=1000,
                          seed=seed)
            _, info = s.solve(dev(p.b))
            s.close()
            assert info["converged"] == 1
            its.append(info["iterations"])
        print(f"iid {m}x{n}: {its} paper {ref}", flush=True)
        assert abs(np.mean(its) - ref) <= 0.1 * ref


# ------------------------------------------------ sparse CG step variants
@pytest.mark.parametrize("kind", ["uniform", "powerlaw"])
def test_sparse_split_cg_finish(rg, kind):
    # the many-workgroup CG step finish (taken by blocks above 16384
    # indices) forced on blocks the oracle can check; the power-law matrix
    # has rows above the long-segment limit in both CG products
    if kind == "uniform":
        p = workloads.sparse_uniform(3000, 1500, density=0.01, seed=3)
        kc, kr, imax = 150, 300, 200
    else:
        p = workloads.sparse_powerlaw(6000, 3000, mean_len=10, max_len=400,
                                      seed=4)
        kc, kr, imax = 300, 600, 1000
    x, z, info, xo, zo = run_both(rg, p, kc, kr, 3, sparse=True,
                                  inner_max=imax, cg_split=True,
                                  sparse_cg=True)
    print(f"split cg {kind}: rel_x={rel(x, xo):.3e} rel_z={rel(z, zo):.3e}", flush=True)
    assert rel(x, xo) <= TRAJ_TOL
    assert rel(z, zo) <= TRAJ_TOL


# ------------------------------------------------ block rules in FP32
@pytest.mark.parametrize("select", ["greedy", "block_law", "iid"])
def test_block_rules_mixed_precision(rg, select):
    # the other block rules inside the FP32 inner iterations (their float
    # kernels) still refine to the FP64 least-squares solution
    p = workloads.dense_least_squares(2000, 500, seed=64)
    kw = dict(eta=0.5) if select == "greedy" else dict(k_col=150, k_row=300)
    s = rg.Solver(dev(p.a), precision="mixed_f32", select=select,
                  stop="err_ref", tol=1e-10, max_iter=20000, **kw)
    x, info = s.solve(dev(p.b), x_ref=dev(p.x_star))
    s.close()
    print(f"mixed {select}: {info}", flush=True)
    assert info["converged"] == 1
    assert rel(x.cpu().numpy(), p.x_star) <= 1e-10


@pytest.mark.parametrize("sparse_cg", [False, True], ids=["gram", "cg"])
def test_block_law_sparse_trajectory(rg, sparse_cg):
    # Lemma 2.1 blocks on a sparse matrix, both small-system projections
    p = workloads.sparse_uniform(3000, 1500, density=0.01, seed=65)
    s = rg.Solver(csr=csr_tensors(p.a), shape=p.a.shape, k_col=150,
                  k_row=300, select="block_law", stop="none", max_iter=3,
                  inner_max=300, sparse_cg=sparse_cg)
    x, _ = s.solve(dev(p.b))
    z = s.get_z().cpu().numpy()
    s.close()
    xo, zo, _ = rgdbek(p.a, p.b, k_col=150, k_row=300, max_iter=3,
                       block_law=True)
    print(f"block law sparse cg={sparse_cg}: rel_x {rel(x.cpu().numpy(), xo):.2e} rel_z {rel(z, zo):.2e}", flush=True)
    assert rel(x.cpu().numpy(), xo) <= TRAJ_TOL
    assert rel(z, zo) <= TRAJ_TOL
