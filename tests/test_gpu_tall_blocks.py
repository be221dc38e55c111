"""Row blocks taller than A is wide (k_row > n), the paper's own setting on
tall systems (Algorithm 1 with eta = 0.5 of Section 3: m*eta rows of an
m x n matrix with m > 2n).  Such a block is generally inconsistent (r^J need
not lie in range(A^J)); the HIP path projects it by CGLS, whose limit is the
pseudoinverse update (A^J)^+ r^J the oracle applies exactly (SVD).  Parity:
iterates within 1e-10 of the oracle after a fixed number of iterations, dense
and sparse, FP64; the mixed form reaches the planted solution; blocks above
the Gram limit run (dense rows only) and the adjoint reports what it cannot
serve."""
import numpy as np
import pytest
import torch

import workloads
from oracle.rgdbek import rgdbek

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
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


def run_both(rg, p, k_col, k_row, iters, seed=0, sparse=False, **kw):
    if sparse:
        s = rg.Solver(csr=csr_tensors(p.a), shape=p.a.shape, k_col=k_col,
                      k_row=k_row, stop="none", max_iter=iters, seed=seed,
                      inner_max=400, graph_iters=1, **kw)
    else:
        s = rg.Solver(dev(p.a), k_col=k_col, k_row=k_row, stop="none",
                      max_iter=iters, seed=seed, inner_max=400, graph_iters=1,
                      **kw)
    x, info = s.solve(dev(p.b))
    z = s.get_z().cpu().numpy()
    s.close()
    xo, zo, _ = rgdbek(p.a, p.b, k_col=k_col, k_row=k_row, max_iter=iters,
                       seed=seed)
    return x.cpu().numpy(), z, info, xo, zo


@pytest.mark.parametrize("kc,kr", [(100, 1000), (250, 1500), (37, 750)])
def test_trajectory_dense_tall_rows(rg, kc, kr):
    # least squares (b has a component in null(A^T)), 2000 x 500
    p = workloads.dense_least_squares(2000, 500, seed=41)
    x, z, info, xo, zo = run_both(rg, p, kc, kr, 3, seed=2)
    print(f"tall dense kc={kc} kr={kr} rel_x={rel(x, xo):.3e} "
          f"rel_z={rel(z, zo):.3e}", flush=True)
    assert info["iterations"] == 3
    assert rel(x, xo) <= TRAJ_TOL
    assert rel(z, zo) <= TRAJ_TOL


def test_trajectory_dense_tall_rows_eta_half(rg):
    # Section 3's setting on a tall system: eta = 0.5 on 4000 x 1000
    p = workloads.dense_consistent(4000, 1000, seed=42)
    x, z, info, xo, zo = run_both(rg, p, 500, 2000, 2, seed=1)
    print(f"tall dense eta=0.5 rel_x={rel(x, xo):.3e} rel_z={rel(z, zo):.3e}",
          flush=True)
    assert rel(x, xo) <= TRAJ_TOL
    assert rel(z, zo) <= TRAJ_TOL


@pytest.mark.parametrize("iters", [1, 3])
def test_trajectory_sparse_tall_rows(rg, iters):
    # the sprandn-like 8000 x 500 matrix of Table 2 at eta = 0.5: blocks of
    # 250 columns and 4000 rows (eight times the width)
    p = workloads.sparse_uniform(8000, 500, density=0.01, seed=43)
    x, z, info, xo, zo = run_both(rg, p, 250, 4000, iters, seed=3,
                                  sparse=True)
    print(f"tall sparse iters={iters} rel_x={rel(x, xo):.3e} "
          f"rel_z={rel(z, zo):.3e}", flush=True)
    assert rel(x, xo) <= TRAJ_TOL
    assert rel(z, zo) <= TRAJ_TOL


def test_sparse_tall_rows_rse_iterations(rg):
    # to RSE <= 1e-6 as in Table 2: same iteration count as the oracle (+-1)
    p = workloads.sparse_uniform(8000, 500, density=0.01, seed=44)
    s = rg.Solver(csr=csr_tensors(p.a), shape=p.a.shape, eta=0.5, stop="rse",
                  tol=1e-6, max_iter=500, inner_max=400)
    x, info = s.solve(dev(p.b))
    s.close()
    xo, _, io = rgdbek(p.a, p.b, eta=0.5, max_iter=500, stop="rse", tol=1e-6)
    print(f"tall sparse rse: gpu {info['iterations']} oracle {io.iterations}",
          flush=True)
    assert info["converged"] == 1
    assert abs(info["iterations"] - io.iterations) <= 1
    assert rel(x.cpu().numpy(), xo) <= 1e-8


def test_mixed_tall_rows_res_ext(rg):
    p = workloads.dense_least_squares(2000, 500, seed=45)
    s = rg.Solver(dev(p.a), k_col=100, k_row=1000, precision="mixed_f32",
                  stop="res_ext", tol=1e-12, max_iter=20000, inner_max=100)
    x, info = s.solve(dev(p.b))
    s.close()
    print("tall mixed", info, flush=True)
    assert info["converged"] == 1
    assert rel(x.cpu().numpy(), p.x_star) <= 1e-10


def test_dense_rows_above_gram_limit(rg):
    # 9000 x 100 with 8500-row blocks: beyond the Gram staging limit, served
    # by CGLS; the adjoint (whose column blocks these are) is refused
    p = workloads.dense_consistent(9000, 100, seed=46)
    x, z, info, xo, zo = run_both(rg, p, 50, 8500, 2, seed=4)
    print(f"rows above limit rel_x={rel(x, xo):.3e} rel_z={rel(z, zo):.3e}",
          flush=True)
    assert rel(x, xo) <= TRAJ_TOL
    assert rel(z, zo) <= TRAJ_TOL
    s = rg.Solver(dev(p.a), k_col=50, k_row=8500, stop="res_ext", tol=1e-10,
                  max_iter=100)
    with pytest.raises(rg.RgdbekError) as ei:
        s.solve_adjoint(dev(np.ones(100)))
    assert ei.value.status == 6
    s.close()
    with pytest.raises(rg.RgdbekError) as ei:
        rg.Solver(dev(workloads.dense_consistent(100, 9000, seed=47).a),
                  k_col=8500, k_row=50)
    assert ei.value.status == 6
