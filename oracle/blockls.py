"""Block projections of RGDBEK -- oracle side.

The update rule RGDBEK takes over from GDBEK (Section 1, the GDBEK update
equation; Algorithm 1, the two "Update" steps):

    z_{k+1} = z_k - A_U A_U^+ z_k
    x_{k+1} = x_k + (A^J)^+ (b^J - z_{k+1}^J - A^J x_k)

with ^+ the Moore-Penrose pseudoinverse.  Both are minimum-norm least-squares
solves on a block: y = A_U^+ z_k minimises ||A_U y - z_k|| with least norm,
and the row correction d = (A^J)^+ r^J minimises ||A^J d - r^J|| with least
norm.  The paper solves these with LSQR (Section 3, remark on the inner
solver) and states no tolerance; the definition is the pseudoinverse, so the
oracle applies it exactly:

* dense blocks, and sparse blocks up to 4096 in both dimensions: LAPACK
  gelsd through ``numpy.linalg.lstsq`` (SVD, minimum norm);
* larger sparse blocks: ``scipy.sparse.linalg.lsqr`` started at zero
  (which converges to the minimum-norm solution) with tolerances at the
  FP64 floor; the reached residual of the normal equations is returned.

Test infrastructure only (see the package docstring).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

DENSE_LIMIT = 4096


def _is_sparse(a):
    return sp.issparse(a)


def pinv_apply(block, rhs):
    """Minimum-norm least-squares solution of block @ y ~= rhs.

    Returns (y, normal_residual) where normal_residual =
    ||block^T (block y - rhs)|| / (||block||_F^2 ||y|| + ||block^T rhs||),
    a scale-free measure of how well the projection was applied."""
    rhs = np.asarray(rhs, dtype=np.float64)
    rows, cols = block.shape
    if rows == 0 or cols == 0:
        return np.zeros(cols), 0.0
    if not _is_sparse(block):
        y = np.linalg.lstsq(np.asarray(block, dtype=np.float64), rhs,
                            rcond=None)[0]
    elif max(rows, cols) <= DENSE_LIMIT:
        y = np.linalg.lstsq(block.toarray(), rhs, rcond=None)[0]
    else:
        out = spla.lsqr(sp.csr_matrix(block), rhs, damp=0.0, atol=1e-16,
                        btol=1e-16, conlim=1e20,
                        iter_lim=20 * max(rows, cols), show=False)
        y = out[0]
    res = block @ y - rhs
    nr = np.linalg.norm(block.T @ res)
    if _is_sparse(block):
        fro2 = float(block.multiply(block).sum())
    else:
        fro2 = float(np.sum(np.asarray(block) ** 2))
    scale = fro2 * np.linalg.norm(y) + np.linalg.norm(block.T @ rhs)
    return y, (nr / scale if scale > 0 else 0.0)


def column_projection(a_u, z):
    """z_{k+1} = z_k - A_U A_U^+ z_k.  Returns (z_next, y, normal_residual)."""
    y, nr = pinv_apply(a_u, z)
    return z - a_u @ y, y, nr


def column_projection_offset(a_u, dz, t_u):
    """Column update of the refinement's correction system.

    The refinement pass (FP64 x, correction (dx, dz) from (0, 0)) runs
    Algorithm 1 on the full residual s + dz with s = b - A x, which it knows
    only through t = A^T s.  The column update of Algorithm 1 applied to it,
    s + dz -> (I - A_U A_U^+)(s + dz), changes dz by -A_U y with
    y = A_U^+ (s + dz) = (A_U^T A_U)^+ (A_U^T dz + t_U).  Any v with
    A_U^T v = t_U inside range(A_U) gives the same y as s; the minimum-norm
    solution of A_U^T v = t_U is one (t_U lies in range(A_U^T)).
    Returns (dz_next, y, normal_residual)."""
    v, _ = pinv_apply(a_u.T, t_u)
    y, nr = pinv_apply(a_u, dz + v)
    return dz - a_u @ y, y, nr


def row_projection(a_j, r_j):
    """d = (A^J)^+ r^J, the correction added to x.  Returns (d, residual)."""
    d, nr = pinv_apply(a_j, r_j)
    return d, nr
