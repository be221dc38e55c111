"""Algorithm 1 of the paper (RGDBEK), iterated step by step in FP64 -- oracle.

Per iteration k (Section 2, Algorithm 1; update rule of GDBEK, Section 1):

  column phase
    eps^z_j = |A_(j)^T z_k|^2 / ||A_(j)||^2          (column residuals)
    U_k     = block of k_col columns drawn with P(j) proportional to eps^z
    z_{k+1} = z_k - A_U A_U^+ z_k
  row phase
    r       = b - z_{k+1} - A x_k
    eps^x_i = |r_i|^2 / ||A^(i)||^2                    (row residuals)
    J_k     = block of k_row rows drawn with P(i) proportional to eps^x
    x_{k+1} = x_k + (A^J)^+ r^J

with x_0 = 0 and z_0 = b.  Readings where the paper is silent:

* the garbled "A^J x_k^J" of the row update is A^J x_k (full x_k), as in
  the convergence proof of Theorem 2.3 and the least-squares step of
  Algorithm 2;
* a zero row or column has weight 0 (never drawn), and so has a weight
  below floor * max (zero up to rounding, see ``select``);
* an empty block (every weight zero) skips that projection, and the
  iteration still counts;
* stopping tests (the paper iterates T times in Algorithm 1 and stops on
  the squared relative residual ||Ax - b||^2/||b||^2 in Sections 3 and 5):
    'none'    run exactly max_iter iterations;
    'err_ref' ||x_k - x_ref|| <= tol ||x_ref||, tested at the top of
              iteration k (the benchmark criterion, planted solution);
    'rse'     ||b - A x_k||^2 <= tol ||b||^2, tested once A x_k is formed
              in iteration k (returns x_k);
    'res_ext' ||b - z_{k+1} - A x_k|| <= tol ||b||, tested at the same
              place (safe for least-squares problems).
* the generator coordinates of iteration k are (seed, it0 + k, phase, sys)
  with phase 0 for columns and 1 for rows; key word 1 = key1 (0 for the
  forward solve, 1 for solves on the adjoint system).

Optional ``col_offset`` t and right-hand side ``b`` make the same loop solve
the correction system of the extended-residual refinement: from an FP64
iterate x with s = b - A x and t = A^T s, Algorithm 1 runs on the
correction (dx, dz) from (0, 0) with right-hand side 0, so that s + dz
plays the role of z: the column residual becomes A^T dz + t, the column
update projects s + dz (``column_projection_offset``), and the row
residual is -dz - A dx.  Its fixed point is x + dx = A^+ b.  With t = 0 and
the true right-hand side it is Algorithm 1 unchanged.

Test infrastructure only (see the package docstring).
"""
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from .select import (select, select_threshold, select_block_law, select_iid,
                     block_size, FLOOR_FP64)
from .blockls import (column_projection, column_projection_offset,
                      row_projection)


@dataclass
class Info:
    iterations: int = 0
    converged: bool = False
    metric: float = float("nan")
    trace: list = field(default_factory=list)


def _sq_norms(a, axis):
    if sp.issparse(a):
        return np.asarray(a.multiply(a).sum(axis=axis)).ravel()
    return np.einsum("ij,ij->j" if axis == 0 else "ij,ij->i", a, a)


def _ratio(num, den):
    """num/den elementwise with 0 where den == 0 (zero rows/columns)."""
    out = np.zeros_like(num)
    nz = den > 0
    out[nz] = num[nz] / den[nz]
    return out


def column_weights(a, z, kappa, col_offset=None):
    """eps^z = (A^T z [+ t])^2 / kappa; returns (eps, g)."""
    g = a.T @ z
    if col_offset is not None:
        g = g + col_offset
    return _ratio(g * g, kappa), g


def row_weights(b, z_next, q, rho):
    """r = b - z_{k+1} - q and eps^x = r^2 / rho; returns (eps, r)."""
    r = (b - z_next) - q
    return _ratio(r * r, rho), r


def rgdbek(a, b, *, k_col=None, k_row=None, eta=None, max_iter=100, seed=0,
           stop="none", tol=0.0, x_ref=None, sys=0, key1=0, it0=0,
           x0=None, z0=None, col_offset=None, record=False,
           floor=FLOOR_FP64, greedy=None, block_law=False, iid=False):
    """Run Algorithm 1.  Returns (x, z, Info).

    a: dense (m, n) ndarray or scipy sparse matrix; b: (m,) FP64.
    Block sizes come from k_col/k_row, or from eta through ``block_size``.
    x0/z0/it0 resume a run (x_0 = 0 and z_0 = b by default).
    greedy: None for Algorithm 1's randomized draws, or a threshold in
    (0, 1] for GDBEK's greedy sets {eps_j >= greedy * max eps} (Section 2),
    with the same update rules and the same order of the two phases.
    block_law: draw the blocks from the law of Lemma 2.1 instead
    (``select_block_law``, block sizes k_col / k_row).
    iid: draw k_col / k_row indices with replacement and keep the distinct
    ones (``select_iid``)."""
    if sp.issparse(a):
        a = sp.csr_matrix(a, dtype=np.float64)
        a_csc = a.tocsc()
    else:
        a = np.asarray(a, dtype=np.float64)
        a_csc = a
    m, n = a.shape
    b = np.asarray(b, dtype=np.float64)
    if k_col is None and greedy is None:
        k_col = block_size(eta, n)
    if k_row is None and greedy is None:
        k_row = block_size(eta, m)
    rho = _sq_norms(a, 1)
    kappa = _sq_norms(a, 0)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    z = b.copy() if z0 is None else np.array(z0, dtype=np.float64)
    info = Info()
    bnorm = np.linalg.norm(b)
    if stop == "err_ref":
        rnorm = np.linalg.norm(x_ref)

    k = 0
    while True:
        if stop == "err_ref":
            info.metric = np.linalg.norm(x - x_ref) / rnorm
            if info.metric <= tol:
                info.converged = True
                break
        if k >= max_iter:
            break
        it = it0 + k
        # column phase
        eps_z, g = column_weights(a, z, kappa, col_offset)
        if greedy is not None:
            u = select_threshold(eps_z, greedy)
        elif block_law:
            u = select_block_law(eps_z, k_col, seed, it, 0, sys, key1, floor)
        elif iid:
            u = select_iid(eps_z, k_col, seed, it, 0, sys, key1, floor)
        else:
            u = select(eps_z, k_col, seed, it, 0, sys, key1, floor)
        z_prev = z
        if u.size and col_offset is not None:
            z, y, nr_c = column_projection_offset(a_csc[:, u], z,
                                                  col_offset[u])
        elif u.size:
            z, y, nr_c = column_projection(a_csc[:, u], z)
        else:
            y, nr_c = np.zeros(0), 0.0
        # row phase
        q = a @ x
        eps_x, r = row_weights(b, z, q, rho)
        if stop == "rse":
            info.metric = np.linalg.norm(b - q) ** 2 / bnorm ** 2
            if info.metric <= tol:
                info.converged = True
                break
        if stop == "res_ext":
            info.metric = np.linalg.norm(r) / bnorm
            if info.metric <= tol:
                info.converged = True
                break
        if greedy is not None:
            j = select_threshold(eps_x, greedy)
        elif block_law:
            j = select_block_law(eps_x, k_row, seed, it, 1, sys, key1, floor)
        elif iid:
            j = select_iid(eps_x, k_row, seed, it, 1, sys, key1, floor)
        else:
            j = select(eps_x, k_row, seed, it, 1, sys, key1, floor)
        x_prev = x
        if j.size:
            d, nr_r = row_projection(a[j, :], r[j])
            x = x + d
        else:
            d, nr_r = np.zeros(n), 0.0
        if record:
            info.trace.append(dict(k=k, U=u, J=j, eps_z=eps_z, eps_x=eps_x,
                                   g=g, r=r, z_prev=z_prev, z=z.copy(),
                                   x_prev=x_prev, x=x.copy(), y=y, d=d,
                                   nr_col=nr_c, nr_row=nr_r))
        k += 1
    info.iterations = k
    if stop == "none":
        info.converged = True
    return x, z, info
