"""Closed-form references -- oracle side.

Theorem 2.3 (Section 2) names the limits RGDBEK converges to: the
minimum-norm solution x* = A^+ b and the optimal residual r = (I - A A^+) b,
which the auxiliary vector z tracks.  These are computed here directly from
the SVD pseudoinverse (``numpy.linalg.pinv``) for small systems.

Differentiation (not part of the paper): for A of full column rank the map
(A, b) -> x = A^+ b has the implicit gradient, for a loss L with
gx = dL/dx,
    w = (A^T)^+ gx = A (A^T A)^{-1} gx          (= dL/db)
    lam = A^+ w = (A^T A)^{-1} gx
    dL/dA = r lam^T - w x^T,    r = b - A x,
obtained by differentiating x = (A^T A)^{-1} A^T b.  For a consistent system
r = 0 and the first term drops.  ``grad_via_solves`` computes the same
quantities with two runs of the oracle solver (the adjoint system A^T w = gx,
then A lam = w) so that a GPU gradient can be compared with either.

Deblurring with Tikhonov rows (Section 6's deblurring problem, solved as
the least-squares system [A; s I] x ~= [b; 0]): for a separable blur
A = T kron T with symmetric T = Q diag(lam) Q^T the normal equations
(A^T A + s^2 I) x = A^T b diagonalise in the basis Q kron Q, so the
solution is written out directly (``tikhonov_kron``).  The same basis
gives the adjoint quantities of the differentiable layer: for a loss with
dL/dx = c, lam = (A^T A + s^2 I)^{-1} c (``tikhonov_kron_lam``), from which
w = [A; s I] lam = dL/db and dL/dA = r lam^T - w x^T follow as above.

Test infrastructure only (see the package docstring).
"""
import numpy as np
import scipy.sparse as sp

from .rgdbek import rgdbek


def pinv_solution(a):
    """(x*, r) as functions of b for a small dense matrix: returns a
    callable b -> (A^+ b, (I - A A^+) b)."""
    a = np.asarray(a, dtype=np.float64)
    p = np.linalg.pinv(a)

    def apply(b):
        x = p @ b
        return x, b - a @ x
    return apply


def grad_reference(a, b, gx):
    """Dense pinv reference of (dL/dA, dL/db) for L with dL/dx = gx."""
    a = np.asarray(a, dtype=np.float64)
    p = np.linalg.pinv(a)
    x = p @ b
    r = b - a @ x
    w = p.T @ gx
    lam = p @ w
    return np.outer(r, lam) - np.outer(w, x), w


def grad_via_solves(a, b, gx, x, *, k_col, k_row, max_iter, seed=0, tol=1e-13,
                    least_squares=True):
    """(dA restricted to A's pattern, w, lam) from two oracle RGDBEK solves.

    The adjoint solve runs Algorithm 1 on A^T (n x m) with right-hand side
    gx and key word 1 = 1; the second solve runs on A with right-hand side w.
    Returns dA as a dense array for dense A and as the values of A's stored
    entries (CSR order) for sparse A."""
    at = a.T.tocsr() if sp.issparse(a) else np.ascontiguousarray(a.T)
    w, _, _ = rgdbek(at, gx, k_col=k_row, k_row=k_col, max_iter=max_iter,
                     seed=seed, key1=1, stop="res_ext", tol=tol)
    r = b - a @ x
    if least_squares:
        lam, _, _ = rgdbek(a, w, k_col=k_col, k_row=k_row, max_iter=max_iter,
                           seed=seed, key1=1, stop="res_ext", tol=tol)
    else:
        lam = np.zeros_like(x)
    if sp.issparse(a):
        c = sp.csr_matrix(a)
        c.sort_indices()
        rows = np.repeat(np.arange(c.shape[0]), np.diff(c.indptr))
        cols = c.indices
        da = r[rows] * lam[cols] - w[rows] * x[cols]
    else:
        da = np.outer(r, lam) - np.outer(w, x)
    return da, w, lam


def tikhonov_kron(t, b_img, s):
    """argmin_x ||(T kron T) x - b||^2 + s^2 ||x||^2 for symmetric T (p x p)
    and one or more right-hand sides b (columns of b_img, p*p rows each,
    row-major image order, so (T kron T) vec(X) = vec(T X T)).  With
    T = Q diag(lam) Q^T, X = Q (F o (Q^T B Q)) Q^T where
    F_ij = lam_i lam_j / ((lam_i lam_j)^2 + s^2)."""
    t = np.asarray(t, dtype=np.float64)
    lam, q = np.linalg.eigh(t)
    p = t.shape[0]
    ll = np.outer(lam, lam)
    f = ll / (ll * ll + s * s)
    b_img = np.asarray(b_img, dtype=np.float64)
    single = b_img.ndim == 1
    bm = b_img.reshape(p * p, -1)
    out = np.empty_like(bm)
    for c in range(bm.shape[1]):
        bimg = np.ascontiguousarray(bm[:, c]).reshape(p, p)
        y = q.T @ bimg @ q
        out[:, c] = (q @ (f * y) @ q.T).ravel()
    return out[:, 0] if single else out


def tikhonov_kron_lam(t, c_img, s):
    """lam = ((T kron T)^T (T kron T) + s^2 I)^{-1} c for symmetric T and
    one or more vectors c (columns of c_img, row-major image order): in the
    basis Q kron Q the matrix is diagonal with entries (lam_i lam_j)^2 + s^2,
    so lam = Q (G o (Q^T C Q)) Q^T with G_ij = 1 / ((lam_i lam_j)^2 + s^2)."""
    t = np.asarray(t, dtype=np.float64)
    ev, q = np.linalg.eigh(t)
    p = t.shape[0]
    ll = np.outer(ev, ev)
    g = 1.0 / (ll * ll + s * s)
    c_img = np.asarray(c_img, dtype=np.float64)
    single = c_img.ndim == 1
    cm = c_img.reshape(p * p, -1)
    out = np.empty_like(cm)
    for k in range(cm.shape[1]):
        cimg = np.ascontiguousarray(cm[:, k]).reshape(p, p)
        y = q.T @ cimg @ q
        out[:, k] = (q @ (g * y) @ q.T).ravel()
    return out[:, 0] if single else out
