"""Seeded generators for the solver's workloads.

The paper evaluates on random sparse matrices (MATLAB ``sprandn`` with
N(0,1) values in Section 3, ``scipy.sparse.rand`` in Section 5), SuiteSparse
matrices, image deblurring with a Gaussian Toeplitz blur (Section 6) and two
FEM problems.  None of those data sets are used here; these generators make
synthetic stand-ins with the shapes and structure of the workloads the
solver is measured on:

* ``dense_consistent``     dense N(0,1) A, planted x*, b = A x*;
* ``dense_least_squares``  dense N(0,1) A, b = A x* + r with r in null(A^T)
                           and ||r|| = ratio * ||A x*|| (an inconsistent
                           system whose least-squares solution is x*);
* ``sparse_powerlaw``      CSR with power-law row lengths, uniform columns,
                           N(0,1) values, unit-norm rows, consistent b;
* ``blur_operator``        2-D separable Gaussian blur (the 1-D point-spread
                           function of Section 6 in both directions), zero
                           boundary, as CSR;
* ``laplacian_batch``      many uneven 5-point Laplacian systems with a
                           random diagonal shift plus extra random rows.

Everything is drawn from ``numpy.random.default_rng(seed)``; nothing here
implements any step of the solver.
"""
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


@dataclass
class Problem:
    name: str
    a: object                  # dense ndarray (m, n) or scipy CSR
    b: np.ndarray              # (m,) or (m, nrhs)
    x_star: np.ndarray         # planted solution (n,) or (n, nrhs)
    r_perp: np.ndarray = None  # least-squares residual part of b, if any
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.a.shape


def to_csr_arrays(a, value_dtype=np.float64):
    """(row_ptr int64, col_idx int32, values) of a scipy sparse matrix,
    with column indices sorted within each row."""
    c = sp.csr_matrix(a)
    c.sort_indices()
    return (c.indptr.astype(np.int64), c.indices.astype(np.int32),
            c.data.astype(value_dtype))


def dense_consistent(m=500, n=250, seed=0):
    """Dense A with i.i.d. N(0,1) entries, x* ~ N(0,1), b = A x*."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((m, n))
    x = rng.standard_normal(n)
    return Problem(f"dense_consistent_{m}x{n}", a, a @ x, x,
                   meta=dict(seed=seed))


def _project_out_range(a, g):
    """g minus its orthogonal projection onto range(a) (full column rank),
    via the Cholesky factor of a^T a, with one correction sweep."""
    gram = a.T @ a
    ch = np.linalg.cholesky(gram)

    def solve(v):
        w = np.linalg.solve(ch, v)
        return np.linalg.solve(ch.T, w)

    r = g - a @ solve(a.T @ g)
    r = r - a @ solve(a.T @ r)
    return r


def dense_least_squares(m=20000, n=5000, seed=0, ratio=0.1):
    """Dense A with i.i.d. N(0,1) entries, x* ~ N(0,1); b = A x* + r with r a
    random N(0, I_m) vector projected onto null(A^T) and scaled to
    ratio * ||A x*||.  x* is then the least-squares solution."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((m, n))
    x = rng.standard_normal(n)
    g = rng.standard_normal(m)
    ax = a @ x
    r = _project_out_range(a, g)
    r *= ratio * np.linalg.norm(ax) / np.linalg.norm(r)
    return Problem(f"dense_least_squares_{m}x{n}", a, ax + r, x, r_perp=r,
                   meta=dict(seed=seed, ratio=ratio))


def sparse_uniform(m, n, density=0.01, seed=0):
    """Uniform random sparsity pattern with N(0,1) values, like MATLAB's
    sprandn(m, n, density) used for the random matrices of Section 3:
    round(density*m*n) distinct positions; x* ~ N(0,1), b = A x*."""
    rng = np.random.default_rng(seed)
    nnz = int(round(density * m * n))
    pos = rng.choice(m * n, size=nnz, replace=False)
    rows, cols = np.divmod(pos, n)
    vals = rng.standard_normal(nnz)
    a = sp.csr_matrix((vals, (rows, cols)), shape=(m, n))
    a.sort_indices()
    x = rng.standard_normal(n)
    return Problem(f"sparse_uniform_{m}x{n}", a, a @ x, x,
                   meta=dict(seed=seed, density=density))


def powerlaw_exponent(mean_len, max_len):
    """alpha with sum_l l * l^-alpha / sum_l l^-alpha = mean_len, l = 1..max."""
    ls = np.arange(1, max_len + 1, dtype=np.float64)
    lo, hi = 0.0, 10.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        w = ls ** -mid
        mean = (ls * w).sum() / w.sum()
        if mean > mean_len:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _distinct_columns(rng, lengths, n):
    """Per-row distinct uniform column indices, rows concatenated and sorted
    within each row."""
    m = lengths.size
    rows = np.repeat(np.arange(m, dtype=np.int64), lengths)
    cols = rng.integers(0, n, size=rows.size, dtype=np.int64)
    while True:
        order = np.lexsort((cols, rows))
        rows, cols = rows[order], cols[order]
        dup = np.zeros(rows.size, dtype=bool)
        dup[1:] = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        nd = int(dup.sum())
        if nd == 0:
            return rows, cols
        cols[dup] = rng.integers(0, n, size=nd, dtype=np.int64)


def sparse_powerlaw(m=1_000_000, n=500_000, mean_len=10.0, max_len=2000,
                    seed=0):
    """CSR (m, n): row lengths l in 1..max_len with P(l) proportional to
    l^-alpha (alpha fitted to the mean), row 0 of length max_len, uniform
    distinct columns, N(0,1) values scaled to unit row norm; x* ~ N(0,1),
    consistent b = A x*."""
    rng = np.random.default_rng(seed)
    max_len = min(max_len, n)
    alpha = powerlaw_exponent(mean_len, max_len)
    ls = np.arange(1, max_len + 1)
    p = ls.astype(np.float64) ** -alpha
    cdf = np.cumsum(p / p.sum())
    lengths = np.searchsorted(cdf, rng.random(m), side="right") + 1
    lengths = np.minimum(lengths, max_len).astype(np.int64)
    lengths[0] = max_len
    rows, cols = _distinct_columns(rng, lengths, n)
    vals = rng.standard_normal(rows.size)
    sq = np.bincount(rows, weights=vals * vals, minlength=m)
    vals /= np.sqrt(sq)[rows]
    indptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lengths, out=indptr[1:])
    a = sp.csr_matrix((vals, cols.astype(np.int32), indptr), shape=(m, n))
    x = rng.standard_normal(n)
    return Problem(f"sparse_powerlaw_{m}x{n}", a, a @ x, x,
                   meta=dict(seed=seed, alpha=alpha, mean_len=mean_len,
                             max_len=max_len))


def gaussian_psf_1d(sigma=2.0, half=7):
    """1-D Gaussian point-spread weights of Section 6:
    exp(-d^2 / (2 sigma^2)) / (sigma sqrt(2 pi)), |d| <= half."""
    d = np.arange(-half, half + 1, dtype=np.float64)
    return np.exp(-d * d / (2.0 * sigma * sigma)) / (sigma * np.sqrt(2 * np.pi))


def blur_operator(npix=512, sigma=2.0, half=7, dtype=np.float32):
    """2-D separable Gaussian blur on an npix x npix image with zero boundary:
    A = T kron T with T the banded Toeplitz matrix of ``gaussian_psf_1d``.
    Square, symmetric, CSR with sorted columns."""
    w = gaussian_psf_1d(sigma, half)
    offs = np.arange(-half, half + 1)
    t = sp.diags([np.full(npix - abs(o), w[i]) for i, o in enumerate(offs)],
                 offs, shape=(npix, npix), format="csr")
    a = sp.kron(t, t, format="csr")
    a.sort_indices()
    return a.astype(dtype)


def smooth_fields(npix, count, seed, corr=8.0):
    """White noise filtered by a Gaussian of std ``corr`` pixels (FFT),
    normalised to zero mean and unit std; shape (npix*npix, count)."""
    rng = np.random.default_rng(seed)
    f = np.fft.fftfreq(npix)
    k2 = f[:, None] ** 2 + f[None, :] ** 2
    filt = np.exp(-2.0 * (np.pi * corr) ** 2 * k2)
    out = np.empty((npix * npix, count))
    for c in range(count):
        noise = rng.standard_normal((npix, npix))
        fld = np.real(np.fft.ifft2(np.fft.fft2(noise) * filt))
        fld = (fld - fld.mean()) / fld.std()
        out[:, c] = fld.ravel()
    return out


def _round_mantissa(v, bits):
    """v rounded to `bits` significant bits (so that products of two such
    numbers are exact in FP32 when 2 * bits <= 24)."""
    m, e = np.frexp(v)
    return np.ldexp(np.round(m * 2.0 ** bits) / 2.0 ** bits, e)


def blur_tikhonov(npix=512, mu=1e-2, sigma=2.0, half=7):
    """The deblurring operator with Tikhonov rows, [A; s I] with A = T kron T
    (``blur_operator``'s structure) and s = sqrt(mu): a least-squares system
    of 2 npix^2 rows whose solution is the regularised deblurred image.  The
    1-D weights are rounded to 12 significant bits, so every entry of A (a
    product of two of them) and s (rounded to FP32) is exact in FP32 storage:
    the stored matrix is exactly T kron T.  Returns (CSR in FP64 with
    FP32-exact values, T as a dense FP64 array, s)."""
    w = _round_mantissa(gaussian_psf_1d(sigma, half), 12)
    offs = np.arange(-half, half + 1)
    t = sp.diags([np.full(npix - abs(o), w[i]) for i, o in enumerate(offs)],
                 offs, shape=(npix, npix), format="csr")
    a = sp.kron(t, t, format="csr")
    s = float(np.float32(np.sqrt(mu)))
    n = npix * npix
    aug = sp.vstack([a, s * sp.identity(n, format="csr")]).tocsr()
    aug.sort_indices()
    assert np.array_equal(aug.data.astype(np.float32).astype(np.float64), aug.data)
    return aug, t.toarray(), s


def blur_rhs(a, npix=512, nrhs=64, seed=0, noise=0.01):
    """Smooth random fields x_true and b = A x_true + noise, the noise std
    being ``noise`` times std(A x_true) per right-hand side."""
    x = smooth_fields(npix, nrhs, seed)
    ax = np.asarray(a.astype(np.float64) @ x)
    rng = np.random.default_rng(seed + 1)
    sd = ax.std(axis=0)
    b = ax + noise * sd[None, :] * rng.standard_normal(ax.shape)
    return b, x


def _laplacian_2d(nx, ny, shift):
    ex = np.ones(nx)
    ey = np.ones(ny)
    lx = sp.diags([-ex[:-1], 2 * ex, -ex[:-1]], [-1, 0, 1])
    ly = sp.diags([-ey[:-1], 2 * ey, -ey[:-1]], [-1, 0, 1])
    lap = sp.kron(sp.identity(ny), lx) + sp.kron(ly, sp.identity(nx))
    return (lap + shift * sp.identity(nx * ny)).tocsr()


def laplacian_batch(count=256, n_min=2000, n_max=200000, extra=0.2,
                    extra_len=8, seed=0):
    """Uneven batch of systems: n_s log-uniform in [n_min, n_max] on an
    nx x ny grid (n_s := nx*ny), 5-point Dirichlet Laplacian (diagonal 4+s,
    off-diagonals -1) with s ~ U[0.1, 1], plus round(extra * n_s) rows of
    ``extra_len`` distinct uniform columns with N(0,1) values.  Each system
    is consistent with a planted x* ~ N(0,1).  Returns a list of Problems."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        ns = int(round(np.exp(rng.uniform(np.log(n_min), np.log(n_max)))))
        nx = max(2, int(round(np.sqrt(ns))))
        ny = max(2, int(round(ns / nx)))
        ns = nx * ny
        shift = rng.uniform(0.1, 1.0)
        lap = _laplacian_2d(nx, ny, shift)
        ne = int(round(extra * ns))
        lens = np.full(ne, min(extra_len, ns), dtype=np.int64)
        rows, cols = _distinct_columns(rng, lens, ns)
        vals = rng.standard_normal(rows.size)
        ext = sp.csr_matrix((vals, (rows, cols)), shape=(ne, ns))
        a = sp.vstack([lap, ext]).tocsr()
        a.sort_indices()
        x = rng.standard_normal(ns)
        out.append(Problem(f"laplacian_{s}", a, a @ x, x,
                           meta=dict(nx=nx, ny=ny, shift=shift)))
    return out


def fem_p1_unit_square(npts, k=0.0, mode=1):
    """P1 finite elements on the unit square (Section 6, finite element
    method): an npts x npts uniform grid of nodes, Delaunay-triangulated
    (2 (npts-1)^2 elements), for -Laplace(u) - k^2 u = f with u = 0 on the
    boundary and the exact solution u = sin(mode pi x) sin(mode pi y).
    Every grid cell has four cocircular corners, so which diagonal splits
    it is the triangulator's choice; scipy's Qhull is used, as its choice
    reproduces the condition number the paper reports for Helmholtz.
    Assembled: stiffness K and consistent mass M; A = K - k^2 M;
    b = M f_I (f interpolated at the nodes); boundary nodes get identity
    rows, and their columns are removed from the other rows (u = 0 there).
    Returns (A csr, b, u_exact at the nodes, coordinates)."""
    from scipy.spatial import Delaunay
    xs = np.linspace(0.0, 1.0, npts)
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    tris = Delaunay(xy).simplices
    rows, cols, kv, mv = [], [], [], []
    for t in tris:
        p = xy[t]
        mat = np.array([[1.0, p[0, 0], p[0, 1]], [1.0, p[1, 0], p[1, 1]],
                        [1.0, p[2, 0], p[2, 1]]])
        area = 0.5 * abs(np.linalg.det(mat))
        grads = np.linalg.inv(mat)[1:, :]          # d(phi_i)/dx, d/dy
        ke = area * grads.T @ grads
        me = area / 12.0 * (np.ones((3, 3)) + np.eye(3))
        for a_ in range(3):
            for b2 in range(3):
                rows.append(t[a_]); cols.append(t[b2])
                kv.append(ke[a_, b2]); mv.append(me[a_, b2])
    N = npts * npts
    K = sp.csr_matrix((kv, (rows, cols)), shape=(N, N))
    M = sp.csr_matrix((mv, (rows, cols)), shape=(N, N))
    w = mode * np.pi
    u = np.sin(w * xy[:, 0]) * np.sin(w * xy[:, 1])
    f = (2.0 * w * w - k * k) * u
    A = (K - (k * k) * M).tolil()
    b = M @ f
    bnd = np.where((xy[:, 0] == 0) | (xy[:, 0] == 1) | (xy[:, 1] == 0) |
                   (xy[:, 1] == 1))[0]
    A[:, bnd] = 0.0
    A[bnd, :] = 0.0
    for i in bnd:
        A[i, i] = 1.0
    b[bnd] = 0.0
    A = A.tocsr()
    A.eliminate_zeros()
    A.data[np.abs(A.data) < 1e-14 * np.abs(A.data).max()] = 0.0
    A.eliminate_zeros()
    return A, b, u, xy
