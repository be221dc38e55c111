"""Python face of the RGDBEK solver: a handle class, block selection, and a
differentiable solve.  Only argument marshalling happens here; every step of
the method runs in librgdbek.so on the GPU.
"""
import ctypes

import torch

from . import _binding as B


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _need_cuda(t, name, dtype=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a tensor on a HIP device")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Solver:
    """A solver handle for one matrix A.

    A is either a dense (m, n) tensor (float64 or float32, row-major) or a
    CSR triple (row_ptr int64, col_idx int32, values float64/float32) with
    shape=(m, n).  Keyword arguments map onto rgdbek_params."""

    def __init__(self, a=None, *, csr=None, shape=None, eta=0.5, k_col=0,
                 k_row=0, tol=1e-8, stop="err_ref", max_iter=10000, seed=0,
                 precision="fp64", inner_max=0, inner_tol=0.0, graph_iters=0,
                 solver=B.SOLVER_AUTO, graph=True, gram_aat=False,
                 weight_floor=0.0, tile_rows=0, select="random",
                 cg_split=False, sparse_cg=False, profile=False, pass_drop=0.0,
                 sparse_full=False, stream=None):
        lib = B.load()
        self._lib = lib
        self._h = ctypes.c_void_p()
        mat = B.Matrix()
        keep = []
        if csr is not None:
            rp, ci, val = csr
            _need_cuda(rp, "row_ptr", torch.int64)
            _need_cuda(ci, "col_idx", torch.int32)
            _need_cuda(val, "values")
            m, n = shape
            mat.m, mat.n, mat.nnz = m, n, val.numel()
            mat.layout = B.CSR
            mat.row_ptr, mat.col_idx = _ptr(rp), _ptr(ci)
            mat.values = _ptr(val)
            mat.value_type = B.F64 if val.dtype == torch.float64 else B.F32
            keep += [rp, ci, val]
        else:
            _need_cuda(a, "A")
            m, n = a.shape
            mat.m, mat.n, mat.nnz = m, n, m * n
            mat.layout = B.DENSE_ROW_MAJOR
            mat.values = _ptr(a)
            mat.row_ptr = None
            mat.col_idx = None
            mat.value_type = B.F64 if a.dtype == torch.float64 else B.F32
            keep.append(a)
        p = B.Params()
        B.check(lib.rgdbek_params_default(ctypes.byref(p)))
        p.k_col, p.k_row, p.eta, p.tol = k_col, k_row, eta, tol
        p.stop = B.STOP_NAMES[stop] if isinstance(stop, str) else int(stop)
        p.precision = (B.PREC_NAMES[precision] if isinstance(precision, str)
                       else int(precision))
        p.max_iter, p.seed = max_iter, seed
        p.inner_max, p.inner_tol, p.graph_iters = inner_max, inner_tol, graph_iters
        p.solver = int(solver)
        p.weight_floor = float(weight_floor)
        p.tile_rows = int(tile_rows)
        p.pass_drop = float(pass_drop)
        p.select_mode = {"random": B.SELECT_RANDOM, "greedy": B.SELECT_GREEDY,
                         "block_law": B.SELECT_BLOCK_LAW,
                         "iid": B.SELECT_IID}[select]
        p.flags = ((B.FLAG_GRAPH if graph else 0) |
                   (B.FLAG_GRAM_AAT if gram_aat else 0) |
                   (B.FLAG_CG_SPLIT if cg_split else 0) |
                   (B.FLAG_SPARSE_CG if sparse_cg else 0) |
                   (B.FLAG_PROFILE if profile else 0) |
                   (B.FLAG_SPARSE_FULL if sparse_full else 0))
        self.m, self.n = int(m), int(n)
        self.params = p
        self.stream = stream
        st = lib.rgdbek_create(ctypes.byref(mat), ctypes.byref(p),
                               _stream(stream), ctypes.byref(self._h))
        B.check(st, None)
        del keep

    # -- solves --------------------------------------------------------
    def _dev(self):
        return torch.device("cuda", torch.cuda.current_device())

    def solve(self, b, x_ref=None, allow_not_converged=True):
        """x = RGDBEK(A, b); returns (x, info dict)."""
        _need_cuda(b, "b", torch.float64)
        x = torch.empty(self.n, dtype=torch.float64, device=b.device)
        if x_ref is not None:
            _need_cuda(x_ref, "x_ref", torch.float64)
        info = B.Info()
        st = self._lib.rgdbek_solve(self._h, _ptr(b), _ptr(x), _ptr(x_ref),
                                    ctypes.byref(info))
        allow = (B.ERR_NOT_CONVERGED,) if allow_not_converged else ()
        B.check(st, self._h, allow)
        return x, info.as_dict()

    def solve_resume(self, b, x, z, it0, x_ref=None):
        """Continue from (x, z) at generator iteration it0 (in place)."""
        _need_cuda(b, "b", torch.float64)
        _need_cuda(x, "x", torch.float64)
        _need_cuda(z, "z", torch.float64)
        info = B.Info()
        st = self._lib.rgdbek_solve_resume(self._h, _ptr(b), _ptr(x), _ptr(z),
                                           int(it0), _ptr(x_ref),
                                           ctypes.byref(info))
        B.check(st, self._h, (B.ERR_NOT_CONVERGED,))
        return info.as_dict()

    def get_z(self):
        z = torch.empty(self.m, dtype=torch.float64, device=self._dev())
        B.check(self._lib.rgdbek_get_z(self._h, _ptr(z)), self._h)
        return z

    def solve_adjoint(self, g):
        """w with A^T w = g (minimum norm), by RGDBEK on the adjoint."""
        _need_cuda(g, "g", torch.float64)
        w = torch.empty(self.m, dtype=torch.float64, device=g.device)
        info = B.Info()
        st = self._lib.rgdbek_solve_adjoint(self._h, _ptr(g), _ptr(w),
                                            ctypes.byref(info))
        B.check(st, self._h, (B.ERR_NOT_CONVERGED,))
        return w, info.as_dict()

    def grad_pattern(self, r, lam, w, x, nnz):
        dA = torch.empty(nnz, dtype=torch.float64, device=w.device)
        st = self._lib.rgdbek_grad_pattern(self._h, _ptr(r), _ptr(lam),
                                           _ptr(w), _ptr(x), _ptr(dA))
        B.check(st, self._h)
        return dA

    def apply(self, x, z, out_ax=None, out_atz=None, precision="f64"):
        """(A x, A^T z) in one residual pass, on the handle's stream (not
        synchronised)."""
        dt = torch.float64 if precision == "f64" else torch.float32
        _need_cuda(x, "x", dt)
        _need_cuda(z, "z", dt)
        ax = out_ax if out_ax is not None else torch.empty(self.m, dtype=dt, device=x.device)
        atz = out_atz if out_atz is not None else torch.empty(self.n, dtype=dt, device=x.device)
        st = self._lib.rgdbek_apply(self._h, B.F64 if precision == "f64" else B.F32,
                                    _ptr(x), _ptr(z), _ptr(ax), _ptr(atz))
        B.check(st, self._h)
        return ax, atz

    def profile(self):
        """Event timing of the last solve of a handle made with
        profile=True: {region: {"launches", "ms", "steps"}} for the steps of
        the iteration (residual passes, draws, block solves, updates, stop
        tests, FP64 refinement passes)."""
        out = {}
        for i, name in enumerate(B.PROF_REGIONS):
            n, ms, steps = ctypes.c_int64(0), ctypes.c_double(0), ctypes.c_int64(0)
            st = self._lib.rgdbek_profile_read(self._h, i, ctypes.byref(n),
                                               ctypes.byref(ms),
                                               ctypes.byref(steps))
            B.check(st, self._h)
            out[name] = {"launches": n.value, "ms": ms.value,
                         "steps": steps.value}
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.rgdbek_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class BatchSolver(Solver):
    """Many independent sparse systems solved together (block-diagonal CSR
    with global indices; system s owns rows row_off[s]:row_off[s+1] and
    columns col_off[s]:col_off[s+1]).  Vectors are the systems' vectors
    concatenated.  Keyword arguments as for Solver (eta/k_col/k_row give
    each system's block sizes)."""

    def __init__(self, csr, row_off, col_off, *, eta=0.1, k_col=0, k_row=0,
                 tol=1e-8, stop="err_ref", max_iter=10000, seed=0,
                 precision="fp64", inner_max=0, inner_tol=0.0, graph_iters=0,
                 graph=True, weight_floor=0.0, select="random", pass_drop=0.0,
                 profile=False, sparse_full=False, stream=None):
        lib = B.load()
        self._lib = lib
        self._h = ctypes.c_void_p()
        rp, ci, val = csr
        _need_cuda(rp, "row_ptr", torch.int64)
        _need_cuda(ci, "col_idx", torch.int32)
        _need_cuda(val, "values")
        ro = (ctypes.c_int64 * len(row_off))(*[int(v) for v in row_off])
        co = (ctypes.c_int64 * len(col_off))(*[int(v) for v in col_off])
        self.nsys = len(row_off) - 1
        m, n = int(row_off[-1]), int(col_off[-1])
        mat = B.Matrix()
        mat.m, mat.n, mat.nnz = m, n, val.numel()
        mat.layout = B.CSR
        mat.row_ptr, mat.col_idx, mat.values = _ptr(rp), _ptr(ci), _ptr(val)
        mat.value_type = B.F64 if val.dtype == torch.float64 else B.F32
        p = B.Params()
        B.check(lib.rgdbek_params_default(ctypes.byref(p)))
        p.k_col, p.k_row, p.eta, p.tol = k_col, k_row, eta, tol
        p.stop = B.STOP_NAMES[stop] if isinstance(stop, str) else int(stop)
        p.precision = (B.PREC_NAMES[precision] if isinstance(precision, str)
                       else int(precision))
        p.max_iter, p.seed = max_iter, seed
        p.inner_max, p.inner_tol, p.graph_iters = inner_max, inner_tol, graph_iters
        p.flags = ((B.FLAG_GRAPH if graph else 0) |
                   (B.FLAG_PROFILE if profile else 0) |
                   (B.FLAG_SPARSE_FULL if sparse_full else 0))
        p.weight_floor = float(weight_floor)
        p.pass_drop = float(pass_drop)
        p.select_mode = {"random": B.SELECT_RANDOM, "greedy": B.SELECT_GREEDY,
                         "block_law": B.SELECT_BLOCK_LAW,
                         "iid": B.SELECT_IID}[select]
        self.m, self.n, self.params, self.stream = m, n, p, stream
        st = lib.rgdbek_create_batched(ctypes.byref(mat), self.nsys, ro, co,
                                       ctypes.byref(p), _stream(stream),
                                       ctypes.byref(self._h))
        B.check(st, None)

    def batch_info(self):
        it = (ctypes.c_int64 * self.nsys)()
        met = (ctypes.c_double * self.nsys)()
        cv = (ctypes.c_int32 * self.nsys)()
        B.check(self._lib.rgdbek_batch_info(self._h, it, met, cv), self._h)
        return list(it), list(met), list(cv)


class MultiRhsSolver(BatchSolver):
    """One sparse matrix, many right-hand sides (RHS-major vectors:
    b[s*m + i], x[s*n + j]); A is stored once and every pass over it serves
    all right-hand sides."""

    def __init__(self, csr, shape, nrhs, *, eta=0.1, k_col=0, k_row=0,
                 tol=1e-8, stop="err_ref", max_iter=10000, seed=0,
                 precision="fp64", inner_max=0, inner_tol=0.0, graph_iters=0,
                 graph=True, weight_floor=0.0, pass_drop=0.0, profile=False,
                 stream=None):
        lib = B.load()
        self._lib = lib
        self._h = ctypes.c_void_p()
        rp, ci, val = csr
        _need_cuda(rp, "row_ptr", torch.int64)
        _need_cuda(ci, "col_idx", torch.int32)
        _need_cuda(val, "values")
        m, n = shape
        mat = B.Matrix()
        mat.m, mat.n, mat.nnz = m, n, val.numel()
        mat.layout = B.CSR
        mat.row_ptr, mat.col_idx, mat.values = _ptr(rp), _ptr(ci), _ptr(val)
        mat.value_type = B.F64 if val.dtype == torch.float64 else B.F32
        p = B.Params()
        B.check(lib.rgdbek_params_default(ctypes.byref(p)))
        p.k_col, p.k_row, p.eta, p.tol = k_col, k_row, eta, tol
        p.stop = B.STOP_NAMES[stop] if isinstance(stop, str) else int(stop)
        p.precision = (B.PREC_NAMES[precision] if isinstance(precision, str)
                       else int(precision))
        p.max_iter, p.seed = max_iter, seed
        p.inner_max, p.inner_tol, p.graph_iters = inner_max, inner_tol, graph_iters
        p.flags = ((B.FLAG_GRAPH if graph else 0) |
                   (B.FLAG_PROFILE if profile else 0))
        p.weight_floor = float(weight_floor)
        p.pass_drop = float(pass_drop)
        self.nsys = int(nrhs)
        self.base_shape = (int(m), int(n))
        self.m, self.n, self.params, self.stream = m * nrhs, n * nrhs, p, stream
        st = lib.rgdbek_create_multirhs(ctypes.byref(mat), int(nrhs),
                                        ctypes.byref(p), _stream(stream),
                                        ctypes.byref(self._h))
        B.check(st, None)


def block_diagonal(mats):
    """Concatenate scipy sparse systems into block-diagonal CSR arrays with
    global indices; returns (row_ptr, col_idx, values, row_off, col_off)."""
    import numpy as np
    import scipy.sparse as sp
    rps, cis, vals = [], [], []
    row_off, col_off = [0], [0]
    nnz = 0
    for a in mats:
        c = sp.csr_matrix(a)
        c.sort_indices()
        rps.append(c.indptr[1:] + nnz if rps else c.indptr + nnz)
        cis.append(c.indices.astype(np.int64) + col_off[-1])
        vals.append(c.data)
        nnz += c.nnz
        row_off.append(row_off[-1] + c.shape[0])
        col_off.append(col_off[-1] + c.shape[1])
    rp = np.concatenate(rps).astype(np.int64)
    ci = np.concatenate(cis).astype(np.int32)
    v = np.concatenate(vals)
    return rp, ci, v, row_off, col_off


def select(eps, k, seed=0, it=0, phase=0, sys=0, key1=0, floor=1e-20,
           stream=None):
    """Block draw on given weights (device FP64 tensor): ascending int32
    indices, exactly as the solver draws them (weights <= floor * max count
    as zero)."""
    lib = B.load()
    _need_cuda(eps, "eps", torch.float64)
    d = eps.numel()
    out = torch.empty(max(1, min(int(k), d)), dtype=torch.int32,
                      device=eps.device)
    cnt = ctypes.c_int64(0)
    st = lib.rgdbek_select(_ptr(eps), d, int(k), float(floor), int(seed),
                           int(key1), int(it),
                           int(phase), int(sys), _ptr(out), ctypes.byref(cnt),
                           _stream(stream))
    B.check(st, None)
    return out[:cnt.value]


def select_noalloc(eps, k, seed=0, it=0, phase=0, sys=0, key1=0, floor=1e-20,
                   out=None, stream=None):
    """select() through the allocation-free entry point: the library's draw
    allocates no device memory (its work space is a static device array;
    overlapping calls on one GPU race).  `out` (device int32, room for
    min(k, d)) may be passed in so that nothing is allocated here either."""
    lib = B.load()
    _need_cuda(eps, "eps", torch.float64)
    d = eps.numel()
    if out is None:
        out = torch.empty(max(1, min(int(k), d)), dtype=torch.int32,
                          device=eps.device)
    cnt = ctypes.c_int64(0)
    st = lib.rgdbek_select_noalloc(_ptr(eps), d, int(k), float(floor),
                                   int(seed), int(key1), int(it), int(phase),
                                   int(sys), _ptr(out), ctypes.byref(cnt),
                                   _stream(stream))
    B.check(st, None)
    return out[:cnt.value]


def select_block_law(eps, s, seed=0, it=0, phase=0, sys=0, key1=0,
                     floor=1e-20, stream=None):
    """Block of size s from the law of Lemma 2.1 on given weights (device
    FP64 tensor): ascending int32 indices, as the solver draws them in the
    block-law mode."""
    lib = B.load()
    _need_cuda(eps, "eps", torch.float64)
    d = eps.numel()
    out = torch.empty(max(1, min(int(s), d)), dtype=torch.int32,
                      device=eps.device)
    cnt = ctypes.c_int64(0)
    st = lib.rgdbek_select_block_law(_ptr(eps), d, int(s), float(floor),
                                     int(seed), int(key1), int(it), int(phase),
                                     int(sys), _ptr(out), ctypes.byref(cnt),
                                     _stream(stream))
    B.check(st, None)
    return out[:cnt.value]


def select_iid(eps, k, seed=0, it=0, phase=0, sys=0, key1=0, floor=1e-20,
               stream=None):
    """Distinct indices of k draws with replacement from P(j) = eps_j /
    sum eps on given weights (device FP64 tensor): ascending int32 indices,
    as the solver draws them in the "iid" mode."""
    lib = B.load()
    _need_cuda(eps, "eps", torch.float64)
    d = eps.numel()
    out = torch.empty(max(1, min(int(k), d)), dtype=torch.int32,
                      device=eps.device)
    cnt = ctypes.c_int64(0)
    st = lib.rgdbek_select_iid(_ptr(eps), d, int(k), float(floor), int(seed),
                               int(key1), int(it), int(phase), int(sys),
                               _ptr(out), ctypes.byref(cnt), _stream(stream))
    B.check(st, None)
    return out[:cnt.value]


def select_threshold(eps, eta, cap=None, stream=None):
    """GDBEK's greedy set on given weights (device FP64 tensor): ascending
    int32 indices j with eps_j > 0 and eps_j >= eta * max(eps), at most cap
    of them (default: all)."""
    lib = B.load()
    _need_cuda(eps, "eps", torch.float64)
    d = eps.numel()
    cap = d if cap is None else int(cap)
    out = torch.empty(max(1, cap), dtype=torch.int32, device=eps.device)
    cnt = ctypes.c_int64(0)
    st = lib.rgdbek_select_threshold(_ptr(eps), d, float(eta), cap, _ptr(out),
                                     ctypes.byref(cnt), _stream(stream))
    B.check(st, None)
    return out[:cnt.value]


class RGDBEKFunction(torch.autograd.Function):
    """x = A^+ b through RGDBEK, differentiable in b and in A's stored
    values.  The forward keeps (b, x, z) only -- z is the method's own
    estimate of the least-squares residual r = (I - A A^+) b -- and no
    iterate history.  The backward runs RGDBEK on the adjoint system
    A^T w = dL/dx (w = dL/db) and, for least-squares systems, once more on A
    (lam = A^+ w); then dL/dA = r lam^T - w x^T on A's pattern.

    The handle must stop on a residual test ('res_ext', 'rse') or run a
    fixed count ('none'): inside a layer there is no reference solution,
    so an 'err_ref' handle is rejected.  Every solve (forward, adjoint,
    second solve) must meet its stopping test; a solve that runs out of
    iterations raises instead of returning a wrong gradient."""

    @staticmethod
    def _checked(what, info):
        if not info.get("converged", False):
            raise RuntimeError(
                f"RGDBEK {what} solve stopped after {info.get('iterations')} "
                f"iterations without meeting its stopping test (metric "
                f"{info.get('final_metric')}); the gradient would be wrong")

    @staticmethod
    def forward(ctx, values, b, solver, least_squares):
        if int(solver.params.stop) == B.STOP_NAMES["err_ref"]:
            raise ValueError("a differentiable solve needs a handle with stop "
                             "'res_ext', 'rse' or 'none' (no reference "
                             "solution exists inside a layer)")
        x, info = solver.solve(b)
        RGDBEKFunction._checked("forward", info)
        z = solver.get_z() if least_squares else None
        ctx.solver = solver
        ctx.least_squares = least_squares
        ctx.nnz = values.numel()
        ctx.save_for_backward(x, z)
        return x

    @staticmethod
    def backward(ctx, gx):
        x, z = ctx.saved_tensors
        s = ctx.solver
        w, info = s.solve_adjoint(gx.contiguous().to(torch.float64))
        RGDBEKFunction._checked("adjoint", info)
        if ctx.least_squares:
            lam, info = s.solve(w)
            RGDBEKFunction._checked("second (lam = A^+ w)", info)
            dA = s.grad_pattern(z, lam, w, x, ctx.nnz)
        else:
            dA = s.grad_pattern(None, None, w, x, ctx.nnz)
        return dA, w, None, None


def solve(solver, values, b, least_squares=False):
    """Differentiable x = A^+ b (A as held by ``solver``, whose stored values
    are ``values``)."""
    return RGDBEKFunction.apply(values, b, solver, least_squares)
