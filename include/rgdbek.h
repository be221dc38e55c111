/*
 * rgdbek.h -- C-ABI of the MI355X (gfx950) RGDBEK solver.
 *
 * RGDBEK (randomized greedy double block extended Kaczmarz, arXiv 2509.19267)
 * solves A x = b for A in R^{m x n}, consistent or in the least-squares sense
 * (the paper's problem statement, eq. (1) of Section 1).  Each iteration
 * (Section 2, Algorithm 1):
 *   column phase: eps^z_j = (A_(j)^T z)^2 / ||A_(j)||^2, draw a block U of
 *                 k_col columns with probability proportional to eps^z,
 *                 z <- z - A_U A_U^+ z;
 *   row phase:    r = b - z - A x, eps^x_i = r_i^2 / ||A^(i)||^2, draw a block
 *                 J of k_row rows the same way, x <- x + (A^J)^+ r^J,
 * starting from x_0 = 0 and z_0 = b.  Block draws are without replacement
 * (successive weighted sampling through exponential keys driven by a
 * counter-based Philox4x64-10 generator keyed by the seed), so a solve is a
 * pure function of (A, b, parameters, seed).
 *
 * Conventions for every entry point:
 *  - Pointers named "device" are HIP device pointers; everything else is host.
 *  - Work is enqueued on the HIP stream given to rgdbek_create; for NULL the
 *    handle creates a private stream (HIP graphs cannot be captured on the
 *    default stream).  Entry points first wait for the caller's stream, and
 *    those that return results synchronise the work stream before returning.
 *  - Status codes only: no C++ exception crosses this interface.  On an error
 *    the handle's message (rgdbek_last_error) says what was wrong.
 *  - A handle is not thread-safe: use one handle per host thread and stream.
 */
#ifndef RGDBEK_H
#define RGDBEK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rgdbek_ctx *rgdbek_handle;

typedef enum {
  RGDBEK_OK = 0,
  RGDBEK_ERR_INVALID_ARG = 1,   /* bad size, pointer, structure or option   */
  RGDBEK_ERR_NUMERIC = 2,       /* NaN/Inf in A or b, or a NaN weight       */
  RGDBEK_ERR_NOT_CONVERGED = 3, /* max_iter reached before the stop test    */
  RGDBEK_ERR_OUT_OF_MEMORY = 4, /* a device allocation failed               */
  RGDBEK_ERR_DEVICE = 5,        /* a HIP call failed (message has details)  */
  RGDBEK_ERR_UNSUPPORTED = 6    /* valid request the library does not serve */
} rgdbek_status;

/* Matrix storage (rgdbek_matrix.layout). */
enum { RGDBEK_DENSE_ROW_MAJOR = 0, RGDBEK_CSR = 1 };
/* Value type of the matrix values given to rgdbek_create. */
enum { RGDBEK_F64 = 0, RGDBEK_F32 = 1 };
/* Stopping tests (rgdbek_params.stop):
 *  NONE     run exactly max_iter iterations;
 *  ERR_REF  ||x_k - x_ref|| <= tol ||x_ref||, tested at the top of iteration k
 *           (needs x_ref: the planted solution of a benchmark);
 *  RSE      ||b - A x_k||^2 <= tol ||b||^2, the paper's squared relative
 *           residual (Sections 3 and 5), tested when A x_k is formed;
 *  RES_EXT  ||b - z_{k+1} - A x_k|| <= tol ||b||, the extended residual that
 *           also goes to zero for inconsistent (least-squares) systems.
 * Every test returns x_k, the iterate it was evaluated on. */
enum { RGDBEK_STOP_NONE = 0, RGDBEK_STOP_ERR_REF = 1, RGDBEK_STOP_RSE = 2,
       RGDBEK_STOP_RES_EXT = 3 };
/* Arithmetic of the solve (rgdbek_params.precision):
 *  FP64       every step in FP64;
 *  MIXED_F32  inner RGDBEK iterations with FP32 matrix values, vectors and
 *             accumulation, inside an FP64 refinement loop.  State (x, z) in
 *             FP64; each pass tests the stop rule in FP64 on it, sets
 *             z = b - A x and forms A^T z in FP64, the FP32 iterations solve
 *             for the correction (dx, dz) from (0, 0), then x += dx and
 *             z += dz in FP64.  A pass ends on residuals alone: when the
 *             FP32 extended residual ||dz + A dx|| (that of the refined
 *             state) has fallen to 1e-5 of its first value in the pass (or
 *             to tol under RES_EXT), or stops improving.  Every stop mode is
 *             served; the test is made in FP64 between passes (RES_EXT from
 *             the second pass on: before the first, z = b and x = 0 meet it
 *             trivially). */
enum { RGDBEK_PREC_FP64 = 0, RGDBEK_PREC_MIXED_F32 = 1 };

/* The coefficient matrix A (m x n).  All pointers are device pointers owned
 * by the caller and read only during rgdbek_create: the library copies and
 * converts what it needs, so the caller may free them once create returns.
 *  dense:  values = m*n entries, row-major (entry (i,j) at i*n + j); nnz is
 *          ignored; row_ptr/col_idx must be NULL.
 *  CSR:    row_ptr[m+1] (int64, row_ptr[0] = 0, non-decreasing,
 *          row_ptr[m] = nnz), col_idx[nnz] in [0, n) and strictly increasing
 *          within each row, values[nnz]. */
typedef struct {
  int64_t m, n, nnz;
  int32_t layout;      /* RGDBEK_DENSE_ROW_MAJOR or RGDBEK_CSR   */
  int32_t value_type;  /* RGDBEK_F64 or RGDBEK_F32               */
  const void *values;
  const int64_t *row_ptr;
  const int32_t *col_idx;
} rgdbek_matrix;

typedef struct {
  int64_t k_col, k_row;  /* block sizes; 0 = derive from eta: k = min(d,
                            max(1, floor(eta*d + 0.5))) for d = n resp. m   */
  double eta;            /* block fraction of Algorithm 1 (0.5 in Section 3,
                            0.1 in Section 5)                              */
  double tol;            /* tolerance of the stopping test                  */
  int32_t stop;          /* RGDBEK_STOP_*                                   */
  int32_t precision;     /* RGDBEK_PREC_*                                   */
  int64_t max_iter;      /* the paper's T: cap on (inner) iterations        */
  uint64_t seed;         /* Philox key word 0                               */
  int32_t inner_max;     /* cap on inner solver steps per projection (0 = 64) */
  int32_t graph_iters;   /* iterations per captured HIP graph (0 = 8)       */
  double inner_tol;      /* relative tolerance of the block projections
                            (0 = 1e-14 in FP64, 1e-7 in FP32)             */
  int32_t solver;        /* RGDBEK_SOLVER_* for dense blocks (0 = auto)     */
  int32_t flags;         /* RGDBEK_FLAG_*                                   */
  double weight_floor;   /* residual weights <= weight_floor * max weight
                            count as zero (zero up to rounding): 0 = default
                            (1e-20 for FP64 weights, 1e-6 for the FP32 inner
                            iterations of the mixed form); < 0 = exact
                            zero test only                                  */
  int32_t tile_rows;     /* rows per workgroup tile of the dense residual
                            pass (rounded up to 16); 0 = sized so one grid
                            round fills the device                          */
  int32_t select_mode;   /* RGDBEK_SELECT_*: 0 = Algorithm 1's randomized
                            draws; 1 = GDBEK's greedy sets (Section 2):
                            indices with weight >= eta * max weight, eta the
                            threshold, k_col/k_row the capacity (0 = the
                            dimension; a larger set keeps its lowest
                            indices); 2 = blocks of size k_col/k_row from
                            the law of Lemma 2.1 (see
                            rgdbek_select_block_law); 3 = k_col/k_row draws
                            with replacement, distinct indices kept (see
                            rgdbek_select_iid; at most 16M rows/columns).
                            Modes 1-3: single systems only.                 */
  double pass_drop;      /* MIXED_F32: a refinement pass ends when its FP32
                            extended residual has fallen to pass_drop times
                            its first value in the pass (0 = 1e-5; in
                            (0, 1))                                         */
} rgdbek_params;

/* Dense block solvers: AUTO picks Cholesky for blocks up to 256 and
 * preconditioned conjugate gradients on the Gram matrix above that. */
enum { RGDBEK_SOLVER_AUTO = 0, RGDBEK_SOLVER_CHOL = 1, RGDBEK_SOLVER_CG = 2 };
/* Flags: GRAPH captures the iteration loop into HIP graphs (default on via
 * rgdbek_params_default); GRAM_AAT precomputes A A^T (m x m, m up to 32768,
 * else ignored) for dense row blocks, as A^T A is always precomputed for
 * dense column blocks of more than 64 columns when n <= 8192; the blocks
 * are then gathered from these matrices instead of formed from A;
 * CG_SPLIT makes the sparse block projections finish every CG step with
 * separate many-workgroup launches whatever the block size (by default only
 * blocks of more than 16384 indices do; smaller ones finish in the last
 * workgroup of the step).  The arithmetic is the same either way.
 * SPARSE_CG keeps the matrix-free CG projections for small sparse single
 * systems (both dimensions up to 4096), which by default, when the inner
 * tolerance is at most 1e-6 (0: the FP64 floor), go through Gram matrices
 * of all columns and rows formed once at create (as dense matrices do). */
enum { RGDBEK_FLAG_GRAPH = 1, RGDBEK_FLAG_GRAM_AAT = 2,
       RGDBEK_FLAG_CG_SPLIT = 4, RGDBEK_FLAG_SPARSE_CG = 8,
       RGDBEK_FLAG_PROFILE = 16, RGDBEK_FLAG_SPARSE_FULL = 32 };
/* RGDBEK_FLAG_SPARSE_FULL: the matrix-free sparse block projections stream
 * all of A in every CG step (as a product with a vector that is zero off the
 * block) instead of a copy of the block's own entries made once per
 * iteration (the default for one stored matrix and for fewer than 16
 * right-hand sides; from 16 on, the many-right-hand-side products read A
 * once for all right-hand sides and make no copies).  The same sums,
 * grouped differently across lanes: results agree to rounding. */
/* RGDBEK_FLAG_PROFILE times every step of every iteration with HIP events on
 * the handle's stream (the launches are then issued one by one, not from
 * captured graphs, so a profiled solve runs a little slower than a plain
 * one; the arithmetic is the same).  Regions, one per step of Algorithm 1's
 * iteration, read back with rgdbek_profile_read after a solve: */
enum { RGDBEK_PROF_COL_RESIDUAL = 0, /* A^T z and eps^z (dense: the fused
                                        pass that also forms A x)          */
       RGDBEK_PROF_COL_DRAW = 1,     /* column block draw                   */
       RGDBEK_PROF_COL_SOLVE = 2,    /* column block least-squares solve    */
       RGDBEK_PROF_COL_UPDATE = 3,   /* z -= A_U y                          */
       RGDBEK_PROF_ROW_RESIDUAL = 4, /* b - z - A x and eps^x               */
       RGDBEK_PROF_ROW_DRAW = 5,     /* row block draw                      */
       RGDBEK_PROF_ROW_SOLVE = 6,    /* row block least-squares solve       */
       RGDBEK_PROF_ROW_UPDATE = 7,   /* x += A^J^T w                        */
       RGDBEK_PROF_STOP = 8,         /* stop tests and iteration counters   */
       RGDBEK_PROF_REFINE = 9,       /* FP64 passes of the mixed form       */
       RGDBEK_PROF_COUNT = 10 };
/* Block rule (rgdbek_params.select_mode). */
enum { RGDBEK_SELECT_RANDOM = 0, RGDBEK_SELECT_GREEDY = 1,
       RGDBEK_SELECT_BLOCK_LAW = 2, RGDBEK_SELECT_IID = 3 };

typedef struct {
  int64_t iterations;        /* RGDBEK iterations run (inner, summed)       */
  int64_t outer_iterations;  /* FP64 refinement passes (mixed precision)    */
  double final_metric;       /* value of the stopping test's left side      */
  int32_t converged;         /* 1 when the stopping test held (NONE: 1)     */
  int32_t status;            /* the status the call returned                */
  double seconds;            /* wall time of the solve (host clock)         */
} rgdbek_info;

/* Fill *p with the defaults: k from eta = 0.5, tol 1e-8, STOP_ERR_REF,
 * FP64, max_iter 10000, seed 0, GRAPH flag on.  INVALID_ARG if p is NULL. */
rgdbek_status rgdbek_params_default(rgdbek_params *p);

/* Build a solver for A: copies A to library-owned device storage (row-major
 * and column-major copies for dense A; CSR and CSC for sparse A), computes
 * the row and column squared norms (the denominators of the residual weights
 * of Section 2) and allocates all work space.  `stream` is a hipStream_t
 * (NULL = default stream).  On success *out receives the handle.
 * Errors: INVALID_ARG (sizes, NULL pointers, k > dimension, CSR structure),
 * NUMERIC (NaN/Inf in A), OUT_OF_MEMORY, DEVICE. */
rgdbek_status rgdbek_create(const rgdbek_matrix *A, const rgdbek_params *p,
                            void *stream, rgdbek_handle *out);

/* A batch of independent sparse systems solved together: A is their
 * block-diagonal concatenation in CSR with global indices -- system s owns
 * rows [row_off[s], row_off[s+1]) and columns [col_off[s], col_off[s+1]) and
 * no entry may leave that block (INVALID_ARG otherwise).  row_off/col_off:
 * host arrays of nsys+1.  Each system gets its own block sizes (from eta, or
 * k_col/k_row capped by the system's dimensions), its own generator stream
 * (system id in Philox counter word 3), iteration counter and stop test;
 * every residual pass and block-projection launch covers all systems.
 * rgdbek_solve then solves all systems (b, x, x_ref concatenated); it is
 * converged when every system is; rgdbek_batch_info gives the per-system
 * figures.  rgdbek_solve_adjoint solves every system's adjoint. */
rgdbek_status rgdbek_create_batched(const rgdbek_matrix *A, int64_t nsys,
                                    const int64_t *row_off,
                                    const int64_t *col_off,
                                    const rgdbek_params *p, void *stream,
                                    rgdbek_handle *out);

/* Many right-hand sides of one sparse matrix: solves A x_s = b_s for
 * s < nrhs.  A is stored once; the batch behaves as the block-diagonal
 * system I_nrhs (x) A with one system per right-hand side (own draws,
 * generator stream, iteration counter and stop test, as for
 * rgdbek_create_batched), and every pass over A serves all right-hand sides.
 * From 16 right-hand sides on, the passes and the CG products run over
 * interleaved copies of the vectors (entry j of right-hand side s at
 * j*nrhs + s), each stored entry read once for all right-hand sides; the
 * handle then holds three such buffers per precision, 3 * max(m, n) * nrhs
 * values.  Below 16, consecutive reads of a stored row belong to different
 * right-hand sides.  Vectors at the boundary are right-hand-side major:
 * b[s*m + i], x[s*n + j].  rgdbek_grad_pattern then sums the pattern
 * gradient over the right-hand sides. */
rgdbek_status rgdbek_create_multirhs(const rgdbek_matrix *A, int64_t nrhs,
                                     const rgdbek_params *p, void *stream,
                                     rgdbek_handle *out);

/* Per-system results of the last solve of a batch (host arrays of nsys, any
 * may be NULL): iterations run, last stop metric, converged flag. */
rgdbek_status rgdbek_batch_info(rgdbek_handle h, int64_t *iterations,
                                double *metric, int32_t *converged);

/* Solve A x = b (Algorithm 1 with the handle's parameters).
 *  b      device, m entries, FP64;
 *  x      device, n entries, FP64, output only (x_0 = 0);
 *  x_ref  device, n entries, FP64, required for STOP_ERR_REF, else NULL;
 *  info   host, may be NULL.
 * Returns OK when the stopping test held (or STOP_NONE ran max_iter),
 * NOT_CONVERGED when max_iter ran out first (x still holds the last iterate),
 * NUMERIC on NaN/Inf in b or a NaN weight during the solve. */
rgdbek_status rgdbek_solve(rgdbek_handle h, const void *b, void *x,
                           const void *x_ref, rgdbek_info *info);

/* As rgdbek_solve but resuming from a saved state: x (n) and z (m) are read
 * as x_{it0}, z_{it0} and overwritten with the final iterates, and the
 * generator counter starts at it0.  Running K iterations, then resuming for
 * K more, reproduces 2K uninterrupted iterations bit for bit. */
rgdbek_status rgdbek_solve_resume(rgdbek_handle h, const void *b, void *x,
                                  void *z, int64_t it0, const void *x_ref,
                                  rgdbek_info *info);

/* Copy the auxiliary vector z (m entries, FP64, device) of the last solve. */
rgdbek_status rgdbek_get_z(rgdbek_handle h, void *z);

/* Solve the adjoint system A^T w = g (n equations, m unknowns) with the same
 * kernels and storage: the roles of rows and columns swap, and the generator
 * uses key word 1 = 1.  g: device, n FP64; w: device, m FP64 (output).
 * Stop test: RES_EXT/RSE/NONE as set in the handle (ERR_REF is treated as
 * RES_EXT with the same tol). */
rgdbek_status rgdbek_solve_adjoint(rgdbek_handle h, const void *g, void *w,
                                   rgdbek_info *info);

/* Gradient of a loss through x = A^+ b restricted to A's sparsity pattern:
 * dA_values[e] = r_i lam_j - w_i x_j for each stored entry e = (i, j) of A
 * (for dense A every entry, row-major).  r, w: device, m FP64; lam, x:
 * device, n FP64; lam may be NULL (consistent systems, r = 0 term dropped);
 * dA_values: device, nnz (dense: m*n) FP64, output. */
rgdbek_status rgdbek_grad_pattern(rgdbek_handle h, const void *r,
                                  const void *lam, const void *w,
                                  const void *x, void *dA_values);

/* One block draw on given weights, exactly as the solver does it (for
 * parity tests): the k indices (ascending) drawn without replacement with
 * probability proportional to eps, through keys E_j / eps_j with
 * E_j = -ln(u_j), u_j from Philox4x64-10 counter (j>>2, it, phase, sys) and
 * key (seed, key1), word j&3 (Section 2 probabilities; Algorithm 1 block
 * draws).  Indices with eps_j <= floor * max(eps) (floor <= 0: eps_j == 0)
 * are never drawn; when at most k weights pass, all of them are returned.
 *  eps: device, d FP64;  out_idx: device, room for min(k, d) int32;
 *  out_count: host, receives the number of indices written.
 * NUMERIC if a weight is NaN, negative or infinite. */
rgdbek_status rgdbek_select(const double *eps, int64_t d, int64_t k,
                            double floor, uint64_t seed, uint64_t key1,
                            uint64_t it,
                            uint32_t phase, uint32_t sys, int32_t *out_idx,
                            int64_t *out_count, void *stream);

/* A block of size s from the law of Lemma 2.1 (Section 2): P(B) proportional
 * to the sum of eps over B among all s-subsets.  Drawn as the one-index draw
 * of rgdbek_select (k = 1, same arguments) followed by the s-1 smallest
 * exponential keys -ln(u'_j) over the other indices, u'_j from the Philox
 * stream of phase + 2; ascending indices; every weight zero (after the
 * floor) gives the empty block; s >= d gives every index.  Arguments as for
 * rgdbek_select (out_idx holds min(s, d) int32). */
rgdbek_status rgdbek_select_block_law(const double *eps, int64_t d, int64_t s,
                                      double floor, uint64_t seed,
                                      uint64_t key1, uint64_t it,
                                      uint32_t phase, uint32_t sys,
                                      int32_t *out_idx, int64_t *out_count,
                                      void *stream);

/* A block drawn with replacement (Section 2 probabilities, Algorithm 1's
 * "select k indices using P" read as k independent draws): the distinct
 * indices of k draws from P(j) = eps_j / sum eps, ascending.  The
 * probabilities are integer weights w_j = floor(eps_j / max(eps) * 2^sh),
 * sh = 63 - ceil(log2 d), zero where eps_j <= floor * max(eps); draw t maps
 * the Philox word u_t of index t (stream phase + 4, otherwise the
 * coordinates of rgdbek_select) to r_t = floor(u_t W / 2^64), W = sum w, and
 * takes the j whose cumulative interval [w_0+..+w_(j-1), w_0+..+w_j) holds
 * r_t.  All integer after the weights: bit-exact.  Every weight zero gives
 * the empty block.
 *  eps: device, d FP64 (d <= 16M);  k >= 1 draws;
 *  out_idx: device, room for min(k, d) int32;  out_count: host.
 * NUMERIC if a weight is NaN, negative or infinite; INVALID_ARG for d or
 * k out of range.  Synchronises the stream before returning. */
rgdbek_status rgdbek_select_iid(const double *eps, int64_t d, int64_t k,
                                double floor, uint64_t seed, uint64_t key1,
                                uint64_t it, uint32_t phase, uint32_t sys,
                                int32_t *out_idx, int64_t *out_count,
                                void *stream);

/* Largest d that rgdbek_select_noalloc accepts. */
#define RGDBEK_NOALLOC_MAX_D 1048576

/* rgdbek_select for callers that cannot allocate device memory (tight
 * serving loops, harnesses that forbid hipMalloc): the same draw, with the
 * same arguments and results bit for bit, but all of its work space lives
 * in one static device array of the library (about 8.6 MB, one copy per
 * GPU, held until the process ends) instead of hipMalloc'ed buffers; the
 * call allocates nothing, host or device.
 *  d must not exceed RGDBEK_NOALLOC_MAX_D (INVALID_ARG otherwise).
 *  Every call on one GPU shares that GPU's array: calls that overlap in
 *  time on one GPU (other threads, other streams) race and must not be
 *  issued; each call clears the parts it needs before its draw and
 *  synchronises the stream before returning.
 * Errors as rgdbek_select. */
rgdbek_status rgdbek_select_noalloc(const double *eps, int64_t d, int64_t k,
                                    double floor, uint64_t seed, uint64_t key1,
                                    uint64_t it, uint32_t phase, uint32_t sys,
                                    int32_t *out_idx, int64_t *out_count,
                                    void *stream);

/* GDBEK's greedy set (Section 2) on a weight vector: the indices j with
 * eps[j] > 0 and eps[j] >= eta * max(eps) (the product and comparison in
 * FP64), in ascending order, at most cap of them (the lowest indices when
 * more pass); every weight zero gives the empty set.
 *  eps      device, d FP64 weights (finite, >= 0; NUMERIC otherwise);
 *  eta      threshold in (0, 1];  cap >= 0;
 *  out_idx  device, cap int32 (may be NULL when cap == 0);
 *  out_count host, receives the set size (after the cap);
 *  stream   hipStream_t (NULL = default); synchronises it before returning. */
rgdbek_status rgdbek_select_threshold(const double *eps, int64_t d, double eta,
                                      int64_t cap, int32_t *out_idx,
                                      int64_t *out_count, void *stream);

/* One residual pass without a solve: ax = A x (m entries) and atz = A^T z
 * (n entries) -- the two products every iteration forms (the column residual
 * A^T z and the A x of the row residual, Section 2).  Dense A: one fused read
 * of the matrix; CSR: one CSR and one CSC pass.  precision RGDBEK_F64 uses
 * the FP64 storage (double vectors); RGDBEK_F32 the FP32 copy of a MIXED_F32
 * handle (float vectors).  All four pointers are device pointers.  Enqueued
 * on the handle's stream with no host synchronisation (for timing): ordered
 * after the work already on the caller's stream, and the caller's stream is
 * ordered after it (events), so results are ready for the caller's later
 * work.  For a batched handle the products are those of the block-diagonal
 * matrix; for a many-RHS handle those of I_nrhs (x) A (vectors of nrhs*n and
 * nrhs*m entries, right-hand side major). */
rgdbek_status rgdbek_apply(rgdbek_handle h, int32_t precision, const void *x,
                           const void *z, void *ax, void *atz);

/* Event timing of the last solve on a handle created with
 * RGDBEK_FLAG_PROFILE (see above): for region `region` (RGDBEK_PROF_*), the
 * number of timed executions in iterations that did work, their summed
 * duration in milliseconds, and the summed inner solver steps (CG steps of
 * the block solves; 0 for other regions).  Any output pointer may be NULL.
 * INVALID_ARG for an unknown region; UNSUPPORTED without the flag. */
rgdbek_status rgdbek_profile_read(rgdbek_handle h, int32_t region,
                                  int64_t *launches, double *ms,
                                  int64_t *steps);

/* Release everything the handle owns.  NULL is a no-op. */
rgdbek_status rgdbek_destroy(rgdbek_handle h);

/* Static description of a status code. */
const char *rgdbek_status_string(rgdbek_status s);

/* Message of the last error on h (empty string if none; h may be NULL for
 * errors raised before a handle existed). */
const char *rgdbek_last_error(rgdbek_handle h);

#ifdef __cplusplus
}
#endif
#endif /* RGDBEK_H */
