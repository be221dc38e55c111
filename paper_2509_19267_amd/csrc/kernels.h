// Launchers of the RGDBEK kernels (host-callable, defined in the .hip files).
// Every launcher enqueues on the given stream and does not synchronise.
// Kernels of the solve loop read Ctrl::done first (respect_done != 0) so that
// a captured graph of several iterations turns into no-ops after the stop.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace rg {

// ------------------------------------------------------------ selection
constexpr int64_t SEL_SMALL_MAX = 65536;  // one workgroup up to this size

// Global scratch of the persistent (one-launch) selection.
struct SelPersist {
  unsigned gh[6][2048];           // digit histograms, one per radix level
  uint64_t ckey[4096];            // candidates of the final bucket
  int64_t cidx[4096];
  double gmax[1024];              // per-workgroup largest weight
  int64_t cnt[1024];              // per-workgroup taken / tie counts
  unsigned long long gpos, ncand; // positive weights, candidates gathered
  int64_t tidx;                   // tie index found by its owner
};
// Largest d the persistent selection takes for `ncu` compute units (0: none).
int64_t select_persist_max(int ncu);

struct SelectScratch {
  SelPersist *pers = nullptr; // persistent selection scratch
  int ncu = 0;                // compute units (grid bound of that launch)
  uint64_t *keys = nullptr;   // d keys
  unsigned *hist = nullptr;   // 2048 bins (zeroed at allocation)
  uint64_t *ckey = nullptr;   // 4096 candidate keys
  int64_t *cidx = nullptr;    // 4096 candidate indices
  int32_t *blk = nullptr;     // per-chunk counts
  double *gmax = nullptr;     // per-chunk maxima (greedy sets)
};
int64_t select_scratch_blocks(int64_t d);
int64_t select_greedy_blocks(int64_t d);

// Block from the law of Lemma 2.1 (Section 2), size s (see select.hip); w:
// d doubles of scratch, tmp: s ints of scratch.
// Draws with replacement (select.hip): integer cumulative weights, flags.
struct IidScratch {
  uint64_t *ploc = nullptr;   // in-chunk inclusive weight sums (d)
  uint64_t *ctot = nullptr;   // chunk totals
  int32_t *flags = nullptr;   // one per index, zero between calls
};
int64_t select_iid_chunks(int64_t d);
int64_t select_iid_max_d();
template <typename T>
void launch_select_iid(const T *eps, int64_t d, int64_t k, double floor,
                       uint64_t seed, uint64_t key1, uint32_t phase,
                       uint32_t sys, int ph, SelectScratch &s, IidScratch &w,
                       int32_t *out, Ctrl *ctrl, int respect_done,
                       hipStream_t st);
template <typename T>
void launch_select_block_law(const T *eps, int64_t d, int64_t s, double floor,
                             uint64_t seed, uint64_t key1, uint32_t phase,
                             uint32_t sys, int ph, SelectScratch &sc,
                             double *w, int32_t *tmp, int32_t *out,
                             Ctrl *ctrl, int respect_done, hipStream_t st);

// GDBEK's greedy set {j : eps_j >= eta * max eps, eps_j > 0} (Section 2),
// ascending, at most cap indices; count to Ctrl::sel_count[ph].
template <typename T>
void launch_select_greedy(const T *eps, int64_t d, double eta, int64_t cap,
                          int ph, SelectScratch &s, int32_t *out, Ctrl *ctrl,
                          int respect_done, hipStream_t st);

// eps: d weights (T promoted to FP64 before the key division); weights not
// above floor * max(eps) count as zero.  ph selects the Ctrl slot (0 columns,
// 1 rows); the iteration number is Ctrl::it.
template <typename T>
void launch_select(const T *eps, int64_t d, int64_t k, double floor,
                   uint64_t seed, uint64_t key1, uint32_t phase, uint32_t sys,
                   int ph, SelectScratch &s, int32_t *out, Ctrl *ctrl,
                   int respect_done, hipStream_t st);

// Per-system draws for a block-diagonal batch (one workgroup per system);
// the concatenated global index list goes to out, its length to
// Ctrl::sel_count[ph].  dmax: the largest system dimension of the phase;
// segmax/tmp/cnt: scratch (nseg / sum of block sizes / nseg).
template <typename T>
void launch_select_seg(const T *eps, const SegInfo *seg, int nseg, int ph,
                       int64_t dmax, double floor, uint64_t seed,
                       uint64_t key1, uint32_t phase, uint64_t *keys,
                       double *segmax, int32_t *tmp, int64_t *cnt,
                       int32_t *out, Ctrl *ctrl, int respect_done,
                       hipStream_t st);

// Per-system control of a batch (batch.hip): reference norms, state reset,
// ERR_REF / RSE / RES_EXT per system, and the fold into Ctrl.
template <typename T>
void launch_seg_ref2(const T *v, SegInfo *seg, int nseg, int cols,
                     hipStream_t st);
void launch_seg_reset(SegInfo *seg, int nseg, int64_t it0, int keep_it,
                      const int32_t *fixed, hipStream_t st);
template <typename T>
void launch_seg_err_ref(const T *x, const double *xr, const double *xb,
                        SegInfo *seg, int nseg, Ctrl *ctrl, int respect_done,
                        hipStream_t st);
template <typename T>
void launch_seg_stop_rowres(const T *r, const T *z, SegInfo *seg, int nseg,
                            int mode, Ctrl *ctrl, int respect_done,
                            hipStream_t st);
void launch_seg_fold(SegInfo *seg, int nseg, Ctrl *ctrl, int end_iter,
                     int64_t cap, int force, hipStream_t st);
void launch_seg_converged(const SegInfo *seg, int nseg, int32_t *flags,
                          hipStream_t st);

// ------------------------------------------------------------ matrices
template <typename T>
struct Csr {                 // CSR (or CSC viewed as CSR of the transpose)
  int64_t rows = 0, cols = 0, nnz = 0;
  const int64_t *ptr = nullptr;
  const int32_t *idx = nullptr;
  const T *val = nullptr;
  int group = 8;             // lanes per segment (power of two)
  const int32_t *longs = nullptr;  // base segments longer than the limit
  int64_t nlong = 0;
  int64_t long_limit = 0;
  // rows handled as long segments, when that is decided by membership rather
  // than by length (the block copies keep the long rows of A as long)
  const uint8_t *long_flag = nullptr;
  // Merge-chunk plan of full passes (rep == 1): chunk c holds nonzeros
  // [c*MP_CH, (c+1)*MP_CH) and owns the rows whose first nonzero position
  // ptr[r] lies in it (mp_rs[c] .. mp_rs[c+1]-1; mp_rs[nchunk] = rows); rows
  // spanning chunks are listed (mp_xrow, first/last chunk) and finished by a
  // second launch from per-chunk head/lead partials.
  const int32_t *mp_rs = nullptr;
  int64_t mp_nchunk = 0;
  const int32_t *mp_xrow = nullptr, *mp_xcs = nullptr, *mp_xce = nullptr;
  int64_t mp_ncross = 0;
  T *mp_head = nullptr, *mp_lead = nullptr;   // nchunk each
  // Replicated operator I_rep (x) A for many right-hand sides: the stored
  // matrix is the base (brows x bcols); rows = rep * brows virtual rows.
  // Virtual segments are visited in RHS-minor order (slot = i * rep + s) so
  // the rep reads of one stored row follow each other and hit in cache.
  int64_t rep = 1, brows = 0, bcols = 0;
  // Interleaved scratch of the many-right-hand-side products (rep >=
  // REP_MM_MIN): max(brows, bcols) * rep entries each, input and output.
  T *rep_in = nullptr, *rep_out = nullptr;
  // Row ends when rows are not contiguous (the block copies of one stored
  // matrix keep A's row starts): row r spans [ptr[r], pend[r]).
  const int64_t *pend = nullptr;
};
template <typename T>
__device__ __forceinline__ int64_t seg_end(const Csr<T> &A, int64_t r) {
  return A.pend ? A.pend[r] : A.ptr[r + 1];
}

// slot of a full sweep -> global row, stored row, column offset
template <typename T>
__device__ __forceinline__ void vrow(const Csr<T> &A, int64_t slot,
                                     int64_t &grow, int64_t &brow,
                                     int64_t &coff) {
  if (A.rep == 1) { grow = slot; brow = slot; coff = 0; return; }
  brow = slot / A.rep;
  const int64_t s = slot - brow * A.rep;
  grow = s * A.brows + brow;
  coff = s * A.bcols;
}
// global row (from an index list) -> stored row, column offset
template <typename T>
__device__ __forceinline__ void gsplit(const Csr<T> &A, int64_t g,
                                       int64_t &brow, int64_t &coff) {
  if (A.rep == 1) { brow = g; coff = 0; return; }
  const int64_t s = g / A.brows;
  brow = g - s * A.brows;
  coff = s * A.bcols;
}

template <typename T>
struct Dense {               // row-major rows x cols with leading dim ld
  int64_t rows = 0, cols = 0, ld = 0;
  const T *a = nullptr;
};

// Scratch for multi-block reductions: `part` holds per-block partials.
struct Reduce {
  double *part = nullptr;    // >= 2 * max blocks
  int64_t cap = 0;
};

// ------------------------------------------------------------ residuals
// Sparse segment dots y_s = sum_e val[e] v[idx[e]] for every segment s (or
// only the segments listed in `list` (count read from *count_dev)), with an
// epilogue selected by `epi`:
enum Epi {
  EPI_STORE = 0,      // out[s] = y
  EPI_COLRES = 1,     // g[s] = y (+ off[s]); eps[s] = g^2 / nrm[s]
  EPI_ROWRES = 2,     // r[s] = b[s] - z[s] - y; eps[s] = r^2 / nrm[s];
                      // partials of ||b - y||^2 and ||r||^2
  EPI_LIST_STORE = 3, // out[k] = y for the k-th listed segment
};
template <typename T>
struct SegArgs {
  const T *v = nullptr;      // vector gathered by idx
  T *out = nullptr;          // EPI_STORE / EPI_LIST_STORE
  T *g = nullptr;            // EPI_COLRES output
  const T *off = nullptr;    // EPI_COLRES offset (nullable)
  T *eps = nullptr;          // weights output
  const double *nrm = nullptr;  // squared norms (FP64)
  const T *b = nullptr, *z = nullptr;  // EPI_ROWRES inputs
  T *r = nullptr;            // EPI_ROWRES output
  double *part = nullptr;    // EPI_ROWRES partials (2 per block)
  const int32_t *list = nullptr;  // listed segments
  const int64_t *count_dev = nullptr;
  int64_t list_cap = 0;
};
template <typename T>
int launch_segdot(const Csr<T> &A, int epi, const SegArgs<T> &a, Ctrl *ctrl,
                  int respect_done, hipStream_t st);   // returns #partials
// nonzeros per merge chunk (one wave); partial slots a full pass may use
constexpr int64_t MP_CH = 256;
int64_t segdot_max_parts(int64_t rows, int64_t nnz, int64_t nchunk,
                         int64_t ncross, int64_t nlong, int64_t rep);

// Dense fused pass: q = A x and g = A^T z from one read of A; then the
// finalise step forms g (+ off), eps^z = g^2/kappa, and q.
template <typename T>
struct DenseWork {
  T *qpart = nullptr;        // nch * rows
  T *gpart = nullptr;        // nrg * ld
  int nch = 0, nrg = 0;      // column chunks, row tiles
  int rpw = 0;               // rows per row tile
};
template <typename T>
void dense_work_shape(const Dense<T> &A, int tile_rows, int target_wgs,
                      int *nch, int *nrg, int *rpw);
template <typename T>
void launch_dense_fused(const Dense<T> &A, const T *x, const T *z,
                        DenseWork<T> &w, const T *off, const double *kappa,
                        T *g, T *eps, T *q, Ctrl *ctrl, int respect_done,
                        hipStream_t st);
// r = b - z - q, eps^x = r^2/rho, partials of ||b-q||^2, ||r||^2
template <typename T>
int launch_rowres_dense(int64_t m, const T *b, const T *z, const T *q,
                        const double *rho, T *r, T *eps, double *part,
                        Ctrl *ctrl, int respect_done, hipStream_t st);

// Stop tests.  ERR_REF at the top of an iteration (x vs x_ref); RSE/RES_EXT
// from the row-residual partials.  Sets Ctrl::done/converged/metric.
template <typename T>
void launch_err_ref(int64_t n, const T *x, const double *x_ref,
                    const double *x_base, Reduce &red, Ctrl *ctrl,
                    int respect_done, hipStream_t st);
// Ctrl::ref2 = sum v_i^2 (FP64), one workgroup.
template <typename T>
void launch_set_ref2(int64_t n, const T *v, Ctrl *ctrl, hipStream_t st);
void launch_stop_rowres(const double *part, int nparts, Ctrl *ctrl,
                        hipStream_t st);
void launch_end_iter(Ctrl *ctrl, hipStream_t st);

// ------------------------------------------------------------ projections
// Dense Gram of listed rows of X (row-major, ld): G[a][b] = <X_la, X_lb>,
// for a, b < count (read from *count_dev, at most cap).
template <typename T>
void launch_gram_rows(const T *X, int64_t ld, int64_t len, const int32_t *list,
                      const int64_t *count_dev, int64_t cap, T *G,
                      Ctrl *ctrl, int respect_done, hipStream_t st);
// Gather G[a][b] = F[l_a * ldf + l_b] from a precomputed Gram F.
template <typename T>
void launch_gram_gather(const T *F, int64_t ldf, const int32_t *list,
                        const int64_t *count_dev, int64_t cap, T *G,
                        Ctrl *ctrl, int respect_done, hipStream_t st);
// Full Gram of all rows of X into F (ld = rows): used once at create.
template <typename T>
void launch_gram_full(const T *X, int64_t ldx, int64_t rows, int64_t len,
                      T *F, hipStream_t st);

// Cholesky factor of G (cap x cap storage, count from *count_dev) in place
// and solve G y = h (h gathered through hlist from hsrc, or given).  One
// workgroup; for counts up to CHOL_MAX.
constexpr int64_t CHOL_MAX = 512;
template <typename T>
void launch_chol_solve(T *G, int64_t cap, const int64_t *count_dev,
                       const T *hsrc, const int32_t *hlist, T *y, int factor,
                       Ctrl *ctrl, int ph, int respect_done, hipStream_t st);

// Preconditioned CG on the gathered Gram G y = h (Jacobi).  init + steps.
template <typename T>
struct CgWork {
  T *res = nullptr, *v = nullptr, *zz = nullptr;
  T *p = nullptr;            // 2 * cap (direction, alternating by step)
  int64_t cap = 0;
  double *pv = nullptr;      // per-block <p, v> partials (cap/4 + 1)
  double *part = nullptr;    // 2 parities x 2 x part_cap (<r,zz>, <r,r>)
  int64_t part_cap = 0;      // cap/256 + 1
  double *rzs = nullptr;     // rz by step parity (2)
  T *v2 = nullptr;           // persistent PCG: G p by step parity (2 * cap)
  double *pv2 = nullptr;     // persistent PCG: <p, v> partials (2 * grid)
};
// Persistent PCG (one launch per projection): largest Gram dimension and
// grid size for a given dimension.
int64_t pcg_persist_cap(bool f64);
int pcg_persist_grid(int64_t cap, int ncu);
template <typename T>
// F != nullptr: G has not been gathered; the first step reads the block
// rows of the full Gram F (leading dimension ldf) through hlist and stores
// them packed into G (cap x cap) for the later steps
void launch_pcg_persist(T *G, int64_t cap, const int64_t *count_dev,
                        const T *hsrc, const int32_t *hlist, T *y,
                        CgWork<T> &w, int grid, int max_steps, double tol,
                        Ctrl *ctrl, int ph, int respect_done, hipStream_t st,
                        const T *F = nullptr, int64_t ldf = 0);
// largest Gram dimension the PCG kernels accept (direction staged in LDS)
int64_t pcg_cap_max();
template <typename T>
void launch_pcg_gram_init(const T *G, int64_t cap, const int64_t *count_dev,
                          const T *hsrc, const int32_t *hlist, T *y,
                          CgWork<T> &w, Ctrl *ctrl, int ph, int respect_done,
                          hipStream_t st);
template <typename T>
void launch_pcg_gram_step(const T *G, int64_t cap, const int64_t *count_dev,
                          T *y, CgWork<T> &w, int step, double tol,
                          Ctrl *ctrl, int ph, int respect_done,
                          hipStream_t st);

// Dense thin updates.
// z[i] -= sum_a y_a * Acm[list_a * ldc + i]   (columns of A, column-major)
// scratch: thin_update_scratch(len, cap) entries of T.
template <typename T>
void launch_col_update(const T *Acm, int64_t ldc, int64_t m,
                       const int32_t *list, const int64_t *count_dev,
                       int64_t cap, const T *y, T *z, T *scratch, Ctrl *ctrl,
                       int respect_done, hipStream_t st);
// x[j] += sum_a w_a * Arm[list_a * ld + j]     (rows of A, row-major)
template <typename T>
void launch_row_update(const T *Arm, int64_t ld, int64_t n,
                       const int32_t *list, const int64_t *count_dev,
                       int64_t cap, const T *w, T *x, T *scratch, Ctrl *ctrl,
                       int respect_done, hipStream_t st);
int64_t thin_update_scratch(int64_t len, int64_t cap);
// s_a = h_{l_a} - <A_{l_a}, v>, listed rows of a row-major matrix against v
// (residual of projected equations, used for one refinement sweep).
// s_a = h1[l_a] - h2[l_a] - <A_{l_a}, v>   (h2 nullable)
template <typename T>
void launch_list_resid(const T *Arm, int64_t ld, int64_t len,
                       const int32_t *list, const int64_t *count_dev,
                       int64_t cap, const T *h1, const T *h2, const T *v,
                       T *s, Ctrl *ctrl, int respect_done, hipStream_t st);

// Sparse block projections (matrix-free CG).  See proj.hip.
template <typename T>
struct SparseCg {
  T *phat = nullptr;    // wide masked direction (n for columns, m for rows)
  T *wide = nullptr;    // wide product (m for columns, n for rows)
  T *p = nullptr, *res = nullptr, *v = nullptr;  // narrow (cap)
  double *part = nullptr;
  int64_t part_cap = 0;     // entries of part
  int32_t *pos = nullptr;   // block position of each index, -1 outside
  double *plong = nullptr;  // one partial per long segment
  int split = 0;            // many-workgroup step finish at any block size
  // many right-hand sides (rep >= REP_MM_MIN): interleaved product buffers,
  // max(brows, bcols) * rep entries each
  T *t0 = nullptr, *t1 = nullptr, *t2 = nullptr;
};
// Small sparse systems (both dimensions up to SPARSE_GRAM_MAX): dense
// copies for the Gram matrices, and the block update out += sign A_L coef
// (A_L the listed columns of A, as rows of the CSR view given).
constexpr int64_t SPARSE_GRAM_MAX = 4096;
template <typename T>
void launch_densify(const Csr<T> &A, T *rm, int64_t ld, T *cm, int64_t ldc,
                    hipStream_t st);
template <typename T>
void launch_sparse_block_update(const Csr<T> &A, const int32_t *list,
                                const int64_t *count_dev, int64_t cap,
                                const T *coef, int sign, T *phat, T *out,
                                Ctrl *ctrl, int respect_done, hipStream_t st);
template <typename T>
void launch_sparse_colproj(const Csr<T> &csr, const Csr<T> &csc,
                           const int32_t *U, const int64_t *count_dev,
                           int64_t cap, const T *g, T *z, SparseCg<T> &w,
                           int max_steps, double tol, Ctrl *ctrl,
                           int respect_done, hipStream_t st);
template <typename T>
void launch_sparse_rowproj(const Csr<T> &csr, const Csr<T> &csc,
                           const int32_t *J, const int64_t *count_dev,
                           int64_t cap, const T *r, const double *rho, T *x,
                           SparseCg<T> &w, int max_steps, double tol,
                           Ctrl *ctrl, int respect_done, hipStream_t st);

// Block-restricted copy of a CSR (or of the CSC, as the CSR of A^T): the
// entries whose column is in the current block, in storage order, with
// their original indices, rebuilt once per iteration so that every CG step
// of the block projection streams only them (see proj.hip).
struct SubWork {
  int64_t *ptr = nullptr;    // rows + 1
  int64_t *cnt = nullptr;    // rows + 1 (counts, then scratch)
  int64_t *tile = nullptr;   // per-tile sums of the scan
  int32_t *idx = nullptr;    // capacity nnz
  void *val = nullptr;       // capacity nnz values
  int32_t *mask = nullptr;   // one flag per column, zero between calls
  uint8_t *long_flag = nullptr;  // rows of A that are long segments
  int64_t cap = 0;           // entry capacity
  int group = 1;             // lanes per row for the compact matrix
};
template <typename T>
Csr<T> launch_sub_matrix(const Csr<T> &A, const int32_t *list,
                         const int64_t *count_dev, int64_t list_cap,
                         SubWork &w, Ctrl *ctrl, hipStream_t st);
int64_t sub_scan_tiles(int64_t n);
// long_flag[r] = 1 for the rows of A longer than A.long_limit
template <typename T>
void launch_mark_long(const Csr<T> &A, uint8_t *flag, hipStream_t st);

// Row blocks taller than A is wide (k_row > n): CGLS on min ||A^J d - r^J||
// (see proj.hip).  d, p, s: n entries; res, q: cap; rhat: m (sparse only:
// the residual scattered onto the block's rows, zero elsewhere).
template <typename T>
struct TallWork {
  T *d = nullptr, *p = nullptr, *s = nullptr;
  T *res = nullptr, *q = nullptr;
  T *rhat = nullptr;
};
template <typename T>
void launch_tall_rowproj_dense(const Dense<T> &A, const int32_t *J,
                               const int64_t *count_dev, int64_t cap,
                               const T *r, T *x, TallWork<T> &w, T *upd,
                               int max_steps, double tol, Ctrl *ctrl,
                               hipStream_t st);
template <typename T>
void launch_tall_rowproj_sparse(const Csr<T> &csr, const Csr<T> &csc,
                                const int32_t *J, const int64_t *count_dev,
                                int64_t cap, const T *r, T *x, TallWork<T> &w,
                                int max_steps, double tol, Ctrl *ctrl,
                                hipStream_t st);

// ------------------------------------------------------------ utilities
template <typename Tout, typename Tin>
void launch_convert(const Tin *in, Tout *out, int64_t n, hipStream_t st);
// copy rows x cols row-major (ld_in) into padded row-major (ld_out) and its
// column-major transpose (ld_t); pads are zero.
template <typename Tout, typename Tin>
void launch_pack_dense(const Tin *in, int64_t rows, int64_t cols,
                       int64_t ld_in, Tout *out_rm, int64_t ld_out,
                       Tout *out_cm, int64_t ld_t, hipStream_t st);
template <typename T>
void launch_sqnorms_dense(const T *Arm, int64_t rows, int64_t cols,
                          int64_t ld, const T *Acm, int64_t ldc,
                          double *rho, double *kappa, hipStream_t st);
template <typename T>
void launch_sqnorms_csr(const Csr<T> &A, double *out, hipStream_t st);
// flag[0] |= any non-finite among n values
template <typename T>
void launch_check_finite(const T *v, int64_t n, int *flag, hipStream_t st);
// CSR -> CSC transpose on the device (stable: rows ascending in a column)
template <typename T>
void launch_csr_to_csc(int64_t m, int64_t n, int64_t nnz, const int64_t *rp,
                       const int32_t *ci, const T *v, int64_t *cp, int32_t *ri,
                       T *cv, int64_t *work, hipStream_t st);
// pattern gradient: dA[e] = sum_s (r_i lam_j - w_i x_j) over stored entries
// (s over the rep right-hand sides sharing A; vectors RHS-major)
void launch_grad_pattern_csr(int64_t m, int64_t n, int64_t rep,
                             const int64_t *rp, const int32_t *ci,
                             const double *r, const double *lam,
                             const double *w, const double *x, double *dA,
                             hipStream_t st);
// out[s*len + i] = in[i] for s < rep (replicate a base vector)
void launch_replicate(const double *in, int64_t len, int64_t rep,
                      double *out, hipStream_t st);
void launch_grad_pattern_dense(int64_t m, int64_t n, const double *r,
                               const double *lam, const double *w,
                               const double *x, double *dA, hipStream_t st);
// y = alpha*y + beta*x (elementwise, FP types mixed through double)
template <typename Ty, typename Tx>
void launch_axpby(int64_t n, double alpha, Ty *y, double beta, const Tx *x,
                  hipStream_t st);
void launch_fill_ctrl_it(Ctrl *ctrl, int64_t it, hipStream_t st);
// Profiling marks (runtime profile mode): post == 0 records whether the
// solve is still running (Ctrl::done clear), post == 1 the CG steps of
// phase ph (ph < 0: none).
struct ProfRec {
  int32_t live;
  int32_t steps;
};
void launch_prof_mark(const Ctrl *ctrl, ProfRec *rec, int post, int ph,
                      hipStream_t st);

// ------------------------------------------------------------ many RHS
// With many right-hand sides sharing A (the replicated operator I_rep (x) A)
// the products run over interleaved vectors -- entry j of right-hand side s
// at j * rep + s -- so one read of each stored entry serves every
// right-hand side and the gathered values of one entry are contiguous.
// Vectors stay right-hand-side-major elsewhere; the transposes convert.
constexpr int64_t REP_MM_MIN = 16;
// out[r * rep + s] = sum_e A.val[e] * in[A.idx[e] * rep + s] over the stored
// rows r < A.brows; part (nullable): per-workgroup sums of out^2, returns
// their count.  ph >= 0: skipped once the CG of that phase is done.
template <typename T>
int launch_rep_mm(const Csr<T> &A, const T *in, T *out, double *part,
                  Ctrl *ctrl, int ph, int respect_done, hipStream_t st);
// in[s * len + i] -> out[i * rep + s]
template <typename T>
void launch_rep_tin(const T *in, T *out, int64_t len, int64_t rep, Ctrl *ctrl,
                    int ph, int respect_done, hipStream_t st);
// in[i * rep + s] -> out[s * len + i]; with x: x += alpha_ph * out (the old
// value) first, alpha_ph = Ctrl::cg_alpha[ph] (the row CG's pending update)
template <typename T>
void launch_rep_tout(const T *in, T *out, T *x, int64_t len, int64_t rep,
                     Ctrl *ctrl, int ph, int respect_done, hipStream_t st);

}  // namespace rg
