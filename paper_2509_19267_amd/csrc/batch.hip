// Per-system control of a batch of independent systems solved together
// (block-diagonal storage).  Every kernel runs one workgroup per system over
// that system's slice of the vectors, so per-system norms are reduced in a
// fixed order with no atomics.  The systems share every residual pass and
// every block-projection launch; only the block draws (select.hip, sel_seg),
// the stop tests and the iteration counters are per system.
#include "common.h"
#include "kernels.h"

namespace rg {

constexpr int BT = 256;

// ref2_s = ||v_s||^2 over the system's column (cols != 0) or row range
template <typename T>
__global__ void __launch_bounds__(BT)
seg_ref2_kernel(const T *__restrict__ v, SegInfo *seg, int cols) {
  __shared__ double sh[BT / WAVE];
  SegInfo &g = seg[blockIdx.x];
  const int64_t off = cols ? g.col_off : g.row_off;
  const int64_t len = cols ? g.ncol : g.nrow;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < len; i += BT) {
    const double a = (double)v[off + i];
    s += a * a;
  }
  s = block_sum<BT>(s, sh);
  if (threadIdx.x == 0) g.ref2 = s;
}

// Reset the per-system state at the start of a solve or refinement pass:
// systems already accepted by an FP64 test (fixed) stay done.
__global__ void seg_reset_kernel(SegInfo *seg, int nseg, int64_t it0,
                                 int keep_it, const int32_t *fixed) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  SegInfo &g = seg[s];
  if (!keep_it) g.it = it0;
  g.iters_run = 0;
  g.pref = 0.0;
  const int f = fixed ? fixed[s] : 0;
  g.done = f;
  g.converged = f;
  g.metric = 0.0;
}

// ERR_REF per system: ||x_base + x - x_ref|| / ||x_ref|| <= tol.
template <typename T>
__global__ void __launch_bounds__(BT)
seg_err_ref_kernel(const T *__restrict__ x, const double *__restrict__ xr,
                   const double *__restrict__ xb, SegInfo *seg, Ctrl *ctrl,
                   int respect_done) {
  const double tol = ctrl->tol;
  if (respect_done && ctrl_done(ctrl)) return;
  __shared__ double sh[BT / WAVE];
  SegInfo &g = seg[blockIdx.x];
  if (respect_done && g.done) return;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < g.ncol; i += BT) {
    const int64_t j = g.col_off + i;
    const double e = (xb ? xb[j] : 0.0) + (double)x[j] - xr[j];
    s += e * e;
  }
  s = block_sum<BT>(s, sh);
  if (threadIdx.x == 0) {
    const double m = g.ref2 > 0.0 ? sqrt(s / g.ref2) : sqrt(s);
    g.metric = m;
    if (m <= tol) { g.done = 1; g.converged = 1; }
  }
}

// RSE / RES_EXT per system from r = b - z - A x and z of the row pass:
// RSE = ||r + z||^2 / ||b_s||^2, RES_EXT = ||r|| / ||b_s||; in a refinement
// pass (Ctrl::pass_drop > 0) also passed at pass_drop times the system's
// first metric of the pass.
template <typename T>
__global__ void __launch_bounds__(BT)
seg_stop_rowres_kernel(const T *__restrict__ r, const T *__restrict__ z,
                       SegInfo *seg, int mode, Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  const double tol = ctrl->tol;
  __shared__ double sh[BT / WAVE];
  SegInfo &g = seg[blockIdx.x];
  if (respect_done && g.done) return;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < g.nrow; i += BT) {
    const int64_t j = g.row_off + i;
    const double v = mode == 2 ? (double)r[j] + (double)z[j] : (double)r[j];
    s += v * v;
  }
  s = block_sum<BT>(s, sh);
  if (threadIdx.x == 0) {
    const double den = g.ref2 > 0.0 ? g.ref2 : 1.0;
    const double m = mode == 2 ? s / den : sqrt(s / den);
    g.metric = m;
    double thr = tol;
    if (ctrl->pass_drop > 0.0) {
      if (g.pref <= 0.0) g.pref = m;
      const double rel = ctrl->pass_drop * g.pref;
      thr = rel > thr ? rel : thr;
    }
    if (m <= thr) { g.done = 1; g.converged = 1; }
  }
}

// Fold the systems: Ctrl::done when every system is done, Ctrl::converged
// when every system passed its test; Ctrl::metric is the largest system
// metric and Ctrl::iters_run the largest per-system iteration count.  With
// end_iter, each running system first advances its counters (and stops at
// the cap).  force evaluates even after Ctrl::done.
__global__ void __launch_bounds__(BT)
seg_fold_kernel(SegInfo *seg, int nseg, Ctrl *ctrl, int end_iter,
                int64_t cap, int force) {
  if (!force && ctrl_done(ctrl)) return;
  __shared__ int s_done[BT], s_conv[BT];
  __shared__ double s_met[BT];
  __shared__ int64_t s_it[BT];
  double met = 0.0;
  int64_t its = 0;
  int all_done = 1, all_conv = 1;
  for (int s = threadIdx.x; s < nseg; s += BT) {
    SegInfo &g = seg[s];
    if (end_iter && !g.done) {
      g.it += 1;
      g.iters_run += 1;
      if (g.iters_run >= cap) g.done = 1;
    }
    all_done &= (g.done != 0);
    all_conv &= (g.converged != 0);
    met = g.metric > met ? g.metric : met;
    its = g.iters_run > its ? g.iters_run : its;
  }
  s_done[threadIdx.x] = all_done;
  s_conv[threadIdx.x] = all_conv;
  s_met[threadIdx.x] = met;
  s_it[threadIdx.x] = its;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < BT; ++i) {
      met = s_met[i] > met ? s_met[i] : met;
      its = s_it[i] > its ? s_it[i] : its;
      all_done &= s_done[i];
      all_conv &= s_conv[i];
    }
    ctrl->metric = met;
    ctrl->iters_run = its;
    ctrl->converged = all_conv;
    if (end_iter) ctrl->it += 1;
    if (all_done || ctrl->numeric || ctrl->sync_fail) ctrl->done = 1;
  }
}

__global__ void seg_converged_kernel(const SegInfo *seg, int nseg,
                                     int32_t *flags) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nseg) flags[s] = seg[s].converged;
}

template <typename T>
void launch_seg_ref2(const T *v, SegInfo *seg, int nseg, int cols,
                     hipStream_t st) {
  hipLaunchKernelGGL(seg_ref2_kernel<T>, dim3(nseg), dim3(BT), 0, st, v, seg,
                     cols);
}
void launch_seg_reset(SegInfo *seg, int nseg, int64_t it0, int keep_it,
                      const int32_t *fixed, hipStream_t st) {
  hipLaunchKernelGGL(seg_reset_kernel, dim3((nseg + 255) / 256), dim3(256), 0,
                     st, seg, nseg, it0, keep_it, fixed);
}
template <typename T>
void launch_seg_err_ref(const T *x, const double *xr, const double *xb,
                        SegInfo *seg, int nseg, Ctrl *ctrl, int respect_done,
                        hipStream_t st) {
  hipLaunchKernelGGL(seg_err_ref_kernel<T>, dim3(nseg), dim3(BT), 0, st, x, xr,
                     xb, seg, ctrl, respect_done);
}
template <typename T>
void launch_seg_stop_rowres(const T *r, const T *z, SegInfo *seg, int nseg,
                            int mode, Ctrl *ctrl, int respect_done,
                            hipStream_t st) {
  hipLaunchKernelGGL(seg_stop_rowres_kernel<T>, dim3(nseg), dim3(BT), 0, st, r,
                     z, seg, mode, ctrl, respect_done);
}
void launch_seg_fold(SegInfo *seg, int nseg, Ctrl *ctrl, int end_iter,
                     int64_t cap, int force, hipStream_t st) {
  hipLaunchKernelGGL(seg_fold_kernel, dim3(1), dim3(BT), 0, st, seg, nseg,
                     ctrl, end_iter, cap, force);
}
void launch_seg_converged(const SegInfo *seg, int nseg, int32_t *flags,
                          hipStream_t st) {
  hipLaunchKernelGGL(seg_converged_kernel, dim3((nseg + 255) / 256), dim3(256),
                     0, st, seg, nseg, flags);
}

template void launch_seg_ref2<double>(const double *, SegInfo *, int, int, hipStream_t);
template void launch_seg_ref2<float>(const float *, SegInfo *, int, int, hipStream_t);
template void launch_seg_err_ref<double>(const double *, const double *, const double *, SegInfo *, int, Ctrl *, int, hipStream_t);
template void launch_seg_err_ref<float>(const float *, const double *, const double *, SegInfo *, int, Ctrl *, int, hipStream_t);
template void launch_seg_stop_rowres<double>(const double *, const double *, SegInfo *, int, int, Ctrl *, int, hipStream_t);
template void launch_seg_stop_rowres<float>(const float *, const float *, SegInfo *, int, int, Ctrl *, int, hipStream_t);

}  // namespace rg
