// Products of one stored sparse matrix with many right-hand sides at once
// (the replicated operator I_rep (x) A of the multi-right-hand-side solver,
// Section 6's deblurring of many images with one blur).
//
// The right-hand sides' vectors are held interleaved here -- entry j of
// right-hand side s at j * rep + s -- so that a wave takes one stored row
// and 64 right-hand sides, one per lane: the row's entries are loaded once
// by the wave and broadcast lane by lane (v_readlane), and the values the
// lanes gather for one entry are 64 contiguous elements (one 512-byte run
// in FP64).  With at most 32 right-hand sides a wave takes 2 or 4 rows, 32
// or 16 lanes each.  The right-hand-side-major layout of the rest of the
// solver would make each lane gather from a different vector, and each
// stored entry would be read once per right-hand side.
#include "common.h"
#include "kernels.h"

namespace rg {

constexpr int REP_NT = 256;            // 4 waves: 4 stored rows per workgroup
constexpr int REP_ROWS = REP_NT / WAVE;
// gathers in flight per lane (measured on the 512^2 blur, 64 right-hand
// sides: 8 gain 16% over 4 in FP32, nothing in FP64)
template <typename T> struct REP_UNR { static constexpr int n = 4; };
template <> struct REP_UNR<float> { static constexpr int n = 8; };

__device__ __forceinline__ int bcast(int v, int j) {
  return __builtin_amdgcn_readlane(v, j);
}
__device__ __forceinline__ float bcast(float v, int j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}
__device__ __forceinline__ double bcast(double v, int j) {
  const int64_t b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), j);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), j);
  return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

// One wave per stored row r, lane = right-hand side s (blockIdx.y selects
// the group of 64).  Lanes past rep gather from right-hand side 0 (in
// bounds) and store nothing.  Every lane of the wave runs the entry loop
// (row and bounds are wave-uniform), as v_readlane needs.
// RC: the right-hand-side count when fixed at compile time (64, one full
// group: the gather stride is a shift), 0 when taken from A.rep.
template <typename T, int RC>
__global__ void __launch_bounds__(REP_NT)
rep_mm_kernel(Csr<T> A, const T *__restrict__ in, T *__restrict__ out,
              double *__restrict__ part, Ctrl *ctrl, int ph,
              int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  if (ph >= 0 && cg_done_at_start(ctrl, ph)) return;
  __shared__ double sh[REP_NT / WAVE];
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t R = RC > 0 ? (int64_t)RC : A.rep;
  const int64_t s = (int64_t)blockIdx.y * WAVE + lane;
  const bool live = s < R;
  const int64_t row = (int64_t)blockIdx.x * REP_ROWS + threadIdx.x / WAVE;
  T acc = (T)0;
  if (row < A.brows) {
    const T *col = in + (live ? s : 0);
    const int64_t e0 = A.ptr[row], e1 = A.ptr[row + 1];
    for (int64_t c0 = e0; c0 < e1; c0 += WAVE) {
      const int64_t e = c0 + lane;
      int ix = 0;
      T v = (T)0;
      if (e < e1) {
        ix = A.idx[e];
        v = A.val[e];
      }
      const int nc = (int)(e1 - c0 < WAVE ? e1 - c0 : WAVE);
      int j = 0;
      // UNR gathers in flight, added in entry order
      for (; j + REP_UNR<T>::n <= nc; j += REP_UNR<T>::n) {
        T g[REP_UNR<T>::n];
#pragma unroll
        for (int u = 0; u < REP_UNR<T>::n; ++u)
          g[u] = col[(int64_t)bcast(ix, j + u) * R];
#pragma unroll
        for (int u = 0; u < REP_UNR<T>::n; ++u) acc += bcast(v, j + u) * g[u];
      }
      for (; j < nc; ++j) acc += bcast(v, j) * col[(int64_t)bcast(ix, j) * R];
    }
    if (live) out[row * R + s] = acc;
  }
  if (part) {
    const double q = (row < A.brows && live) ? (double)acc * (double)acc : 0.0;
    const double t = block_sum<REP_NT>(q, sh);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
  }
}

// At most 32 right-hand sides: a wave takes 64/GR stored rows, GR lanes
// each (lane = right-hand side), so that few right-hand sides do not leave
// most lanes idle.  Each lane loads its row's entries itself (the lanes of
// a group read the same address) and gathers GR contiguous values per
// entry.
template <typename T, int GR>
__global__ void __launch_bounds__(REP_NT)
rep_mm_group_kernel(Csr<T> A, const T *__restrict__ in, T *__restrict__ out,
                    double *__restrict__ part, Ctrl *ctrl, int ph,
                    int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  if (ph >= 0 && cg_done_at_start(ctrl, ph)) return;
  __shared__ double sh[REP_NT / WAVE];
  constexpr int RPW = WAVE / GR;          // stored rows per wave
  const int lane = threadIdx.x & (WAVE - 1);
  const int ls = lane % GR;
  const int64_t R = A.rep;                // R <= GR
  const bool live = ls < R;
  const int64_t row = ((int64_t)blockIdx.x * REP_ROWS + threadIdx.x / WAVE) * RPW +
                      lane / GR;
  T acc = (T)0;
  if (row < A.brows) {
    const T *col = in + (live ? ls : 0);
    const int64_t e0 = A.ptr[row], e1 = A.ptr[row + 1];
    int64_t e = e0;
    for (; e + 4 <= e1; e += 4) {
      int32_t ix[4];
      T v[4], g[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        ix[u] = A.idx[e + u];
        v[u] = A.val[e + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) g[u] = col[(int64_t)ix[u] * R];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc += v[u] * g[u];
    }
    for (; e < e1; ++e) acc += A.val[e] * col[(int64_t)A.idx[e] * R];
    if (live) out[row * R + ls] = acc;
  }
  if (part) {
    const double q = (row < A.brows && live) ? (double)acc * (double)acc : 0.0;
    const double t = block_sum<REP_NT>(q, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
  }
}

template <typename T>
int launch_rep_mm(const Csr<T> &A, const T *in, T *out, double *part,
                  Ctrl *ctrl, int ph, int respect_done, hipStream_t st) {
  if (A.rep <= 32) {
    const int gr = A.rep <= 16 ? 16 : 32;
    const int64_t rows_per_block = (int64_t)REP_ROWS * (WAVE / gr);
    const int64_t gx = (A.brows + rows_per_block - 1) / rows_per_block;
    if (gx <= 0) return 0;
    if (gr == 16)
      hipLaunchKernelGGL((rep_mm_group_kernel<T, 16>), dim3((unsigned)gx),
                         dim3(REP_NT), 0, st, A, in, out, part, ctrl, ph,
                         respect_done);
    else
      hipLaunchKernelGGL((rep_mm_group_kernel<T, 32>), dim3((unsigned)gx),
                         dim3(REP_NT), 0, st, A, in, out, part, ctrl, ph,
                         respect_done);
    return (int)gx;
  }
  const int64_t gx = (A.brows + REP_ROWS - 1) / REP_ROWS;
  const int64_t gy = (A.rep + WAVE - 1) / WAVE;
  if (gx <= 0 || gy <= 0) return 0;
  if (A.rep == WAVE)
    hipLaunchKernelGGL((rep_mm_kernel<T, WAVE>), dim3((unsigned)gx, (unsigned)gy),
                       dim3(REP_NT), 0, st, A, in, out, part, ctrl, ph,
                       respect_done);
  else
    hipLaunchKernelGGL((rep_mm_kernel<T, 0>), dim3((unsigned)gx, (unsigned)gy),
                       dim3(REP_NT), 0, st, A, in, out, part, ctrl, ph,
                       respect_done);
  return (int)(gx * gy);
}

// 64 x 64 tiles through LDS (one padding column against bank conflicts)
template <typename T>
__global__ void __launch_bounds__(REP_NT)
rep_tin_kernel(const T *__restrict__ in, T *__restrict__ out, int64_t len,
               int64_t R, Ctrl *ctrl, int ph, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  if (ph >= 0 && cg_done_at_start(ctrl, ph)) return;
  __shared__ T tile[WAVE][WAVE + 1];
  const int64_t i0 = (int64_t)blockIdx.x * WAVE, s0 = (int64_t)blockIdx.y * WAVE;
  const int tx = threadIdx.x & (WAVE - 1), ty = threadIdx.x / WAVE;
  for (int r = ty; r < WAVE; r += REP_ROWS) {
    const int64_t s = s0 + r, i = i0 + tx;
    tile[r][tx] = (s < R && i < len) ? in[s * len + i] : (T)0;
  }
  __syncthreads();
  for (int r = ty; r < WAVE; r += REP_ROWS) {
    const int64_t i = i0 + r, s = s0 + tx;
    if (i < len && s < R) out[i * R + s] = tile[tx][r];
  }
}

template <typename T>
__global__ void __launch_bounds__(REP_NT)
rep_tout_kernel(const T *__restrict__ in, T *__restrict__ out,
                T *__restrict__ x, int64_t len, int64_t R, Ctrl *ctrl, int ph,
                int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  if (ph >= 0 && cg_done_at_start(ctrl, ph)) return;
  __shared__ T tile[WAVE][WAVE + 1];
  const double alpha = (x && ph >= 0) ? ctrl->cg_alpha[ph] : 0.0;
  const int64_t i0 = (int64_t)blockIdx.x * WAVE, s0 = (int64_t)blockIdx.y * WAVE;
  const int tx = threadIdx.x & (WAVE - 1), ty = threadIdx.x / WAVE;
  for (int r = ty; r < WAVE; r += REP_ROWS) {
    const int64_t i = i0 + r, s = s0 + tx;
    tile[r][tx] = (i < len && s < R) ? in[i * R + s] : (T)0;
  }
  __syncthreads();
  for (int r = ty; r < WAVE; r += REP_ROWS) {
    const int64_t s = s0 + r, i = i0 + tx;
    if (s < R && i < len) {
      const int64_t o = s * len + i;
      if (alpha != 0.0) x[o] += (T)alpha * out[o];
      out[o] = tile[tx][r];
    }
  }
}

template <typename T>
void launch_rep_tin(const T *in, T *out, int64_t len, int64_t rep, Ctrl *ctrl,
                    int ph, int respect_done, hipStream_t st) {
  const int64_t gx = (len + WAVE - 1) / WAVE, gy = (rep + WAVE - 1) / WAVE;
  if (gx <= 0 || gy <= 0) return;
  hipLaunchKernelGGL(rep_tin_kernel<T>, dim3((unsigned)gx, (unsigned)gy),
                     dim3(REP_NT), 0, st, in, out, len, rep, ctrl, ph,
                     respect_done);
}

template <typename T>
void launch_rep_tout(const T *in, T *out, T *x, int64_t len, int64_t rep,
                     Ctrl *ctrl, int ph, int respect_done, hipStream_t st) {
  const int64_t gx = (len + WAVE - 1) / WAVE, gy = (rep + WAVE - 1) / WAVE;
  if (gx <= 0 || gy <= 0) return;
  hipLaunchKernelGGL(rep_tout_kernel<T>, dim3((unsigned)gx, (unsigned)gy),
                     dim3(REP_NT), 0, st, in, out, x, len, rep, ctrl, ph,
                     respect_done);
}

template int launch_rep_mm<double>(const Csr<double> &, const double *,
                                   double *, double *, Ctrl *, int, int,
                                   hipStream_t);
template int launch_rep_mm<float>(const Csr<float> &, const float *, float *,
                                  double *, Ctrl *, int, int, hipStream_t);
template void launch_rep_tin<double>(const double *, double *, int64_t,
                                     int64_t, Ctrl *, int, int, hipStream_t);
template void launch_rep_tin<float>(const float *, float *, int64_t, int64_t,
                                    Ctrl *, int, int, hipStream_t);
template void launch_rep_tout<double>(const double *, double *, double *,
                                      int64_t, int64_t, Ctrl *, int, int,
                                      hipStream_t);
template void launch_rep_tout<float>(const float *, float *, float *, int64_t,
                                     int64_t, Ctrl *, int, int, hipStream_t);

}  // namespace rg
