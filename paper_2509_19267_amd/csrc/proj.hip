// Block projections of RGDBEK on gfx950 (the pseudoinverse updates of the
// GDBEK rule that Algorithm 1 reuses):
//   column block: y = argmin ||A_U y - z||,  z <- z - A_U y
//   row block:    d = (A^J)^+ r^J,           x <- x + d
// The column right-hand side A_U^T z is g restricted to U, already produced
// by the column residual pass.  For the row block with independent rows,
// d = A^J^T w with (A^J A^J^T) w = r^J.
//
// Dense blocks: Gram matrix (gathered from a precomputed A^T A / A A^T, or
// formed from the listed rows), then a one-workgroup blocked Cholesky with an
// optional corrected semi-normal-equations sweep (ill-conditioned square row
// blocks), or Jacobi-preconditioned CG with one launch per step (the last
// workgroup of each step carries the vector recurrences).
// Sparse blocks: matrix-free CGLS (columns, z updated as the CGLS residual)
// and CGNE on A^J A^J^T (rows), the wide products streaming the full CSR/CSC
// with a direction vector that is zero outside the block.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace rg {

// ------------------------------------------------------------ Gram
template <typename T>
__global__ void __launch_bounds__(256)
gram_gather_kernel(const T *__restrict__ F, int64_t ldf,
                   const int32_t *__restrict__ list,
                   const int64_t *__restrict__ cnt, int64_t cap,
                   T *__restrict__ G, Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  const int64_t c = *cnt;
  const int64_t a = blockIdx.y;
  if (a >= c) return;
  const int64_t la = list[a];
  for (int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x; b < c;
       b += (int64_t)gridDim.x * 256)
    G[a * cap + b] = F[la * ldf + list[b]];
}
template <typename T>
void launch_gram_gather(const T *F, int64_t ldf, const int32_t *list,
                        const int64_t *count_dev, int64_t cap, T *G,
                        Ctrl *ctrl, int respect_done, hipStream_t st) {
  int gx = (int)((cap + 255) / 256);
  if (gx > 8) gx = 8;
  hipLaunchKernelGGL(gram_gather_kernel<T>, dim3(gx, (unsigned)cap), dim3(256),
                     0, st, F, ldf, list, count_dev, cap, G, ctrl,
                     respect_done);
}

// G[a][b] = <X_{l_a}, X_{l_b}> (list == nullptr: identity) on the matrix
// cores (MFMA 16x16x4, FP64 or FP32): one
// workgroup of 4 waves per 64 x 64 lower tile (mirrored on store), each wave
// a 32 x 32 quarter as 2 x 2 MFMA blocks.  K advances 16 at a time through
// double-buffered LDS stages stored k-major (tile[k][row]), so the 16 lanes
// that feed one MFMA row group read consecutive words; the next stage is
// loaded from global memory into registers while the current one is
// multiplied.  Operand layout of v_mfma_*_16x16x4 (both precisions): lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator element r of
// lane l is D[row(l / 16, r)][l % 16], row = 4 (l / 16) + r for FP32 and
// 4 r + l / 16 for FP64 (measured on gfx950).
template <typename T> struct Mfma16;
template <> struct Mfma16<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * r + lk; }
};
template <> struct Mfma16<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};
constexpr int SY_B = 64;             // output tile (rows = columns)
constexpr int SY_K = 16;             // k per LDS stage
constexpr int SY_P = SY_B + 16;      // LDS row pitch (k-major rows of 64)
constexpr int SY_NT = 256;

template <typename T>
__device__ __forceinline__ void sy_load(const T *__restrict__ X, int64_t ld,
                                        int64_t len,
                                        const int32_t *__restrict__ list,
                                        int64_t c, int64_t r0, int64_t k0,
                                        T (&v)[4]) {
  // thread t: row r0 + t / 4, k = k0 + 4 (t % 4) .. + 3
  const int64_t r = r0 + (threadIdx.x >> 2);
  const int64_t k = k0 + 4 * (threadIdx.x & 3);
#pragma unroll
  for (int u = 0; u < 4; ++u) v[u] = (T)0;
  if (r >= c) return;
  const T *row = X + (list ? (int64_t)list[r] : r) * ld;
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (k + u < len) v[u] = row[k + u];
}

template <typename T>
__global__ void __launch_bounds__(SY_NT)
gram_mfma_kernel(const T *__restrict__ X, int64_t ld, int64_t len,
                 const int32_t *__restrict__ list,
                 const int64_t *__restrict__ cnt, int64_t cap, int64_t ldg,
                 T *__restrict__ G, Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  typedef typename Mfma16<T>::v4 v4;
  const int64_t c = cnt ? *cnt : cap;
  const int64_t ta = (int64_t)blockIdx.y * SY_B, tb = (int64_t)blockIdx.x * SY_B;
  if (ta >= c || tb >= c || tb > ta) return;   // lower tiles only
  __shared__ T sa[2][SY_K][SY_P], sb[2][SY_K][SY_P];
  const int lane = threadIdx.x & (WAVE - 1);
  const int w = threadIdx.x / WAVE;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  const int sr = threadIdx.x >> 2, sk = 4 * (threadIdx.x & 3);
  v4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (v4){0, 0, 0, 0};
  T va[4], vb[4];
  sy_load<T>(X, ld, len, list, c, ta, 0, va);
  sy_load<T>(X, ld, len, list, c, tb, 0, vb);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    sa[0][sk + u][sr] = va[u];
    sb[0][sk + u][sr] = vb[u];
  }
  __syncthreads();
  const int64_t nst = (len + SY_K - 1) / SY_K;
  for (int64_t st = 0; st < nst; ++st) {
    const int cur = (int)(st & 1);
    const bool more = st + 1 < nst;
    if (more) {
      sy_load<T>(X, ld, len, list, c, ta, (st + 1) * SY_K, va);
      sy_load<T>(X, ld, len, list, c, tb, (st + 1) * SY_K, vb);
    }
#pragma unroll
    for (int kk = 0; kk < SY_K / 4; ++kk) {
      const int k = 4 * kk + lk;
      T fa[2], fb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        fa[i] = sa[cur][k][wr + 16 * i + li];
        fb[i] = sb[cur][k][wc + 16 * i + li];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = Mfma16<T>::mma(fa[i], fb[j], acc[i][j]);
    }
    if (more) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        sa[cur ^ 1][sk + u][sr] = va[u];
        sb[cur ^ 1][sk + u][sr] = vb[u];
      }
    }
    __syncthreads();
  }
  const bool diag = (ta == tb);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = ta + wr + 16 * i + Mfma16<T>::row(lk, r);
        const int64_t gj = tb + wc + 16 * j + li;
        if (gi >= c || gj >= c || (diag && gj > gi)) continue;
        const T v = acc[i][j][r];
        G[gi * ldg + gj] = v;
        G[gj * ldg + gi] = v;
      }
}

template <typename T>
void launch_gram_rows(const T *X, int64_t ld, int64_t len, const int32_t *list,
                      const int64_t *count_dev, int64_t cap, T *G, Ctrl *ctrl,
                      int respect_done, hipStream_t st) {
  const unsigned nt = (unsigned)((cap + SY_B - 1) / SY_B);
  hipLaunchKernelGGL(gram_mfma_kernel<T>, dim3(nt, nt), dim3(SY_NT), 0, st, X,
                     ld, len, list, count_dev, cap, cap, G, ctrl,
                     respect_done);
}
template <typename T>
void launch_gram_full(const T *X, int64_t ldx, int64_t rows, int64_t len,
                      T *F, hipStream_t st) {
  const unsigned nt = (unsigned)((rows + SY_B - 1) / SY_B);
  hipLaunchKernelGGL(gram_mfma_kernel<T>, dim3(nt, nt), dim3(SY_NT), 0, st, X,
                     ldx, len, (const int32_t *)nullptr,
                     (const int64_t *)nullptr, rows, rows, F, (Ctrl *)nullptr,
                     0);
}

// ------------------------------------------------------------ Cholesky
// One workgroup of 256 threads, blocked left-looking with 32-column panels
// in LDS.  A pivot below 1e-13 of the largest diagonal marks the column as
// dependent (its unknown is set to zero), which keeps the projection onto the
// span of the block exact for rank-deficient blocks.
constexpr int CNB = 32;
constexpr int CNT = 256;

template <typename T>
__global__ void __launch_bounds__(CNT)
chol_solve_kernel(T *__restrict__ G, int64_t ldg,
                  const int64_t *__restrict__ cnt,
                  const T *__restrict__ hsrc, const int32_t *__restrict__ hl,
                  T *__restrict__ y, int factor, Ctrl *ctrl, int ph,
                  int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  const int c = (int)*cnt;
  if (c <= 0) return;
  __shared__ T P[CHOL_MAX][CNB + 1];
  __shared__ T Lb[CNB][CNB + 1];
  __shared__ T vec[CHOL_MAX];
  __shared__ T dmax;
  const int tid = threadIdx.x;
  if (factor) {
    if (tid == 0) {
      T mx = 0;
      for (int i = 0; i < c; ++i) mx = G[(int64_t)i * ldg + i] > mx ? G[(int64_t)i * ldg + i] : mx;
      dmax = mx;
    }
    __syncthreads();
    const T thr = dmax * (T)1e-13;
    for (int p = 0; p < c; p += CNB) {
      const int w = (c - p) < CNB ? (c - p) : CNB;
      const int h = c - p;
      // load panel rows p..c-1, columns p..p+w-1
      for (int e = tid; e < h * CNB; e += CNT) {
        const int r = e / CNB, cc = e % CNB;
        P[r][cc] = (cc < w) ? G[(int64_t)(p + r) * ldg + p + cc] : (T)0;
      }
      __syncthreads();
      // left-looking update with previous panels: P -= L[p:, 0:p] L[p:p+w, 0:p]^T
      for (int t0 = 0; t0 < p; t0 += CNB) {
        for (int e = tid; e < CNB * CNB; e += CNT) {
          const int rr = e / CNB, kk = e % CNB;
          Lb[rr][kk] = (rr < w) ? G[(int64_t)(p + rr) * ldg + t0 + kk] : (T)0;
        }
        __syncthreads();
        for (int r = tid; r < h; r += CNT) {
          T lr[CNB];
#pragma unroll
          for (int kk = 0; kk < CNB; ++kk) lr[kk] = G[(int64_t)(p + r) * ldg + t0 + kk];
          for (int cc = 0; cc < w && cc <= r; ++cc) {
            T s = 0;
#pragma unroll
            for (int kk = 0; kk < CNB; ++kk) s += lr[kk] * Lb[cc][kk];
            P[r][cc] -= s;
          }
        }
        __syncthreads();
      }
      // factor the panel (right-looking inside LDS)
      for (int j = 0; j < w; ++j) {
        __syncthreads();
        const T dj = P[j][j];
        const bool dep = !(dj > thr);
        const T sq = dep ? (T)0 : sqrt(dj);
        __syncthreads();   // every wave has read the pivot before it changes
        for (int r = j + tid; r < h; r += CNT) {
          if (r == j) P[j][j] = sq;
          else P[r][j] = dep ? (T)0 : P[r][j] / sq;
        }
        __syncthreads();
        for (int r = j + 1 + tid; r < h; r += CNT) {
          const T lrj = P[r][j];
          const int kmax = r < w - 1 ? r : w - 1;
          for (int k = j + 1; k <= kmax; ++k) P[r][k] -= lrj * P[k][j];
        }
      }
      __syncthreads();
      for (int e = tid; e < h * CNB; e += CNT) {
        const int r = e / CNB, cc = e % CNB;
        if (cc < w && cc <= r) G[(int64_t)(p + r) * ldg + p + cc] = P[r][cc];
      }
      __syncthreads();
    }
  }
  // forward solve L v = h
  for (int i = tid; i < c; i += CNT) vec[i] = hl ? hsrc[hl[i]] : hsrc[i];
  __syncthreads();
  for (int p = 0; p < c; p += CNB) {
    const int w = (c - p) < CNB ? (c - p) : CNB;
    // subtract contributions of solved entries 0..p-1 from rows p..p+w-1
    if (tid < w) {
      T s = 0;
      for (int t = 0; t < p; ++t) s += G[(int64_t)(p + tid) * ldg + t] * vec[t];
      vec[p + tid] -= s;
    }
    __syncthreads();
    if (tid < WAVE) {
      for (int j = 0; j < w; ++j) {
        const T d = G[(int64_t)(p + j) * ldg + p + j];
        T vj = vec[p + j];
        vj = d != (T)0 ? vj / d : (T)0;
        if (tid == 0) vec[p + j] = vj;
        __builtin_amdgcn_wave_barrier();
        if (tid > j && tid < w) vec[p + tid] -= G[(int64_t)(p + tid) * ldg + p + j] * vj;
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
  }
  // backward solve L^T y = v
  for (int p = ((c - 1) / CNB) * CNB; p >= 0; p -= CNB) {
    const int w = (c - p) < CNB ? (c - p) : CNB;
    if (tid < w) {
      T s = 0;
      for (int t = p + w; t < c; ++t) s += G[(int64_t)t * ldg + p + tid] * vec[t];
      vec[p + tid] -= s;
    }
    __syncthreads();
    if (tid < WAVE) {
      for (int j = w - 1; j >= 0; --j) {
        const T d = G[(int64_t)(p + j) * ldg + p + j];
        T vj = vec[p + j];
        vj = d != (T)0 ? vj / d : (T)0;
        if (tid == 0) vec[p + j] = vj;
        __builtin_amdgcn_wave_barrier();
        if (tid < j) vec[p + tid] -= G[(int64_t)(p + j) * ldg + p + tid] * vj;
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
  }
  for (int i = tid; i < c; i += CNT) y[i] = vec[i];
}

template <typename T>
void launch_chol_solve(T *G, int64_t cap, const int64_t *count_dev,
                       const T *hsrc, const int32_t *hlist, T *y, int factor,
                       Ctrl *ctrl, int ph, int respect_done, hipStream_t st) {
  hipLaunchKernelGGL(chol_solve_kernel<T>, dim3(1), dim3(CNT), 0, st, G, cap,
                     count_dev, hsrc, hlist, y, factor, ctrl, ph,
                     respect_done);
}

// ------------------------------------------------------------ PCG on Gram
// Jacobi-preconditioned CG on G y = h with two fence-free launches per step.
// Scalars are never broadcast through memory within a launch: every block
// re-derives them from small arrays of per-block partials of the previous
// launch, in a fixed order, so all blocks hold identical bits.
//   step t, launch A (one wave per row of G, 4 rows per block):
//     t > 0: rz_t = sum rz partials, rr = sum rr partials; stop when
//            rr <= tol^2 rr_0 (every block reaches the same verdict);
//            beta = rz_t / rz_{t-1};  p_t = zz + beta p_{t-1}  (whole vector,
//            rebuilt in LDS by every block; block 0 stores it)
//     v = G p_t on the block's rows; partial <p_t, v>
//   step t, launch B (k/256 blocks):
//     alpha = rz_t / sum <p,v> partials; y += alpha p_t; res -= alpha v;
//     zz = res / diag(G); partials of <res, zz> and <res, res>
// p alternates between two buffers by step parity.
constexpr int PG_NT = 256;
constexpr int PG_ROWS = PG_NT / WAVE;     // rows per block in launch A
constexpr int64_t PG_LDS_MAX = 8192;      // p staged in LDS (FP64: 64 KB)

template <typename T>
__global__ void __launch_bounds__(PG_NT)
pcg_init_kernel(const T *__restrict__ G, int64_t ldg,
                const int64_t *__restrict__ cnt, const T *__restrict__ hsrc,
                const int32_t *__restrict__ hl, T *__restrict__ y,
                CgWork<T> w, Ctrl *ctrl, int ph, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  __shared__ double sh[PG_NT / WAVE];
  const int64_t c = *cnt;
  double rz = 0.0, rr = 0.0;
  for (int64_t a = threadIdx.x; a < c; a += PG_NT) {
    const T h = hl ? hsrc[hl[a]] : hsrc[a];
    const T dg = G[a * ldg + a];
    const T zz = dg > (T)0 ? h / dg : (T)0;
    y[a] = (T)0;
    w.res[a] = h;
    w.zz[a] = zz;
    w.p[a] = zz;               // p_0 in buffer 0
    rz += (double)h * (double)zz;
    rr += (double)h * (double)h;
  }
  rz = block_sum<PG_NT>(rz, sh);
  rr = block_sum<PG_NT>(rr, sh);
  if (threadIdx.x == 0) {
    ctrl->cg_rz[ph] = rz;      // rz_0
    ctrl->cg_rz0[ph] = rr;     // ||h||^2
    ctrl->cg_done[ph] = (rr == 0.0 || c == 0) ? 1 : 0;
    ctrl->cg_steps[ph] = 0;
  }
}

template <typename T>
__global__ void __launch_bounds__(PG_NT)
pcg_step_a(const T *__restrict__ G, int64_t ldg, const int64_t *__restrict__ cnt,
           CgWork<T> w, int t, int nb_b, double tol, Ctrl *ctrl, int ph,
           int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  if (ctrl->cg_done[ph]) return;
  __shared__ T ps[PG_LDS_MAX];
  __shared__ double sh[PG_NT / WAVE];
  const int64_t c = *cnt;
  const T *pold = w.p + (int64_t)((t + 1) & 1) * w.cap;
  T *pnew = w.p + (int64_t)(t & 1) * w.cap;
  if (t > 0) {
    const double *part = w.part + (int64_t)((t - 1) & 1) * 2 * w.part_cap;
    double rz = 0.0, rr = 0.0;
    for (int b = threadIdx.x; b < nb_b; b += PG_NT) {
      rz += part[2 * b];
      rr += part[2 * b + 1];
    }
    rz = block_sum<PG_NT>(rz, sh);
    rr = block_sum<PG_NT>(rr, sh);
    const double rz_prev = w.rzs[(t - 1) & 1];
    if (rr <= tol * tol * ctrl->cg_rz0[ph] || rz_prev == 0.0) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctrl->cg_done[ph] = 1;
        ctrl->cg_steps[ph] = t;
      }
      return;
    }
    const double beta = rz / rz_prev;
    for (int64_t a = threadIdx.x; a < c; a += PG_NT) {
      const T pv = w.zz[a] + (T)beta * pold[a];
      ps[a] = pv;
      if (blockIdx.x == 0) pnew[a] = pv;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) w.rzs[t & 1] = rz;
  } else {
    for (int64_t a = threadIdx.x; a < c; a += PG_NT) ps[a] = pnew[a];
    if (blockIdx.x == 0 && threadIdx.x == 0) w.rzs[0] = ctrl->cg_rz[ph];
  }
  __syncthreads();
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t row = (int64_t)blockIdx.x * PG_ROWS + threadIdx.x / WAVE;
  double pv = 0.0;
  if (row < c) {
    T s = 0;
    const T *gr = G + row * ldg;
    for (int64_t b = lane; b < c; b += WAVE) s += gr[b] * ps[b];
    s = wave_sum(s);
    if (lane == 0) {
      w.v[row] = s;
      pv = (double)s * (double)ps[row];
    }
  }
  pv = block_sum<PG_NT>(pv, sh);
  if (threadIdx.x == 0) w.pv[blockIdx.x] = pv;
}

template <typename T>
__global__ void __launch_bounds__(PG_NT)
pcg_step_b(const T *__restrict__ G, int64_t ldg, const int64_t *__restrict__ cnt,
           T *__restrict__ y, CgWork<T> w, int t, int nb_a, Ctrl *ctrl, int ph,
           int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  if (ctrl->cg_done[ph]) return;
  __shared__ double sh[PG_NT / WAVE];
  const int64_t c = *cnt;
  const T *pt = w.p + (int64_t)(t & 1) * w.cap;
  double pv = 0.0;
  for (int b = threadIdx.x; b < nb_a; b += PG_NT) pv += w.pv[b];
  pv = block_sum<PG_NT>(pv, sh);
  const double rz = w.rzs[t & 1];
  const double alpha = pv != 0.0 ? rz / pv : 0.0;
  double rzn = 0.0, rr = 0.0;
  const int64_t a = (int64_t)blockIdx.x * PG_NT + threadIdx.x;
  if (a < c) {
    y[a] += (T)alpha * pt[a];
    const T r = w.res[a] - (T)alpha * w.v[a];
    w.res[a] = r;
    const T dg = G[a * ldg + a];
    const T zz = dg > (T)0 ? r / dg : (T)0;
    w.zz[a] = zz;
    rzn = (double)r * (double)zz;
    rr = (double)r * (double)r;
  }
  rzn = block_sum<PG_NT>(rzn, sh);
  rr = block_sum<PG_NT>(rr, sh);
  if (threadIdx.x == 0) {
    double *part = w.part + (int64_t)(t & 1) * 2 * w.part_cap;
    part[2 * blockIdx.x] = rzn;
    part[2 * blockIdx.x + 1] = rr;
  }
}

template <typename T>
void launch_pcg_gram_init(const T *G, int64_t cap, const int64_t *count_dev,
                          const T *hsrc, const int32_t *hlist, T *y,
                          CgWork<T> &w, Ctrl *ctrl, int ph, int respect_done,
                          hipStream_t st) {
  hipLaunchKernelGGL(pcg_init_kernel<T>, dim3(1), dim3(PG_NT), 0, st, G, cap,
                     count_dev, hsrc, hlist, y, w, ctrl, ph, respect_done);
}
template <typename T>
void launch_pcg_gram_step(const T *G, int64_t cap, const int64_t *count_dev,
                          T *y, CgWork<T> &w, int step, double tol,
                          Ctrl *ctrl, int ph, int respect_done,
                          hipStream_t st) {
  const int nb_a = (int)((cap + PG_ROWS - 1) / PG_ROWS);
  const int nb_b = (int)((cap + PG_NT - 1) / PG_NT);
  hipLaunchKernelGGL(pcg_step_a<T>, dim3(nb_a), dim3(PG_NT), 0, st, G, cap,
                     count_dev, w, step, nb_b, tol, ctrl, ph, respect_done);
  hipLaunchKernelGGL(pcg_step_b<T>, dim3(nb_b), dim3(PG_NT), 0, st, G, cap,
                     count_dev, y, w, step, nb_a, ctrl, ph, respect_done);
}
int64_t pcg_cap_max() { return PG_LDS_MAX; }

// ------------------------------------------------------------ persistent PCG
// The whole Jacobi-preconditioned CG of one block projection in one launch of
// P co-resident workgroups (P <= compute units).  Workgroup w owns rows
// [w*rpw, (w+1)*rpw) of G and of y.  Every workgroup keeps the full direction
// p, residual res and diagonal of G in LDS and updates them redundantly
// (O(c) work per step, identical bits in every workgroup); per step only the
// product v = G p on the owned rows and a partial of <p, v> are exchanged,
// through double-buffered global arrays and one grid barrier.  The stopping
// test ||res|| <= tol ||h|| is evaluated identically by every workgroup, so
// all leave the loop together.  The barrier waits are bounded: after
// GRID_SPIN_MAX polls a workgroup raises Ctrl::sync_fail and leaves, so the
// launch always drains.
constexpr int PP_NT = 1024;                      // 16 waves: one row of G each
constexpr int PP_RPW = 16;                       // rows of G per workgroup
constexpr int PP_UNROLL = 8;                     // row loads in flight per lane
template <typename T> struct PpCap;
template <> struct PpCap<double> { static constexpr int64_t v = 4096; };
template <> struct PpCap<float> { static constexpr int64_t v = 8192; };
// 16-byte row loads of the packed block (rows start 16-byte aligned when
// the leading dimension is a multiple of the vector width)
typedef double pp_d2 __attribute__((ext_vector_type(2)));
typedef float pp_f4 __attribute__((ext_vector_type(4)));
template <typename T> struct PpVec;
template <> struct PpVec<double> { using type = pp_d2; static constexpr int n = 2; };
template <> struct PpVec<float> { using type = pp_f4; static constexpr int n = 4; };

template <typename T>
__global__ void __launch_bounds__(PP_NT)
pcg_persist_kernel(T *__restrict__ G, int64_t ldg,
                   const int64_t *__restrict__ cnt, const T *__restrict__ hsrc,
                   const int32_t *__restrict__ hl, T *__restrict__ y,
                   T *__restrict__ vbuf, double *__restrict__ pvbuf,
                   int64_t cap, int max_steps, double tol, Ctrl *ctrl, int ph,
                   int respect_done, const T *__restrict__ F, int64_t ldf) {
  if (respect_done && ctrl_done(ctrl)) return;
  constexpr int64_t CAP = PpCap<T>::v;
  __shared__ T ps[CAP], rs[CAP], dg[CAP];
  __shared__ int32_t sl[CAP];
  __shared__ double sh[PP_NT / WAVE];
  const int64_t c = *cnt;
  const int P = (int)gridDim.x;
  const int64_t rpw = (c + P - 1) / P;
  const int64_t r0 = (int64_t)blockIdx.x * rpw;
  const int64_t r1 = r0 + rpw < c ? r0 + rpw : c;
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  double rz = 0.0, rr = 0.0;
  // F != nullptr: G is not gathered yet.  Every workgroup reads its own
  // rows of the block straight from the full Gram F (the block list in
  // LDS) during the first step and stores them packed for the later steps,
  // which read only the rows the same threads wrote.
  for (int64_t a = threadIdx.x; a < c; a += PP_NT) {
    const T h = hl ? hsrc[hl[a]] : hsrc[a];
    T d;
    if (F) {
      const int32_t l = hl[a];
      sl[a] = l;
      d = F[(int64_t)l * ldf + l];
    } else {
      d = G[a * ldg + a];
    }
    const T z = d > (T)0 ? h / d : (T)0;
    rs[a] = h;
    dg[a] = d;
    ps[a] = z;
    rz += (double)h * (double)z;
    rr += (double)h * (double)h;
  }
  for (int64_t a = r0 + threadIdx.x; a < r1; a += PP_NT) y[a] = (T)0;
  rz = block_sum<PP_NT>(rz, sh);
  rr = block_sum<PP_NT>(rr, sh);
  const double rr0 = rr;
  const uint64_t base = ctrl->cg_barbase[ph];
  int nbar = 0, t = 0;
  bool run = !(rr0 == 0.0 || c == 0);
  while (run && t < max_steps) {
    const int par = t & 1;
    T *vb = vbuf + (int64_t)par * cap;
    double *pvb = pvbuf + (int64_t)par * P;
    double pvp = 0.0;
    for (int64_t row = r0 + wv; row < r1; row += PP_NT / WAVE) {
      T *gr = G + row * ldg;
      T s = (T)0;
      int64_t b = lane;
      if (F && t == 0) {
        const T *fr = F + (int64_t)sl[row] * ldf;
        for (; b + (PP_UNROLL - 1) * WAVE < c; b += PP_UNROLL * WAVE) {
          T gv[PP_UNROLL];
#pragma unroll
          for (int u = 0; u < PP_UNROLL; ++u) gv[u] = fr[sl[b + u * WAVE]];
#pragma unroll
          for (int u = 0; u < PP_UNROLL; ++u) {
            gr[b + u * WAVE] = gv[u];
            s += gv[u] * ps[b + u * WAVE];
          }
        }
        for (; b < c; b += WAVE) {
          const T gv = fr[sl[b]];
          gr[b] = gv;
          s += gv * ps[b];
        }
      } else if (ldg % PpVec<T>::n == 0) {
        using V = typename PpVec<T>::type;
        constexpr int VN = PpVec<T>::n;
        const V *grv = reinterpret_cast<const V *>(gr);
        const int64_t cv = c / VN;
        int64_t q = lane;
        for (; q + (PP_UNROLL - 1) * WAVE < cv; q += PP_UNROLL * WAVE) {
          V gv[PP_UNROLL];
#pragma unroll
          for (int u = 0; u < PP_UNROLL; ++u) gv[u] = grv[q + u * WAVE];
#pragma unroll
          for (int u = 0; u < PP_UNROLL; ++u)
#pragma unroll
            for (int v = 0; v < VN; ++v)
              s += gv[u][v] * ps[(q + u * WAVE) * VN + v];
        }
        for (; q < cv; q += WAVE) {
          const V g = grv[q];
#pragma unroll
          for (int v = 0; v < VN; ++v) s += g[v] * ps[q * VN + v];
        }
        for (b = cv * VN + lane; b < c; b += WAVE) s += gr[b] * ps[b];
      } else {
        for (; b + (PP_UNROLL - 1) * WAVE < c; b += PP_UNROLL * WAVE) {
          T gv[PP_UNROLL];
#pragma unroll
          for (int u = 0; u < PP_UNROLL; ++u) gv[u] = gr[b + u * WAVE];
#pragma unroll
          for (int u = 0; u < PP_UNROLL; ++u) s += gv[u] * ps[b + u * WAVE];
        }
        for (; b < c; b += WAVE) s += gr[b] * ps[b];
      }
      s = wave_sum(s);
      if (lane == 0) {
        vb[row] = s;
        pvp += (double)s * (double)ps[row];
      }
    }
    pvp = block_sum<PP_NT>(pvp, sh);
    if (threadIdx.x == 0) pvb[blockIdx.x] = pvp;
    ++nbar;
    if (!grid_barrier(&ctrl->cg_bar[ph], base + (uint64_t)nbar * P,
                      &ctrl->sync_fail))
      return;
    double pv = 0.0;
    for (int b = threadIdx.x; b < P; b += PP_NT) pv += ld_agent(&pvb[b]);
    pv = block_sum<PP_NT>(pv, sh);
    const double alpha = pv != 0.0 ? rz / pv : 0.0;
    for (int64_t a = r0 + threadIdx.x; a < r1; a += PP_NT)
      y[a] += (T)alpha * ps[a];
    double rz1 = 0.0;
    rr = 0.0;
    for (int64_t a = threadIdx.x; a < c; a += PP_NT) {
      const T r = rs[a] - (T)alpha * ld_agent(&vb[a]);
      rs[a] = r;
      const T z = dg[a] > (T)0 ? r / dg[a] : (T)0;
      rz1 += (double)r * (double)z;
      rr += (double)r * (double)r;
    }
    rz1 = block_sum<PP_NT>(rz1, sh);
    rr = block_sum<PP_NT>(rr, sh);
    ++t;
    if (rr <= tol * tol * rr0 || rz == 0.0 || pv == 0.0) break;
    const double beta = rz1 / rz;
    rz = rz1;
    for (int64_t a = threadIdx.x; a < c; a += PP_NT) {
      const T z = dg[a] > (T)0 ? rs[a] / dg[a] : (T)0;
      ps[a] = z + (T)beta * ps[a];
    }
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctrl->cg_barbase[ph] = base + (uint64_t)nbar * P;
    ctrl->cg_steps[ph] = t;
    ctrl->cg_done[ph] = 1;
  }
}

int64_t pcg_persist_cap(bool f64) {
  return f64 ? PpCap<double>::v : PpCap<float>::v;
}
int pcg_persist_grid(int64_t cap, int ncu) {
  int64_t p = (cap + PP_RPW - 1) / PP_RPW;
  if (p > ncu) p = ncu;
  if (p < 1) p = 1;
  return (int)p;
}

template <typename T>
void launch_pcg_persist(T *G, int64_t cap, const int64_t *count_dev,
                        const T *hsrc, const int32_t *hlist, T *y,
                        CgWork<T> &w, int grid, int max_steps, double tol,
                        Ctrl *ctrl, int ph, int respect_done, hipStream_t st,
                        const T *F, int64_t ldf) {
  hipLaunchKernelGGL(pcg_persist_kernel<T>, dim3(grid), dim3(PP_NT), 0, st, G,
                     cap, count_dev, hsrc, hlist, y, w.v2, w.pv2, cap,
                     max_steps, tol, ctrl, ph, respect_done, F, ldf);
}

// ------------------------------------------------------------ thin updates
// out[i] (+)= sign * sum_a coef_a * M[list_a * ldm + i]: blockIdx.y takes a
// chunk of UP_CHUNK list entries, each thread two consecutive i (one 16-byte
// load per listed row when T is double; rows are padded, so i + 1 is always
// inside the row), with UP_UNROLL rows in flight; partials are combined in a
// fixed order by upd_finish.
constexpr int UP_NT = 256;
constexpr int UP_CHUNK = 32;
constexpr int UP_UNROLL = 8;
template <typename T>
__global__ void __launch_bounds__(UP_NT)
upd_partial(const T *__restrict__ M, int64_t ldm, int64_t len,
            const int32_t *__restrict__ list, const int64_t *__restrict__ cnt,
            const T *__restrict__ coef, T *__restrict__ part, Ctrl *ctrl,
            int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  typedef T v2 __attribute__((ext_vector_type(2)));
  const int64_t c = *cnt;
  const int64_t a0 = (int64_t)blockIdx.y * UP_CHUNK;
  if (a0 >= c) return;
  const int64_t a1 = a0 + UP_CHUNK < c ? a0 + UP_CHUNK : c;
  const int64_t i = 2 * ((int64_t)blockIdx.x * UP_NT + threadIdx.x);
  if (i >= len) return;
  T s0 = 0, s1 = 0;
  int64_t a = a0;
  for (; a + UP_UNROLL <= a1; a += UP_UNROLL) {
    v2 mv[UP_UNROLL];
    T cf[UP_UNROLL];
#pragma unroll
    for (int u = 0; u < UP_UNROLL; ++u) {
      mv[u] = *reinterpret_cast<const v2 *>(M + (int64_t)list[a + u] * ldm + i);
      cf[u] = coef[a + u];
    }
#pragma unroll
    for (int u = 0; u < UP_UNROLL; ++u) {
      s0 += cf[u] * mv[u].x;
      s1 += cf[u] * mv[u].y;
    }
  }
  for (; a < a1; ++a) {
    const v2 mv = *reinterpret_cast<const v2 *>(M + (int64_t)list[a] * ldm + i);
    s0 += coef[a] * mv.x;
    s1 += coef[a] * mv.y;
  }
  T *pp = part + (int64_t)blockIdx.y * len;
  pp[i] = s0;
  if (i + 1 < len) pp[i + 1] = s1;
}
template <typename T>
__global__ void __launch_bounds__(UP_NT)
upd_finish(int64_t len, const int64_t *__restrict__ cnt, int nsplit,
           const T *__restrict__ part, T sign, T *__restrict__ out,
           Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  const int64_t i = (int64_t)blockIdx.x * UP_NT + threadIdx.x;
  if (i >= len) return;
  const int64_t c = *cnt;
  int ns = (int)((c + UP_CHUNK - 1) / UP_CHUNK);
  if (ns > nsplit) ns = nsplit;
  T s = 0;
  int b = 0;
  for (; b + 8 <= ns; b += 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(b + u) * len + i];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; b < ns; ++b) s += part[(int64_t)b * len + i];
  out[i] += sign * s;
}

template <typename T>
static void thin_update(const T *M, int64_t ldm, int64_t len,
                        const int32_t *list, const int64_t *cnt, int64_t cap,
                        const T *coef, T *out, T sign, T *part, Ctrl *ctrl,
                        int respect_done, hipStream_t st) {
  const unsigned gx = (unsigned)((len + 2 * UP_NT - 1) / (2 * UP_NT));
  const unsigned gy = (unsigned)((cap + UP_CHUNK - 1) / UP_CHUNK);
  hipLaunchKernelGGL(upd_partial<T>, dim3(gx, gy), dim3(UP_NT), 0, st, M, ldm,
                     len, list, cnt, coef, part, ctrl, respect_done);
  const unsigned gf = (unsigned)((len + UP_NT - 1) / UP_NT);
  hipLaunchKernelGGL(upd_finish<T>, dim3(gf), dim3(UP_NT), 0, st, len, cnt,
                     (int)gy, part, sign, out, ctrl, respect_done);
}

template <typename T>
void launch_col_update(const T *Acm, int64_t ldc, int64_t m,
                       const int32_t *list, const int64_t *count_dev,
                       int64_t cap, const T *y, T *z, T *scratch, Ctrl *ctrl,
                       int respect_done, hipStream_t st) {
  thin_update<T>(Acm, ldc, m, list, count_dev, cap, y, z, (T)-1, scratch,
                 ctrl, respect_done, st);
}
template <typename T>
void launch_row_update(const T *Arm, int64_t ld, int64_t n,
                       const int32_t *list, const int64_t *count_dev,
                       int64_t cap, const T *w, T *x, T *scratch, Ctrl *ctrl,
                       int respect_done, hipStream_t st) {
  thin_update<T>(Arm, ld, n, list, count_dev, cap, w, x, (T)1, scratch, ctrl,
                 respect_done, st);
}
int64_t thin_update_scratch(int64_t len, int64_t cap) {
  return len * ((cap + UP_CHUNK - 1) / UP_CHUNK);
}

// s_a = h1[l_a] - h2[l_a] - <A_{l_a}, v>  (one wave per listed row)
template <typename T>
__global__ void __launch_bounds__(256)
list_resid_kernel(const T *__restrict__ A, int64_t ld, int64_t len,
                  const int32_t *__restrict__ list,
                  const int64_t *__restrict__ cnt, const T *__restrict__ h1,
                  const T *__restrict__ h2, const T *__restrict__ v,
                  T *__restrict__ s, Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t a = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
  if (a >= *cnt) return;
  const int64_t l = list[a];
  T acc = 0;
  for (int64_t t = lane; t < len; t += WAVE) acc += A[l * ld + t] * v[t];
  acc = wave_sum(acc);
  if (lane == 0) s[a] = h1[l] - (h2 ? h2[l] : (T)0) - acc;
}
template <typename T>
void launch_list_resid(const T *Arm, int64_t ld, int64_t len,
                       const int32_t *list, const int64_t *count_dev,
                       int64_t cap, const T *h1, const T *h2, const T *v,
                       T *s, Ctrl *ctrl, int respect_done, hipStream_t st) {
  hipLaunchKernelGGL(list_resid_kernel<T>, dim3((unsigned)((cap + 3) / 4)),
                     dim3(256), 0, st, Arm, ld, len, list, count_dev, h1, h2,
                     v, s, ctrl, respect_done);
}

// ------------------------------------------------------------ sparse CG
// Column block, CGLS with z as the running residual:
//   s = A_U^T z (= g_U), p = s, gam = ||s||^2
//   step: q = A phat (phat = p on U, zero elsewhere)   [wide, CSR rows]
//         alpha = gam / ||q||^2                         [last block]
//         z -= alpha q ; s -= alpha A_U^T q             [narrow + elementwise]
//         gam' = ||s||^2, p = s + (gam'/gam) p          [last block]
// Row block, CG on A^J A^J^T w = r^J with Jacobi rho_J, d accumulated:
//   step: u = A^T phat (phat = p on J)                  [wide, CSC columns]
//         x += alpha_prev u_prev (fused before u is overwritten)
//         v = A^J u, alpha = rz / <p, v>                [narrow, last block]
//         res -= alpha v, zz = res/rho, beta, p = zz + beta p
constexpr int SC_NT = 256;
constexpr unsigned SC_MAXB = 512;   // blocks of a launch that ends in a ticket
constexpr unsigned SC_WIDE_MAXB = 512;   // blocks of the columns' wide product
constexpr unsigned SC_WIDE_GRID_MIN = 8;  // slots per group above which the
                                          // wide product takes a full grid
// Larger blocks update the CG vectors with separate many-workgroup launches
// (sc_cupd, sc_rupd1/2) instead of a walk by the last workgroup.
constexpr int64_t SC_SERIAL_MAX = 16384;
constexpr int SC_UNROLL = 8;        // loads in flight in one-block list walks

template <typename T, int G>
__global__ void __launch_bounds__(SC_NT)
sc_wide_col(Csr<T> A, const T *__restrict__ phat, T *__restrict__ q,
            double *__restrict__ part, const double *__restrict__ plong,
            int64_t nlong, Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  if (cg_done_at_start(ctrl, 0)) return;
  __shared__ double sh[SC_NT / WAVE];
  constexpr int SPB = SC_NT / G;
  const int lg = threadIdx.x & (G - 1);
  double qq = 0.0;
  // grid-stride over row segments: a bounded grid keeps the final ticket
  // and the partials to reduce few
  for (int64_t slot0 = (int64_t)blockIdx.x * SPB; slot0 < A.rows;
       slot0 += (int64_t)gridDim.x * SPB) {
    const int64_t slot = slot0 + threadIdx.x / G;
    int64_t s = 0, br = 0, co = 0;
    T acc = 0;
    bool mine = slot < A.rows;
    if (mine) {
      vrow(A, slot, s, br, co);
      const T *ph = phat + co;
      const int64_t e0 = A.ptr[br], e1 = seg_end(A, br);
      if (nlong && (A.long_flag ? A.long_flag[br] != 0 : e1 - e0 > A.long_limit))
        mine = false;   // sc_long_wide
      else
        for (int64_t e = e0 + lg; e < e1; e += G) acc += A.val[e] * ph[A.idx[e]];
    }
    acc = group_sum<G>(acc);
    if (mine && lg == 0) {
      q[s] = acc;
      qq += (double)acc * (double)acc;
    }
  }
  qq = block_sum<SC_NT>(qq, sh);
  if (threadIdx.x == 0) st_agent(&part[blockIdx.x], qq);
  if (!last_block(&ctrl->ticket[3])) return;
  double tot = 0.0, tl = 0.0;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += SC_NT) tot += ld_agent(&part[b]);
  for (int64_t i = threadIdx.x; i < nlong; i += SC_NT) tl += plong[i];
  tot = block_sum<SC_NT>(tot, sh);
  tot += block_sum<SC_NT>(tl, sh);
  if (threadIdx.x == 0) {
    const double gam = ctrl->cg_rz[0];
    ctrl->cg_alpha[0] = tot > 0.0 ? gam / tot : 0.0;
    if (tot == 0.0) ctrl->cg_done[0] = 1;
  }
}

// The same product over a full grid (one row slot per thread group, no
// grid-stride loop) for matrices with many rows, where a bounded grid walks
// its rows as a long chain of dependent loads; each workgroup leaves its
// partial of ||q||^2, and sc_wide_col_fin sums them (in block order, then
// the long segments) and forms alpha.
template <typename T, int G>
__global__ void __launch_bounds__(SC_NT)
sc_wide_col_grid(Csr<T> A, const T *__restrict__ phat, T *__restrict__ q,
                 double *__restrict__ part, int64_t nlong, Ctrl *ctrl,
                 int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  if (cg_done_at_start(ctrl, 0)) return;
  __shared__ double sh[SC_NT / WAVE];
  constexpr int SPB = SC_NT / G;
  const int lg = threadIdx.x & (G - 1);
  const int64_t slot = (int64_t)blockIdx.x * SPB + threadIdx.x / G;
  double qq = 0.0;
  int64_t s = 0, br = 0, co = 0;
  T acc = 0;
  bool mine = slot < A.rows;
  if (mine) {
    vrow(A, slot, s, br, co);
    const T *ph = phat + co;
    const int64_t e0 = A.ptr[br], e1 = seg_end(A, br);
    if (nlong && (A.long_flag ? A.long_flag[br] != 0 : e1 - e0 > A.long_limit))
      mine = false;   // sc_long_wide
    else
      for (int64_t e = e0 + lg; e < e1; e += G) acc += A.val[e] * ph[A.idx[e]];
  }
  acc = group_sum<G>(acc);
  if (mine && lg == 0) {
    q[s] = acc;
    qq = (double)acc * (double)acc;
  }
  qq = block_sum<SC_NT>(qq, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = qq;
}
template <typename T>
__global__ void __launch_bounds__(1024)
sc_wide_col_fin(const double *__restrict__ part, int64_t nb,
                const double *__restrict__ plong, int64_t nlong, Ctrl *ctrl,
                int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  if (cg_done_at_start(ctrl, 0)) return;
  __shared__ double sh[1024 / WAVE];
  double tot = 0.0, tl = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += 1024) tot += part[b];
  for (int64_t i = threadIdx.x; i < nlong; i += 1024) tl += plong[i];
  tot = block_sum<1024>(tot, sh);
  tot += block_sum<1024>(tl, sh);
  if (threadIdx.x == 0) {
    const double gam = ctrl->cg_rz[0];
    ctrl->cg_alpha[0] = tot > 0.0 ? gam / tot : 0.0;
    if (tot == 0.0) ctrl->cg_done[0] = 1;
  }
}

// narrow: w_a = <A_(U_a), q> over listed CSC columns; s -= alpha w;
// and z -= alpha q over a slice of rows; last block: gam', beta, p, phat.
template <typename T, int G>
__global__ void __launch_bounds__(SC_NT)
sc_narrow_col(Csr<T> At, const int32_t *__restrict__ U,
              const int64_t *__restrict__ cnt, const T *__restrict__ q,
              T *__restrict__ z, int64_t m, T *__restrict__ sres,
              T *__restrict__ p, T *__restrict__ phat,
              double *__restrict__ part, const double *__restrict__ plong,
              int64_t nlong, double tol, int par, int gridm,
              const T *__restrict__ pre, Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  if (cg_done_at_start(ctrl, 0)) return;
  __shared__ double sh[SC_NT / WAVE];
  const double alpha = ctrl->cg_alpha[0];
  const int64_t c = *cnt;
  // elementwise part: z -= alpha q on this block's slice of rows
  const int64_t per = (m + gridDim.x - 1) / gridDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * per;
  for (int64_t i = i0 + threadIdx.x; i < i0 + per && i < m; i += SC_NT)
    z[i] -= (T)alpha * q[i];
  // narrow part (grid-stride over the listed columns)
  constexpr int SPB = SC_NT / G;
  const int lg = threadIdx.x & (G - 1);
  double ss = 0.0;
  for (int64_t a0 = (int64_t)blockIdx.x * SPB; a0 < c;
       a0 += (int64_t)gridDim.x * SPB) {
    const int64_t a = a0 + threadIdx.x / G;
    T acc = 0;
    bool mine = a < c;
    if (mine) {
      int64_t bc, ro;
      gsplit(At, (int64_t)U[a], bc, ro);
      if (pre) {   // many right-hand sides: A^T q formed interleaved
        if (lg == 0) acc = pre[bc * At.rep + (int64_t)U[a] / At.brows];
      } else {
        const T *qv = q + ro;
        const int64_t e0 = At.ptr[bc], e1 = At.ptr[bc + 1];
        if (nlong && e1 - e0 > At.long_limit) mine = false;   // sc_long_narrow
        else
          for (int64_t e = e0 + lg; e < e1; e += G) acc += At.val[e] * qv[At.idx[e]];
      }
    }
    acc = group_sum<G>(acc);
    if (mine && lg == 0) {
      const T sv = sres[a] - (T)alpha * acc;
      sres[a] = sv;
      ss += (double)sv * (double)sv;
    }
  }
  ss = block_sum<SC_NT>(ss, sh);
  if (gridm) {   // full grid: sc_narrow_col_fin reduces the partials
    if (threadIdx.x == 0) part[blockIdx.x] = ss;
    return;
  }
  if (threadIdx.x == 0) st_agent(&part[blockIdx.x], ss);
  if (!last_block(&ctrl->ticket[4])) return;
  double tot = 0.0, tl = 0.0;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += SC_NT) tot += ld_agent(&part[b]);
  for (int64_t i = threadIdx.x; i < nlong; i += SC_NT) tl += plong[i];
  tot = block_sum<SC_NT>(tot, sh);
  tot += block_sum<SC_NT>(tl, sh);
  const double gam = ctrl->cg_rz[0];
  const double beta = gam > 0.0 ? tot / gam : 0.0;
  // one block walks the whole list: keep SC_UNROLL loads in flight
  for (int64_t k0 = threadIdx.x; !par && k0 < c; k0 += SC_UNROLL * SC_NT) {
    T sv[SC_UNROLL], po[SC_UNROLL];
    int32_t ix[SC_UNROLL];
#pragma unroll
    for (int u = 0; u < SC_UNROLL; ++u) {
      const int64_t k = k0 + (int64_t)u * SC_NT;
      if (k < c) { sv[u] = ld_agent(&sres[k]); po[u] = p[k]; ix[u] = U[k]; }
    }
#pragma unroll
    for (int u = 0; u < SC_UNROLL; ++u) {
      const int64_t k = k0 + (int64_t)u * SC_NT;
      if (k < c) {
        const T pv = sv[u] + (T)beta * po[u];
        p[k] = pv;
        phat[ix[u]] = pv;
      }
    }
  }
  if (threadIdx.x == 0) {
    ctrl->cg_beta[0] = beta;
    ctrl->cg_rz[0] = tot;
    ctrl->cg_steps[0] += 1;
    if (tot <= tol * tol * ctrl->cg_rz0[0]) ctrl->cg_done[0] = 1;
  }
}

template <typename T>
__global__ void __launch_bounds__(SC_NT)
sc_init(const int32_t *__restrict__ list, const int64_t *__restrict__ cnt,
        const T *__restrict__ rhs_src, const double *__restrict__ jac,
        T *__restrict__ sres, T *__restrict__ zz_or_null, T *__restrict__ p,
        T *__restrict__ phat, int32_t *__restrict__ pos,
        double *__restrict__ part, Ctrl *ctrl, int ph, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  __shared__ double sh[SC_NT / WAVE];
  const int64_t c = *cnt;
  double rz = 0.0, rr = 0.0;
  for (int64_t a = (int64_t)blockIdx.x * SC_NT + threadIdx.x; a < c;
       a += (int64_t)gridDim.x * SC_NT) {
    const int64_t l = list[a];
    if (pos) pos[l] = (int32_t)a;
    const T h = rhs_src[l];
    sres[a] = h;
    T zz = h;
    if (jac) {
      const double dj = jac[l];
      zz = dj > 0.0 ? (T)((double)h / dj) : (T)0;
      zz_or_null[a] = zz;
    }
    p[a] = zz;
    phat[l] = zz;
    rz += (double)h * (double)zz;
    rr += (double)h * (double)h;
  }
  rz = block_sum<SC_NT>(rz, sh);
  rr = block_sum<SC_NT>(rr, sh);
  if (threadIdx.x == 0) {
    st_agent(&part[2 * blockIdx.x], rz);
    st_agent(&part[2 * blockIdx.x + 1], rr);
  }
  if (!last_block(&ctrl->ticket[6])) return;
  rz = 0.0;
  rr = 0.0;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += SC_NT) {
    rz += ld_agent(&part[2 * b]);
    rr += ld_agent(&part[2 * b + 1]);
  }
  rz = block_sum<SC_NT>(rz, sh);
  rr = block_sum<SC_NT>(rr, sh);
  if (threadIdx.x == 0) {
    ctrl->cg_rz[ph] = rz;
    ctrl->cg_rz0[ph] = rr;
    ctrl->cg_alpha[ph] = 0.0;
    ctrl->cg_done[ph] = (rr == 0.0 || c == 0) ? 1 : 0;
    ctrl->cg_steps[ph] = 0;
  }
}

template <typename T>
__global__ void __launch_bounds__(SC_NT)
sc_clear(const int32_t *__restrict__ list, const int64_t *__restrict__ cnt,
         int64_t cap, T *__restrict__ phat, int32_t *__restrict__ pos,
         Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  const int64_t c = *cnt;
  for (int64_t a = (int64_t)blockIdx.x * SC_NT + threadIdx.x; a < c;
       a += (int64_t)gridDim.x * SC_NT) {
    phat[list[a]] = (T)0;
    if (pos) pos[list[a]] = -1;
  }
}

// Finish of a listed product launched over a full grid (large blocks, many
// listed segments): the partials in block order, then the long segments,
// give what the last workgroup of the bounded launch forms.
//   columns: gam' = ||s||^2, beta = gam'/gam, stop at gam' <= tol^2 gam_0
//   rows:    alpha = rz / <p, v>
__global__ void __launch_bounds__(1024)
sc_narrow_col_fin(const double *__restrict__ part, int64_t nb,
                  const double *__restrict__ plong, int64_t nlong, double tol,
                  Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  if (cg_done_at_start(ctrl, 0)) return;
  __shared__ double sh[1024 / WAVE];
  double tot = 0.0, tl = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += 1024) tot += part[b];
  for (int64_t i = threadIdx.x; i < nlong; i += 1024) tl += plong[i];
  tot = block_sum<1024>(tot, sh);
  tot += block_sum<1024>(tl, sh);
  if (threadIdx.x == 0) {
    const double gam = ctrl->cg_rz[0];
    ctrl->cg_beta[0] = gam > 0.0 ? tot / gam : 0.0;
    ctrl->cg_rz[0] = tot;
    ctrl->cg_steps[0] += 1;
    if (tot <= tol * tol * ctrl->cg_rz0[0]) ctrl->cg_done[0] = 1;
  }
}
__global__ void __launch_bounds__(1024)
sc_narrow_row_fin(const double *__restrict__ part, int64_t nb,
                  const double *__restrict__ plong, int64_t nlong, Ctrl *ctrl,
                  int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  if (cg_done_at_start(ctrl, 1)) return;
  __shared__ double sh[1024 / WAVE];
  double tot = 0.0, tl = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += 1024) tot += part[b];
  for (int64_t i = threadIdx.x; i < nlong; i += 1024) tl += plong[i];
  tot = block_sum<1024>(tot, sh);
  tot += block_sum<1024>(tl, sh);
  if (threadIdx.x == 0) {
    const double rz = ctrl->cg_rz[1];
    ctrl->cg_alpha[1] = tot != 0.0 ? rz / tot : 0.0;
    ctrl->cg_steps[1] += 1;
    if (tot == 0.0) ctrl->cg_done[1] = 1;
  }
}

// Many-workgroup finish of a CG step for large blocks (SC_SERIAL_MAX).  Each
// runs only when the narrow kernel of the same step completed (the step
// counter equals step + 1), so steps after convergence stay no-ops.
template <typename T>
__global__ void __launch_bounds__(SC_NT)
sc_cupd(const int32_t *__restrict__ U, const int64_t *__restrict__ cnt,
        const T *__restrict__ sres, T *__restrict__ p, T *__restrict__ phat,
        Ctrl *ctrl, int step, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  if (ctrl->cg_steps[0] != step + 1) return;
  const double beta = ctrl->cg_beta[0];
  const int64_t c = *cnt;
  for (int64_t a = (int64_t)blockIdx.x * SC_NT + threadIdx.x; a < c;
       a += (int64_t)gridDim.x * SC_NT) {
    const T pv = sres[a] + (T)beta * p[a];
    p[a] = pv;
    phat[U[a]] = pv;
  }
}

// rows: res -= alpha v, zz = res / rho, partials of <res, zz> and ||res||^2;
// the last block forms beta and the stopping test
template <typename T>
__global__ void __launch_bounds__(SC_NT)
sc_rupd1(const int32_t *__restrict__ J, const int64_t *__restrict__ cnt,
         const double *__restrict__ rho, T *__restrict__ res,
         T *__restrict__ zz, const T *__restrict__ v,
         double *__restrict__ part, double tol, Ctrl *ctrl, int step,
         int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  if (ctrl->cg_steps[1] != step + 1) return;
  __shared__ double sh[SC_NT / WAVE];
  const double alpha = ctrl->cg_alpha[1];
  const int64_t c = *cnt;
  double rz1 = 0.0, rr = 0.0;
  for (int64_t a = (int64_t)blockIdx.x * SC_NT + threadIdx.x; a < c;
       a += (int64_t)gridDim.x * SC_NT) {
    const T r = res[a] - (T)alpha * v[a];
    res[a] = r;
    const double dj = rho[J[a]];
    const T zv = dj > 0.0 ? (T)((double)r / dj) : (T)0;
    zz[a] = zv;
    rz1 += (double)r * (double)zv;
    rr += (double)r * (double)r;
  }
  rz1 = block_sum<SC_NT>(rz1, sh);
  rr = block_sum<SC_NT>(rr, sh);
  if (threadIdx.x == 0) {
    st_agent(&part[2 * blockIdx.x], rz1);
    st_agent(&part[2 * blockIdx.x + 1], rr);
  }
  if (!last_block(&ctrl->ticket[7])) return;
  rz1 = 0.0;
  rr = 0.0;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += SC_NT) {
    rz1 += ld_agent(&part[2 * b]);
    rr += ld_agent(&part[2 * b + 1]);
  }
  rz1 = block_sum<SC_NT>(rz1, sh);
  rr = block_sum<SC_NT>(rr, sh);
  if (threadIdx.x == 0) {
    const double rz = ctrl->cg_rz[1];
    ctrl->cg_beta[1] = rz != 0.0 ? rz1 / rz : 0.0;
    ctrl->cg_rz[1] = rz1;
    if (rr <= tol * tol * ctrl->cg_rz0[1]) ctrl->cg_done[1] = 1;
  }
}

template <typename T>
__global__ void __launch_bounds__(SC_NT)
sc_rupd2(const int32_t *__restrict__ J, const int64_t *__restrict__ cnt,
         const T *__restrict__ zz, T *__restrict__ p, T *__restrict__ phat,
         Ctrl *ctrl, int step, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  if (ctrl->cg_steps[1] != step + 1) return;
  const double beta = ctrl->cg_beta[1];
  const int64_t c = *cnt;
  for (int64_t a = (int64_t)blockIdx.x * SC_NT + threadIdx.x; a < c;
       a += (int64_t)gridDim.x * SC_NT) {
    const T pn = zz[a] + (T)beta * p[a];
    p[a] = pn;
    phat[J[a]] = pn;
  }
}

// Long segments of the CG products (one replica of A, rep == 1): one
// workgroup each, so that a few power-law rows do not hold up the launch
// that walks all the short ones with G lanes per segment.  The main kernels
// skip every segment longer than the limit the long lists were built with.
// Wide products take every long segment (A.longs); listed products only
// the long segments whose position in the block list is recorded in pos
// (-1: not in the block).  Each workgroup writes its result and one
// partial (q^2 for columns' wide product, s^2 or <p, v> for the listed
// ones) that the main kernel's last block adds in index order.
template <typename T>
__global__ void __launch_bounds__(SC_NT)
sc_long_wide(Csr<T> A, const T *__restrict__ phat, T *__restrict__ out,
             T *__restrict__ x, double *__restrict__ plong, Ctrl *ctrl,
             int ph, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  if (cg_done_at_start(ctrl, ph)) return;
  __shared__ double sh[SC_NT / WAVE];
  const int64_t r = A.longs[blockIdx.x];
  const int64_t e0 = A.ptr[r], e1 = seg_end(A, r);
  T acc = 0;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += SC_NT)
    acc += A.val[e] * phat[A.idx[e]];
  const T sv = (T)block_sum<SC_NT>((double)acc, sh);
  if (threadIdx.x == 0) {
    if (x) {   // rows: this column's pending x += alpha_prev u_prev first
      const double alpha = ctrl->cg_alpha[ph];
      if (alpha != 0.0) x[r] += (T)alpha * out[r];
    }
    out[r] = sv;
    plong[blockIdx.x] = (double)sv * (double)sv;
  }
}

template <typename T>
__global__ void __launch_bounds__(SC_NT)
sc_long_narrow(Csr<T> A, const int32_t *__restrict__ pos,
               const T *__restrict__ vec, T *__restrict__ dst,
               const T *__restrict__ p, double *__restrict__ plong,
               Ctrl *ctrl, int ph, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  if (cg_done_at_start(ctrl, ph)) return;
  __shared__ double sh[SC_NT / WAVE];
  const int64_t r = A.longs[blockIdx.x];
  const int32_t a = pos[r];
  if (a < 0) {
    if (threadIdx.x == 0) plong[blockIdx.x] = 0.0;
    return;
  }
  const int64_t e0 = A.ptr[r], e1 = A.ptr[r + 1];
  T acc = 0;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += SC_NT)
    acc += A.val[e] * vec[A.idx[e]];
  const T w = (T)block_sum<SC_NT>((double)acc, sh);
  if (threadIdx.x == 0) {
    if (ph == 0) {   // columns: s_a -= alpha w
      const T sv = dst[a] - (T)ctrl->cg_alpha[0] * w;
      dst[a] = sv;
      plong[blockIdx.x] = (double)sv * (double)sv;
    } else {         // rows: v_a = w
      dst[a] = w;
      plong[blockIdx.x] = (double)w * (double)p[a];
    }
  }
}

// rows: wide product u = A^T phat over CSC columns, with the pending update
// x += alpha_prev * u_prev applied first (same column, same thread).
template <typename T, int G>
__global__ void __launch_bounds__(SC_NT)
sc_wide_row(Csr<T> At, const T *__restrict__ phat, T *__restrict__ u,
            T *__restrict__ x, int64_t nlong, Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  if (cg_done_at_start(ctrl, 1)) return;
  const double alpha = ctrl->cg_alpha[1];
  constexpr int SPB = SC_NT / G;
  const int lg = threadIdx.x & (G - 1);
  const int64_t slot = (int64_t)blockIdx.x * SPB + threadIdx.x / G;
  int64_t s = 0, br = 0, co = 0;
  T acc = 0;
  bool mine = slot < At.rows;
  if (mine) {
    vrow(At, slot, s, br, co);
    const T *ph = phat + co;
    const int64_t e0 = At.ptr[br], e1 = seg_end(At, br);
    if (nlong && (At.long_flag ? At.long_flag[br] != 0 : e1 - e0 > At.long_limit))
      mine = false;   // sc_long_wide
    else
      for (int64_t e = e0 + lg; e < e1; e += G) acc += At.val[e] * ph[At.idx[e]];
  }
  acc = group_sum<G>(acc);
  if (mine && lg == 0) {
    if (alpha != 0.0) x[s] += (T)alpha * u[s];
    u[s] = acc;
  }
}

template <typename T, int G>
__global__ void __launch_bounds__(SC_NT)
sc_narrow_row(Csr<T> A, const int32_t *__restrict__ J,
              const int64_t *__restrict__ cnt, const T *__restrict__ u,
              const double *__restrict__ rho, T *__restrict__ res,
              T *__restrict__ zz, T *__restrict__ p, T *__restrict__ v,
              T *__restrict__ phat, double *__restrict__ part,
              const double *__restrict__ plong, int64_t nlong, double tol,
              int par, int gridm, const T *__restrict__ pre, Ctrl *ctrl,
              int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  if (cg_done_at_start(ctrl, 1)) return;
  __shared__ double sh[SC_NT / WAVE];
  const int64_t c = *cnt;
  constexpr int SPB = SC_NT / G;
  const int lg = threadIdx.x & (G - 1);
  double pv = 0.0;
  for (int64_t a0 = (int64_t)blockIdx.x * SPB; a0 < c;
       a0 += (int64_t)gridDim.x * SPB) {
    const int64_t a = a0 + threadIdx.x / G;
    T acc = 0;
    bool mine = a < c;
    if (mine) {
      int64_t brw, co;
      gsplit(A, (int64_t)J[a], brw, co);
      if (pre) {   // many right-hand sides: A u formed interleaved
        if (lg == 0) acc = pre[brw * A.rep + (int64_t)J[a] / A.brows];
      } else {
        const T *uv = u + co;
        const int64_t e0 = A.ptr[brw], e1 = A.ptr[brw + 1];
        if (nlong && e1 - e0 > A.long_limit) mine = false;   // sc_long_narrow
        else
          for (int64_t e = e0 + lg; e < e1; e += G) acc += A.val[e] * uv[A.idx[e]];
      }
    }
    acc = group_sum<G>(acc);
    if (mine && lg == 0) {
      v[a] = acc;
      pv += (double)acc * (double)p[a];
    }
  }
  pv = block_sum<SC_NT>(pv, sh);
  if (gridm) {   // full grid: sc_narrow_row_fin reduces the partials
    if (threadIdx.x == 0) part[blockIdx.x] = pv;
    return;
  }
  if (threadIdx.x == 0) st_agent(&part[blockIdx.x], pv);
  if (!last_block(&ctrl->ticket[5])) return;
  double tot = 0.0, tl = 0.0;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += SC_NT) tot += ld_agent(&part[b]);
  for (int64_t i = threadIdx.x; i < nlong; i += SC_NT) tl += plong[i];
  tot = block_sum<SC_NT>(tot, sh);
  tot += block_sum<SC_NT>(tl, sh);
  const double rz = ctrl->cg_rz[1];
  const double alpha = tot != 0.0 ? rz / tot : 0.0;
  if (par) {   // sc_rupd1 and sc_rupd2 finish the step
    if (threadIdx.x == 0) {
      ctrl->cg_alpha[1] = alpha;
      ctrl->cg_steps[1] += 1;
      if (tot == 0.0) ctrl->cg_done[1] = 1;
    }
    return;
  }
  double rz1 = 0.0, rr = 0.0;
  // one block walks the whole list: keep SC_UNROLL loads in flight
  for (int64_t k0 = threadIdx.x; k0 < c; k0 += SC_UNROLL * SC_NT) {
    T rv[SC_UNROLL], vv[SC_UNROLL];
    double dj[SC_UNROLL];
#pragma unroll
    for (int u = 0; u < SC_UNROLL; ++u) {
      const int64_t k = k0 + (int64_t)u * SC_NT;
      if (k < c) { rv[u] = res[k]; vv[u] = ld_agent(&v[k]); dj[u] = rho[J[k]]; }
    }
#pragma unroll
    for (int u = 0; u < SC_UNROLL; ++u) {
      const int64_t k = k0 + (int64_t)u * SC_NT;
      if (k < c) {
        const T r = rv[u] - (T)alpha * vv[u];
        res[k] = r;
        const T zv = dj[u] > 0.0 ? (T)((double)r / dj[u]) : (T)0;
        zz[k] = zv;
        rz1 += (double)r * (double)zv;
        rr += (double)r * (double)r;
      }
    }
  }
  rz1 = block_sum<SC_NT>(rz1, sh);
  rr = block_sum<SC_NT>(rr, sh);
  const double beta = rz != 0.0 ? rz1 / rz : 0.0;
  for (int64_t k0 = threadIdx.x; k0 < c; k0 += SC_UNROLL * SC_NT) {
    T zv[SC_UNROLL], po[SC_UNROLL];
    int32_t ix[SC_UNROLL];
#pragma unroll
    for (int u = 0; u < SC_UNROLL; ++u) {
      const int64_t k = k0 + (int64_t)u * SC_NT;
      if (k < c) { zv[u] = zz[k]; po[u] = p[k]; ix[u] = J[k]; }
    }
#pragma unroll
    for (int u = 0; u < SC_UNROLL; ++u) {
      const int64_t k = k0 + (int64_t)u * SC_NT;
      if (k < c) {
        const T pn = zv[u] + (T)beta * po[u];
        p[k] = pn;
        phat[ix[u]] = pn;
      }
    }
  }
  if (threadIdx.x == 0) {
    ctrl->cg_alpha[1] = alpha;
    ctrl->cg_rz[1] = rz1;
    ctrl->cg_steps[1] += 1;
    if (rr <= tol * tol * ctrl->cg_rz0[1] || tot == 0.0) ctrl->cg_done[1] = 1;
  }
}

// final pending update x += alpha u (always exactly once per row phase)
template <typename T>
__global__ void __launch_bounds__(SC_NT)
sc_row_finish(int64_t n, const T *__restrict__ u, T *__restrict__ x,
              Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  const double alpha = ctrl->cg_alpha[1];
  const int64_t j = (int64_t)blockIdx.x * SC_NT + threadIdx.x;
  if (j < n && alpha != 0.0) x[j] += (T)alpha * u[j];
}

static unsigned sc_init_blocks(int64_t cap) {
  int64_t b = (cap + SC_NT - 1) / SC_NT;
  if (b > 256) b = 256;
  return (unsigned)(b < 1 ? 1 : b);
}

template <typename T>
static unsigned seg_blocks(int64_t nseg, int G) {
  return (unsigned)((nseg + (SC_NT / G) - 1) / (SC_NT / G));
}

#define RG_SWITCH_G(GV, CALL)                 \
  switch (GV) {                               \
    case 1: { constexpr int GG = 1; CALL; } break;   \
    case 2: { constexpr int GG = 2; CALL; } break;   \
    case 4: { constexpr int GG = 4; CALL; } break;   \
    case 8: { constexpr int GG = 8; CALL; } break;   \
    case 16: { constexpr int GG = 16; CALL; } break; \
    case 32: { constexpr int GG = 32; CALL; } break; \
    default: { constexpr int GG = 64; CALL; } break; \
  }

template <typename T>
void launch_sparse_colproj(const Csr<T> &csr, const Csr<T> &csc,
                           const int32_t *U, const int64_t *count_dev,
                           int64_t cap, const T *g, T *z, SparseCg<T> &w,
                           int max_steps, double tol, Ctrl *ctrl,
                           int respect_done, hipStream_t st) {
  // long segments apart only for one replica of A (the lists are built
  // for it); a replicated operator walks every segment with G lanes
  const int64_t nlw = csr.rep == 1 && w.pos ? csr.nlong : 0;
  const int64_t nln = csc.rep == 1 && w.pos ? csc.nlong : 0;
  hipLaunchKernelGGL(sc_init<T>, dim3(sc_init_blocks(cap)), dim3(SC_NT), 0, st,
                     U, count_dev, g, (const double *)nullptr, w.res,
                     (T *)nullptr, w.p, w.phat, nln ? w.pos : (int32_t *)nullptr,
                     w.part, ctrl, 0, respect_done);
  const unsigned nbw = std::min<unsigned>(seg_blocks<T>(csr.rows, csr.group), SC_WIDE_MAXB);
  // many rows: a full grid and a separate reduction instead of a bounded
  // grid walking SC_WIDE_GRID_MIN or more row slots per thread group
  const unsigned nbg = seg_blocks<T>(csr.rows, csr.group);
  const bool wide_grid = nbg >= SC_WIDE_GRID_MIN * SC_WIDE_MAXB &&
                         (int64_t)nbg <= w.part_cap;
  // many right-hand sides: both products over interleaved vectors, and the
  // listed product reads its value from them (one lane per listed column)
  const bool mm = csr.rep >= REP_MM_MIN && w.t0 != nullptr;
  const int gn = mm ? 1 : csc.group;
  unsigned nbn = std::min<unsigned>(seg_blocks<T>(cap, gn), SC_MAXB);
  if (nbn < 64) nbn = 64;
  const int par = (w.split || cap > SC_SERIAL_MAX) ? 1 : 0;
  // large blocks: the listed product over a full grid, reduced by a
  // separate launch (no grid-stride walk, no last-workgroup ticket)
  const unsigned nbnf = seg_blocks<T>(cap, gn);
  const bool narrow_grid = par && nbnf > SC_MAXB && (int64_t)nbnf <= w.part_cap;
  const unsigned nbu = std::min<unsigned>(
      (unsigned)((cap + SC_NT - 1) / SC_NT), SC_MAXB);
  for (int s = 0; s < max_steps; ++s) {
    if (mm) {
      // q = A phat for every right-hand side, ||q||^2 -> alpha; then A^T q
      launch_rep_tin<T>(w.phat, w.t0, csr.bcols, csr.rep, ctrl, 0,
                        respect_done, st);
      const int nbm = launch_rep_mm<T>(csr, w.t0, w.t1, w.part, ctrl, 0,
                                       respect_done, st);
      hipLaunchKernelGGL(sc_wide_col_fin<T>, dim3(1), dim3(1024), 0, st,
                         (const double *)w.part, (int64_t)nbm,
                         (const double *)nullptr, (int64_t)0, ctrl,
                         respect_done);
      launch_rep_tout<T>(w.t1, w.wide, (T *)nullptr, csr.brows, csr.rep, ctrl,
                         0, respect_done, st);
      launch_rep_mm<T>(csc, w.t1, w.t2, (double *)nullptr, ctrl, 0,
                       respect_done, st);
    } else {
    if (nlw)
      hipLaunchKernelGGL(sc_long_wide<T>, dim3((unsigned)nlw), dim3(SC_NT), 0,
                         st, csr, w.phat, w.wide, (T *)nullptr, w.plong, ctrl,
                         0, respect_done);
    if (wide_grid) {
      RG_SWITCH_G(csr.group,
                  hipLaunchKernelGGL((sc_wide_col_grid<T, GG>), dim3(nbg),
                                     dim3(SC_NT), 0, st, csr, w.phat, w.wide,
                                     w.part, nlw, ctrl, respect_done));
      hipLaunchKernelGGL(sc_wide_col_fin<T>, dim3(1), dim3(1024), 0, st,
                         (const double *)w.part, (int64_t)nbg,
                         (const double *)w.plong, nlw, ctrl, respect_done);
    } else {
      RG_SWITCH_G(csr.group, hipLaunchKernelGGL((sc_wide_col<T, GG>), dim3(nbw),
                                                dim3(SC_NT), 0, st, csr, w.phat,
                                                w.wide, w.part, w.plong, nlw,
                                                ctrl, respect_done));
    }
    }
    if (nln)
      hipLaunchKernelGGL(sc_long_narrow<T>, dim3((unsigned)nln), dim3(SC_NT),
                         0, st, csc, w.pos, w.wide, w.res, w.p, w.plong, ctrl,
                         0, respect_done);
    RG_SWITCH_G(gn,
                hipLaunchKernelGGL((sc_narrow_col<T, GG>),
                                   dim3(narrow_grid ? nbnf : nbn),
                                   dim3(SC_NT), 0, st, csc, U, count_dev,
                                   w.wide, z, csr.rows, w.res, w.p, w.phat,
                                   w.part, w.plong, nln, tol, par,
                                   narrow_grid ? 1 : 0,
                                   mm ? (const T *)w.t2 : (const T *)nullptr,
                                   ctrl, respect_done));
    if (narrow_grid)
      hipLaunchKernelGGL(sc_narrow_col_fin, dim3(1), dim3(1024), 0, st,
                         (const double *)w.part, (int64_t)nbnf,
                         (const double *)w.plong, nln, tol, ctrl,
                         respect_done);
    if (par)
      hipLaunchKernelGGL(sc_cupd<T>, dim3(nbu), dim3(SC_NT), 0, st, U,
                         count_dev, w.res, w.p, w.phat, ctrl, s, respect_done);
  }
  hipLaunchKernelGGL(sc_clear<T>, dim3(64), dim3(SC_NT), 0, st, U, count_dev,
                     cap, w.phat, nln ? w.pos : (int32_t *)nullptr, ctrl,
                     respect_done);
}

template <typename T>
void launch_sparse_rowproj(const Csr<T> &csr, const Csr<T> &csc,
                           const int32_t *J, const int64_t *count_dev,
                           int64_t cap, const T *r, const double *rho, T *x,
                           SparseCg<T> &w, int max_steps, double tol,
                           Ctrl *ctrl, int respect_done, hipStream_t st) {
  const int64_t nlw = csc.rep == 1 && w.pos ? csc.nlong : 0;
  const int64_t nln = csr.rep == 1 && w.pos ? csr.nlong : 0;
  hipLaunchKernelGGL(sc_init<T>, dim3(sc_init_blocks(cap)), dim3(SC_NT), 0, st,
                     J, count_dev, r, rho, w.res, w.v, w.p, w.phat,
                     nln ? w.pos : (int32_t *)nullptr, w.part, ctrl, 1,
                     respect_done);
  // w.v doubles as the Jacobi-scaled residual buffer zz during steps
  const unsigned nbw = seg_blocks<T>(csc.rows, csc.group);
  const bool mm = csr.rep >= REP_MM_MIN && w.t0 != nullptr;
  const int gn = mm ? 1 : csr.group;
  const unsigned nbn = std::min<unsigned>(seg_blocks<T>(cap, gn), SC_MAXB);
  const int par = (w.split || cap > SC_SERIAL_MAX) ? 1 : 0;
  const unsigned nbnf = seg_blocks<T>(cap, gn);
  const bool narrow_grid = par && nbnf > SC_MAXB && (int64_t)nbnf <= w.part_cap;
  const unsigned nbu = std::min<unsigned>(
      (unsigned)((cap + SC_NT - 1) / SC_NT), SC_MAXB);
  for (int s = 0; s < max_steps; ++s) {
    if (mm) {
      // u = A^T phat for every right-hand side (the pending x += alpha u
      // applied as u is replaced), then A u
      launch_rep_tin<T>(w.phat, w.t0, csr.brows, csr.rep, ctrl, 1,
                        respect_done, st);
      launch_rep_mm<T>(csc, w.t0, w.t1, (double *)nullptr, ctrl, 1,
                       respect_done, st);
      launch_rep_tout<T>(w.t1, w.wide, x, csc.brows, csr.rep, ctrl, 1,
                         respect_done, st);
      launch_rep_mm<T>(csr, w.t1, w.t2, (double *)nullptr, ctrl, 1,
                       respect_done, st);
    } else {
    if (nlw)
      hipLaunchKernelGGL(sc_long_wide<T>, dim3((unsigned)nlw), dim3(SC_NT), 0,
                         st, csc, w.phat, w.wide, x, w.plong, ctrl, 1,
                         respect_done);
    RG_SWITCH_G(csc.group, hipLaunchKernelGGL((sc_wide_row<T, GG>), dim3(nbw),
                                              dim3(SC_NT), 0, st, csc, w.phat,
                                              w.wide, x, nlw, ctrl,
                                              respect_done));
    }
    if (nln)
      hipLaunchKernelGGL(sc_long_narrow<T>, dim3((unsigned)nln), dim3(SC_NT),
                         0, st, csr, w.pos, w.wide, w.v + cap, w.p, w.plong,
                         ctrl, 1, respect_done);
    RG_SWITCH_G(gn,
                hipLaunchKernelGGL((sc_narrow_row<T, GG>),
                                   dim3(narrow_grid ? nbnf : nbn),
                                   dim3(SC_NT), 0, st, csr, J, count_dev,
                                   w.wide, rho, w.res, w.v, w.p,
                                   w.v + cap, w.phat, w.part, w.plong, nln,
                                   tol, par, narrow_grid ? 1 : 0,
                                   mm ? (const T *)w.t2 : (const T *)nullptr,
                                   ctrl, respect_done));
    if (narrow_grid)
      hipLaunchKernelGGL(sc_narrow_row_fin, dim3(1), dim3(1024), 0, st,
                         (const double *)w.part, (int64_t)nbnf,
                         (const double *)w.plong, nln, ctrl, respect_done);
    if (par) {
      hipLaunchKernelGGL(sc_rupd1<T>, dim3(nbu), dim3(SC_NT), 0, st, J,
                         count_dev, rho, w.res, w.v, w.v + cap, w.part, tol,
                         ctrl, s, respect_done);
      hipLaunchKernelGGL(sc_rupd2<T>, dim3(nbu), dim3(SC_NT), 0, st, J,
                         count_dev, w.v, w.p, w.phat, ctrl, s, respect_done);
    }
  }
  hipLaunchKernelGGL(sc_row_finish<T>, dim3((unsigned)((csc.rows + SC_NT - 1) / SC_NT)),
                     dim3(SC_NT), 0, st, csc.rows, w.wide, x, ctrl,
                     respect_done);
  hipLaunchKernelGGL(sc_clear<T>, dim3(64), dim3(SC_NT), 0, st, J, count_dev,
                     cap, w.phat, nln ? w.pos : (int32_t *)nullptr, ctrl,
                     respect_done);
}

// ------------------------------------------------------------ small sparse
// Dense row- and column-major copies of a sparse A (one thread per row,
// repeated entries summed in storage order; the buffers come zeroed).
template <typename T>
__global__ void __launch_bounds__(256)
densify_kernel(Csr<T> A, T *__restrict__ rm, int64_t ld, T *__restrict__ cm,
               int64_t ldc) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= A.rows) return;
  for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
    const int64_t j = A.idx[e];
    rm[i * ld + j] += A.val[e];
    cm[j * ldc + i] += A.val[e];
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
list_scatter(const int32_t *__restrict__ list, const int64_t *__restrict__ cnt,
             const T *__restrict__ coef, T *__restrict__ dst, Ctrl *ctrl,
             int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  const int64_t c = *cnt;
  for (int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x; a < c;
       a += (int64_t)gridDim.x * 256)
    dst[list[a]] = coef[a];
}

// out_i += sign * sum_e A_ie phat_(idx e), one thread per row of the view
// (small systems only), in storage order
template <typename T>
__global__ void __launch_bounds__(256)
rows_axpy(Csr<T> A, const T *__restrict__ phat, int sign, T *__restrict__ out,
          Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= A.rows) return;
  T acc = 0;
  bool any = false;
  for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
    const T v = phat[A.idx[e]];
    if (v != (T)0) {
      acc += A.val[e] * v;
      any = true;
    }
  }
  if (any) out[i] += sign > 0 ? acc : -acc;
}

template <typename T>
void launch_densify(const Csr<T> &A, T *rm, int64_t ld, T *cm, int64_t ldc,
                    hipStream_t st) {
  const unsigned nb = (unsigned)((A.rows + 255) / 256);
  hipLaunchKernelGGL(densify_kernel<T>, dim3(nb > 0 ? nb : 1), dim3(256), 0, st,
                     A, rm, ld, cm, ldc);
}

template <typename T>
void launch_sparse_block_update(const Csr<T> &A, const int32_t *list,
                                const int64_t *count_dev, int64_t cap,
                                const T *coef, int sign, T *phat, T *out,
                                Ctrl *ctrl, int respect_done, hipStream_t st) {
  const unsigned nl = (unsigned)std::max<int64_t>(1, std::min<int64_t>(
      (cap + 255) / 256, 256));
  hipLaunchKernelGGL(list_scatter<T>, dim3(nl), dim3(256), 0, st, list,
                     count_dev, coef, phat, ctrl, respect_done);
  const unsigned nr = (unsigned)((A.rows + 255) / 256);
  hipLaunchKernelGGL(rows_axpy<T>, dim3(nr > 0 ? nr : 1), dim3(256), 0, st, A,
                     phat, sign, out, ctrl, respect_done);
  hipLaunchKernelGGL(sc_clear<T>, dim3(64), dim3(SC_NT), 0, st, list,
                     count_dev, cap, phat, (int32_t *)nullptr, ctrl,
                     respect_done);
}

// ------------------------------------------------------------ instantiate
#define RG_INST(T)                                                            \
  template void launch_gram_gather<T>(const T *, int64_t, const int32_t *,   \
                                      const int64_t *, int64_t, T *, Ctrl *,  \
                                      int, hipStream_t);                      \
  template void launch_gram_rows<T>(const T *, int64_t, int64_t,             \
                                    const int32_t *, const int64_t *,        \
                                    int64_t, T *, Ctrl *, int, hipStream_t);  \
  template void launch_gram_full<T>(const T *, int64_t, int64_t, int64_t,    \
                                    T *, hipStream_t);                        \
  template void launch_chol_solve<T>(T *, int64_t, const int64_t *,          \
                                     const T *, const int32_t *, T *, int,   \
                                     Ctrl *, int, int, hipStream_t);          \
  template void launch_pcg_gram_init<T>(const T *, int64_t, const int64_t *, \
                                        const T *, const int32_t *, T *,     \
                                        CgWork<T> &, Ctrl *, int, int,        \
                                        hipStream_t);                         \
  template void launch_pcg_gram_step<T>(const T *, int64_t, const int64_t *, \
                                        T *, CgWork<T> &, int, double,       \
                                        Ctrl *, int, int, hipStream_t);       \
  template void launch_pcg_persist<T>(T *, int64_t, const int64_t *,         \
                                      const T *, const int32_t *, T *,       \
                                      CgWork<T> &, int, int, double, Ctrl *, \
                                      int, int, hipStream_t, const T *,      \
                                      int64_t);                               \
  template void launch_col_update<T>(const T *, int64_t, int64_t,            \
                                     const int32_t *, const int64_t *,       \
                                     int64_t, const T *, T *, T *, Ctrl *,   \
                                     int, hipStream_t);                       \
  template void launch_row_update<T>(const T *, int64_t, int64_t,            \
                                     const int32_t *, const int64_t *,       \
                                     int64_t, const T *, T *, T *, Ctrl *,   \
                                     int, hipStream_t);                       \
  template void launch_list_resid<T>(const T *, int64_t, int64_t,            \
                                     const int32_t *, const int64_t *,       \
                                     int64_t, const T *, const T *,          \
                                     const T *, T *, Ctrl *, int,            \
                                     hipStream_t);                            \
  template void launch_sparse_colproj<T>(const Csr<T> &, const Csr<T> &,     \
                                         const int32_t *, const int64_t *,   \
                                         int64_t, const T *, T *,            \
                                         SparseCg<T> &, int, double, Ctrl *, \
                                         int, hipStream_t);                   \
  template void launch_sparse_rowproj<T>(const Csr<T> &, const Csr<T> &,     \
                                         const int32_t *, const int64_t *,   \
                                         int64_t, const T *, const double *, \
                                         T *, SparseCg<T> &, int, double,    \
                                         Ctrl *, int, hipStream_t);
RG_INST(double)
RG_INST(float)
template void launch_densify<double>(const Csr<double> &, double *, int64_t,
                                     double *, int64_t, hipStream_t);
template void launch_densify<float>(const Csr<float> &, float *, int64_t,
                                    float *, int64_t, hipStream_t);
template void launch_sparse_block_update<double>(
    const Csr<double> &, const int32_t *, const int64_t *, int64_t,
    const double *, int, double *, double *, Ctrl *, int, hipStream_t);
template void launch_sparse_block_update<float>(
    const Csr<float> &, const int32_t *, const int64_t *, int64_t,
    const float *, int, float *, float *, Ctrl *, int, hipStream_t);
#undef RG_INST

// ------------------------------------------------------------ block restriction
// The wide products of the sparse CG (columns: q = A phat over CSR rows;
// rows: u = A^T phat over CSC columns) multiply by a vector that is zero
// outside the block, so only the entries of the block's columns (rows) can
// contribute.  Once per iteration those entries are copied, in storage
// order and with their original indices, into a compact matrix of the same
// row count; every CG step then streams it instead of all of A (about the
// block's share of the nonzeros).  The long rows of A (one workgroup each
// in the CG products) stay long in the copy.  The sums drop only zero terms
// and stay deterministic; their grouping across lanes differs from the full
// pass's, so the two agree to rounding.
// One stored matrix: the copy keeps A's row starts ("gapped"), so one pass
// suffices:
//   mark:   mask[list_a] = 1
//   fill:   each row's marked entries, in order, from A.ptr_r (ballot
//           ranks); end_r = A.ptr_r + their count
//   unmark: mask[list_a] = 0
// For the replicated operator I_rep (x) A of a few right-hand sides the copy
// is a compact matrix over the virtual rows and columns (each right-hand
// side keeps the entries of its own block; the capacity is the k longest
// columns' entries per right-hand side, not A's):
//   mark
//   count:  cnt_r = #{e in row r : mask[idx_e]}            (G lanes per row)
//   scan:   ptr = exclusive prefix sum of cnt             (three launches)
//   fill:   each row's marked entries, in order, to ptr_r
//   unmark
constexpr int SB_NT = 256;
constexpr int SB_TILE = 2048;          // scan elements per workgroup

__global__ void __launch_bounds__(SB_NT)
sub_mark(const int32_t *__restrict__ list, const int64_t *__restrict__ cnt,
         int32_t *__restrict__ mask, int32_t v, Ctrl *ctrl) {
  if (ctrl_done(ctrl)) return;
  const int64_t c = *cnt;
  for (int64_t a = (int64_t)blockIdx.x * SB_NT + threadIdx.x; a < c;
       a += (int64_t)gridDim.x * SB_NT)
    mask[list[a]] = v;
}

template <typename T, int G>
__global__ void __launch_bounds__(SB_NT)
sub_count(Csr<T> A, const int32_t *__restrict__ mask, int64_t *__restrict__ cnt,
          const uint8_t *__restrict__ long_flag, Ctrl *ctrl) {
  if (ctrl_done(ctrl)) return;
  constexpr int SPB = SB_NT / G;
  const int lg = threadIdx.x & (G - 1);
  const int64_t r = (int64_t)blockIdx.x * SPB + threadIdx.x / G;
  int64_t k = 0;
  const bool mine = r < A.rows && !(long_flag && long_flag[r]);   // sub_count_long
  if (mine) {
    int64_t br, co;      // stored row and column offset (replicated A)
    gsplit(A, r, br, co);
    const int32_t *mk = mask + co;
    const int64_t e0 = A.ptr[br], e1 = A.ptr[br + 1];
    for (int64_t e = e0 + lg; e < e1; e += G) k += mk[A.idx[e]] ? 1 : 0;
  }
  k = group_sum<G>(k);
  if (mine && lg == 0) cnt[r] = k;
  if (r == A.rows && lg == 0) cnt[r] = 0;   // sentinel: ptr[rows] = total
}

// exclusive scan of n int64 values: per-tile sums, scan of the tile sums in
// one workgroup, then per-tile scans with the tile offset
__global__ void __launch_bounds__(SB_NT)
sub_scan_a(const int64_t *__restrict__ v, int64_t n,
           int64_t *__restrict__ tile, Ctrl *ctrl) {
  if (ctrl_done(ctrl)) return;
  __shared__ int64_t sh[SB_NT / WAVE];
  const int64_t i0 = (int64_t)blockIdx.x * SB_TILE;
  int64_t s = 0;
  for (int64_t i = i0 + threadIdx.x; i < i0 + SB_TILE && i < n; i += SB_NT)
    s += v[i];
  s = block_sum_i64<SB_NT>(s, sh);
  if (threadIdx.x == 0) tile[blockIdx.x] = s;
}
__global__ void __launch_bounds__(1024)
sub_scan_b(int64_t *__restrict__ tile, int64_t ntile, Ctrl *ctrl) {
  if (ctrl_done(ctrl)) return;
  __shared__ int64_t sh[1024];
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < ntile; b0 += 1024) {
    const int64_t b = b0 + threadIdx.x;
    const int64_t v = b < ntile ? tile[b] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int64_t t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
      __syncthreads();
      sh[threadIdx.x] += t;
      __syncthreads();
    }
    if (b < ntile) tile[b] = carry + sh[threadIdx.x] - v;   // exclusive
    const int64_t tot = sh[1023];
    __syncthreads();
    carry += tot;
  }
}
__global__ void __launch_bounds__(SB_NT)
sub_scan_c(const int64_t *__restrict__ v, int64_t n,
           const int64_t *__restrict__ tile, int64_t *__restrict__ out,
           Ctrl *ctrl) {
  if (ctrl_done(ctrl)) return;
  constexpr int PER = SB_TILE / SB_NT;   // consecutive elements per thread
  __shared__ int64_t sh[SB_NT];
  const int64_t i0 = (int64_t)blockIdx.x * SB_TILE + (int64_t)threadIdx.x * PER;
  int64_t loc[PER];
  int64_t s = 0;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int64_t i = i0 + u;
    loc[u] = s;
    s += i < n ? v[i] : 0;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < SB_NT; o <<= 1) {
    const int64_t t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  const int64_t base = tile[blockIdx.x] + sh[threadIdx.x] - s;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int64_t i = i0 + u;
    if (i < n) out[i] = base + loc[u];
  }
}

// ptr == nullptr: the gapped copy of one stored matrix -- row r's entries
// start at A.ptr[r] and end[r] receives their end (no count or scan)
template <typename T, int G>
__global__ void __launch_bounds__(SB_NT)
sub_fill(Csr<T> A, const int32_t *__restrict__ mask,
         const int64_t *__restrict__ ptr, int32_t *__restrict__ idx,
         T *__restrict__ val, const uint8_t *__restrict__ long_flag,
         int64_t *__restrict__ end, Ctrl *ctrl) {
  if (ctrl_done(ctrl)) return;
  constexpr int SPB = SB_NT / G;
  const int lane = threadIdx.x & (WAVE - 1);
  const int lg = threadIdx.x & (G - 1);
  const int gbase = lane & ~(G - 1);          // first lane of the group
  const int64_t r = (int64_t)blockIdx.x * SPB + threadIdx.x / G;
  const bool live = r < A.rows && !(long_flag && long_flag[r]);  // sub_fill_long
  int64_t br = 0, co = 0;   // stored row and column offset (replicated A)
  if (live) gsplit(A, r, br, co);
  const int64_t e0 = live ? A.ptr[br] : 0, e1 = live ? A.ptr[br + 1] : 0;
  int64_t pos = live ? (ptr ? ptr[r] : e0) : 0;
  // every lane of a wave runs the same trip count (ballots need the whole
  // wave): the longest segment of the wave's groups
  int64_t len = e1 - e0;
  for (int o = 32; o > 0; o >>= 1) {
    const int64_t t = __shfl_xor(len, o, WAVE);
    len = t > len ? t : len;
  }
  const unsigned long long gmask =
      (G == 64) ? ~0ull : (((1ull << G) - 1ull) << gbase);
  for (int64_t c = 0; c < len; c += G) {
    const int64_t e = e0 + c + lg;
    const bool in = e < e1;
    const int32_t j = in ? (int32_t)(co + A.idx[e]) : 0;
    const bool take = in && mask[j] != 0;
    const unsigned long long bal = __ballot(take);
    const unsigned long long mine = bal & gmask;
    const unsigned long long below = mine & ((1ull << lane) - 1ull);
    if (take) {
      const int64_t o = pos + __popcll(below);
      idx[o] = j;
      val[o] = A.val[e];
    }
    pos += __popcll(mine);
  }
  if (!ptr && live && lg == 0) end[r] = pos;
}

// long rows (A.longs): one workgroup each, in storage order
template <typename T>
__global__ void __launch_bounds__(SB_NT)
sub_count_long(Csr<T> A, const int32_t *__restrict__ mask,
               int64_t *__restrict__ cnt, Ctrl *ctrl) {
  if (ctrl_done(ctrl)) return;
  __shared__ int64_t sh[SB_NT / WAVE];
  const int64_t r = A.longs[blockIdx.x];
  const int64_t e0 = A.ptr[r], e1 = A.ptr[r + 1];
  int64_t k = 0;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += SB_NT)
    k += mask[A.idx[e]] ? 1 : 0;
  k = block_sum_i64<SB_NT>(k, sh);
  if (threadIdx.x == 0) cnt[r] = k;
}
template <typename T>
__global__ void __launch_bounds__(SB_NT)
sub_fill_long(Csr<T> A, const int32_t *__restrict__ mask,
              const int64_t *__restrict__ ptr, int32_t *__restrict__ idx,
              T *__restrict__ val, int64_t *__restrict__ end, Ctrl *ctrl) {
  if (ctrl_done(ctrl)) return;
  __shared__ int64_t wsum[SB_NT / WAVE];
  const int lane = threadIdx.x & (WAVE - 1);
  const int w = threadIdx.x / WAVE;
  const int64_t r = A.longs[blockIdx.x];
  const int64_t e0 = A.ptr[r], e1 = A.ptr[r + 1];
  int64_t pos = ptr ? ptr[r] : e0;
  for (int64_t c = e0; c < e1; c += SB_NT) {
    const int64_t e = c + threadIdx.x;
    const bool in = e < e1;
    const int32_t j = in ? A.idx[e] : 0;
    const bool take = in && mask[j] != 0;
    const unsigned long long bal = __ballot(take);
    if (lane == 0) wsum[w] = __popcll(bal);
    __syncthreads();
    int64_t before = 0, tot = 0;
    for (int i = 0; i < SB_NT / WAVE; ++i) {
      before += i < w ? wsum[i] : 0;
      tot += wsum[i];
    }
    if (take) {
      const int64_t o = pos + before + __popcll(bal & ((1ull << lane) - 1ull));
      idx[o] = j;
      val[o] = A.val[e];
    }
    pos += tot;
    __syncthreads();
  }
  if (!ptr && threadIdx.x == 0) end[r] = pos;
}

int64_t sub_scan_tiles(int64_t n) { return (n + SB_TILE - 1) / SB_TILE; }

template <typename T>
__global__ void __launch_bounds__(SB_NT)
mark_long_kernel(Csr<T> A, uint8_t *__restrict__ flag) {
  const int64_t r = (int64_t)blockIdx.x * SB_NT + threadIdx.x;
  if (r < A.rows)
    flag[r] = (A.long_limit > 0 && A.ptr[r + 1] - A.ptr[r] > A.long_limit) ? 1 : 0;
}
template <typename T>
void launch_mark_long(const Csr<T> &A, uint8_t *flag, hipStream_t st) {
  hipLaunchKernelGGL(mark_long_kernel<T>, dim3((unsigned)((A.rows + SB_NT - 1) / SB_NT)),
                     dim3(SB_NT), 0, st, A, flag);
}
template void launch_mark_long<double>(const Csr<double> &, uint8_t *, hipStream_t);
template void launch_mark_long<float>(const Csr<float> &, uint8_t *, hipStream_t);

template <typename T>
Csr<T> launch_sub_matrix(const Csr<T> &A, const int32_t *list,
                         const int64_t *count_dev, int64_t list_cap,
                         SubWork &w, Ctrl *ctrl, hipStream_t st) {
  const unsigned gm = (unsigned)std::min<int64_t>(
      std::max<int64_t>((list_cap + SB_NT - 1) / SB_NT, 1), 1024);
  hipLaunchKernelGGL(sub_mark, dim3(gm), dim3(SB_NT), 0, st, list, count_dev,
                     w.mask, 1, ctrl);
  const int64_t rows = A.rows;
  const int G = A.group;
  const unsigned nb = (unsigned)((rows + 1 + SB_NT / G - 1) / (SB_NT / G));
  const uint8_t *lf = (A.nlong && A.rep == 1) ? w.long_flag : nullptr;
  if (A.rep == 1) {
    // one stored matrix: the gapped copy, each row's block entries at the
    // start of its own span of A (row ends in w.cnt), in one pass
    RG_SWITCH_G(G, hipLaunchKernelGGL((sub_fill<T, GG>), dim3(nb), dim3(SB_NT),
                                      0, st, A, w.mask, (const int64_t *)nullptr,
                                      w.idx, (T *)w.val, lf, w.cnt, ctrl));
    if (lf)
      hipLaunchKernelGGL(sub_fill_long<T>, dim3((unsigned)A.nlong), dim3(SB_NT),
                         0, st, A, w.mask, (const int64_t *)nullptr, w.idx,
                         (T *)w.val, w.cnt, ctrl);
    hipLaunchKernelGGL(sub_mark, dim3(gm), dim3(SB_NT), 0, st, list, count_dev,
                       w.mask, 0, ctrl);
    Csr<T> B = A;
    B.idx = w.idx;
    B.val = (const T *)w.val;
    B.pend = w.cnt;
    B.group = w.group;
    // A's long rows stay long segments (one workgroup each) in the copy
    B.long_flag = w.long_flag;
    B.mp_rs = nullptr;     // no merge plan: row-split passes only
    B.mp_nchunk = 0;
    return B;
  }
  RG_SWITCH_G(G, hipLaunchKernelGGL((sub_count<T, GG>), dim3(nb), dim3(SB_NT),
                                    0, st, A, w.mask, w.cnt, lf, ctrl));
  if (lf)
    hipLaunchKernelGGL(sub_count_long<T>, dim3((unsigned)A.nlong), dim3(SB_NT),
                       0, st, A, w.mask, w.cnt, ctrl);
  const int64_t nt = sub_scan_tiles(rows + 1);
  hipLaunchKernelGGL(sub_scan_a, dim3((unsigned)nt), dim3(SB_NT), 0, st, w.cnt,
                     rows + 1, w.tile, ctrl);
  hipLaunchKernelGGL(sub_scan_b, dim3(1), dim3(1024), 0, st, w.tile, nt, ctrl);
  hipLaunchKernelGGL(sub_scan_c, dim3((unsigned)nt), dim3(SB_NT), 0, st, w.cnt,
                     rows + 1, w.tile, w.ptr, ctrl);
  RG_SWITCH_G(G, hipLaunchKernelGGL((sub_fill<T, GG>), dim3(nb), dim3(SB_NT),
                                    0, st, A, w.mask, (const int64_t *)w.ptr,
                                    w.idx, (T *)w.val, lf, (int64_t *)nullptr,
                                    ctrl));
  if (lf)
    hipLaunchKernelGGL(sub_fill_long<T>, dim3((unsigned)A.nlong), dim3(SB_NT),
                       0, st, A, w.mask, (const int64_t *)w.ptr, w.idx,
                       (T *)w.val, (int64_t *)nullptr, ctrl);
  hipLaunchKernelGGL(sub_mark, dim3(gm), dim3(SB_NT), 0, st, list, count_dev,
                     w.mask, 0, ctrl);
  Csr<T> B = A;
  B.ptr = w.ptr;
  B.idx = w.idx;
  B.val = (const T *)w.val;
  B.nnz = w.cap;
  B.group = w.group;
  // the replicated operator I_rep (x) A: the copy is a plain matrix over
  // the virtual rows and columns (column indices already offset)
  B.rep = 1;
  B.brows = A.rows;
  B.bcols = A.cols;
  B.longs = nullptr;
  B.nlong = 0;
  B.long_limit = 0;
  B.long_flag = nullptr;
  B.mp_rs = nullptr;     // no merge plan: row-split passes only
  B.mp_nchunk = 0;
  return B;
}
template Csr<double> launch_sub_matrix<double>(const Csr<double> &, const int32_t *, const int64_t *, int64_t, SubWork &, Ctrl *, hipStream_t);
template Csr<float> launch_sub_matrix<float>(const Csr<float> &, const int32_t *, const int64_t *, int64_t, SubWork &, Ctrl *, hipStream_t);

// ------------------------------------------------------------ tall row blocks
// A row block with more rows than A has columns (k_row > n) is in general
// inconsistent: r^J need not lie in range(A^J), and CG on A^J A^J^T does not
// reach the pseudoinverse update there.  Such blocks are projected by CGLS on
// min ||A^J d - r^J|| started at d = 0, whose limit is the minimum-norm
// least-squares solution (A^J)^+ r^J (for independent columns,
// (A^J^T A^J)^-1 A^J^T r^J):
//   res = r^J, s = A^J^T res, p = s, gam = ||s||^2
//   step: q = A^J p; alpha = gam / ||q||^2; d += alpha p; res -= alpha q;
//         s = A^J^T res; gam' = ||s||^2 (stop when gam' <= tol^2 gam_0);
//         p = s + (gam'/gam) p
//   x += d
// The vector recurrences and their norms run in one workgroup (fixed
// order); the products are listed-row dots and the thin row update (dense),
// or listed CSR segment dots and a CSC pass over the residual scattered
// onto the block's rows (sparse).  Ctrl::cg_rz[1] holds gam, cg_rz0[1] gam_0.
constexpr int TL_NT = 1024;

// d = 0, s = 0 (n); rhat = 0 (m); CG flags of the row phase reset
template <typename T>
__global__ void __launch_bounds__(256)
tall_init(int64_t n, int64_t m, T *__restrict__ d, T *__restrict__ s,
          T *__restrict__ rhat, Ctrl *ctrl) {
  if (ctrl_done(ctrl)) return;
  const int64_t stride = (int64_t)gridDim.x * 256;
  const int64_t i0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (int64_t i = i0; i < n; i += stride) { d[i] = (T)0; s[i] = (T)0; }
  if (rhat)
    for (int64_t i = i0; i < m; i += stride) rhat[i] = (T)0;
  if (i0 == 0) { ctrl->cg_done[1] = 0; ctrl->cg_steps[1] = 0; }
}

// res_a = r[J_a] (and rhat[J_a] = res_a)
template <typename T>
__global__ void __launch_bounds__(256)
tall_load(const int32_t *__restrict__ J, const int64_t *__restrict__ cnt,
          const T *__restrict__ r, T *__restrict__ res, T *__restrict__ rhat,
          Ctrl *ctrl) {
  if (ctrl_done(ctrl)) return;
  const int64_t c = *cnt;
  for (int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x; a < c;
       a += (int64_t)gridDim.x * 256) {
    const T v = r[J[a]];
    res[a] = v;
    if (rhat) rhat[J[a]] = v;
  }
}

// gam = gam_0 = ||s||^2, p = s
template <typename T>
__global__ void __launch_bounds__(TL_NT)
tall_start(int64_t n, const T *__restrict__ s, T *__restrict__ p, Ctrl *ctrl) {
  if (ctrl_done(ctrl)) return;
  __shared__ double sh[TL_NT / WAVE];
  double g = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += TL_NT) {
    const T v = s[i];
    p[i] = v;
    g += (double)v * (double)v;
  }
  g = block_sum<TL_NT>(g, sh);
  if (threadIdx.x == 0) {
    ctrl->cg_rz[1] = g;
    ctrl->cg_rz0[1] = g;
    if (!(g > 0.0)) ctrl->cg_done[1] = 1;
  }
}

// dense q_a = <A_{J_a}, p>: one wave per listed row
template <typename T>
__global__ void __launch_bounds__(256)
tall_rowdot(const T *__restrict__ A, int64_t ld, int64_t n,
            const int32_t *__restrict__ J, const int64_t *__restrict__ cnt,
            const T *__restrict__ p, T *__restrict__ q, Ctrl *ctrl) {
  if (ctrl_done(ctrl) || ctrl->cg_done[1]) return;
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t a = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
  if (a >= *cnt) return;
  const T *row = A + (int64_t)J[a] * ld;
  T acc = (T)0;
  for (int64_t t = lane; t < n; t += WAVE) acc += row[t] * p[t];
  acc = wave_sum(acc);
  if (lane == 0) q[a] = acc;
}

// alpha = gam / ||q||^2; d += alpha p; res -= alpha q; then the input of the
// next transpose product: s = 0 (dense, accumulated into) or rhat[J_a] = res_a
template <typename T>
__global__ void __launch_bounds__(TL_NT)
tall_mid(int64_t n, const int32_t *__restrict__ J,
         const int64_t *__restrict__ cnt, const T *__restrict__ p,
         const T *__restrict__ q, T *__restrict__ d, T *__restrict__ res,
         T *__restrict__ s, T *__restrict__ rhat, Ctrl *ctrl) {
  if (ctrl_done(ctrl) || ctrl->cg_done[1]) return;
  __shared__ double sh[TL_NT / WAVE];
  const int64_t c = *cnt;
  double qq = 0.0;
  for (int64_t a = threadIdx.x; a < c; a += TL_NT)
    qq += (double)q[a] * (double)q[a];
  qq = block_sum<TL_NT>(qq, sh);
  const double gam = ctrl->cg_rz[1];
  if (!(qq > 0.0)) {
    if (threadIdx.x == 0) ctrl->cg_done[1] = 1;
    return;
  }
  const T alpha = (T)(gam / qq);
  for (int64_t i = threadIdx.x; i < n; i += TL_NT) {
    d[i] += alpha * p[i];
    if (!rhat) s[i] = (T)0;
  }
  for (int64_t a = threadIdx.x; a < c; a += TL_NT) {
    const T v = res[a] - alpha * q[a];
    res[a] = v;
    if (rhat) rhat[J[a]] = v;
  }
}

// gam' = ||s||^2; stop at gam' <= tol^2 gam_0; p = s + (gam'/gam) p
template <typename T>
__global__ void __launch_bounds__(TL_NT)
tall_end(int64_t n, const T *__restrict__ s, T *__restrict__ p, double tol,
         int max_steps, Ctrl *ctrl) {
  if (ctrl_done(ctrl) || ctrl->cg_done[1]) return;
  __shared__ double sh[TL_NT / WAVE];
  double g = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += TL_NT)
    g += (double)s[i] * (double)s[i];
  g = block_sum<TL_NT>(g, sh);
  const double gam = ctrl->cg_rz[1];
  const int steps = ctrl->cg_steps[1] + 1;
  const bool stop = g <= tol * tol * ctrl->cg_rz0[1] || steps >= max_steps ||
                    !(gam > 0.0);
  if (!stop) {
    const T beta = (T)(g / gam);
    for (int64_t i = threadIdx.x; i < n; i += TL_NT) p[i] = s[i] + beta * p[i];
  }
  __syncthreads();   // every thread has read gam before it is replaced
  if (threadIdx.x == 0) {
    ctrl->cg_rz[1] = g;
    ctrl->cg_steps[1] = steps;
    if (stop) ctrl->cg_done[1] = 1;
  }
}

// x += d
template <typename T>
__global__ void __launch_bounds__(256)
tall_finish(int64_t n, const T *__restrict__ d, T *__restrict__ x, Ctrl *ctrl) {
  if (ctrl_done(ctrl)) return;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256)
    x[i] += d[i];
}

static unsigned tall_grid(int64_t len) {
  int64_t g = (len + 255) / 256;
  if (g > 1024) g = 1024;
  return (unsigned)(g < 1 ? 1 : g);
}

template <typename T>
void launch_tall_rowproj_dense(const Dense<T> &A, const int32_t *J,
                               const int64_t *count_dev, int64_t cap,
                               const T *r, T *x, TallWork<T> &w, T *upd,
                               int max_steps, double tol, Ctrl *ctrl,
                               hipStream_t st) {
  const int64_t n = A.cols;
  hipLaunchKernelGGL(tall_init<T>, dim3(tall_grid(n)), dim3(256), 0, st, n,
                     (int64_t)0, w.d, w.s, (T *)nullptr, ctrl);
  hipLaunchKernelGGL(tall_load<T>, dim3(tall_grid(cap)), dim3(256), 0, st, J,
                     count_dev, r, w.res, (T *)nullptr, ctrl);
  thin_update<T>(A.a, A.ld, n, J, count_dev, cap, w.res, w.s, (T)1, upd, ctrl,
                 1, st);
  hipLaunchKernelGGL(tall_start<T>, dim3(1), dim3(TL_NT), 0, st, n,
                     (const T *)w.s, w.p, ctrl);
  const unsigned gq = (unsigned)((cap + 3) / 4);
  for (int k = 0; k < max_steps; ++k) {
    hipLaunchKernelGGL(tall_rowdot<T>, dim3(gq), dim3(256), 0, st, A.a, A.ld,
                       n, J, count_dev, (const T *)w.p, w.q, ctrl);
    hipLaunchKernelGGL(tall_mid<T>, dim3(1), dim3(TL_NT), 0, st, n, J,
                       count_dev, (const T *)w.p, (const T *)w.q, w.d, w.res,
                       w.s, (T *)nullptr, ctrl);
    thin_update<T>(A.a, A.ld, n, J, count_dev, cap, w.res, w.s, (T)1, upd,
                   ctrl, 1, st);
    hipLaunchKernelGGL(tall_end<T>, dim3(1), dim3(TL_NT), 0, st, n,
                       (const T *)w.s, w.p, tol, max_steps, ctrl);
  }
  hipLaunchKernelGGL(tall_finish<T>, dim3(tall_grid(n)), dim3(256), 0, st, n,
                     (const T *)w.d, x, ctrl);
}

template <typename T>
void launch_tall_rowproj_sparse(const Csr<T> &csr, const Csr<T> &csc,
                                const int32_t *J, const int64_t *count_dev,
                                int64_t cap, const T *r, T *x, TallWork<T> &w,
                                int max_steps, double tol, Ctrl *ctrl,
                                hipStream_t st) {
  const int64_t n = csr.cols, m = csr.rows;
  hipLaunchKernelGGL(tall_init<T>, dim3(tall_grid(std::max(n, m))), dim3(256),
                     0, st, n, m, w.d, w.s, w.rhat, ctrl);
  hipLaunchKernelGGL(tall_load<T>, dim3(tall_grid(cap)), dim3(256), 0, st, J,
                     count_dev, r, w.res, w.rhat, ctrl);
  SegArgs<T> tp;            // s = A^T rhat over the CSC
  tp.v = w.rhat;
  tp.out = w.s;
  launch_segdot<T>(csc, EPI_STORE, tp, ctrl, 1, st);
  hipLaunchKernelGGL(tall_start<T>, dim3(1), dim3(TL_NT), 0, st, n,
                     (const T *)w.s, w.p, ctrl);
  SegArgs<T> lp;            // q = A^J p over the listed CSR rows
  lp.v = w.p;
  lp.out = w.q;
  lp.list = J;
  lp.count_dev = count_dev;
  lp.list_cap = cap;
  for (int k = 0; k < max_steps; ++k) {
    launch_segdot<T>(csr, EPI_LIST_STORE, lp, ctrl, 1, st);
    hipLaunchKernelGGL(tall_mid<T>, dim3(1), dim3(TL_NT), 0, st, n, J,
                       count_dev, (const T *)w.p, (const T *)w.q, w.d, w.res,
                       w.s, w.rhat, ctrl);
    launch_segdot<T>(csc, EPI_STORE, tp, ctrl, 1, st);
    hipLaunchKernelGGL(tall_end<T>, dim3(1), dim3(TL_NT), 0, st, n,
                       (const T *)w.s, w.p, tol, max_steps, ctrl);
  }
  hipLaunchKernelGGL(tall_finish<T>, dim3(tall_grid(n)), dim3(256), 0, st, n,
                     (const T *)w.d, x, ctrl);
}

template void launch_tall_rowproj_dense<double>(const Dense<double> &, const int32_t *, const int64_t *, int64_t, const double *, double *, TallWork<double> &, double *, int, double, Ctrl *, hipStream_t);
template void launch_tall_rowproj_dense<float>(const Dense<float> &, const int32_t *, const int64_t *, int64_t, const float *, float *, TallWork<float> &, float *, int, double, Ctrl *, hipStream_t);
template void launch_tall_rowproj_sparse<double>(const Csr<double> &, const Csr<double> &, const int32_t *, const int64_t *, int64_t, const double *, double *, TallWork<double> &, int, double, Ctrl *, hipStream_t);
template void launch_tall_rowproj_sparse<float>(const Csr<float> &, const Csr<float> &, const int32_t *, const int64_t *, int64_t, const float *, float *, TallWork<float> &, int, double, Ctrl *, hipStream_t);

}  // namespace rg
