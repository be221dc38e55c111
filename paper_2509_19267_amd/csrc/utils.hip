// Set-up and elementwise kernels: storage conversion (row-major/column-major
// dense copies, CSR -> CSC), the squared row and column norms that
// normalise the residual weights (Section 2), finiteness checks, the
// pattern-restricted gradient, and small vector updates.
#include "common.h"
#include "kernels.h"

namespace rg {

template <typename Tout, typename Tin>
__global__ void convert_kernel(const Tin *__restrict__ in, Tout *__restrict__ out,
                               int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256)
    out[i] = (Tout)in[i];
}
static unsigned grid_for(int64_t n, int nt = 256, int64_t cap = 1 << 16) {
  int64_t g = (n + nt - 1) / nt;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (unsigned)g;
}
template <typename Tout, typename Tin>
void launch_convert(const Tin *in, Tout *out, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((convert_kernel<Tout, Tin>), dim3(grid_for(n)), dim3(256),
                     0, st, in, out, n);
}

// 32x32 tiles through LDS: coalesced reads of the input rows and coalesced
// writes of both the padded row-major copy and the transposed copy.
template <typename Tout, typename Tin>
__global__ void __launch_bounds__(256)
pack_dense_kernel(const Tin *__restrict__ in, int64_t rows, int64_t cols,
                  int64_t ld_in, Tout *__restrict__ orm, int64_t ldo,
                  Tout *__restrict__ ocm, int64_t ldt) {
  __shared__ Tout t[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int64_t r = r0 + k, c = c0 + tx;
    Tout v = (r < rows && c < cols) ? (Tout)in[r * ld_in + c] : (Tout)0;
    t[k][tx] = v;
    if (orm && r < rows && c < ldo) orm[r * ldo + c] = v;
  }
  __syncthreads();
  if (!ocm) return;
  for (int k = ty; k < 32; k += 8) {
    const int64_t c = c0 + k, r = r0 + tx;
    if (c < cols && r < ldt) ocm[c * ldt + r] = t[tx][k];
  }
}
template <typename Tout, typename Tin>
void launch_pack_dense(const Tin *in, int64_t rows, int64_t cols,
                       int64_t ld_in, Tout *out_rm, int64_t ld_out,
                       Tout *out_cm, int64_t ld_t, hipStream_t st) {
  // cover the padded extents so pads are written as zeros
  const int64_t gr = ((ld_t > rows ? ld_t : rows) + 31) / 32;
  const int64_t gc = ((ld_out > cols ? ld_out : cols) + 31) / 32;
  hipLaunchKernelGGL((pack_dense_kernel<Tout, Tin>), dim3((unsigned)gc, (unsigned)gr),
                     dim3(256), 0, st, in, rows, cols, ld_in, out_rm, ld_out,
                     out_cm, ld_t);
}

// one wave per row of a row-major matrix: out[i] = sum_j M[i][j]^2 (FP64)
template <typename T>
__global__ void __launch_bounds__(256)
rownorm2_kernel(const T *__restrict__ M, int64_t rows, int64_t len, int64_t ld,
                double *__restrict__ out) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
  if (i >= rows) return;
  double s = 0.0;
  for (int64_t j = lane; j < len; j += WAVE) {
    const double v = (double)M[i * ld + j];
    s += v * v;
  }
  s = wave_sum(s);
  if (lane == 0) out[i] = s;
}
template <typename T>
void launch_sqnorms_dense(const T *Arm, int64_t rows, int64_t cols, int64_t ld,
                          const T *Acm, int64_t ldc, double *rho,
                          double *kappa, hipStream_t st) {
  hipLaunchKernelGGL(rownorm2_kernel<T>, dim3((unsigned)((rows + 3) / 4)),
                     dim3(256), 0, st, Arm, rows, cols, ld, rho);
  hipLaunchKernelGGL(rownorm2_kernel<T>, dim3((unsigned)((cols + 3) / 4)),
                     dim3(256), 0, st, Acm, cols, rows, ldc, kappa);
}

template <typename T>
__global__ void __launch_bounds__(256)
segnorm2_kernel(Csr<T> A, double *__restrict__ out) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t s = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
  if (s >= A.rows) return;
  double acc = 0.0;
  for (int64_t e = A.ptr[s] + lane; e < A.ptr[s + 1]; e += WAVE) {
    const double v = (double)A.val[e];
    acc += v * v;
  }
  acc = wave_sum(acc);
  if (lane == 0) out[s] = acc;
}
template <typename T>
void launch_sqnorms_csr(const Csr<T> &A, double *out, hipStream_t st) {
  hipLaunchKernelGGL(segnorm2_kernel<T>, dim3((unsigned)((A.rows + 3) / 4)),
                     dim3(256), 0, st, A, out);
}

template <typename T>
__global__ void check_finite_kernel(const T *__restrict__ v, int64_t n,
                                    int *flag) {
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    const double x = (double)v[i];
    if (!(x == x) || x > 1.7976931348623157e308 || x < -1.7976931348623157e308) bad = 1;
  }
  if (__any(bad) && (threadIdx.x & (WAVE - 1)) == 0) atomicOr(flag, 1);
}
template <typename T>
void launch_check_finite(const T *v, int64_t n, int *flag, hipStream_t st) {
  hipLaunchKernelGGL(check_finite_kernel<T>, dim3(grid_for(n, 256, 4096)),
                     dim3(256), 0, st, v, n, flag);
}

// ------------------------------------------------------------ CSR -> CSC
__global__ void col_count_kernel(int64_t nnz, const int32_t *__restrict__ ci,
                                 int64_t *__restrict__ cnt) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * 256)
    atomicAdd((unsigned long long *)&cnt[ci[e]], 1ull);
}
// exclusive scan of cnt[0..n) into ptr[0..n], one workgroup
__global__ void __launch_bounds__(1024)
scan_kernel(int64_t n, const int64_t *__restrict__ cnt, int64_t *__restrict__ ptr) {
  __shared__ int64_t sh[1024];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < n; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const int64_t v = i < n ? cnt[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int64_t add = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
      __syncthreads();
      sh[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < n) ptr[i] = carry + sh[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += sh[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) ptr[n] = carry;
}
// one wave per row: place entries with an atomic cursor per column
template <typename T>
__global__ void __launch_bounds__(256)
csc_fill_kernel(int64_t m, const int64_t *__restrict__ rp,
                const int32_t *__restrict__ ci, const T *__restrict__ v,
                int64_t *__restrict__ cursor, int32_t *__restrict__ ri,
                T *__restrict__ cv) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
  if (i >= m) return;
  for (int64_t e = rp[i] + lane; e < rp[i + 1]; e += WAVE) {
    const int32_t j = ci[e];
    const unsigned long long pos =
        atomicAdd((unsigned long long *)&cursor[j], 1ull);
    ri[pos] = (int32_t)i;
    cv[pos] = v[e];
  }
}
// sort each column segment by row (shell sort; the placement order above
// depends on scheduling, the sorted result does not)
template <typename T>
__global__ void __launch_bounds__(256)
csc_sort_kernel(int64_t n, const int64_t *__restrict__ cp,
                int32_t *__restrict__ ri, T *__restrict__ cv) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  const int64_t b = cp[j], len = cp[j + 1] - cp[j];
  int64_t gap = 1;
  while (gap < len / 3) gap = 3 * gap + 1;
  for (; gap >= 1; gap /= 3) {
    for (int64_t i = gap; i < len; ++i) {
      const int32_t kr = ri[b + i];
      const T kv = cv[b + i];
      int64_t k = i;
      while (k >= gap && ri[b + k - gap] > kr) {
        ri[b + k] = ri[b + k - gap];
        cv[b + k] = cv[b + k - gap];
        k -= gap;
      }
      ri[b + k] = kr;
      cv[b + k] = kv;
    }
  }
}
template <typename T>
void launch_csr_to_csc(int64_t m, int64_t n, int64_t nnz, const int64_t *rp,
                       const int32_t *ci, const T *v, int64_t *cp, int32_t *ri,
                       T *cv, int64_t *work, hipStream_t st) {
  hipMemsetAsync(work, 0, sizeof(int64_t) * (size_t)n, st);
  if (nnz > 0)
    hipLaunchKernelGGL(col_count_kernel, dim3(grid_for(nnz, 256, 8192)),
                       dim3(256), 0, st, nnz, ci, work);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, n, work, cp);
  hipMemcpyAsync(work, cp, sizeof(int64_t) * (size_t)n,
                 hipMemcpyDeviceToDevice, st);
  if (m > 0)
    hipLaunchKernelGGL(csc_fill_kernel<T>, dim3((unsigned)((m + 3) / 4)),
                       dim3(256), 0, st, m, rp, ci, v, work, ri, cv);
  if (n > 0)
    hipLaunchKernelGGL(csc_sort_kernel<T>, dim3((unsigned)((n + 255) / 256)),
                       dim3(256), 0, st, n, cp, ri, cv);
}

// ------------------------------------------------------------ gradient
__global__ void __launch_bounds__(256)
grad_csr_kernel(int64_t m, int64_t n, int64_t rep,
                const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                const double *__restrict__ r, const double *__restrict__ lam,
                const double *__restrict__ w, const double *__restrict__ x,
                double *__restrict__ dA) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
  if (i >= m) return;
  for (int64_t e = rp[i] + lane; e < rp[i + 1]; e += WAVE) {
    const int64_t j = ci[e];
    double acc = 0.0;
    for (int64_t s = 0; s < rep; ++s) {
      const int64_t gi = s * m + i, gj = s * n + j;
      acc += (lam ? r[gi] * lam[gj] : 0.0) - w[gi] * x[gj];
    }
    dA[e] = acc;
  }
}
void launch_grad_pattern_csr(int64_t m, int64_t n, int64_t rep,
                             const int64_t *rp, const int32_t *ci,
                             const double *r, const double *lam,
                             const double *w, const double *x, double *dA,
                             hipStream_t st) {
  hipLaunchKernelGGL(grad_csr_kernel, dim3((unsigned)((m + 3) / 4)), dim3(256),
                     0, st, m, n, rep, rp, ci, r, lam, w, x, dA);
}
__global__ void replicate_kernel(const double *__restrict__ in, int64_t len,
                                 int64_t rep, double *__restrict__ out) {
  const int64_t tot = len * rep;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < tot;
       t += (int64_t)gridDim.x * 256)
    out[t] = in[t % len];
}
void launch_replicate(const double *in, int64_t len, int64_t rep, double *out,
                      hipStream_t st) {
  hipLaunchKernelGGL(replicate_kernel, dim3(grid_for(len * rep, 256, 8192)),
                     dim3(256), 0, st, in, len, rep, out);
}
__global__ void __launch_bounds__(256)
grad_dense_kernel(int64_t m, int64_t n, const double *__restrict__ r,
                  const double *__restrict__ lam, const double *__restrict__ w,
                  const double *__restrict__ x, double *__restrict__ dA) {
  const int64_t tot = m * n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / n, j = e - i * n;
    dA[e] = (lam ? r[i] * lam[j] : 0.0) - w[i] * x[j];
  }
}
void launch_grad_pattern_dense(int64_t m, int64_t n, const double *r,
                               const double *lam, const double *w,
                               const double *x, double *dA, hipStream_t st) {
  hipLaunchKernelGGL(grad_dense_kernel, dim3(grid_for(m * n, 256, 16384)),
                     dim3(256), 0, st, m, n, r, lam, w, x, dA);
}

template <typename Ty, typename Tx>
__global__ void axpby_kernel(int64_t n, double alpha, Ty *__restrict__ y,
                             double beta, const Tx *__restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    const double xv = x ? (double)x[i] : 0.0;
    // alpha == 0 overwrites y without reading it (y may hold anything)
    const double yv = alpha != 0.0 ? alpha * (double)y[i] : 0.0;
    y[i] = (Ty)(yv + beta * xv);
  }
}
template <typename Ty, typename Tx>
void launch_axpby(int64_t n, double alpha, Ty *y, double beta, const Tx *x,
                  hipStream_t st) {
  hipLaunchKernelGGL((axpby_kernel<Ty, Tx>), dim3(grid_for(n, 256, 8192)),
                     dim3(256), 0, st, n, alpha, y, beta, x);
}

#define RG_UT(T)                                                             \
  template void launch_sqnorms_dense<T>(const T *, int64_t, int64_t, int64_t, \
                                        const T *, int64_t, double *,        \
                                        double *, hipStream_t);              \
  template void launch_sqnorms_csr<T>(const Csr<T> &, double *, hipStream_t); \
  template void launch_check_finite<T>(const T *, int64_t, int *,           \
                                       hipStream_t);                         \
  template void launch_csr_to_csc<T>(int64_t, int64_t, int64_t,             \
                                     const int64_t *, const int32_t *,      \
                                     const T *, int64_t *, int32_t *, T *,  \
                                     int64_t *, hipStream_t);
RG_UT(double)
RG_UT(float)
#undef RG_UT
template void launch_convert<float, double>(const double *, float *, int64_t, hipStream_t);
template void launch_convert<double, float>(const float *, double *, int64_t, hipStream_t);
template void launch_convert<double, double>(const double *, double *, int64_t, hipStream_t);
template void launch_convert<float, float>(const float *, float *, int64_t, hipStream_t);
template void launch_pack_dense<double, double>(const double *, int64_t, int64_t, int64_t, double *, int64_t, double *, int64_t, hipStream_t);
template void launch_pack_dense<float, double>(const double *, int64_t, int64_t, int64_t, float *, int64_t, float *, int64_t, hipStream_t);
template void launch_pack_dense<double, float>(const float *, int64_t, int64_t, int64_t, double *, int64_t, double *, int64_t, hipStream_t);
template void launch_pack_dense<float, float>(const float *, int64_t, int64_t, int64_t, float *, int64_t, float *, int64_t, hipStream_t);
template void launch_axpby<double, double>(int64_t, double, double *, double, const double *, hipStream_t);
template void launch_axpby<double, float>(int64_t, double, double *, double, const float *, hipStream_t);
template void launch_axpby<float, double>(int64_t, double, float *, double, const double *, hipStream_t);
template void launch_axpby<float, float>(int64_t, double, float *, double, const float *, hipStream_t);

}  // namespace rg
