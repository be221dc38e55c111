// Residual passes of RGDBEK on gfx950: the column residual A^T z and the row
// residual b - z - A x with their weights (Section 2, the two residual
// definitions of the randomized selection; Algorithm 1), plus the stop tests.
//
// Sparse A: row-split segment dots over CSR (rows) and CSC (columns, i.e.
// the CSR of A^T), G lanes per segment (G from the mean segment length),
// segments longer than a limit handed to a one-workgroup-per-segment kernel,
// so power-law rows do not stall a wave.  Deterministic: fixed-order shuffle
// reductions, no floating-point atomics.
// Dense A: one read of the row-major matrix gives both A x_k and A^T z_k
// (the row phase needs A x_k, not A x_{k+1}, so both products of an
// iteration can share the pass); 16-byte loads, each wave streams whole row
// segments, column partials meet in LDS, row-block partials are summed in a
// fixed order by the finalise kernel.
#include "common.h"
#include "kernels.h"

namespace rg {

constexpr int SEG_NT = 256;

template <typename T>
__device__ __forceinline__ void seg_epilogue(int epi, const SegArgs<T> &a,
                                             int64_t s, int64_t slot, T acc,
                                             double &pb, double &pr) {
  if (epi == EPI_STORE) {
    a.out[s] = acc;
  } else if (epi == EPI_LIST_STORE) {
    a.out[slot] = acc;
  } else if (epi == EPI_COLRES) {
    T g = acc;
    if (a.off) g += a.off[s];
    a.g[s] = g;
    const double nr = a.nrm[s];
    a.eps[s] = nr > 0.0 ? (T)((double)g * (double)g / nr) : (T)0;
  } else {  // EPI_ROWRES
    const T bb = a.b[s];
    const T r = bb - a.z[s] - acc;
    a.r[s] = r;
    const double nr = a.nrm[s];
    a.eps[s] = nr > 0.0 ? (T)((double)r * (double)r / nr) : (T)0;
    const double bq = (double)bb - (double)acc;
    pb += bq * bq;
    pr += (double)r * (double)r;
  }
}

template <typename T, int G, int EPI>
__global__ void __launch_bounds__(SEG_NT)
segdot_kernel(Csr<T> A, SegArgs<T> a, Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  constexpr int SPB = SEG_NT / G;
  const int lg = threadIdx.x & (G - 1);
  const int64_t slot = (int64_t)blockIdx.x * SPB + threadIdx.x / G;
  const bool listed = (a.list != nullptr);
  const int64_t nseg = listed ? *a.count_dev : A.rows;
  bool active = slot < nseg;
  int64_t s = 0, br = 0, co = 0;
  T acc = (T)0;
  if (active) {
    if (listed) {
      s = (int64_t)a.list[slot];
      gsplit(A, s, br, co);
    } else {
      vrow(A, slot, s, br, co);
    }
    const int64_t e0 = A.ptr[br], e1 = A.ptr[br + 1];
    if (!listed && A.long_limit > 0 && e1 - e0 > A.long_limit) {
      active = false;   // handled by segdot_long
    } else {
      const T *v = a.v + co;
      for (int64_t e = e0 + lg; e < e1; e += G)
        acc += A.val[e] * v[A.idx[e]];
    }
  }
  acc = group_sum<G>(acc);
  double pb = 0.0, pr = 0.0;
  if (active && lg == 0) seg_epilogue<T>(EPI, a, s, slot, acc, pb, pr);
  if (EPI == EPI_ROWRES) {
    __shared__ double sh[SEG_NT / WAVE];
    pb = block_sum<SEG_NT>(pb, sh);
    pr = block_sum<SEG_NT>(pr, sh);
    if (threadIdx.x == 0) {
      a.part[2 * blockIdx.x] = pb;
      a.part[2 * blockIdx.x + 1] = pr;
    }
  }
}

// one workgroup per long segment (from A.longs)
template <typename T, int EPI>
__global__ void __launch_bounds__(SEG_NT)
segdot_long(Csr<T> A, SegArgs<T> a, int64_t part_base, Ctrl *ctrl,
            int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  __shared__ double sh[SEG_NT / WAVE];
  const int64_t li = blockIdx.x / A.rep, rs = blockIdx.x - li * A.rep;
  const int64_t br = A.longs[li];
  const int64_t s = rs * A.brows + br;
  const T *v = a.v + rs * A.bcols;
  const int64_t e0 = A.ptr[br], e1 = A.ptr[br + 1];
  T acc = (T)0;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += SEG_NT)
    acc += A.val[e] * v[A.idx[e]];
  const double tot = block_sum<SEG_NT>((double)acc, sh);
  double pb = 0.0, pr = 0.0;
  if (threadIdx.x == 0) seg_epilogue<T>(EPI, a, s, s, (T)tot, pb, pr);
  if (EPI == EPI_ROWRES && threadIdx.x == 0) {
    a.part[2 * (part_base + blockIdx.x)] = pb;
    a.part[2 * (part_base + blockIdx.x) + 1] = pr;
  }
}

// ------------------------------------------------------------ merge pass
// Full passes (rep == 1) balanced by nonzeros, not by rows, so power-law row
// lengths cost nothing extra: each wave streams one chunk of MP_CH nonzeros
// (MP_K consecutive per lane: 16-byte index loads, coalesced value loads),
// stages the products in LDS, and finishes the rows the chunk owns (those
// whose first nonzero lies in it; empty rows included).  A row running past
// its chunk leaves a head partial; every chunk leaves the lead partial of the
// row entering it; mp_cross sums head + leads in chunk order for the listed
// spanning rows.  Fixed summation order: deterministic.
constexpr int MP_NT = 256;
constexpr int MP_K = (int)(MP_CH / WAVE);
constexpr int MP_WPB = MP_NT / WAVE;

template <typename T>
__device__ __forceinline__ void mp_finish(int epi, const SegArgs<T> &a,
                                          int64_t r, T acc, double &pb,
                                          double &pr) {
  seg_epilogue<T>(epi, a, r, r, acc, pb, pr);
}

template <typename T, int EPI>
__global__ void __launch_bounds__(MP_NT)
mp_chunks(Csr<T> A, SegArgs<T> a, Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  __shared__ T sp[MP_WPB][MP_CH];
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  const int64_t c = (int64_t)blockIdx.x * MP_WPB + wv;
  double pb = 0.0, pr = 0.0;
  if (c < A.mp_nchunk) {
    const int64_t e0 = c * MP_CH;
    const int64_t eh = A.nnz < e0 + MP_CH ? A.nnz : e0 + MP_CH;   // data end
    // products of this lane's MP_K consecutive nonzeros
    const int64_t eb = e0 + (int64_t)lane * MP_K;
    T pv[MP_K];
    if (eh == e0 + MP_CH) {
      // full chunk: one 16-byte index load and MP_K*sizeof(T) value bytes
      typedef int32_t i4 __attribute__((ext_vector_type(MP_K)));
      typedef T tv __attribute__((ext_vector_type(MP_K)));
      const i4 ix = *reinterpret_cast<const i4 *>(A.idx + eb);
      const tv vv = *reinterpret_cast<const tv *>(A.val + eb);
#pragma unroll
      for (int j = 0; j < MP_K; ++j) pv[j] = vv[j] * a.v[ix[j]];
    } else {
#pragma unroll
      for (int j = 0; j < MP_K; ++j) {
        const int64_t e = eb + j;
        pv[j] = (T)0;
        if (e < eh) pv[j] = A.val[e] * a.v[A.idx[e]];
      }
    }
#pragma unroll
    for (int j = 0; j < MP_K; ++j) sp[wv][lane * MP_K + j] = pv[j];
    // lead partial: the row that began before e0 and continues here
    const int64_t rs = A.mp_rs[c], re = A.mp_rs[c + 1];
    T lead = (T)0;
    if (c > 0 && rs > 0) {
      const int64_t pe = A.ptr[rs] - e0;     // where the entering row stops
      const int64_t lim = pe < MP_CH ? pe : MP_CH;
#pragma unroll
      for (int j = 0; j < MP_K; ++j)
        if (lane * MP_K + j < lim) lead += pv[j];
    }
    lead = wave_sum(lead);
    if (lane == 0) A.mp_lead[c] = lead;
    // the products of the whole wave are read back below: order the LDS
    // stores before the loads (one wave, so a wave-scope fence suffices)
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // owned rows: lane-strided, each summed in element order from LDS
    for (int64_t r = rs + lane; r < re; r += WAVE) {
      const int64_t s0 = A.ptr[r] - e0, t0 = A.ptr[r + 1] - e0;
      const int64_t t = t0 < MP_CH ? t0 : MP_CH;
      T acc = (T)0;
      for (int64_t q = s0; q < t; ++q) acc += sp[wv][q];
      if (t0 > MP_CH) {
        A.mp_head[c] = acc;                  // finished by mp_cross
      } else {
        mp_finish<T>(EPI, a, r, acc, pb, pr);
      }
    }
  }
  if (EPI == EPI_ROWRES) {
    __shared__ double sh[MP_NT / WAVE];
    pb = block_sum<MP_NT>(pb, sh);
    pr = block_sum<MP_NT>(pr, sh);
    if (threadIdx.x == 0) {
      a.part[2 * blockIdx.x] = pb;
      a.part[2 * blockIdx.x + 1] = pr;
    }
  }
}

template <typename T, int EPI>
__global__ void __launch_bounds__(MP_NT)
mp_cross(Csr<T> A, SegArgs<T> a, int64_t part_base, Ctrl *ctrl,
         int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  const int64_t x = (int64_t)blockIdx.x * MP_NT + threadIdx.x;
  double pb = 0.0, pr = 0.0;
  if (x < A.mp_ncross) {
    const int64_t r = A.mp_xrow[x];
    const int64_t cs = A.mp_xcs[x], ce = A.mp_xce[x];
    T acc = A.mp_head[cs];
    for (int64_t c = cs + 1; c <= ce; ++c) acc += A.mp_lead[c];
    mp_finish<T>(EPI, a, r, acc, pb, pr);
  }
  if (EPI == EPI_ROWRES) {
    __shared__ double sh[MP_NT / WAVE];
    pb = block_sum<MP_NT>(pb, sh);
    pr = block_sum<MP_NT>(pr, sh);
    if (threadIdx.x == 0) {
      a.part[2 * (part_base + blockIdx.x)] = pb;
      a.part[2 * (part_base + blockIdx.x) + 1] = pr;
    }
  }
}

template <typename T, int EPI>
static int merge_dispatch(const Csr<T> &A, const SegArgs<T> &a, Ctrl *ctrl,
                          int respect_done, hipStream_t st) {
  const int nb = (int)((A.mp_nchunk + MP_WPB - 1) / MP_WPB);
  hipLaunchKernelGGL((mp_chunks<T, EPI>), dim3(nb), dim3(MP_NT), 0, st, A, a,
                     ctrl, respect_done);
  int nparts = nb;
  if (A.mp_ncross > 0) {
    const int nx = (int)((A.mp_ncross + MP_NT - 1) / MP_NT);
    hipLaunchKernelGGL((mp_cross<T, EPI>), dim3(nx), dim3(MP_NT), 0, st, A, a,
                       (int64_t)nb, ctrl, respect_done);
    nparts += nx;
  }
  return nparts;
}

int64_t segdot_max_parts(int64_t rows, int64_t nnz, int64_t nchunk,
                         int64_t ncross, int64_t nlong, int64_t rep) {
  (void)nnz;
  const int64_t seg = rows * rep + nlong * rep + 1024;   // G >= 1 lanes
  const int64_t mer = (nchunk + MP_WPB - 1) / MP_WPB +
                      (ncross + MP_NT - 1) / MP_NT + 16;
  return seg > mer ? seg : mer;
}

// Full passes of many right-hand sides (A.rep >= REP_MM_MIN): the vector
// is interleaved, the product formed for all right-hand sides at once
// (launch_rep_mm), and this epilogue turns the interleaved result back to
// right-hand-side-major order through a 64 x 64 LDS tile while it applies
// the pass's epilogue to every (right-hand side, stored row).  Partials: one
// pair per workgroup.
template <typename T, int EPI>
__global__ void __launch_bounds__(SEG_NT)
rep_epi_kernel(Csr<T> A, SegArgs<T> a, const T *__restrict__ prod, Ctrl *ctrl,
               int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  __shared__ T tile[WAVE][WAVE + 1];
  __shared__ double sh[SEG_NT / WAVE];
  const int64_t R = A.rep, len = A.brows;
  const int64_t i0 = (int64_t)blockIdx.x * WAVE, s0 = (int64_t)blockIdx.y * WAVE;
  const int tx = threadIdx.x & (WAVE - 1), ty = threadIdx.x / WAVE;
  for (int r = ty; r < WAVE; r += SEG_NT / WAVE) {
    const int64_t i = i0 + r, s = s0 + tx;
    tile[r][tx] = (i < len && s < R) ? prod[i * R + s] : (T)0;
  }
  __syncthreads();
  double pb = 0.0, pr = 0.0;
  for (int r = ty; r < WAVE; r += SEG_NT / WAVE) {
    const int64_t s = s0 + r, i = i0 + tx;
    if (s < R && i < len) {
      const int64_t g = s * len + i;
      seg_epilogue<T>(EPI, a, g, g, tile[tx][r], pb, pr);
    }
  }
  if (EPI == EPI_ROWRES) {
    pb = block_sum<SEG_NT>(pb, sh);
    pr = block_sum<SEG_NT>(pr, sh);
    if (threadIdx.x == 0) {
      const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
      a.part[2 * b] = pb;
      a.part[2 * b + 1] = pr;
    }
  }
}

template <typename T, int EPI>
static int rep_dispatch(const Csr<T> &A, const SegArgs<T> &a, Ctrl *ctrl,
                        int respect_done, hipStream_t st) {
  launch_rep_tin<T>(a.v, A.rep_in, A.bcols, A.rep, ctrl, -1, respect_done, st);
  launch_rep_mm<T>(A, A.rep_in, A.rep_out, nullptr, ctrl, -1, respect_done, st);
  const int64_t gx = (A.brows + WAVE - 1) / WAVE, gy = (A.rep + WAVE - 1) / WAVE;
  if (gx <= 0 || gy <= 0) return 0;
  hipLaunchKernelGGL((rep_epi_kernel<T, EPI>), dim3((unsigned)gx, (unsigned)gy),
                     dim3(SEG_NT), 0, st, A, a, (const T *)A.rep_out, ctrl,
                     respect_done);
  return (int)(gx * gy);
}

template <typename T, int EPI>
static int segdot_dispatch(const Csr<T> &A, const SegArgs<T> &a, Ctrl *ctrl,
                           int respect_done, hipStream_t st) {
  if (!a.list && A.rep >= REP_MM_MIN && A.rep_in && EPI != EPI_LIST_STORE)
    return rep_dispatch<T, EPI>(A, a, ctrl, respect_done, st);
  if (!a.list && A.rep == 1 && A.mp_rs &&
      (EPI == EPI_STORE || EPI == EPI_COLRES || EPI == EPI_ROWRES))
    return merge_dispatch<T, EPI>(A, a, ctrl, respect_done, st);
  const int64_t nseg = a.list ? a.list_cap : A.rows;
  const int G = A.group;
  const int spb = SEG_NT / G;
  const int nb = (int)((nseg + spb - 1) / spb);
  int nparts = 0;
  if (nb > 0) {
    switch (G) {
#define RG_SEG(GG)                                                          \
  case GG:                                                                  \
    hipLaunchKernelGGL((segdot_kernel<T, GG, EPI>), dim3(nb), dim3(SEG_NT), \
                       0, st, A, a, ctrl, respect_done);                    \
    break;
      RG_SEG(1) RG_SEG(2) RG_SEG(4) RG_SEG(8) RG_SEG(16) RG_SEG(32) RG_SEG(64)
#undef RG_SEG
      default: break;
    }
    nparts = nb;
  }
  if (!a.list && A.nlong > 0) {
    hipLaunchKernelGGL((segdot_long<T, EPI>), dim3((unsigned)(A.nlong * A.rep)),
                       dim3(SEG_NT), 0, st, A, a, (int64_t)nparts, ctrl,
                       respect_done);
    nparts += (int)(A.nlong * A.rep);
  }
  return nparts;
}

template <typename T>
int launch_segdot(const Csr<T> &A, int epi, const SegArgs<T> &a, Ctrl *ctrl,
                  int respect_done, hipStream_t st) {
  switch (epi) {
    case EPI_STORE:
      return segdot_dispatch<T, EPI_STORE>(A, a, ctrl, respect_done, st);
    case EPI_COLRES:
      return segdot_dispatch<T, EPI_COLRES>(A, a, ctrl, respect_done, st);
    case EPI_ROWRES:
      return segdot_dispatch<T, EPI_ROWRES>(A, a, ctrl, respect_done, st);
    default:
      return segdot_dispatch<T, EPI_LIST_STORE>(A, a, ctrl, respect_done, st);
  }
}
template int launch_segdot<double>(const Csr<double> &, int,
                                   const SegArgs<double> &, Ctrl *, int,
                                   hipStream_t);
template int launch_segdot<float>(const Csr<float> &, int,
                                  const SegArgs<float> &, Ctrl *, int,
                                  hipStream_t);

// ------------------------------------------------------------ dense pass
typedef double df_d2 __attribute__((ext_vector_type(2)));
typedef float df_f4 __attribute__((ext_vector_type(4)));
template <typename T> struct Vec;
template <> struct Vec<double> { using type = df_d2; static constexpr int n = 2; };
template <> struct Vec<float> { using type = df_f4; static constexpr int n = 4; };

constexpr int DF_NT = 256;     // 4 waves
// 16-byte loads per lane per row (NL) and rows in flight per wave (RG)
template <typename T> struct DfShape;
template <> struct DfShape<double> { static constexpr int NL = 4, RG = 4; };
template <> struct DfShape<float> { static constexpr int NL = 4, RG = 4; };
// rows per workgroup sweep
template <typename T>
constexpr int df_rstep() { return (DF_NT / WAVE) * DfShape<T>::RG; }

template <typename T>
constexpr int df_cb() { return WAVE * Vec<T>::n * DfShape<T>::NL; }

// Work split of the fused pass: column chunks of df_cb() columns (one per
// grid column) times row tiles of `rpw` rows (one per grid row).  With
// tile_rows = 0 the tile height is chosen so that the grid holds about
// `target_wgs` workgroups of equal size (one full round on the device),
// which keeps the last round from running half empty.
template <typename T>
void dense_work_shape(const Dense<T> &A, int tile_rows, int target_wgs,
                      int *nch, int *nrg, int *rpw) {
  const int64_t cb = df_cb<T>();
  *nch = (int)((A.ld + cb - 1) / cb);
  int64_t r;
  if (tile_rows > 0) {
    r = tile_rows;
  } else {
    int64_t want = target_wgs / *nch;
    if (want < 1) want = 1;
    r = (A.rows + want - 1) / want;
  }
  constexpr int64_t RS = df_rstep<T>();
  r = (r + RS - 1) / RS * RS;
  if (r < RS) r = RS;
  *rpw = (int)r;
  *nrg = (int)((A.rows + r - 1) / r);
  if (*nrg < 1) *nrg = 1;
}
template void dense_work_shape<double>(const Dense<double> &, int, int, int *,
                                       int *, int *);
template void dense_work_shape<float>(const Dense<float> &, int, int, int *,
                                      int *, int *);

template <typename T>
__device__ __forceinline__ T vget(const typename Vec<T>::type &v, int i) {
  return v[i];
}

// One workgroup: columns [c0, c0 + df_cb()) of rows [r0, r0 + rpw).  Each
// wave streams DF_RG rows at a time with DF_NL 16-byte loads per lane per
// row; q_i partials are wave sums (one per row and column chunk), g_j
// partials stay in registers over the whole tile and are summed over the
// four waves in LDS (one per column and row tile).
template <typename T>
__global__ void __launch_bounds__(DF_NT)
dense_fused_kernel(Dense<T> A, int rpw, const T *__restrict__ x,
                   const T *__restrict__ z, T *__restrict__ qpart,
                   T *__restrict__ gpart, Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  using V = typename Vec<T>::type;
  constexpr int VN = Vec<T>::n;
  constexpr int CB = df_cb<T>();
  constexpr int DF_NL = DfShape<T>::NL, DF_RG = DfShape<T>::RG;
  constexpr int DF_RSTEP = df_rstep<T>();
  __shared__ T sg[DF_NT / WAVE][CB];
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  const int64_t c0 = (int64_t)blockIdx.x * CB;
  const int64_t r0 = (int64_t)blockIdx.y * rpw;
  const int64_t ld = A.ld;
  T xs[DF_NL][VN], ga[DF_NL][VN];
  bool cok[DF_NL];
#pragma unroll
  for (int t = 0; t < DF_NL; ++t) {
    const int64_t c = c0 + (int64_t)(t * WAVE + lane) * VN;
    cok[t] = c < ld;
#pragma unroll
    for (int v = 0; v < VN; ++v) {
      xs[t][v] = cok[t] ? x[c + v] : (T)0;
      ga[t][v] = (T)0;
    }
  }
  for (int rr = wv * DF_RG; rr < rpw; rr += DF_RSTEP) {
    V av[DF_RG][DF_NL];
    T zr[DF_RG];
#pragma unroll
    for (int u = 0; u < DF_RG; ++u) {
      const int64_t i = r0 + rr + u;
      const bool rok = i < A.rows;
      zr[u] = rok ? z[i] : (T)0;
      const V *row = reinterpret_cast<const V *>(A.a + (rok ? i : 0) * ld + c0);
#pragma unroll
      for (int t = 0; t < DF_NL; ++t) {
        if (rok && cok[t]) av[u][t] = __builtin_nontemporal_load(&row[t * WAVE + lane]);
        else av[u][t] = V{};
      }
    }
#pragma unroll
    for (int u = 0; u < DF_RG; ++u) {
      T qa = (T)0;
#pragma unroll
      for (int t = 0; t < DF_NL; ++t)
#pragma unroll
        for (int v = 0; v < VN; ++v) {
          const T a = vget<T>(av[u][t], v);
          qa += a * xs[t][v];
          ga[t][v] += zr[u] * a;
        }
      qa = wave_sum(qa);
      const int64_t i = r0 + rr + u;
      if (lane == 0 && i < A.rows) qpart[(int64_t)blockIdx.x * A.rows + i] = qa;
    }
  }
#pragma unroll
  for (int t = 0; t < DF_NL; ++t)
#pragma unroll
    for (int v = 0; v < VN; ++v) sg[wv][(t * WAVE + lane) * VN + v] = ga[t][v];
  __syncthreads();
  for (int c = threadIdx.x; c < CB; c += DF_NT) {
    const int64_t col = c0 + c;
    if (col < ld) {
      T s = (T)0;
#pragma unroll
      for (int w = 0; w < DF_NT / WAVE; ++w) s += sg[w][c];
      gpart[(int64_t)blockIdx.y * ld + col] = s;
    }
  }
}

// Sums the partials in a fixed order.  The first ceil(cols/64) workgroups
// handle 64 columns each, the four waves taking every fourth row tile and
// meeting in LDS; the rest handle 256 rows each.
template <typename T>
__global__ void __launch_bounds__(256)
dense_finalize(int64_t rows, int64_t cols, int64_t ld, int nch, int nrg,
               int ncb, const T *__restrict__ qpart,
               const T *__restrict__ gpart, const T *__restrict__ off,
               const double *__restrict__ kappa, T *__restrict__ g,
               T *__restrict__ eps, T *__restrict__ q, Ctrl *ctrl,
               int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  if ((int)blockIdx.x < ncb) {
    __shared__ T sh[4][WAVE];
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const int64_t t = (int64_t)blockIdx.x * WAVE + lane;
    T s0 = (T)0, s1 = (T)0;
    if (t < cols) {
      // s0 takes tiles wv, wv + 8, ... and s1 tiles wv + 4, wv + 12, ...;
      // four of those steps load together (eight loads in flight), the
      // additions keep their order
      int b = wv;
      for (; b + 28 < nrg; b += 32) {
        T v0[4], v1[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          v0[j] = gpart[(int64_t)(b + 8 * j) * ld + t];
          v1[j] = gpart[(int64_t)(b + 8 * j + 4) * ld + t];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          s0 += v0[j];
          s1 += v1[j];
        }
      }
      for (; b + 4 < nrg; b += 8) {
        s0 += gpart[(int64_t)b * ld + t];
        s1 += gpart[(int64_t)(b + 4) * ld + t];
      }
      if (b < nrg) s0 += gpart[(int64_t)b * ld + t];
    }
    sh[wv][lane] = s0 + s1;
    __syncthreads();
    if (wv == 0 && t < cols) {
      T s = (sh[0][lane] + sh[1][lane]) + (sh[2][lane] + sh[3][lane]);
      if (off) s += off[t];
      g[t] = s;
      const double k = kappa[t];
      eps[t] = k > 0.0 ? (T)((double)s * (double)s / k) : (T)0;
    }
    return;
  }
  const int64_t t = (int64_t)(blockIdx.x - ncb) * 256 + threadIdx.x;
  if (t < rows) {
    T s = (T)0;
    int c = 0;
    for (; c + 4 <= nch; c += 4) {
      T v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = qpart[(int64_t)(c + j) * rows + t];
#pragma unroll
      for (int j = 0; j < 4; ++j) s += v[j];
    }
    for (; c < nch; ++c) s += qpart[(int64_t)c * rows + t];
    q[t] = s;
  }
}

template <typename T>
void launch_dense_fused(const Dense<T> &A, const T *x, const T *z,
                        DenseWork<T> &w, const T *off, const double *kappa,
                        T *g, T *eps, T *q, Ctrl *ctrl, int respect_done,
                        hipStream_t st) {
  hipLaunchKernelGGL(dense_fused_kernel<T>, dim3(w.nch, w.nrg), dim3(DF_NT),
                     0, st, A, w.rpw, x, z, w.qpart, w.gpart, ctrl,
                     respect_done);
  const int ncb = (int)((A.cols + WAVE - 1) / WAVE);
  const int nrw = (int)((A.rows + 255) / 256);
  hipLaunchKernelGGL(dense_finalize<T>, dim3((unsigned)(ncb + nrw)),
                     dim3(256), 0, st, A.rows, A.cols, A.ld, w.nch, w.nrg,
                     ncb, w.qpart, w.gpart, off, kappa, g, eps, q, ctrl,
                     respect_done);
}
template void launch_dense_fused<double>(const Dense<double> &, const double *,
                                         const double *, DenseWork<double> &,
                                         const double *, const double *,
                                         double *, double *, double *, Ctrl *,
                                         int, hipStream_t);
template void launch_dense_fused<float>(const Dense<float> &, const float *,
                                        const float *, DenseWork<float> &,
                                        const float *, const double *, float *,
                                        float *, float *, Ctrl *, int,
                                        hipStream_t);

template <typename T>
__global__ void __launch_bounds__(256)
rowres_dense_kernel(int64_t m, const T *__restrict__ b,
                    const T *__restrict__ z, const T *__restrict__ q,
                    const double *__restrict__ rho, T *__restrict__ r,
                    T *__restrict__ eps, double *__restrict__ part,
                    Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  __shared__ double sh[256 / WAVE];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double pb = 0.0, pr = 0.0;
  if (i < m) {
    const T bb = b[i], qq = q[i];
    const T rr = bb - z[i] - qq;
    r[i] = rr;
    const double nr = rho[i];
    eps[i] = nr > 0.0 ? (T)((double)rr * (double)rr / nr) : (T)0;
    const double bq = (double)bb - (double)qq;
    pb = bq * bq;
    pr = (double)rr * (double)rr;
  }
  pb = block_sum<256>(pb, sh);
  pr = block_sum<256>(pr, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = pb;
    part[2 * blockIdx.x + 1] = pr;
  }
}

template <typename T>
int launch_rowres_dense(int64_t m, const T *b, const T *z, const T *q,
                        const double *rho, T *r, T *eps, double *part,
                        Ctrl *ctrl, int respect_done, hipStream_t st) {
  const int nb = (int)((m + 255) / 256);
  hipLaunchKernelGGL(rowres_dense_kernel<T>, dim3(nb), dim3(256), 0, st, m, b,
                     z, q, rho, r, eps, part, ctrl, respect_done);
  return nb;
}
template int launch_rowres_dense<double>(int64_t, const double *,
                                         const double *, const double *,
                                         const double *, double *, double *,
                                         double *, Ctrl *, int, hipStream_t);
template int launch_rowres_dense<float>(int64_t, const float *, const float *,
                                        const float *, const double *, float *,
                                        float *, double *, Ctrl *, int,
                                        hipStream_t);

// ------------------------------------------------------------ stop tests
// ||x_base + x - x_ref||^2 / ||x_ref||^2 at the top of an iteration; the last
// block compares with tol^2 and raises done/converged.  `final_check`
// (respect_done == 0) evaluates even when done is already set.
template <typename T>
__global__ void __launch_bounds__(256)
err_ref_kernel(int64_t n, const T *__restrict__ x,
               const double *__restrict__ xr, const double *__restrict__ xb,
               double *__restrict__ part, Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  __shared__ double sh[256 / WAVE];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    const double v = (xb ? xb[i] : 0.0) + (double)x[i];
    const double e = v - xr[i];
    s += e * e;
  }
  s = block_sum<256>(s, sh);
  if (threadIdx.x == 0) st_agent(&part[blockIdx.x], s);
  if (last_block(&ctrl->ticket[0])) {
    double t = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += 256) t += ld_agent(&part[b]);
    t = block_sum<256>(t, sh);
    if (threadIdx.x == 0) {
      const double metric = ctrl->ref2 > 0.0 ? sqrt(t / ctrl->ref2) : sqrt(t);
      ctrl->metric = metric;
      if (metric <= ctrl->tol) { ctrl->done = 1; ctrl->converged = 1; }
    }
  }
}

template <typename T>
void launch_err_ref(int64_t n, const T *x, const double *x_ref,
                    const double *x_base, Reduce &red, Ctrl *ctrl,
                    int respect_done, hipStream_t st) {
  int nb = (int)((n + 255) / 256);
  if (nb > 512) nb = 512;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(err_ref_kernel<T>, dim3(nb), dim3(256), 0, st, n, x,
                     x_ref, x_base, red.part, ctrl, respect_done);
}
template void launch_err_ref<double>(int64_t, const double *, const double *,
                                     const double *, Reduce &, Ctrl *, int,
                                     hipStream_t);
template void launch_err_ref<float>(int64_t, const float *, const double *,
                                    const double *, Reduce &, Ctrl *, int,
                                    hipStream_t);

template <typename T>
__global__ void __launch_bounds__(1024)
set_ref2_kernel(int64_t n, const T *__restrict__ v, Ctrl *ctrl) {
  __shared__ double sh[1024 / WAVE];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const double a = (double)v[i];
    s += a * a;
  }
  s = block_sum<1024>(s, sh);
  if (threadIdx.x == 0) ctrl->ref2 = s;
}
template <typename T>
void launch_set_ref2(int64_t n, const T *v, Ctrl *ctrl, hipStream_t st) {
  hipLaunchKernelGGL(set_ref2_kernel<T>, dim3(1), dim3(1024), 0, st, n, v,
                     ctrl);
}
template void launch_set_ref2<double>(int64_t, const double *, Ctrl *,
                                      hipStream_t);
template void launch_set_ref2<float>(int64_t, const float *, Ctrl *,
                                     hipStream_t);

// RSE  : sum(b - Ax)^2 / ||b||^2 <= tol
// RES_EXT: sqrt(sum r^2 / ||b||^2) <= tol
// (or <= pass_drop times the first metric of a mixed-form refinement pass)
__global__ void __launch_bounds__(256)
stop_rowres_kernel(const double *__restrict__ part, int nparts, Ctrl *ctrl) {
  if (ctrl_done(ctrl)) return;
  const int mode = ctrl->stop_mode;
  if (mode != 2 && mode != 3) return;
  __shared__ double sh[256 / WAVE];
  double pb = 0.0, pr = 0.0;
  for (int b = threadIdx.x; b < nparts; b += 256) {
    pb += part[2 * b];
    pr += part[2 * b + 1];
  }
  pb = block_sum<256>(pb, sh);
  pr = block_sum<256>(pr, sh);
  if (threadIdx.x == 0) {
    const double den = ctrl->ref2 > 0.0 ? ctrl->ref2 : 1.0;
    const double metric = (mode == 2) ? pb / den : sqrt(pr / den);
    ctrl->metric = metric;
    double thr = ctrl->tol;
    if (ctrl->pass_drop > 0.0) {
      if (ctrl->pass_ref <= 0.0) ctrl->pass_ref = metric;
      const double rel = ctrl->pass_drop * ctrl->pass_ref;
      thr = rel > thr ? rel : thr;
    }
    if (metric <= thr) { ctrl->done = 1; ctrl->converged = 1; }
  }
}
void launch_stop_rowres(const double *part, int nparts, Ctrl *ctrl,
                        hipStream_t st) {
  hipLaunchKernelGGL(stop_rowres_kernel, dim3(1), dim3(256), 0, st, part,
                     nparts, ctrl);
}

__global__ void end_iter_kernel(Ctrl *ctrl) {
  if (threadIdx.x != 0 || ctrl->done) return;
  ctrl->it += 1;
  ctrl->iters_run += 1;
  if (ctrl->iters_run >= ctrl->it_end || ctrl->numeric || ctrl->sync_fail)
    ctrl->done = 1;
}
void launch_end_iter(Ctrl *ctrl, hipStream_t st) {
  hipLaunchKernelGGL(end_iter_kernel, dim3(1), dim3(64), 0, st, ctrl);
}

__global__ void fill_it_kernel(Ctrl *ctrl, int64_t it) {
  if (threadIdx.x == 0) ctrl->it = it;
}
void launch_fill_ctrl_it(Ctrl *ctrl, int64_t it, hipStream_t st) {
  hipLaunchKernelGGL(fill_it_kernel, dim3(1), dim3(64), 0, st, ctrl, it);
}

__global__ void prof_mark_kernel(const Ctrl *ctrl, ProfRec *rec, int post,
                                 int ph) {
  if (threadIdx.x != 0) return;
  if (post == 0) rec->live = ctrl->done ? 0 : 1;
  else rec->steps = ph >= 0 ? ctrl->cg_steps[ph] : 0;
}
void launch_prof_mark(const Ctrl *ctrl, ProfRec *rec, int post, int ph,
                      hipStream_t st) {
  hipLaunchKernelGGL(prof_mark_kernel, dim3(1), dim3(64), 0, st, ctrl, rec,
                     post, ph);
}

}  // namespace rg
