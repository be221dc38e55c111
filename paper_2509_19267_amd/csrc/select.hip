// Block selection of RGDBEK on gfx950 (Section 2: column/row set
// probabilities and the "select n*eta columns / m*eta rows" steps of
// Algorithm 1).
//
// Draw k distinct indices without replacement with probability proportional
// to the residual weights eps, via exponential clocks (Efraimidis & Spirakis,
// IPL 2006): the block is the k smallest keys E_j / eps_j, E_j = -ln(u_j),
// ties ordered by index, returned in ascending index order.  u_j comes from
// Philox4x64-10 (Salmon et al., SC'11) with counter (j>>2, it, phase, sys),
// key (seed, key1), word j&3, mapped to (2*(w>>12)+1)*2^-53.
//
// Bit-exactness: this file is compiled with -ffp-contract=off; the logarithm
// uses only correctly rounded +,-,*,/ in a fixed order (atanh series on
// [sqrt(1/2), sqrt(2))), and the key is one correctly rounded division.
//
// Weights below floor * max(eps) count as zero (a weight that a projection
// has just annihilated is zero up to rounding); the largest weight comes from
// a max-reduction that runs before the keys.
//
// Pipeline (both forms end in the same predicate
//   take j  <=>  key_j < lo  ||  (key_j == tkey && j <= tidx)):
//  small d (one workgroup): keys -> 8 radix passes of 8 bits with LDS
//    histograms -> ordered tie resolution -> ballot/popcount compaction;
//  large d (multi-workgroup): keys + histogram of bits 62..52 -> scan ->
//    histogram of bits 51..41 -> scan -> gather the few candidates left ->
//    one-workgroup bitonic sort -> per-chunk counts -> ordered compaction.
#include <cmath>

#include "common.h"
#include "kernels.h"

namespace rg {

// ---------------------------------------------------------------- Philox
struct P4 { uint64_t v[4]; };

__device__ __forceinline__ P4 philox4x64_10(uint64_t c0, uint64_t c1,
                                            uint64_t c2, uint64_t c3,
                                            uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    const uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
    const uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  P4 o; o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
  return o;
}

// ---------------------------------------------------------------- ln
// ln(u) for u in [2^-53, 1): frexp by exponent bits (u is normal), reduce the
// mantissa to [sqrt(1/2), sqrt(2)), s = (f-1)/(f+1), t = s*s,
// ln f = 2s + 2s*t*P(t) with P(t) = sum_{i=1..11} t^(i-1)/(2i+1) by Horner,
// ln u = e*ln2 + ln f.  Coefficients are the correctly rounded quotients.
__device__ __forceinline__ double ln_unit(double u) {
  const uint64_t bits = (uint64_t)__double_as_longlong(u);
  int e = (int)((bits >> 52) & 0x7ff) - 1022;
  double f = __longlong_as_double(
      (long long)((bits & 0x800FFFFFFFFFFFFFull) | (1022ull << 52)));
  if (f < 0.7071067811865476) { f = f * 2.0; e -= 1; }
  const double s = (f - 1.0) / (f + 1.0);
  const double t = s * s;
  double p = 1.0 / 23.0;
  p = p * t; p = p + 1.0 / 21.0;
  p = p * t; p = p + 1.0 / 19.0;
  p = p * t; p = p + 1.0 / 17.0;
  p = p * t; p = p + 1.0 / 15.0;
  p = p * t; p = p + 1.0 / 13.0;
  p = p * t; p = p + 1.0 / 11.0;
  p = p * t; p = p + 1.0 / 9.0;
  p = p * t; p = p + 1.0 / 7.0;
  p = p * t; p = p + 1.0 / 5.0;
  p = p * t; p = p + 1.0 / 3.0;
  const double s2 = s + s;
  const double tp = t * p;
  const double lnf = s2 + s2 * tp;
  const double el = (double)e * 0.6931471805599453;
  return el + lnf;
}

__device__ __forceinline__ double unit_from_word(uint64_t w) {
  return (double)((w >> 12) * 2ull + 1ull) * 0x1p-53;
}

constexpr uint64_t SENT = ~0ull;   // key of a zero weight: never selected

// key of index j with weight e (already promoted to FP64); sets *bad on a
// NaN, negative or infinite weight.  Weights not above `cut` (the relative
// floor times the largest weight) count as zero.
__device__ __forceinline__ uint64_t make_key(double e, uint64_t w, double cut,
                                             int *bad) {
  if (!(e >= 0.0) || e > 1.7976931348623157e308) { *bad = 1; return SENT; }
  if (!(e > cut)) return SENT;
  const double E = -ln_unit(unit_from_word(w));
  const double k = E / e;
  return (uint64_t)__double_as_longlong(k);
}

__device__ __forceinline__ bool take(uint64_t key, int64_t j, uint64_t lo,
                                     uint64_t tkey, int64_t tidx) {
  return key < lo || (key == tkey && j <= tidx);
}

// Ordered compaction of one workgroup-sized chunk [base, base+NT) with the
// predicate above: ballot + popcount inside waves, wave totals via LDS.
// Returns the number taken in the chunk; writes at out[offset + rank].
template <int NT>
__device__ __forceinline__ int64_t compact_chunk(const uint64_t *keys,
                                                 int64_t base, int64_t d,
                                                 uint64_t lo, uint64_t tkey,
                                                 int64_t tidx, int32_t *out,
                                                 int64_t offset, int *wtot) {
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  const int64_t j = base + threadIdx.x;
  bool f = false;
  if (j < d) f = take(keys[j], j, lo, tkey, tidx);
  const uint64_t mask = __ballot(f);
  const int before = __popcll(mask & ((1ull << lane) - 1ull));
  __syncthreads();
  if (lane == 0) wtot[wv] = __popcll(mask);
  __syncthreads();
  int wbase = 0, total = 0;
#pragma unroll
  for (int i = 0; i < NT / WAVE; ++i) {
    if (i < wv) wbase += wtot[i];
    total += wtot[i];
  }
  if (f) out[offset + wbase + before] = (int32_t)j;
  return total;
}

// ------------------------------------------------ one-workgroup selection
// One workgroup of 1024 threads draws the block from d weights.  keys:
// scratch of d entries (written once, then read by the radix levels);
// writes out[0..count) (local indices), returns count (the same value in
// every thread); raises *numeric on a bad weight.  Radix levels of 11, 11,
// 11, 11, 11, 9 bits with LDS histograms until the bucket holding rank k has
// at most WG_CAND keys; those are gathered into LDS (any order) and ranked
// by counting (O(WG_CAND^2) LDS reads, so the bucket is refined further
// rather than ranked large), giving the k-th pair (key, index); an ordered
// ballot/scan compaction writes the block.  More than WG_CAND equal keys:
// the tie index comes from an ordered scan.  Up to WG_LDS_KEYS keys are
// kept in LDS instead of the global scratch.
constexpr int WG_NT = 1024;
constexpr int WG_CAND = 256;
constexpr int WG_UNROLL = 8;
constexpr int WG_LDS_KEYS = 8192;

__device__ __forceinline__ int wg_shift(int lev) { return lev < 5 ? 53 - 11 * lev : 0; }
__device__ __forceinline__ int wg_width(int lev) { return lev < 5 ? 11 : 9; }

// exclusive prefix of v over the workgroup (thread order); *tot = sum
__device__ __forceinline__ int64_t wg_scan(int64_t v, int64_t *sh, int64_t *tot) {
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  int64_t inc = v;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int64_t u = __shfl_up(inc, o, WAVE);
    if (lane >= o) inc += u;
  }
  __syncthreads();
  if (lane == WAVE - 1) sh[wv] = inc;
  __syncthreads();
  int64_t before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < WG_NT / WAVE; ++i) {
    if (i < wv) before += sh[i];
    all += sh[i];
  }
  *tot = all;
  return before + inc - v;
}

// From keys (d of them, SENT for zero weights), the count of positive keys
// and the LDS histogram of their top 11 bits: find the threshold pair and
// write the ordered block to out; returns its size (same in every thread).
__device__ __forceinline__ int64_t resolve_compact(const uint64_t *__restrict__ keys,
                                   int64_t d, int64_t k, int64_t pos,
                                   unsigned *hist, int32_t *__restrict__ out) {
  constexpr int NT = WG_NT;
  __shared__ int64_t sh64[NT / WAVE];
  __shared__ uint64_t s_ck[WG_CAND];
  __shared__ int32_t s_ci[WG_CAND];
  __shared__ unsigned s_nc;
  __shared__ int64_t s_b, s_acc, s_cb, s_tidx;
  __shared__ uint64_t s_tkey;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  uint64_t lo, tkey;
  int64_t tidx;
  if (pos <= k) {
    lo = SENT; tkey = SENT; tidx = -1;
  } else {
    uint64_t prefix = 0;
    int64_t krem = k;
    int lev = 0;
    while (true) {
      const int sh = wg_shift(lev), wd = wg_width(lev);
      const int nb = 1 << wd;
      if (wv == 0) {
        const int per = nb / WAVE;
        int64_t ls = 0;
        for (int i = 0; i < per; ++i) ls += hist[lane * per + i];
        int64_t inc = ls;
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
          const int64_t u = __shfl_up(inc, o, WAVE);
          if (lane >= o) inc += u;
        }
        const int64_t exc = inc - ls;
        if (exc < krem && krem <= inc) {
          int64_t acc = exc;
          int b = lane * per;
          for (;; ++b) {
            if (acc + (int64_t)hist[b] >= krem) break;
            acc += hist[b];
          }
          s_b = b;
          s_acc = acc;
          s_cb = hist[b];
        }
      }
      if (tid == 0) s_nc = 0u;
      __syncthreads();
      prefix = (prefix << wd) | (uint64_t)s_b;
      krem -= s_acc;
      const int64_t cb = s_cb;
      __syncthreads();
      if (cb == krem) {
        lo = (prefix + 1ull) << sh;
        tkey = SENT; tidx = -1;
        break;
      }
      if (cb <= WG_CAND) {
        // gather the bucket into LDS (any order) and rank by counting
        for (int64_t j0 = tid; j0 < d; j0 += WG_UNROLL * NT) {
          uint64_t kv[WG_UNROLL];
#pragma unroll
          for (int u = 0; u < WG_UNROLL; ++u) {
            const int64_t j = j0 + (int64_t)u * NT;
            kv[u] = j < d ? keys[j] : SENT;
          }
#pragma unroll
          for (int u = 0; u < WG_UNROLL; ++u)
            if (kv[u] != SENT && (kv[u] >> sh) == prefix) {
              const unsigned slot = atomicAdd(&s_nc, 1u);
              s_ck[slot] = kv[u];
              s_ci[slot] = (int32_t)(j0 + (int64_t)u * NT);
            }
        }
        __syncthreads();
        const int nc = (int)cb;
        if (tid < nc) {
          const uint64_t a = s_ck[tid];
          const int32_t ai = s_ci[tid];
          int64_t rank = 0;
          for (int u = 0; u < nc; ++u) {
            const uint64_t b = s_ck[u];
            rank += (b < a) || (b == a && s_ci[u] < ai);
          }
          if (rank == krem - 1) { s_tkey = a; s_tidx = ai; }
        }
        __syncthreads();
        tkey = s_tkey;
        tidx = s_tidx;
        lo = tkey;
        break;
      }
      if (sh == 0) {
        // more than WG_CAND equal keys: the krem-th of them in index order
        tkey = prefix;
        if (tid == 0) s_tidx = -1;
        int64_t seen = 0;
        for (int64_t base = 0; base < d && seen < krem; base += NT) {
          const int64_t j = base + tid;
          const int64_t f = (j < d && keys[j] == tkey) ? 1 : 0;
          int64_t tot;
          const int64_t r = seen + wg_scan(f, sh64, &tot);
          if (f && r == krem - 1) s_tidx = j;
          seen += tot;
        }
        __syncthreads();
        tidx = s_tidx;
        lo = tkey;
        break;
      }
      // histogram of the next digit inside the bucket
      const int nsh = wg_shift(lev + 1), nwd = wg_width(lev + 1);
      for (int i = tid; i < (1 << nwd); i += NT) hist[i] = 0u;
      __syncthreads();
      for (int64_t j0 = tid; j0 < d; j0 += WG_UNROLL * NT) {
        uint64_t kv[WG_UNROLL];
#pragma unroll
        for (int u = 0; u < WG_UNROLL; ++u) {
          const int64_t j = j0 + (int64_t)u * NT;
          kv[u] = j < d ? keys[j] : SENT;
        }
#pragma unroll
        for (int u = 0; u < WG_UNROLL; ++u)
          if (kv[u] != SENT && (kv[u] >> sh) == prefix)
            atomicAdd(&hist[(kv[u] >> nsh) & ((1u << nwd) - 1u)], 1u);
      }
      __syncthreads();
      ++lev;
    }
  }
  // ordered compaction, four consecutive indices per thread per pass
  int64_t off = 0;
  for (int64_t base = 0; base < d; base += 4 * NT) {
    const int64_t j0 = base + 4 * (int64_t)tid;
    bool f[4];
    int64_t c = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t j = j0 + q;
      f[q] = j < d && take(keys[j], j, lo, tkey, tidx);
      c += f[q];
    }
    int64_t tot;
    int64_t r = off + wg_scan(c, sh64, &tot);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (f[q]) out[r++] = (int32_t)(j0 + q);
    off += tot;
  }
  return off;
}

template <typename T>
__device__ __forceinline__ int64_t select_wg(const T *__restrict__ eps, int64_t d, int64_t k,
                             double floor, uint64_t seed, uint64_t key1,
                             uint64_t it, uint32_t phase, uint32_t sys,
                             uint64_t *__restrict__ keys,
                             int32_t *__restrict__ out, int *numeric) {
  constexpr int NT = WG_NT;
  __shared__ unsigned hist[2048];
  __shared__ int64_t sh64[NT / WAVE];
  __shared__ double shmax[NT / WAVE];
  __shared__ uint64_t s_keys[WG_LDS_KEYS];
  if (d <= WG_LDS_KEYS) keys = s_keys;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  // 1. largest finite weight
  // (the passes over d issue WG_UNROLL independent loads per thread at a
  // time: one workgroup has no other latency hiding)
  double mx = 0.0;
  for (int64_t j0 = tid; j0 < d; j0 += WG_UNROLL * NT) {
    double e[WG_UNROLL];
#pragma unroll
    for (int u = 0; u < WG_UNROLL; ++u) {
      const int64_t j = j0 + (int64_t)u * NT;
      e[u] = j < d ? (double)eps[j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < WG_UNROLL; ++u)
      if (e[u] <= 1.7976931348623157e308) mx = e[u] > mx ? e[u] : mx;
  }
  mx = wave_max(mx);
  if (lane == 0) shmax[wv] = mx;
  for (int i = tid; i < 2048; i += NT) hist[i] = 0u;
  __syncthreads();
  mx = 0.0;
  for (int i = 0; i < NT / WAVE; ++i) mx = shmax[i] > mx ? shmax[i] : mx;
  const double cut = floor > 0.0 ? floor * mx : 0.0;
  // 2. keys and the top-digit histogram
  int bad = 0;
  int64_t pos = 0;
  for (int64_t g = tid; g * 4 < d; g += NT) {
    double ev[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t j = g * 4 + q;
      ev[q] = j < d ? (double)eps[j] : 0.0;
    }
    const P4 r = philox4x64_10((uint64_t)g, it, phase, sys, seed, key1);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t j = g * 4 + q;
      if (j < d) {
        const uint64_t kk = make_key(ev[q], r.v[q], cut, &bad);
        keys[j] = kk;
        if (kk != SENT) {
          ++pos;
          atomicAdd(&hist[kk >> 53], 1u);
        }
      }
    }
  }
  if (bad) atomicOr(numeric, 1);
  pos = block_sum_i64<NT>(pos, sh64);   // (also orders keys/hist writes)
  return resolve_compact(keys, d, k, pos, hist, out);
}

template <typename T>
__global__ void __launch_bounds__(1024)
sel_small(const T *__restrict__ eps, int64_t d, int64_t k, double floor,
          uint64_t seed, uint64_t key1, int ph, uint32_t phase, uint32_t sys,
          uint64_t *__restrict__ keys, int32_t *__restrict__ out, Ctrl *ctrl,
          int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  const int64_t cnt = select_wg<T>(eps, d, k, floor, seed, key1,
                                   (uint64_t)ctrl->it, phase, sys, keys, out,
                                   &ctrl->numeric);
  if (threadIdx.x == 0) ctrl->sel_count[ph] = cnt;
}

// Per-system draws of a batch: each system draws from its own weights
// (eps[off_s .. off_s + d_s)) with its own block size, iteration counter and
// generator stream (system id in counter word 3); a finished system draws
// nothing.  Three launches: the largest weight of every system (one
// workgroup each), the keys of all systems (many workgroups per system),
// and the threshold search and ordered compaction (one workgroup each).
// Local indices go to tmp[koff_s ..]; counts to cnt[s].
template <typename T>
__global__ void __launch_bounds__(256)
sel_seg_max(const T *__restrict__ eps, const SegInfo *__restrict__ seg, int ph,
            double *__restrict__ segmax, Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  const SegInfo &g = seg[blockIdx.x];
  if (g.done) return;
  __shared__ double sh[256 / WAVE];
  const int64_t off = ph == 0 ? g.col_off : g.row_off;
  const int64_t d = ph == 0 ? g.ncol : g.nrow;
  double mx = 0.0;
  for (int64_t j0 = threadIdx.x; j0 < d; j0 += WG_UNROLL * 256) {
    double e[WG_UNROLL];
#pragma unroll
    for (int u = 0; u < WG_UNROLL; ++u) {
      const int64_t j = j0 + (int64_t)u * 256;
      e[u] = j < d ? (double)eps[off + j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < WG_UNROLL; ++u)
      if (e[u] <= 1.7976931348623157e308) mx = e[u] > mx ? e[u] : mx;
  }
  mx = wave_max(mx);
  if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < 256 / WAVE; ++i) mx = sh[i] > mx ? sh[i] : mx;
    segmax[blockIdx.x] = mx;
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
sel_seg_keys(const T *__restrict__ eps, const SegInfo *__restrict__ seg,
             int ph, double floor, uint64_t seed, uint64_t key1,
             uint32_t phase, const double *__restrict__ segmax,
             uint64_t *__restrict__ keys, Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  const int sidx = blockIdx.y;
  const SegInfo &g = seg[sidx];
  if (g.done) return;
  const int64_t off = ph == 0 ? g.col_off : g.row_off;
  const int64_t d = ph == 0 ? g.ncol : g.nrow;
  const int64_t gl = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gl * 4 >= d) return;
  const double mx = segmax[sidx];
  const double cut = floor > 0.0 ? floor * mx : 0.0;
  double ev[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t j = gl * 4 + q;
    ev[q] = j < d ? (double)eps[off + j] : 0.0;
  }
  const P4 r = philox4x64_10((uint64_t)gl, (uint64_t)g.it, phase,
                             (uint32_t)sidx, seed, key1);
  int bad = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t j = gl * 4 + q;
    if (j < d) keys[off + j] = make_key(ev[q], r.v[q], cut, &bad);
  }
  if (bad) atomicOr(&ctrl->numeric, 1);
}

__global__ void __launch_bounds__(WG_NT)
sel_seg_resolve(const SegInfo *__restrict__ seg, int ph,
                const uint64_t *__restrict__ keys, int32_t *__restrict__ tmp,
                int64_t *__restrict__ cnt, Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  const SegInfo &g = seg[blockIdx.x];
  if (g.done) {
    if (threadIdx.x == 0) cnt[blockIdx.x] = 0;
    return;
  }
  __shared__ unsigned hist[2048];
  __shared__ int64_t sh64[WG_NT / WAVE];
  const int64_t off = ph == 0 ? g.col_off : g.row_off;
  const int64_t d = ph == 0 ? g.ncol : g.nrow;
  const int64_t k = ph == 0 ? g.kc : g.kr;
  const int64_t ko = ph == 0 ? g.kc_off : g.kr_off;
  const uint64_t *kk = keys + off;
  __shared__ uint64_t s_keys[WG_LDS_KEYS];
  const bool lds = d <= WG_LDS_KEYS;     // later passes read the LDS copy
  for (int i = threadIdx.x; i < 2048; i += WG_NT) hist[i] = 0u;
  __syncthreads();
  int64_t pos = 0;
  for (int64_t j0 = threadIdx.x; j0 < d; j0 += WG_UNROLL * WG_NT) {
    uint64_t kv[WG_UNROLL];
#pragma unroll
    for (int u = 0; u < WG_UNROLL; ++u) {
      const int64_t j = j0 + (int64_t)u * WG_NT;
      kv[u] = j < d ? kk[j] : SENT;
    }
#pragma unroll
    for (int u = 0; u < WG_UNROLL; ++u) {
      const int64_t j = j0 + (int64_t)u * WG_NT;
      if (lds && j < d) s_keys[j] = kv[u];
      if (kv[u] != SENT) {
        ++pos;
        atomicAdd(&hist[kv[u] >> 53], 1u);
      }
    }
  }
  pos = block_sum_i64<WG_NT>(pos, sh64);   // (also orders the LDS copy)
  const int64_t c = resolve_compact(lds ? s_keys : kk, d, k, pos, hist,
                                    tmp + ko);
  if (threadIdx.x == 0) cnt[blockIdx.x] = c;
}

// Concatenate the per-system draws into one list of global indices and set
// Ctrl::sel_count[ph] to the total.
__global__ void __launch_bounds__(256)
sel_seg_pack(const SegInfo *__restrict__ seg, int nseg, int ph,
             const int32_t *__restrict__ tmp, const int64_t *__restrict__ cnt,
             int32_t *__restrict__ out, Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  __shared__ int64_t sh64[256 / WAVE];
  const int s = blockIdx.x;
  int64_t before = 0, total = 0;
  for (int q = threadIdx.x; q < nseg; q += 256) {
    total += cnt[q];
    if (q < s) before += cnt[q];
  }
  before = block_sum_i64<256>(before, sh64);
  total = block_sum_i64<256>(total, sh64);
  const SegInfo &g = seg[s];
  const int64_t off = ph == 0 ? g.col_off : g.row_off;
  const int64_t ko = ph == 0 ? g.kc_off : g.kr_off;
  const int64_t c = cnt[s];
  for (int64_t a = threadIdx.x; a < c; a += 256)
    out[before + a] = (int32_t)(tmp[ko + a] + off);
  if (s == 0 && threadIdx.x == 0) ctrl->sel_count[ph] = total;
}

// ------------------------------------------------ multi-workgroup selection
constexpr int SEL_NT = 1024;
constexpr int SEL_CHUNK = 4 * SEL_NT;       // indices per workgroup
constexpr int SEL_BITS = 11;
constexpr int SEL_BINS = 1 << SEL_BITS;
constexpr int SEL_CAND = 4096;              // candidates sorted in LDS

// mode values stored in ctrl->sel_mode
enum { M_RADIX = 0, M_ALL = 1, M_RESOLVED = 2, M_GATHER = 3, M_FALLBACK = 4,
       M_EXACT = 5 };

// largest non-negative finite weight, as its (order-preserving) bit pattern
template <typename T>
__global__ void __launch_bounds__(SEL_NT)
sel_max(const T *__restrict__ eps, int64_t d, Ctrl *ctrl, int ph,
        int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  __shared__ double sh[SEL_NT / WAVE];
  const int64_t base = (int64_t)blockIdx.x * SEL_CHUNK;
  double mx = 0.0;
  for (int q = 0; q < 4; ++q) {
    const int64_t j = base + q * SEL_NT + threadIdx.x;
    if (j < d) {
      const double e = (double)eps[j];
      if (e <= 1.7976931348623157e308) mx = e > mx ? e : mx;
    }
  }
  mx = wave_max(mx);
  if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < SEL_NT / WAVE; ++i) mx = sh[i] > mx ? sh[i] : mx;
    if (mx > 0.0)
      atomicMax((unsigned long long *)&ctrl->sel_maxbits[ph],
                (unsigned long long)__double_as_longlong(mx));
  }
}

template <typename T>
__global__ void __launch_bounds__(SEL_NT)
sel_keys_hist(const T *__restrict__ eps, int64_t d, double floor,
              uint64_t seed, uint64_t key1, uint32_t phase, uint32_t sys,
              uint64_t *__restrict__ keys, unsigned *__restrict__ hist,
              Ctrl *ctrl, int ph, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  __shared__ unsigned h[SEL_BINS];
  __shared__ int64_t sh64[SEL_NT / WAVE];
  for (int i = threadIdx.x; i < SEL_BINS; i += SEL_NT) h[i] = 0;
  __syncthreads();
  const uint64_t it = (uint64_t)ctrl->it;
  const double mx = __longlong_as_double((long long)ctrl->sel_maxbits[ph]);
  const double cut = floor > 0.0 ? floor * mx : 0.0;
  const int64_t g = (int64_t)blockIdx.x * SEL_NT + threadIdx.x;
  int bad = 0;
  int64_t pos = 0;
  if (g * 4 < d) {
    const P4 r = philox4x64_10((uint64_t)g, it, phase, sys, seed, key1);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t j = g * 4 + q;
      if (j < d) {
        const uint64_t kk = make_key((double)eps[j], r.v[q], cut, &bad);
        keys[j] = kk;
        if (kk != SENT) {
          ++pos;
          atomicAdd(&h[(kk >> 52) & (SEL_BINS - 1)], 1u);
        }
      }
    }
  }
  if (bad) atomicOr(&ctrl->numeric, 1);
  pos = block_sum_i64<SEL_NT>(pos, sh64);
  if (threadIdx.x == 0 && pos) atomicAdd((unsigned long long *)&ctrl->sel_pos[ph],
                                         (unsigned long long)pos);
  __syncthreads();
  for (int i = threadIdx.x; i < SEL_BINS; i += SEL_NT)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

// One workgroup: pick the bucket holding rank krem, clear the histogram.
__global__ void __launch_bounds__(SEL_NT)
sel_scan(unsigned *__restrict__ hist, int64_t k, Ctrl *ctrl, int ph,
         int first, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  __shared__ unsigned h[SEL_BINS];
  const int mode = first ? M_RADIX : ctrl->sel_mode[ph];
  for (int i = threadIdx.x; i < SEL_BINS; i += SEL_NT) {
    h[i] = hist[i];
    hist[i] = 0;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  if (first) {
    const int64_t pos = ctrl->sel_pos[ph];
    ctrl->sel_pos[ph] = 0;
    ctrl->sel_maxbits[ph] = 0;
    if (pos <= k) {
      ctrl->sel_mode[ph] = M_ALL;
      ctrl->sel_tkey[ph] = SENT; ctrl->sel_tidx[ph] = -1;
      ctrl->sel_prefix[ph] = SENT; ctrl->sel_shift[ph] = 0;
      return;
    }
    ctrl->sel_krem[ph] = k;
    ctrl->sel_prefix[ph] = 0;
    ctrl->sel_shift[ph] = 63;
  } else if (mode != M_RADIX) {
    return;
  }
  const int64_t kr = ctrl->sel_krem[ph];
  int64_t acc = 0;
  int b = 0;
  for (; b < SEL_BINS; ++b) {
    if (acc + (int64_t)h[b] >= kr) break;
    acc += h[b];
  }
  const int shift = ctrl->sel_shift[ph] - SEL_BITS;   // 52, then 41
  const uint64_t prefix = (ctrl->sel_prefix[ph] << SEL_BITS) | (uint64_t)b;
  const int64_t krem = kr - acc;
  const int64_t cnt = h[b];
  ctrl->sel_prefix[ph] = prefix;
  ctrl->sel_shift[ph] = shift;
  ctrl->sel_krem[ph] = krem;
  if (cnt == krem) {
    ctrl->sel_mode[ph] = M_RESOLVED;
    ctrl->sel_prefix[ph] = (prefix + 1) << shift;   // lo bound
  } else if (!first) {
    ctrl->sel_mode[ph] = (cnt <= SEL_CAND) ? M_GATHER : M_FALLBACK;
    ctrl->sel_cand[ph] = 0;
  } else {
    ctrl->sel_mode[ph] = M_RADIX;
  }
}

__global__ void __launch_bounds__(SEL_NT)
sel_hist(const uint64_t *__restrict__ keys, int64_t d,
         unsigned *__restrict__ hist, Ctrl *ctrl, int ph, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  if (ctrl->sel_mode[ph] != M_RADIX) return;
  __shared__ unsigned h[SEL_BINS];
  for (int i = threadIdx.x; i < SEL_BINS; i += SEL_NT) h[i] = 0;
  __syncthreads();
  const int shift = ctrl->sel_shift[ph];            // 52
  const uint64_t pre = ctrl->sel_prefix[ph];
  const int64_t base = (int64_t)blockIdx.x * SEL_CHUNK;
  for (int q = 0; q < 4; ++q) {
    const int64_t j = base + q * SEL_NT + threadIdx.x;
    if (j < d) {
      const uint64_t kk = keys[j];
      if (kk != SENT && (kk >> shift) == pre)
        atomicAdd(&h[(kk >> (shift - SEL_BITS)) & (SEL_BINS - 1)], 1u);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < SEL_BINS; i += SEL_NT)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

__global__ void __launch_bounds__(SEL_NT)
sel_gather(const uint64_t *__restrict__ keys, int64_t d,
           uint64_t *__restrict__ ckey, int64_t *__restrict__ cidx,
           Ctrl *ctrl, int ph, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  if (ctrl->sel_mode[ph] != M_GATHER) return;
  const int shift = ctrl->sel_shift[ph];            // 41
  const uint64_t pre = ctrl->sel_prefix[ph];
  const int64_t base = (int64_t)blockIdx.x * SEL_CHUNK;
  for (int q = 0; q < 4; ++q) {
    const int64_t j = base + q * SEL_NT + threadIdx.x;
    if (j < d) {
      const uint64_t kk = keys[j];
      if (kk != SENT && (kk >> shift) == pre) {
        const unsigned long long slot =
            atomicAdd((unsigned long long *)&ctrl->sel_cand[ph], 1ull);
        if (slot < (unsigned long long)SEL_CAND) { ckey[slot] = kk; cidx[slot] = j; }
      }
    }
  }
}

// One workgroup: find (tkey, tidx), the krem-th smallest candidate pair.
__global__ void __launch_bounds__(SEL_NT)
sel_resolve(const uint64_t *__restrict__ keys, int64_t d,
            const uint64_t *__restrict__ ckey, const int64_t *__restrict__ cidx,
            Ctrl *ctrl, int ph, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  const int mode = ctrl->sel_mode[ph];
  if (mode == M_ALL) {
    if (threadIdx.x == 0) { ctrl->sel_prefix[ph] = SENT; }
    return;
  }
  if (mode == M_RESOLVED) {
    if (threadIdx.x == 0) { ctrl->sel_tkey[ph] = SENT; ctrl->sel_tidx[ph] = -1; }
    return;
  }
  __shared__ uint64_t sk[SEL_CAND];
  __shared__ int64_t si[SEL_CAND];
  __shared__ unsigned h[256];
  __shared__ uint64_t s_pre;
  __shared__ int64_t s_krem, s_tidx;
  __shared__ int wtot[SEL_NT / WAVE];
  if (mode == M_GATHER) {
    const int64_t nc = ctrl->sel_cand[ph];
    for (int i = threadIdx.x; i < SEL_CAND; i += SEL_NT) {
      if (i < nc) { sk[i] = ckey[i]; si[i] = cidx[i]; }
      else { sk[i] = SENT; si[i] = INT64_MAX; }
    }
    __syncthreads();
    // bitonic sort of (key, idx) pairs ascending
    for (int size = 2; size <= SEL_CAND; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int i = threadIdx.x; i < SEL_CAND; i += SEL_NT) {
          const int p = i ^ stride;
          if (p > i) {
            const bool up = ((i & size) == 0);
            const uint64_t a = sk[i], b = sk[p];
            const int64_t ai = si[i], bi = si[p];
            const bool gt = (a > b) || (a == b && ai > bi);
            if (gt == up) { sk[i] = b; sk[p] = a; si[i] = bi; si[p] = ai; }
          }
        }
        __syncthreads();
      }
    }
    if (threadIdx.x == 0) {
      const int64_t kr = ctrl->sel_krem[ph];
      ctrl->sel_tkey[ph] = sk[kr - 1];
      ctrl->sel_tidx[ph] = si[kr - 1];
      ctrl->sel_prefix[ph] = sk[kr - 1];    // lo bound = tkey
      ctrl->sel_mode[ph] = M_EXACT;
    }
    return;
  }
  // M_FALLBACK: finish the radix select over all keys with this workgroup
  // (8-bit digits below the resolved prefix), then locate the tie index.
  if (threadIdx.x == 0) {
    s_pre = ctrl->sel_prefix[ph];
    s_krem = ctrl->sel_krem[ph];
  }
  int shift = ctrl->sel_shift[ph];
  __syncthreads();
  while (shift > 0) {
    const int step = shift >= 8 ? 8 : shift;
    const int nshift = shift - step;
    for (int i = threadIdx.x; i < 256; i += SEL_NT) h[i] = 0;
    __syncthreads();
    const uint64_t pre = s_pre;
    for (int64_t j = threadIdx.x; j < d; j += SEL_NT) {
      const uint64_t kk = keys[j];
      if (kk != SENT && (kk >> shift) == pre)
        atomicAdd(&h[(kk >> nshift) & ((1u << step) - 1u)], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t kr = s_krem, acc = 0;
      int b = 0;
      for (; b < (1 << step); ++b) {
        if (acc + (int64_t)h[b] >= kr) break;
        acc += h[b];
      }
      s_pre = (pre << step) | (uint64_t)b;
      s_krem = kr - acc;
    }
    __syncthreads();
    shift = nshift;
  }
  const uint64_t tkey = s_pre;
  const int64_t krem = s_krem;
  int64_t seen = 0;
  if (threadIdx.x == 0) s_tidx = -1;
  __syncthreads();
  for (int64_t base = 0; base < d && seen < krem; base += SEL_NT) {
    const int64_t j = base + threadIdx.x;
    const bool f = (j < d) && keys[j] == tkey;
    const uint64_t mask = __ballot(f);
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    __syncthreads();
    if (lane == 0) wtot[wv] = __popcll(mask);
    __syncthreads();
    int64_t wb = 0, tot = 0;
    for (int i = 0; i < SEL_NT / WAVE; ++i) {
      if (i < wv) wb += wtot[i];
      tot += wtot[i];
    }
    const int64_t rank = seen + wb + __popcll(mask & ((1ull << lane) - 1ull));
    if (f && rank == krem - 1) s_tidx = j;
    seen += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    ctrl->sel_tkey[ph] = tkey;
    ctrl->sel_tidx[ph] = s_tidx;
    ctrl->sel_prefix[ph] = tkey;
    ctrl->sel_mode[ph] = M_EXACT;
  }
}

__global__ void __launch_bounds__(SEL_NT)
sel_count(const uint64_t *__restrict__ keys, int64_t d,
          int32_t *__restrict__ blk, Ctrl *ctrl, int ph, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  __shared__ int64_t sh64[SEL_NT / WAVE];
  const uint64_t lo = ctrl->sel_prefix[ph];
  const uint64_t tkey = ctrl->sel_tkey[ph];
  const int64_t tidx = ctrl->sel_tidx[ph];
  const int64_t base = (int64_t)blockIdx.x * SEL_CHUNK;
  int64_t c = 0;
  for (int q = 0; q < 4; ++q) {
    const int64_t j = base + q * SEL_NT + threadIdx.x;
    if (j < d) c += take(keys[j], j, lo, tkey, tidx);
  }
  c = block_sum_i64<SEL_NT>(c, sh64);
  if (threadIdx.x == 0) blk[blockIdx.x] = (int32_t)c;
}

__global__ void __launch_bounds__(SEL_NT)
sel_write(const uint64_t *__restrict__ keys, int64_t d,
          const int32_t *__restrict__ blk, int32_t *__restrict__ out,
          Ctrl *ctrl, int ph, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  __shared__ int64_t sh64[SEL_NT / WAVE];
  __shared__ int wtot[SEL_NT / WAVE];
  const uint64_t lo = ctrl->sel_prefix[ph];
  const uint64_t tkey = ctrl->sel_tkey[ph];
  const int64_t tidx = ctrl->sel_tidx[ph];
  int64_t before = 0, total = 0;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += SEL_NT) {
    const int64_t v = blk[b];
    total += v;
    if (b < (int)blockIdx.x) before += v;
  }
  before = block_sum_i64<SEL_NT>(before, sh64);
  total = block_sum_i64<SEL_NT>(total, sh64);
  const int64_t base = (int64_t)blockIdx.x * SEL_CHUNK;
  int64_t off = before;
  for (int q = 0; q < 4; ++q)
    off += compact_chunk<SEL_NT>(keys, base + q * SEL_NT, d, lo, tkey, tidx,
                                 out, off, wtot);
  if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->sel_count[ph] = total;
}

// ------------------------------------------------ persistent selection
// One launch of P co-resident workgroups; workgroup w owns indices
// [w*L, (w+1)*L) with L = KPT*SP_NT and keeps their keys in registers
// (thread t holds the Philox groups t, t + SP_NT, ... of its chunk, four
// consecutive indices each).  Grid barriers separate: the max-reduction;
// keys + histogram of the top 11 key bits; each further radix level (11, 11,
// 11, 11, 9 bits) while the bucket holding rank k is larger than SP_CAND;
// the gather of that bucket (every workgroup then finds the same k-th pair
// (key, index) in LDS); the per-workgroup taken counts.  The taken indices
// are written in ascending order from per-workgroup offsets.  Same draw and
// same predicate as the other forms, so the same block, bit for bit.
constexpr int SP_NT = 256;
constexpr int SP_CAND = SP_NT;   // candidates ranked in LDS (one per thread)
constexpr int SP_MAXG = 1024;

__device__ __forceinline__ int sp_shift(int lev) { return lev < 5 ? 53 - 11 * lev : 0; }
__device__ __forceinline__ int sp_width(int lev) { return lev < 5 ? 11 : 9; }

// exclusive prefix of v over the workgroup (thread order); *tot = sum
__device__ __forceinline__ int64_t sp_scan(int64_t v, int64_t *sh, int64_t *tot) {
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  int64_t inc = v;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int64_t u = __shfl_up(inc, o, WAVE);
    if (lane >= o) inc += u;
  }
  __syncthreads();
  if (lane == WAVE - 1) sh[wv] = inc;
  __syncthreads();
  int64_t before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < SP_NT / WAVE; ++i) {
    if (i < wv) before += sh[i];
    all += sh[i];
  }
  *tot = all;
  return before + inc - v;
}

template <typename T, int KPT>
__global__ void __launch_bounds__(SP_NT)
sel_persist_kernel(const T *__restrict__ eps, int64_t d, int64_t k,
                   double floor, uint64_t seed, uint64_t key1, uint32_t phase,
                   uint32_t sys, int ph, SelPersist *sp,
                   int32_t *__restrict__ out, Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  constexpr int NG = KPT / 4;
  __shared__ unsigned hist[2048];
  __shared__ uint64_t s_ck[SP_CAND];
  __shared__ int32_t s_ci[SP_CAND];
  __shared__ double shd[SP_NT / WAVE];
  __shared__ int64_t sh64[SP_NT / WAVE];
  __shared__ int64_t s_b, s_acc, s_cb, s_tidx;
  __shared__ uint64_t s_tkey;
  const int P = (int)gridDim.x;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int64_t L = (int64_t)KPT * SP_NT;
  const int64_t base = (int64_t)blockIdx.x * L;
  const uint64_t it = (uint64_t)ctrl->it;
  const uint64_t bbase = ctrl->sel_barbase[ph];
  uint64_t nbar = 0;
  uint64_t *bar = &ctrl->sel_bar[ph];
  int32_t *fail = &ctrl->sync_fail;

  if (blockIdx.x == 0) {
    unsigned *gh = &sp->gh[0][0];
    for (int i = tid; i < 6 * 2048; i += SP_NT) gh[i] = 0u;
    if (tid == 0) { sp->gpos = 0ull; sp->ncand = 0ull; sp->tidx = -1; }
  }
  // 1. largest finite weight
  double mx = 0.0;
#pragma unroll
  for (int i = 0; i < NG; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t j = base + 4 * ((int64_t)i * SP_NT + tid) + q;
      if (j < d) {
        const double e = (double)eps[j];
        if (e <= 1.7976931348623157e308) mx = e > mx ? e : mx;
      }
    }
  mx = wave_max(mx);
  if (lane == 0) shd[wv] = mx;
  __syncthreads();
  if (tid == 0) {
    for (int i = 0; i < SP_NT / WAVE; ++i) mx = shd[i] > mx ? shd[i] : mx;
    sp->gmax[blockIdx.x] = mx;
  }
  if (!grid_barrier(bar, bbase + (++nbar) * P, fail)) return;
  double gm = 0.0;
  for (int b = tid; b < P; b += SP_NT) {
    const double v = ld_agent(&sp->gmax[b]);
    gm = v > gm ? v : gm;
  }
  gm = wave_max(gm);
  __syncthreads();
  if (lane == 0) shd[wv] = gm;
  __syncthreads();
  gm = 0.0;
  for (int i = 0; i < SP_NT / WAVE; ++i) gm = shd[i] > gm ? shd[i] : gm;
  const double cut = floor > 0.0 ? floor * gm : 0.0;

  // 2. keys and the top-digit histogram
  for (int i = tid; i < 2048; i += SP_NT) hist[i] = 0u;
  __syncthreads();
  uint64_t key[KPT];
  int bad = 0;
  int64_t pos = 0;
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    const int64_t g = base / 4 + (int64_t)i * SP_NT + tid;
    if (g * 4 < d) {
      const P4 r = philox4x64_10((uint64_t)g, it, phase, sys, seed, key1);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t j = g * 4 + q;
        uint64_t kk = SENT;
        if (j < d) kk = make_key((double)eps[j], r.v[q], cut, &bad);
        key[4 * i + q] = kk;
        if (kk != SENT) {
          ++pos;
          atomicAdd(&hist[kk >> 53], 1u);
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) key[4 * i + q] = SENT;
    }
  }
  if (bad) atomicOr(&ctrl->numeric, 1);
  pos = block_sum_i64<SP_NT>(pos, sh64);
  for (int i = tid; i < 2048; i += SP_NT)
    if (hist[i]) atomicAdd(&sp->gh[0][i], hist[i]);
  if (tid == 0 && pos) atomicAdd(&sp->gpos, (unsigned long long)pos);
  if (!grid_barrier(bar, bbase + (++nbar) * P, fail)) return;

  // 3. threshold pair (tkey, tidx) and bound lo
  uint64_t lo, tkey;
  int64_t tidx;
  const int64_t gpos = (int64_t)ld_agent(&sp->gpos);
  if (gpos <= k) {
    lo = SENT; tkey = SENT; tidx = -1;
  } else {
    uint64_t prefix = 0;
    int64_t krem = k;
    int lev = 0;
    while (true) {
      const int sh = sp_shift(lev), wd = sp_width(lev);
      const int nb = 1 << wd;
      for (int i = tid; i < nb; i += SP_NT) hist[i] = ld_agent(&sp->gh[lev][i]);
      __syncthreads();
      if (wv == 0) {
        // bucket holding rank krem: lane sums of nb/64 bins, wave scan
        const int per = nb / WAVE;
        int64_t ls = 0;
        for (int i = 0; i < per; ++i) ls += hist[lane * per + i];
        int64_t inc = ls;
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
          const int64_t u = __shfl_up(inc, o, WAVE);
          if (lane >= o) inc += u;
        }
        const int64_t exc = inc - ls;
        if (exc < krem && krem <= inc) {
          int64_t acc = exc;
          int b = lane * per;
          for (;; ++b) {
            if (acc + (int64_t)hist[b] >= krem) break;
            acc += hist[b];
          }
          s_b = b;
          s_acc = acc;
          s_cb = hist[b];
        }
      }
      __syncthreads();
      prefix = (prefix << wd) | (uint64_t)s_b;
      krem -= s_acc;
      const int64_t cb = s_cb;
      __syncthreads();
      if (cb == krem) {
        lo = (prefix + 1ull) << sh;
        tkey = SENT; tidx = -1;
        break;
      }
      if (cb <= SP_CAND) {
        // gather the bucket (one slot reservation per workgroup), then every
        // workgroup ranks the candidates in LDS by counting
        int64_t mc = 0;
#pragma unroll
        for (int i = 0; i < KPT; ++i)
          mc += (key[i] != SENT && (key[i] >> sh) == prefix);
        int64_t wtot;
        const int64_t wex = sp_scan(mc, sh64, &wtot);
        if (tid == 0 && wtot > 0)
          s_b = (int64_t)atomicAdd(&sp->ncand, (unsigned long long)wtot);
        __syncthreads();
        int64_t slot = s_b + wex;
#pragma unroll
        for (int i = 0; i < NG; ++i)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const uint64_t kk = key[4 * i + q];
            if (kk != SENT && (kk >> sh) == prefix) {
              if (slot < SP_CAND) {
                sp->ckey[slot] = kk;
                sp->cidx[slot] = base + 4 * ((int64_t)i * SP_NT + tid) + q;
              }
              ++slot;
            }
          }
        if (!grid_barrier(bar, bbase + (++nbar) * P, fail)) return;
        const int nc = (int)cb;
        for (int i = tid; i < nc; i += SP_NT) {
          s_ck[i] = ld_agent(&sp->ckey[i]);
          s_ci[i] = (int32_t)ld_agent(&sp->cidx[i]);
        }
        __syncthreads();
        if (tid < nc) {
          const uint64_t a = s_ck[tid];
          const int32_t ai = s_ci[tid];
          int64_t rank = 0;
          for (int u = 0; u < nc; ++u) {
            const uint64_t b = s_ck[u];
            rank += (b < a) || (b == a && s_ci[u] < ai);
          }
          if (rank == krem - 1) { s_tkey = a; s_tidx = ai; }
        }
        __syncthreads();
        tkey = s_tkey;
        tidx = s_tidx;
        lo = tkey;
        break;
      }
      if (sh == 0) {
        // more than SP_CAND equal keys: the krem-th of them in index order
        tkey = prefix;
        int64_t mine = 0;
#pragma unroll
        for (int i = 0; i < KPT; ++i) mine += key[i] == tkey;
        mine = block_sum_i64<SP_NT>(mine, sh64);
        if (tid == 0) sp->cnt[blockIdx.x] = mine;
        if (!grid_barrier(bar, bbase + (++nbar) * P, fail)) return;
        int64_t before = 0;
        for (int b = tid; b < (int)blockIdx.x; b += SP_NT) before += ld_agent(&sp->cnt[b]);
        before = block_sum_i64<SP_NT>(before, sh64);
        if (before < krem && krem <= before + mine) {
          int64_t seen = before;
          for (int i = 0; i < NG; ++i) {
            int64_t c = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) c += key[4 * i + q] == tkey;
            int64_t tot;
            const int64_t ex = sp_scan(c, sh64, &tot);
            int64_t r = seen + ex;
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (key[4 * i + q] == tkey) {
                if (r == krem - 1)
                  st_agent(&sp->tidx, base + 4 * ((int64_t)i * SP_NT + tid) + q);
                ++r;
              }
            seen += tot;
          }
        }
        if (!grid_barrier(bar, bbase + (++nbar) * P, fail)) return;
        tidx = ld_agent(&sp->tidx);
        lo = tkey;
        break;
      }
      // histogram of the next digit inside the bucket
      const int nsh = sp_shift(lev + 1), nwd = sp_width(lev + 1);
      for (int i = tid; i < (1 << nwd); i += SP_NT) hist[i] = 0u;
      __syncthreads();
#pragma unroll
      for (int i = 0; i < KPT; ++i) {
        const uint64_t kk = key[i];
        if (kk != SENT && (kk >> sh) == prefix)
          atomicAdd(&hist[(kk >> nsh) & ((1u << nwd) - 1u)], 1u);
      }
      __syncthreads();
      for (int i = tid; i < (1 << nwd); i += SP_NT)
        if (hist[i]) atomicAdd(&sp->gh[lev + 1][i], hist[i]);
      if (!grid_barrier(bar, bbase + (++nbar) * P, fail)) return;
      ++lev;
    }
  }

  // 4. counts per workgroup, then ordered compaction
  int64_t mine = 0;
#pragma unroll
  for (int i = 0; i < NG; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      mine += take(key[4 * i + q], base + 4 * ((int64_t)i * SP_NT + tid) + q,
                   lo, tkey, tidx);
  mine = block_sum_i64<SP_NT>(mine, sh64);
  if (tid == 0) sp->cnt[blockIdx.x] = mine;
  if (!grid_barrier(bar, bbase + (++nbar) * P, fail)) return;
  int64_t before = 0, total = 0;
  for (int b = tid; b < P; b += SP_NT) {
    const int64_t v = ld_agent(&sp->cnt[b]);
    total += v;
    if (b < (int)blockIdx.x) before += v;
  }
  before = block_sum_i64<SP_NT>(before, sh64);
  total = block_sum_i64<SP_NT>(total, sh64);
  int64_t off = before;
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    int64_t c = 0;
    bool f[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t j = base + 4 * ((int64_t)i * SP_NT + tid) + q;
      f[q] = take(key[4 * i + q], j, lo, tkey, tidx);
      c += f[q];
    }
    int64_t tot;
    int64_t r = off + sp_scan(c, sh64, &tot);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (f[q]) out[r++] = (int32_t)(base + 4 * ((int64_t)i * SP_NT + tid) + q);
    off += tot;
  }
  if (blockIdx.x == 0 && tid == 0) {
    ctrl->sel_count[ph] = total;
    ctrl->sel_barbase[ph] = bbase + nbar * (uint64_t)P;
  }
}

// keys per thread and grid of the persistent selection (kpt 0: not taken)
static void sel_persist_shape(int64_t d, int ncu, int *kpt, int *grid) {
  *kpt = 0;
  *grid = 0;
  if (ncu <= 0) return;
  const int64_t lim = ncu < SP_MAXG ? ncu : SP_MAXG;
  for (int kk : {4, 16}) {
    const int64_t L = (int64_t)kk * SP_NT;
    const int64_t g = (d + L - 1) / L;
    if (g <= lim) { *kpt = kk; *grid = (int)(g < 1 ? 1 : g); return; }
  }
}
int64_t select_persist_max(int ncu) {
  const int64_t lim = ncu < SP_MAXG ? ncu : SP_MAXG;
  return ncu > 0 ? lim * 16 * SP_NT : 0;
}
// smallest d that takes the persistent form (below: one workgroup, keys in
// LDS)
constexpr int64_t SP_MIN_D = WG_LDS_KEYS + 1;

// ------------------------------------------------ Lemma 2.1 block law
// P(B) proportional to sum_{j in B} eps_j over the s-subsets: the one-index
// draw j* of launch_select (k = 1, same coordinates), then a uniform
// (s-1)-subset of the other indices -- launch_select with k = s-1 on unit
// weights (zero at j*), generator phase + 2 -- merged into one ascending
// list.  Every weight zero: the empty block.
__global__ void __launch_bounds__(256)
bl_weights(int64_t d, const int32_t *__restrict__ first,
           double *__restrict__ w, Ctrl *ctrl, int ph, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  const int64_t js = ctrl->sel_count[ph] > 0 ? (int64_t)first[0] : -1;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < d;
       j += (int64_t)gridDim.x * 256)
    w[j] = (js < 0 || j == js) ? 0.0 : 1.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->bl_first[ph] = js;
}

__global__ void __launch_bounds__(1024)
bl_merge(const int32_t *__restrict__ tmp, int32_t *__restrict__ out,
         int with_subset, Ctrl *ctrl, int ph, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  const int64_t js = ctrl->bl_first[ph];
  const int64_t c2 = with_subset ? ctrl->sel_count[ph] : 0;
  __syncthreads();
  if (js < 0) {
    if (threadIdx.x == 0) ctrl->sel_count[ph] = 0;
    return;
  }
  int64_t below = 0;
  for (int64_t a = threadIdx.x; a < c2; a += 1024) {
    const int32_t v = tmp[a];
    out[a + (v > js ? 1 : 0)] = v;
    below += v < js;
  }
  __shared__ int64_t sh64[1024 / WAVE];
  below = block_sum_i64<1024>(below, sh64);
  if (threadIdx.x == 0) {
    out[below] = (int32_t)js;
    ctrl->sel_count[ph] = c2 + 1;
  }
}

template <typename T>
void launch_select_block_law(const T *eps, int64_t d, int64_t s, double floor,
                             uint64_t seed, uint64_t key1, uint32_t phase,
                             uint32_t sys, int ph, SelectScratch &sc,
                             double *w, int32_t *tmp, int32_t *out,
                             Ctrl *ctrl, int respect_done, hipStream_t st) {
  launch_select<T>(eps, d, 1, floor, seed, key1, phase, sys, ph, sc, out, ctrl,
                   respect_done, st);
  unsigned g = (unsigned)((d + 255) / 256);
  if (g > 1024) g = 1024;
  hipLaunchKernelGGL(bl_weights, dim3(g > 0 ? g : 1), dim3(256), 0, st, d, out,
                     w, ctrl, ph, respect_done);
  const int with_subset = s > 1 ? 1 : 0;
  if (with_subset)
    launch_select<double>(w, d, s - 1, 0.0, seed, key1, phase + 2, sys, ph, sc,
                          tmp, ctrl, respect_done, st);
  hipLaunchKernelGGL(bl_merge, dim3(1), dim3(1024), 0, st, tmp, out,
                     with_subset, ctrl, ph, respect_done);
}
template void launch_select_block_law<double>(const double *, int64_t, int64_t,
                                              double, uint64_t, uint64_t,
                                              uint32_t, uint32_t, int,
                                              SelectScratch &, double *,
                                              int32_t *, int32_t *, Ctrl *,
                                              int, hipStream_t);
template void launch_select_block_law<float>(const float *, int64_t, int64_t,
                                             double, uint64_t, uint64_t,
                                             uint32_t, uint32_t, int,
                                             SelectScratch &, double *,
                                             int32_t *, int32_t *, Ctrl *,
                                             int, hipStream_t);

// ------------------------------------------------ greedy (GDBEK) sets
// GDBEK's threshold sets (Section 2): {j : eps_j >= eta * max eps, eps_j > 0}
// in ascending order, at most `cap` of them (the lowest indices when more
// pass).  Three launches, no atomics: per-chunk maxima; per-chunk counts
// (every block re-reduces the maxima in the same order); ordered writes from
// per-chunk offsets.  The comparison is one FP64 product and compare, as in
// the oracle, so the set is bit-exact.
constexpr int GR_NT = 256;
constexpr int GR_PT = 16;                       // weights per thread
constexpr int64_t GR_CH = (int64_t)GR_NT * GR_PT;

template <typename T>
__global__ void __launch_bounds__(GR_NT)
gr_max(const T *__restrict__ eps, int64_t d, double *__restrict__ pmax,
       Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  __shared__ double sh[GR_NT / WAVE];
  const int64_t base = (int64_t)blockIdx.x * GR_CH;
  double mx = 0.0;
#pragma unroll
  for (int q = 0; q < GR_PT; ++q) {
    const int64_t j = base + (int64_t)q * GR_NT + threadIdx.x;
    if (j < d) {
      const double e = (double)eps[j];
      if (e <= 1.7976931348623157e308) mx = e > mx ? e : mx;
    }
  }
  mx = wave_max(mx);
  if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < GR_NT / WAVE; ++i) mx = sh[i] > mx ? sh[i] : mx;
    pmax[blockIdx.x] = mx;
  }
}

__device__ __forceinline__ double gr_threshold(const double *pmax, int nb,
                                               double eta, double *sh) {
  double gm = 0.0;
  for (int b = threadIdx.x; b < nb; b += GR_NT) gm = pmax[b] > gm ? pmax[b] : gm;
  gm = wave_max(gm);
  __syncthreads();
  if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE] = gm;
  __syncthreads();
  gm = 0.0;
  for (int i = 0; i < GR_NT / WAVE; ++i) gm = sh[i] > gm ? sh[i] : gm;
  return gm > 0.0 ? eta * gm : -1.0;    // -1: every weight is zero
}

__device__ __forceinline__ bool gr_take(double e, double thr) {
  return thr >= 0.0 && e > 0.0 && e >= thr;
}

template <typename T>
__global__ void __launch_bounds__(GR_NT)
gr_count(const T *__restrict__ eps, int64_t d, double eta,
         const double *__restrict__ pmax, int32_t *__restrict__ blk,
         Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  __shared__ double sh[GR_NT / WAVE];
  __shared__ int64_t sh64[GR_NT / WAVE];
  const double thr = gr_threshold(pmax, (int)gridDim.x, eta, sh);
  const int64_t base = (int64_t)blockIdx.x * GR_CH;
  int64_t c = 0;
  int bad = 0;
#pragma unroll
  for (int q = 0; q < GR_PT; ++q) {
    const int64_t j = base + (int64_t)q * GR_NT + threadIdx.x;
    if (j < d) {
      const double e = (double)eps[j];
      if (!(e >= 0.0) || e > 1.7976931348623157e308) bad = 1;
      c += gr_take(e, thr);
    }
  }
  if (bad) atomicOr(&ctrl->numeric, 1);
  c = block_sum_i64<GR_NT>(c, sh64);
  if (threadIdx.x == 0) blk[blockIdx.x] = (int32_t)c;
}

template <typename T>
__global__ void __launch_bounds__(GR_NT)
gr_write(const T *__restrict__ eps, int64_t d, double eta, int64_t cap,
         const double *__restrict__ pmax, const int32_t *__restrict__ blk,
         int32_t *__restrict__ out, Ctrl *ctrl, int ph, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  __shared__ double sh[GR_NT / WAVE];
  __shared__ int64_t sh64[GR_NT / WAVE];
  __shared__ int wtot[GR_NT / WAVE];
  const double thr = gr_threshold(pmax, (int)gridDim.x, eta, sh);
  int64_t before = 0, total = 0;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += GR_NT) {
    total += blk[b];
    if (b < (int)blockIdx.x) before += blk[b];
  }
  before = block_sum_i64<GR_NT>(before, sh64);
  total = block_sum_i64<GR_NT>(total, sh64);
  const int64_t base = (int64_t)blockIdx.x * GR_CH;
  int64_t off = before;
  for (int q = 0; q < GR_PT; ++q) {
    const int64_t j = base + (int64_t)q * GR_NT + threadIdx.x;
    const bool f = j < d && gr_take((double)eps[j], thr);
    const uint64_t mask = __ballot(f);
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    __syncthreads();
    if (lane == 0) wtot[wv] = __popcll(mask);
    __syncthreads();
    int wb = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < GR_NT / WAVE; ++i) {
      if (i < wv) wb += wtot[i];
      tot += wtot[i];
    }
    const int64_t r = off + wb + __popcll(mask & ((1ull << lane) - 1ull));
    if (f && r < cap) out[r] = (int32_t)j;
    off += tot;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0)
    ctrl->sel_count[ph] = total < cap ? total : cap;
}

template <typename T>
void launch_select_greedy(const T *eps, int64_t d, double eta, int64_t cap,
                          int ph, SelectScratch &s, int32_t *out, Ctrl *ctrl,
                          int respect_done, hipStream_t st) {
  const int nb = (int)((d + GR_CH - 1) / GR_CH);
  const unsigned g = (unsigned)(nb > 0 ? nb : 1);
  hipLaunchKernelGGL(gr_max<T>, dim3(g), dim3(GR_NT), 0, st, eps, d, s.gmax,
                     ctrl, respect_done);
  hipLaunchKernelGGL(gr_count<T>, dim3(g), dim3(GR_NT), 0, st, eps, d, eta,
                     s.gmax, s.blk, ctrl, respect_done);
  hipLaunchKernelGGL(gr_write<T>, dim3(g), dim3(GR_NT), 0, st, eps, d, eta,
                     cap, s.gmax, s.blk, out, ctrl, ph, respect_done);
}
template void launch_select_greedy<double>(const double *, int64_t, double,
                                           int64_t, int, SelectScratch &,
                                           int32_t *, Ctrl *, int, hipStream_t);
template void launch_select_greedy<float>(const float *, int64_t, double,
                                          int64_t, int, SelectScratch &,
                                          int32_t *, Ctrl *, int, hipStream_t);
int64_t select_greedy_blocks(int64_t d) { return (d + GR_CH - 1) / GR_CH; }

// ------------------------------------------------ draws with replacement
// k independent draws from P(j) = eps_j / sum eps, the distinct indices kept
// in ascending order.  Integer weights w_j = floor(eps_j / max eps * 2^sh)
// (one FP64 division, an exact scaling and an exact floor), zero at or below
// floor * max eps, with sh = 63 - ceil(log2 d): the total W stays below
// 2^63 and every cumulative sum is exact in any order.  Draw t takes the
// Philox word u_t of index t in the stream of phase + 4, r_t =
// floor(u_t W / 2^64), and the index j with P_(j-1) <= r_t < P_j.  Five
// launches, no float atomics: chunk maxima (gr_max); integer weights with
// in-chunk inclusive sums and chunk totals; the draws (the chunk by a binary
// search over the chunk prefix held in LDS, then a binary search inside the
// chunk) set one flag per drawn index; per-chunk flag counts; ordered
// writes that also clear the flags for the next call.
constexpr int ID_NT = GR_NT;
constexpr int ID_PT = GR_PT;                    // consecutive weights per thread
constexpr int64_t ID_CH = GR_CH;                // chunk = gr_max's chunk
constexpr int ID_MAXCH = 4096;                  // chunks: d <= 16M
constexpr int ID_DRAW_NT = 256;

__device__ __forceinline__ double id_gmax(const double *pmax, int nb,
                                          double *sh) {
  double gm = 0.0;
  for (int b = threadIdx.x; b < nb; b += ID_NT) gm = pmax[b] > gm ? pmax[b] : gm;
  gm = wave_max(gm);
  __syncthreads();
  if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE] = gm;
  __syncthreads();
  gm = 0.0;
  for (int i = 0; i < ID_NT / WAVE; ++i) gm = sh[i] > gm ? sh[i] : gm;
  return gm;
}

// exclusive scan of one uint64 per thread over the block; *tot = the sum
__device__ __forceinline__ uint64_t id_scan(uint64_t v, uint64_t *sh,
                                            uint64_t *tot) {
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  uint64_t inc = v;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const uint64_t u = __shfl_up(inc, o, WAVE);
    if (lane >= o) inc += u;
  }
  __syncthreads();
  if (lane == WAVE - 1) sh[wv] = inc;
  __syncthreads();
  uint64_t before = 0, all = 0;
  for (int i = 0; i < (int)(blockDim.x / WAVE); ++i) {
    if (i < wv) before += sh[i];
    all += sh[i];
  }
  *tot = all;
  return before + inc - v;
}

template <typename T>
__global__ void __launch_bounds__(ID_NT)
id_weights(const T *__restrict__ eps, int64_t d, double flr, double scale,
           const double *__restrict__ pmax, uint64_t *__restrict__ ploc,
           uint64_t *__restrict__ ctot, Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  __shared__ double sh[ID_NT / WAVE];
  __shared__ uint64_t shu[ID_NT / WAVE];
  const double gm = id_gmax(pmax, (int)gridDim.x, sh);
  const double cut = flr * gm;
  const int64_t j0 = (int64_t)blockIdx.x * ID_CH + (int64_t)threadIdx.x * ID_PT;
  uint64_t w[ID_PT];
  uint64_t acc = 0;
  int bad = 0;
#pragma unroll
  for (int q = 0; q < ID_PT; ++q) {
    const int64_t j = j0 + q;
    uint64_t v = 0;
    if (j < d) {
      const double e = (double)eps[j];
      if (!(e >= 0.0) || e > 1.7976931348623157e308) bad = 1;
      else if (gm > 0.0 && e > cut) v = (uint64_t)__builtin_floor((e / gm) * scale);
    }
    acc += v;
    w[q] = acc;                                  // in-thread inclusive sums
  }
  if (bad) atomicOr(&ctrl->numeric, 1);
  uint64_t tot;
  const uint64_t before = id_scan(acc, shu, &tot);
#pragma unroll
  for (int q = 0; q < ID_PT; ++q)
    if (j0 + q < d) ploc[j0 + q] = before + w[q];
  if (threadIdx.x == 0) ctot[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(ID_DRAW_NT)
id_draw(int64_t k, int64_t d, int nb, uint64_t seed, uint64_t key1,
        uint32_t phase, uint32_t sys, const uint64_t *__restrict__ ploc,
        const uint64_t *__restrict__ ctot, int32_t *__restrict__ flags,
        Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  __shared__ uint64_t cp[ID_MAXCH];
  __shared__ uint64_t shu[ID_DRAW_NT / WAVE];
  // inclusive prefix of the chunk totals: consecutive runs per thread
  const int per = (nb + ID_DRAW_NT - 1) / ID_DRAW_NT;
  const int b0 = threadIdx.x * per;
  uint64_t run = 0;
  for (int i = 0; i < per; ++i)
    if (b0 + i < nb) run += ctot[b0 + i];
  uint64_t all;
  uint64_t pre = id_scan(run, shu, &all);
  for (int i = 0; i < per; ++i)
    if (b0 + i < nb) { pre += ctot[b0 + i]; cp[b0 + i] = pre; }
  __syncthreads();
  const uint64_t W = all;
  if (W == 0) return;
  const uint64_t it = (uint64_t)ctrl->it;
  for (int64_t t = (int64_t)blockIdx.x * ID_DRAW_NT + threadIdx.x; t < k;
       t += (int64_t)gridDim.x * ID_DRAW_NT) {
    const P4 rw = philox4x64_10((uint64_t)(t >> 2), it, phase, sys, seed, key1);
    const int q = (int)(t & 3);                        // no dynamic index
    const uint64_t u = q == 0 ? rw.v[0] : q == 1 ? rw.v[1] : q == 2 ? rw.v[2] : rw.v[3];
    const uint64_t r = __umul64hi(u, W);               // r < W
    int lo = 0, hi = nb - 1;                         // first chunk with cp > r
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (cp[mid] > r) hi = mid; else lo = mid + 1;
    }
    const uint64_t r2 = r - (lo ? cp[lo - 1] : 0ull);
    int64_t a = (int64_t)lo * ID_CH;
    int64_t b = a + ID_CH < d ? a + ID_CH - 1 : d - 1;  // ploc[b] = chunk total > r2
    while (a < b) {
      const int64_t mid = (a + b) >> 1;
      if (ploc[mid] > r2) b = mid; else a = mid + 1;
    }
    flags[a] = 1;
  }
}

__global__ void __launch_bounds__(ID_NT)
id_count(const int32_t *__restrict__ flags, int64_t d,
         int32_t *__restrict__ blk, Ctrl *ctrl, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  __shared__ int64_t sh64[ID_NT / WAVE];
  const int64_t base = (int64_t)blockIdx.x * ID_CH;
  int64_t c = 0;
#pragma unroll
  for (int q = 0; q < ID_PT; ++q) {
    const int64_t j = base + (int64_t)q * ID_NT + threadIdx.x;
    if (j < d) c += flags[j] != 0;
  }
  c = block_sum_i64<ID_NT>(c, sh64);
  if (threadIdx.x == 0) blk[blockIdx.x] = (int32_t)c;
}

__global__ void __launch_bounds__(ID_NT)
id_write(int32_t *__restrict__ flags, int64_t d,
         const int32_t *__restrict__ blk, int32_t *__restrict__ out,
         Ctrl *ctrl, int ph, int respect_done) {
  if (respect_done && ctrl_done(ctrl)) return;
  __shared__ int64_t sh64[ID_NT / WAVE];
  __shared__ int wtot[ID_NT / WAVE];
  int64_t before = 0, total = 0;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += ID_NT) {
    total += blk[b];
    if (b < (int)blockIdx.x) before += blk[b];
  }
  before = block_sum_i64<ID_NT>(before, sh64);
  total = block_sum_i64<ID_NT>(total, sh64);
  const int64_t base = (int64_t)blockIdx.x * ID_CH;
  int64_t off = before;
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  for (int q = 0; q < ID_PT; ++q) {
    const int64_t j = base + (int64_t)q * ID_NT + threadIdx.x;
    const bool f = j < d && flags[j] != 0;
    const uint64_t mask = __ballot(f);
    __syncthreads();
    if (lane == 0) wtot[wv] = __popcll(mask);
    __syncthreads();
    int wb = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < ID_NT / WAVE; ++i) {
      if (i < wv) wb += wtot[i];
      tot += wtot[i];
    }
    if (f) {
      out[off + wb + __popcll(mask & ((1ull << lane) - 1ull))] = (int32_t)j;
      flags[j] = 0;
    }
    off += tot;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->sel_count[ph] = total;
}

int64_t select_iid_chunks(int64_t d) { return (d + ID_CH - 1) / ID_CH; }
int64_t select_iid_max_d() { return (int64_t)ID_MAXCH * ID_CH; }

template <typename T>
void launch_select_iid(const T *eps, int64_t d, int64_t k, double floor,
                       uint64_t seed, uint64_t key1, uint32_t phase,
                       uint32_t sys, int ph, SelectScratch &s, IidScratch &w,
                       int32_t *out, Ctrl *ctrl, int respect_done,
                       hipStream_t st) {
  const int nb = (int)select_iid_chunks(d);
  int sh = 63;
  while (sh > 0 && (((int64_t)1) << (63 - sh)) < d) --sh;   // 63 - ceil(log2 d)
  const double scale = std::ldexp(1.0, sh);
  hipLaunchKernelGGL(gr_max<T>, dim3(nb), dim3(GR_NT), 0, st, eps, d, s.gmax,
                     ctrl, respect_done);
  hipLaunchKernelGGL(id_weights<T>, dim3(nb), dim3(ID_NT), 0, st, eps, d,
                     floor, scale, s.gmax, w.ploc, w.ctot, ctrl, respect_done);
  int64_t g = (k + ID_DRAW_NT - 1) / ID_DRAW_NT;
  if (g > 1024) g = 1024;
  hipLaunchKernelGGL(id_draw, dim3((unsigned)(g > 0 ? g : 1)), dim3(ID_DRAW_NT),
                     0, st, k > 0 ? k : 0, d, nb, seed, key1, phase + 4u, sys,
                     w.ploc, w.ctot, w.flags, ctrl, respect_done);
  hipLaunchKernelGGL(id_count, dim3(nb), dim3(ID_NT), 0, st, w.flags, d, s.blk,
                     ctrl, respect_done);
  hipLaunchKernelGGL(id_write, dim3(nb), dim3(ID_NT), 0, st, w.flags, d, s.blk,
                     out, ctrl, ph, respect_done);
}
template void launch_select_iid<double>(const double *, int64_t, int64_t,
                                        double, uint64_t, uint64_t, uint32_t,
                                        uint32_t, int, SelectScratch &,
                                        IidScratch &, int32_t *, Ctrl *, int,
                                        hipStream_t);
template void launch_select_iid<float>(const float *, int64_t, int64_t, double,
                                       uint64_t, uint64_t, uint32_t, uint32_t,
                                       int, SelectScratch &, IidScratch &,
                                       int32_t *, Ctrl *, int, hipStream_t);

// ------------------------------------------------ launcher
template <typename T>
void launch_select(const T *eps, int64_t d, int64_t k, double floor,
                   uint64_t seed, uint64_t key1, uint32_t phase, uint32_t sys,
                   int ph, SelectScratch &s, int32_t *out, Ctrl *ctrl,
                   int respect_done, hipStream_t st) {
  int kpt = 0, grid = 0;
  if (s.pers && d >= SP_MIN_D) sel_persist_shape(d, s.ncu, &kpt, &grid);
  if (kpt == 4) {
    hipLaunchKernelGGL((sel_persist_kernel<T, 4>), dim3(grid), dim3(SP_NT), 0,
                       st, eps, d, k, floor, seed, key1, phase, sys, ph,
                       s.pers, out, ctrl, respect_done);
    return;
  }
  if (kpt == 16) {
    hipLaunchKernelGGL((sel_persist_kernel<T, 16>), dim3(grid), dim3(SP_NT),
                       0, st, eps, d, k, floor, seed, key1, phase, sys, ph,
                       s.pers, out, ctrl, respect_done);
    return;
  }
  if (d <= SEL_SMALL_MAX) {
    hipLaunchKernelGGL(sel_small<T>, dim3(1), dim3(1024), 0, st, eps, d, k,
                       floor, seed, key1, ph, phase, sys, s.keys, out, ctrl,
                       respect_done);
    return;
  }
  const int nb = (int)((d + SEL_CHUNK - 1) / SEL_CHUNK);
  hipLaunchKernelGGL(sel_max<T>, dim3(nb), dim3(SEL_NT), 0, st, eps, d, ctrl,
                     ph, respect_done);
  hipLaunchKernelGGL(sel_keys_hist<T>, dim3(nb), dim3(SEL_NT), 0, st, eps, d,
                     floor, seed, key1, phase, sys, s.keys, s.hist, ctrl, ph,
                     respect_done);
  hipLaunchKernelGGL(sel_scan, dim3(1), dim3(SEL_NT), 0, st, s.hist, k, ctrl,
                     ph, 1, respect_done);
  hipLaunchKernelGGL(sel_hist, dim3(nb), dim3(SEL_NT), 0, st, s.keys, d,
                     s.hist, ctrl, ph, respect_done);
  hipLaunchKernelGGL(sel_scan, dim3(1), dim3(SEL_NT), 0, st, s.hist, k, ctrl,
                     ph, 0, respect_done);
  hipLaunchKernelGGL(sel_gather, dim3(nb), dim3(SEL_NT), 0, st, s.keys, d,
                     s.ckey, s.cidx, ctrl, ph, respect_done);
  hipLaunchKernelGGL(sel_resolve, dim3(1), dim3(SEL_NT), 0, st, s.keys, d,
                     s.ckey, s.cidx, ctrl, ph, respect_done);
  hipLaunchKernelGGL(sel_count, dim3(nb), dim3(SEL_NT), 0, st, s.keys, d,
                     s.blk, ctrl, ph, respect_done);
  hipLaunchKernelGGL(sel_write, dim3(nb), dim3(SEL_NT), 0, st, s.keys, d,
                     s.blk, out, ctrl, ph, respect_done);
}

template void launch_select<double>(const double *, int64_t, int64_t, double,
                                    uint64_t, uint64_t, uint32_t, uint32_t,
                                    int, SelectScratch &, int32_t *, Ctrl *,
                                    int, hipStream_t);
template void launch_select<float>(const float *, int64_t, int64_t, double,
                                   uint64_t, uint64_t, uint32_t, uint32_t, int,
                                   SelectScratch &, int32_t *, Ctrl *, int,
                                   hipStream_t);

int64_t select_scratch_blocks(int64_t d) {
  return (d + SEL_CHUNK - 1) / SEL_CHUNK;
}

template <typename T>
void launch_select_seg(const T *eps, const SegInfo *seg, int nseg, int ph,
                       int64_t dmax, double floor, uint64_t seed,
                       uint64_t key1, uint32_t phase, uint64_t *keys,
                       double *segmax, int32_t *tmp, int64_t *cnt,
                       int32_t *out, Ctrl *ctrl, int respect_done,
                       hipStream_t st) {
  hipLaunchKernelGGL(sel_seg_max<T>, dim3(nseg), dim3(256), 0, st, eps, seg,
                     ph, segmax, ctrl, respect_done);
  const unsigned gx = (unsigned)((dmax + 4 * 256 - 1) / (4 * 256));
  hipLaunchKernelGGL(sel_seg_keys<T>, dim3(gx > 0 ? gx : 1, nseg), dim3(256),
                     0, st, eps, seg, ph, floor, seed, key1, phase, segmax,
                     keys, ctrl, respect_done);
  hipLaunchKernelGGL(sel_seg_resolve, dim3(nseg), dim3(WG_NT), 0, st, seg, ph,
                     keys, tmp, cnt, ctrl, respect_done);
  hipLaunchKernelGGL(sel_seg_pack, dim3(nseg), dim3(256), 0, st, seg, nseg, ph,
                     tmp, cnt, out, ctrl, respect_done);
}
template void launch_select_seg<double>(const double *, const SegInfo *, int,
                                        int, int64_t, double, uint64_t,
                                        uint64_t, uint32_t, uint64_t *,
                                        double *, int32_t *, int64_t *,
                                        int32_t *, Ctrl *, int, hipStream_t);
template void launch_select_seg<float>(const float *, const SegInfo *, int,
                                       int, int64_t, double, uint64_t,
                                       uint64_t, uint32_t, uint64_t *,
                                       double *, int32_t *, int64_t *,
                                       int32_t *, Ctrl *, int, hipStream_t);

}  // namespace rg
