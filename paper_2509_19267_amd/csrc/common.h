// Shared device helpers for the RGDBEK kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rg {

constexpr int WAVE = 64;

// Device-wide control block of one solve.  Lives in device memory; every
// kernel of an iteration reads `done` first and returns when it is set, so a
// captured graph of several iterations becomes a no-op after the stop test.
struct Ctrl {
  int64_t it;          // generator iteration counter of the current iteration
  int64_t it_end;      // iterations stop when it reaches it_end
  int64_t iters_run;   // iterations completed in this solve
  int32_t done;        // 1: stop test held or cap reached -> skip all work
  int32_t converged;   // 1: stop test held
  int32_t numeric;     // 1: NaN/negative/Inf weight met
  int32_t stop_mode;   // RGDBEK_STOP_* of the running solve
  double tol;          // tolerance of the stop test
  double ref2;         // ||x_ref||^2 or ||b||^2 (denominator of the test)
  double metric;       // last evaluated stop metric
  // refinement passes of the mixed form: a residual test (RSE/RES_EXT) also
  // holds once metric <= pass_drop * pass_ref, pass_ref being the first
  // metric the pass evaluated (pass_drop 0: off)
  double pass_drop;
  double pass_ref;
  // block selection state (one per phase: 0 = columns, 1 = rows)
  int64_t sel_count[2];   // indices selected
  int64_t sel_pos[2];     // positive weights seen
  int64_t sel_krem[2];    // remaining rank inside the current radix bucket
  uint64_t sel_prefix[2]; // resolved high bits of the threshold key
  int32_t sel_shift[2];   // bits still unresolved below the prefix
  int32_t sel_mode[2];    // 0 radix, 1 all positives, 2 resolved, 3 fallback
  uint64_t sel_tkey[2];   // threshold key (k-th smallest)
  int64_t sel_tidx[2];    // threshold index (ties broken by index)
  int64_t sel_cand[2];    // candidates gathered for the final sort
  uint64_t sel_maxbits[2]; // bits of the largest weight (non-negative)
  int64_t bl_first[2];    // block law: the weighted index (-1: none)
  // inner solver state (one per phase)
  double cg_rz[2], cg_rz0[2], cg_alpha[2], cg_beta[2];
  int32_t cg_done[2], cg_steps[2];
  uint64_t sel_bar[2];    // grid-barrier arrivals of the persistent selection
  uint64_t sel_barbase[2];
  uint64_t cg_bar[2];     // grid-barrier arrivals of the persistent PCG
  uint64_t cg_barbase[2]; // arrivals completed by earlier launches
  int32_t sync_fail;      // a grid-barrier wait timed out
  int32_t pad0;
  unsigned ticket[8];     // last-block tickets (reset by the last block)
};

// Per-system state of a batch of independent systems stored block-diagonally
// (system s owns rows [row_off, row_off + nrow) and columns [col_off,
// col_off + ncol)).  Block sizes kc/kr; kc_off/kr_off: offsets of the
// system's slots in the per-phase draw scratch.
struct SegInfo {
  int64_t row_off, nrow, col_off, ncol;
  int64_t kc, kr, kc_off, kr_off;
  int64_t it;          // generator iteration counter of this system
  int64_t iters_run;   // iterations this system has run in the solve
  int32_t done;        // 1: this system stopped (tested or capped)
  int32_t converged;
  double metric;
  double ref2;
  double pref;         // first residual metric of a refinement pass
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double w = __shfl_xor(v, o, WAVE);
    v = w > v ? w : v;
  }
  return v;
}
__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}
// Sum within aligned groups of G lanes (G a power of two <= 64).
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// Block-wide sum, fixed order (waves reduced by shuffles, then wave partials
// summed in wave order by every thread).  `sh` needs NT/64 doubles.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *sh) {
  v = wave_sum(v);
  const int w = threadIdx.x / WAVE;
  __syncthreads();
  if ((threadIdx.x & (WAVE - 1)) == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NT / WAVE; ++i) s += sh[i];
  return s;
}
template <int NT>
__device__ __forceinline__ int64_t block_sum_i64(int64_t v, int64_t *sh) {
  v = wave_sum_i64(v);
  const int w = threadIdx.x / WAVE;
  __syncthreads();
  if ((threadIdx.x & (WAVE - 1)) == 0) sh[w] = v;
  __syncthreads();
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < NT / WAVE; ++i) s += sh[i];
  return s;
}

// Agent-scope (device-wide) relaxed accesses for values exchanged between
// blocks of one launch.
template <typename T>
__device__ __forceinline__ void st_agent(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_agent(const T *p) {
  return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// "Last block" election: every thread releases its prior global writes at
// agent scope, thread 0 takes a ticket, and the block that takes the final
// ticket acquires them and returns true (and re-arms the ticket).
__device__ __forceinline__ bool last_block(unsigned *ticket) {
  __shared__ int is_last;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned nb = gridDim.x * gridDim.y * gridDim.z;
    unsigned t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL,
                                        __HIP_MEMORY_SCOPE_AGENT);
    is_last = (t == nb - 1);
    if (is_last)
      __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  if (is_last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return is_last != 0;
}

// Flags tested once at a kernel's start (Ctrl::done, the CG's done flag of
// a phase), written only by earlier launches of the stream: kernel
// boundaries order and publish those writes, so a plain load suffices.  It
// is uniform and takes the scalar cache, and the many workgroups of a
// launch with nothing left to do (a captured CG step after the CG has met
// its tolerance) leave without each waiting on an L2 round trip.
__device__ __forceinline__ bool ctrl_done(const Ctrl *c) {
  return c->done != 0;
}
__device__ __forceinline__ bool cg_done_at_start(const Ctrl *c, int ph) {
  return c->cg_done[ph] != 0;
}

// Grid barrier of a persistent launch (every workgroup resident): arrivals
// are counted in a 64-bit counter that only grows; barrier number b of a
// launch completes when the counter reaches base + b * gridDim.x.  Thread 0
// releases the workgroup's writes at agent scope, arrives, polls, and
// acquires.  Polls are bounded (GRID_SPIN_MAX, seconds): a timed-out wait
// sets *fail, which also ends the waits of the other workgroups, so the
// launch always drains.
constexpr int64_t GRID_SPIN_MAX = 1ll << 22;
// Arrive at barrier number `target` (counter value after every workgroup
// arrived); returns false after a timed-out wait.
__device__ __forceinline__ bool grid_barrier(uint64_t *ctr, uint64_t target,
                                             int32_t *fail) {
  __shared__ int s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(ctr, (uint64_t)1, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    int64_t spins = 0;
    int ok = 1;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
           target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > GRID_SPIN_MAX || ld_agent(fail) != 0) { ok = 0; break; }
    }
    if (!ok) st_agent(fail, 1);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}


}  // namespace rg
