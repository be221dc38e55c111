// Host runtime of the RGDBEK solver: handle lifecycle, device storage, the
// per-iteration kernel sequence of Algorithm 1, HIP-graph capture of several
// iterations at a time, the FP64 refinement loop of the mixed-precision form,
// and the C-ABI entry points declared in include/rgdbek.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <string>
#include <vector>

#include "../../include/rgdbek.h"
#include "common.h"
#include "kernels.h"

using namespace rg;

namespace {

struct HipError {
  hipError_t e;
  const char *what;
};
struct ApiError {
  rgdbek_status s;
  std::string msg;
};

#define HIPCHK(x)                                 \
  do {                                            \
    hipError_t _e = (x);                          \
    if (_e != hipSuccess) throw HipError{_e, #x}; \
  } while (0)

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

int pick_group(double mean_len) {
  int g = 1;
  while (g < 64 && g < mean_len * 0.5) g <<= 1;
  return g;
}

// Device allocation list owned by a handle.
// Nonzero-balanced chunking of one CSR (see Csr::mp_*), device arrays.
struct MergePlan {
  int32_t *rs = nullptr;                 // nchunk + 1 owned-row starts
  int32_t *xrow = nullptr, *xcs = nullptr, *xce = nullptr;
  int64_t nchunk = 0, ncross = 0;
};

struct Pool {
  std::vector<void *> ptrs;
  hipStream_t st = nullptr;   // zero-fills are ordered on this stream
  template <typename T>
  T *alloc(int64_t count, bool zero = true) {
    if (count <= 0) count = 1;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, sizeof(T) * (size_t)count);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw ApiError{RGDBEK_ERR_OUT_OF_MEMORY,
                     "device allocation of " +
                         std::to_string(sizeof(T) * (size_t)count) +
                         " bytes failed"};
    }
    ptrs.push_back(p);
    if (zero) HIPCHK(hipMemsetAsync(p, 0, sizeof(T) * (size_t)count, st));
    return (T *)p;
  }
  void release() {
    for (void *p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

// Work space and matrix views of one arithmetic precision.
template <typename T>
struct Engine {
  bool ready = false;
  bool dense = false;
  int64_t m = 0, n = 0, kc = 0, kr = 0;
  Dense<T> arm, acm;          // row-major A (ld), column-major A (ldc)
  Csr<T> csr, csc;
  const T *ata = nullptr, *aat = nullptr;  // precomputed Grams (nullable)
  bool sgram = false;         // sparse A projected through the Grams
  const double *rho = nullptr, *kappa = nullptr;
  // vectors
  T *x = nullptr, *z = nullptr, *b = nullptr, *q = nullptr, *g = nullptr;
  T *r = nullptr, *eps_x = nullptr, *eps_z = nullptr, *off = nullptr;
  int32_t *U = nullptr, *J = nullptr;
  // dense block work
  DenseWork<T> dw;
  T *GU = nullptr, *GJ = nullptr, *y = nullptr, *w = nullptr, *s = nullptr;
  T *upd = nullptr;
  CgWork<T> cgc, cgr;
  // sparse block work
  SparseCg<T> scc, scr;
  TallWork<T> tall;          // row blocks taller than A is wide (CGLS)
  SubWork subc, subr;        // block-restricted CSR (columns U) / CSC (rows J)
  bool tall_rows = false;
  SelectScratch sel;
  Reduce red;
  double *part = nullptr;     // row-residual partials
  double floor = 0.0;         // relative weight floor of the block draws
  int32_t *seltmp = nullptr;  // per-system draws before packing (batch)
  double *segmax = nullptr;   // per-system largest weight (batch)
  double *blw = nullptr;      // block law: unit weights of the subset draw
  int32_t *bltmp = nullptr;   // block law: the subset before the merge
  IidScratch iid;             // draws with replacement
  int64_t seg_dmax[2] = {0, 0};  // largest system dimension per phase
  int64_t *selcnt = nullptr;  // per-system draw counts (batch)
  int nseg = 0;               // systems (0: a single system)
  SegInfo *seg = nullptr;
};

}  // namespace

struct rgdbek_ctx {
  int64_t m = 0, n = 0, nnz = 0;
  bool dense = false;
  rgdbek_params p{};
  int64_t kc = 0, kr = 0;
  int ncu = 256;                  // compute units of the device
  hipStream_t user_st = nullptr;  // caller's stream (inputs are ordered on it)
  hipStream_t st = nullptr;       // the stream all work is enqueued on
  bool own_stream = false;        // st was created by the handle
  std::string err;
  Pool pool;
  // FP64 storage
  double *a_rm = nullptr, *a_cm = nullptr;
  int64_t ld = 0, ldc = 0;
  int64_t *csr_ptr = nullptr, *csc_ptr = nullptr;
  int32_t *csr_idx = nullptr, *csc_idx = nullptr;
  double *csr_val = nullptr, *csc_val = nullptr;
  int32_t *csr_longs = nullptr, *csc_longs = nullptr;
  int64_t csr_nlong = 0, csc_nlong = 0;
  MergePlan csr_mp, csc_mp;   // nonzero-balanced full-pass plans
  double *rho = nullptr, *kappa = nullptr;
  Engine<double> e64;
  Engine<double> e64t;        // adjoint system (A^T), built on demand
  Engine<float> e32;          // inner engine of the mixed form
  Ctrl *ctrl = nullptr;
  Ctrl *hctrl = nullptr;      // pinned host mirror
  // batch of independent systems (block-diagonal storage); nseg == 0 for a
  // single system
  int nseg = 0;
  SegInfo *seg = nullptr;     // per-system state, forward engines
  SegInfo *seg_t = nullptr;   // per-system state, adjoint engine
  std::vector<SegInfo> hseg;
  int64_t rep = 1;            // right-hand sides sharing one stored A
  int64_t bm = 0, bn = 0;     // stored (base) dimensions of A
  int32_t *fixed = nullptr;   // systems accepted by an FP64 test (mixed form)
  double *xref = nullptr, *x64 = nullptr, *z64 = nullptr, *zero64 = nullptr,
         *t64 = nullptr;
  // captured graphs, keyed by (engine, key1, stop)
  struct GraphEntry {
    int which = 0;
    uint64_t key1 = 0;
    int stop = 0;
    int use_xref = 0;
    int with_base = 0;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
  };
  std::vector<GraphEntry> graphs;
  // RGDBEK_FLAG_PROFILE: event-timed regions of the last solve
  struct ProfRegion {
    int cat = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
  };
  std::vector<ProfRegion> prof_regions;   // enqueued this solve
  std::vector<hipEvent_t> prof_events;    // pool, reused across solves
  size_t prof_used_events = 0;
  ProfRec *prof_log = nullptr;            // device: live flag, CG steps
  int64_t prof_cap = 0;
  struct ProfSum {
    int64_t launches = 0;
    double ms = 0.0;
    int64_t steps = 0;
  } prof[RGDBEK_PROF_COUNT];
};

static thread_local std::string g_global_err;

// RGDBEK_TRACE=1 prints one line per refinement pass / inner graph to stderr.
static bool trace_on() {
  static int v = -1;
  if (v < 0) {
    const char *e = std::getenv("RGDBEK_TRACE");
    v = (e && e[0] == '1') ? 1 : 0;
  }
  return v == 1;
}

namespace {

void set_err(rgdbek_ctx *h, const std::string &m) {
  if (h) h->err = m;
  else g_global_err = m;
}

// ------------------------------------------------------------ engine set-up
// the forward engine of precision T (the adjoint engine shares its Grams)
template <typename T> Engine<T> &forward_engine(rgdbek_ctx *h);
template <> Engine<double> &forward_engine<double>(rgdbek_ctx *h) { return h->e64; }
template <> Engine<float> &forward_engine<float>(rgdbek_ctx *h) { return h->e32; }

// Gram-block solve work (dense engines, and sparse engines small enough for
// the Gram matrices of all columns and rows).
template <typename T>
void alloc_gram_blocks(rgdbek_ctx *h, Engine<T> &e) {
  Pool &P = h->pool;
  e.GU = P.alloc<T>(e.kc * e.kc);
  if (!e.tall_rows) e.GJ = P.alloc<T>(e.kr * e.kr);
  e.y = P.alloc<T>(e.kc);
  e.w = P.alloc<T>(e.kr);
  e.s = P.alloc<T>(e.kr);
  for (CgWork<T> *cw : {&e.cgc, &e.cgr}) {
    const int64_t cap = (cw == &e.cgc) ? e.kc : e.kr;
    cw->cap = cap;
    cw->res = P.alloc<T>(cap);
    cw->p = P.alloc<T>(2 * cap);
    cw->v = P.alloc<T>(cap);
    cw->zz = P.alloc<T>(cap);
    cw->pv = P.alloc<double>(cap / 4 + 64);
    cw->part_cap = cap / 256 + 2;
    cw->part = P.alloc<double>(4 * cw->part_cap);
    cw->rzs = P.alloc<double>(2);
    cw->v2 = P.alloc<T>(2 * cap);
    cw->pv2 = P.alloc<double>(2 * pcg_persist_grid(cap, h->ncu));
  }
}

template <typename T>
void build_engine(rgdbek_ctx *h, Engine<T> &e, bool transpose) {
  Pool &P = h->pool;
  e.dense = h->dense;
  e.m = transpose ? h->n : h->m;
  e.n = transpose ? h->m : h->n;
  e.kc = transpose ? h->kr : h->kc;
  e.kr = transpose ? h->kc : h->kr;
  // row blocks with more rows than there are columns: CGLS projections
  e.tall_rows = e.kr > e.n;
  for (const SegInfo &g : h->hseg) {
    const int64_t kr = transpose ? g.kc : g.kr;
    const int64_t nc = transpose ? g.nrow : g.ncol;
    if (kr > nc) e.tall_rows = true;
  }
  const bool f64 = std::is_same<T, double>::value;
  const double wf = h->p.weight_floor;
  e.floor = wf > 0.0 ? wf : (wf < 0.0 ? 0.0 : (f64 ? 1e-20 : 1e-6));
  if (h->dense) {
    // row-major and column-major copies in precision T
    const int64_t ld = transpose ? h->ldc : h->ld;
    const int64_t ldc = transpose ? h->ld : h->ldc;
    T *rm, *cm;
    if (f64) {
      rm = (T *)(transpose ? h->a_cm : h->a_rm);
      cm = (T *)(transpose ? h->a_rm : h->a_cm);
    } else {
      rm = P.alloc<T>(e.m * ld, false);
      cm = P.alloc<T>(e.n * ldc, false);
      launch_convert<T, double>(transpose ? h->a_cm : h->a_rm, rm, e.m * ld,
                                h->st);
      launch_convert<T, double>(transpose ? h->a_rm : h->a_cm, cm, e.n * ldc,
                                h->st);
    }
    e.arm = Dense<T>{e.m, e.n, ld, rm};
    e.acm = Dense<T>{e.n, e.m, ldc, cm};
    int nch, nrg, rpw;
    dense_work_shape<T>(e.arm, h->p.tile_rows, 4 * h->ncu, &nch, &nrg, &rpw);
    e.dw.nch = nch;
    e.dw.nrg = nrg;
    e.dw.rpw = rpw;
    e.dw.qpart = P.alloc<T>((int64_t)nch * e.m);
    e.dw.gpart = P.alloc<T>((int64_t)nrg * ld);
    // Gram of all columns (A^T A) when the column blocks are large enough to
    // be worth a gather; rows: A A^T only on request.  The adjoint engine
    // (A^T) takes the forward engine's Grams with the roles swapped: its
    // columns are the rows of A.
    const T *ata = nullptr, *aat = nullptr;
    if (transpose) {
      const Engine<T> &f = forward_engine<T>(h);
      ata = f.aat;
      aat = f.ata;
    }
    // the FP64 engine of a mixed handle only runs the refinement's residual
    // passes: its block solves (a resumed solve) form their Grams from A
    const bool mixed64 = f64 && !transpose &&
                         h->p.precision == RGDBEK_PREC_MIXED_F32;
    const bool gram_cols = !mixed64 && e.kc > 64 && (ata || e.n <= 8192);
    if (gram_cols) {
      if (!ata) {
        T *F = P.alloc<T>(e.n * e.n, false);
        launch_gram_full<T>(cm, ldc, e.n, e.m, F, h->st);
        ata = F;
      }
      e.ata = ata;
    }
    const bool gram_rows = !mixed64 &&
        (aat || ((h->p.flags & RGDBEK_FLAG_GRAM_AAT) && e.m <= 32768));
    if (gram_rows) {
      if (!aat) {
        T *F = P.alloc<T>(e.m * e.m, false);
        launch_gram_full<T>(rm, ld, e.m, e.n, F, h->st);
        aat = F;
      }
      e.aat = aat;
    }
    alloc_gram_blocks(h, e);
    e.upd = P.alloc<T>(std::max(thin_update_scratch(e.m, e.kc),
                                thin_update_scratch(e.n, e.kr)));
  } else {
    // CSR / CSC views; the adjoint swaps them
    Csr<T> a, at;
    const double *vr = transpose ? h->csc_val : h->csr_val;
    const double *vc = transpose ? h->csr_val : h->csc_val;
    const T *vrT, *vcT;
    if (f64) {
      vrT = (const T *)vr;
      vcT = (const T *)vc;
    } else {
      T *t1 = P.alloc<T>(h->nnz, false), *t2 = P.alloc<T>(h->nnz, false);
      launch_convert<T, double>(vr, t1, h->nnz, h->st);
      launch_convert<T, double>(vc, t2, h->nnz, h->st);
      vrT = t1;
      vcT = t2;
    }
    a.rep = at.rep = h->rep;
    a.brows = at.bcols = transpose ? h->bn : h->bm;
    a.bcols = at.brows = transpose ? h->bm : h->bn;
    a.rows = e.m; a.cols = e.n; a.nnz = h->nnz;
    a.ptr = transpose ? h->csc_ptr : h->csr_ptr;
    a.idx = transpose ? h->csc_idx : h->csr_idx;
    a.val = vrT;
    at.rows = e.n; at.cols = e.m; at.nnz = h->nnz;
    at.ptr = transpose ? h->csr_ptr : h->csc_ptr;
    at.idx = transpose ? h->csr_idx : h->csc_idx;
    at.val = vcT;
    const double mr = a.brows ? (double)h->nnz / (double)a.brows : 1.0;
    const double mc = a.bcols ? (double)h->nnz / (double)a.bcols : 1.0;
    a.group = pick_group(mr);
    at.group = pick_group(mc);
    // the long-segment lists were built with these same limits (the
    // adjoint's rows are the forward columns and vice versa)
    a.long_limit = 32LL * a.group;
    at.long_limit = 32LL * at.group;
    a.longs = transpose ? h->csc_longs : h->csr_longs;
    a.nlong = transpose ? h->csc_nlong : h->csr_nlong;
    at.longs = transpose ? h->csr_longs : h->csc_longs;
    at.nlong = transpose ? h->csr_nlong : h->csc_nlong;
    if (h->rep == 1) {
      auto plan = [&](Csr<T> &c, const MergePlan &mp) {
        c.mp_rs = mp.rs;
        c.mp_nchunk = mp.nchunk;
        c.mp_xrow = mp.xrow;
        c.mp_xcs = mp.xcs;
        c.mp_xce = mp.xce;
        c.mp_ncross = mp.ncross;
        c.mp_head = P.alloc<T>(mp.nchunk);
        c.mp_lead = P.alloc<T>(mp.nchunk);
      };
      plan(a, transpose ? h->csc_mp : h->csr_mp);
      plan(at, transpose ? h->csr_mp : h->csc_mp);
    }
    // many right-hand sides: three interleaved buffers shared by the full
    // passes (input, product) and the CG steps (direction, two products)
    T *rb[3] = {nullptr, nullptr, nullptr};
    if (h->rep >= REP_MM_MIN) {
      const int64_t len = std::max(a.brows, a.bcols) * h->rep;
      for (int i = 0; i < 3; ++i) rb[i] = P.alloc<T>(len, false);
      a.rep_in = at.rep_in = rb[0];
      a.rep_out = at.rep_out = rb[1];
    }
    e.csr = a;
    e.csc = at;
    for (int ph = 0; ph < 2; ++ph) {
      SparseCg<T> &sc = ph == 0 ? e.scc : e.scr;
      const int64_t cap = ph == 0 ? e.kc : e.kr;
      sc.phat = P.alloc<T>(ph == 0 ? e.n : e.m);
      sc.wide = P.alloc<T>(ph == 0 ? e.m : e.n);
      sc.p = P.alloc<T>(cap);
      sc.res = P.alloc<T>(cap);
      sc.v = P.alloc<T>(2 * cap);
      const int64_t nb = std::max(e.m, e.n) / 4 + cap / 4 + 1024;
      sc.part = P.alloc<double>(nb);
      sc.part_cap = nb;
      sc.split = (h->p.flags & RGDBEK_FLAG_CG_SPLIT) ? 1 : 0;
      sc.t0 = rb[0];
      sc.t1 = rb[1];
      sc.t2 = rb[2];
      // long segments (one replica of A): block positions, -1 outside
      if (h->rep == 1 && (a.nlong || at.nlong)) {
        const int64_t d = ph == 0 ? e.n : e.m;
        sc.pos = P.alloc<int32_t>(d, false);
        HIPCHK(hipMemsetAsync(sc.pos, 0xff, sizeof(int32_t) * d, h->st));
        sc.plong = P.alloc<double>(std::max(a.nlong, at.nlong) + 64);
      }
    }
    // block-restricted copies for the CG's wide products.  Entry capacity
    // of the copies: all of A for one stored matrix; for a few right-hand
    // sides, per right-hand side the entries of its k longest columns
    // (rows), times the right-hand sides.
    int64_t capc = h->nnz, capr = h->nnz;
    if (h->rep > 1 && h->rep < REP_MM_MIN) {
      auto topk = [&](const int64_t *ptr_dev, int64_t len, int64_t k) {
        std::vector<int64_t> pp(len + 1), ln(len);
        HIPCHK(hipMemcpy(pp.data(), ptr_dev, sizeof(int64_t) * (len + 1),
                         hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < len; ++i) ln[i] = pp[i + 1] - pp[i];
        k = std::min<int64_t>(k, len);
        std::nth_element(ln.begin(), ln.begin() + (k > 0 ? k - 1 : 0), ln.end(),
                         std::greater<int64_t>());
        int64_t t = 0;
        for (int64_t i = 0; i < k; ++i) t += ln[i];
        return t;
      };
      const int64_t kcs = e.kc / h->rep, krs = e.kr / h->rep;
      // forward engine: columns of A are CSC segments, rows CSR segments
      capc = h->rep * topk(transpose ? h->csr_ptr : h->csc_ptr,
                           transpose ? h->bm : h->bn, kcs);
      capr = h->rep * topk(transpose ? h->csc_ptr : h->csr_ptr,
                           transpose ? h->bn : h->bm, krs);
    }
    const double sub_bytes = (double)(capc + capr) * (4.0 + sizeof(T));
    // (not for many right-hand sides past REP_MM_MIN: their products read
    // A once for all right-hand sides, a copy per right-hand side would not)
    if (!(h->p.flags & RGDBEK_FLAG_SPARSE_FULL) &&
        (h->rep == 1 ||
         (h->rep < REP_MM_MIN && sub_bytes <= 48.0 * (1ull << 30)))) {
      double share = 1.0;
      auto sub = [&](SubWork &w, const Csr<T> &M, int64_t cap, int64_t dcol) {
        w.cap = cap;
        w.ptr = P.alloc<int64_t>(M.rows + 2);
        w.cnt = P.alloc<int64_t>(M.rows + 2);
        w.tile = P.alloc<int64_t>(sub_scan_tiles(M.rows + 1) + 2);
        w.idx = P.alloc<int32_t>(w.cap + 64, false);
        w.val = P.alloc<T>(w.cap + 64, false);
        w.mask = P.alloc<int32_t>(dcol + 64);
        if (M.rep == 1) {   // long rows of one stored matrix
          w.long_flag = P.alloc<uint8_t>(M.rows + 64);
          launch_mark_long<T>(M, w.long_flag, h->st);
        }
        // lanes per row of the copy from its expected row length (the
        // block's share of each stored row's entries)
        w.group = pick_group(M.brows ? (double)h->nnz / (double)M.brows * share
                                     : 1.0);
      };
      share = e.n ? (double)e.kc / (double)e.n : 1.0;
      sub(e.subc, a, capc, e.n);
      share = e.m ? (double)e.kr / (double)e.m : 1.0;
      sub(e.subr, at, capr, e.m);
    }
    // Small single systems: the Gram matrices of all columns and all rows,
    // formed once through a dense copy, turn each block projection into a
    // gather, one Cholesky or persistent PCG launch and one sparse update,
    // instead of two launches per CG step.
    // (worth it when the projections are solved to the FP64 floor, i.e. many
    // CG steps; with a loose inner tolerance a few matrix-free CG steps cost
    // less than the gather)
    const bool exact_inner = !(h->p.inner_tol > 1e-6);
    if (!(h->p.flags & RGDBEK_FLAG_SPARSE_CG) && h->rep == 1 && h->nseg == 0 &&
        exact_inner && e.m <= SPARSE_GRAM_MAX && e.n <= SPARSE_GRAM_MAX) {
      const int64_t ld = round_up(e.n, 8), ldc = round_up(e.m, 8);
      T *rm = P.alloc<T>(e.m * ld);
      T *cm = P.alloc<T>(e.n * ldc);
      launch_densify<T>(a, rm, ld, cm, ldc, h->st);
      T *F1 = P.alloc<T>(e.n * e.n, false);
      launch_gram_full<T>(cm, ldc, e.n, e.m, F1, h->st);
      T *F2 = P.alloc<T>(e.m * e.m, false);
      launch_gram_full<T>(rm, ld, e.m, e.n, F2, h->st);
      e.ata = F1;
      e.aat = F2;
      alloc_gram_blocks(h, e);
      e.sgram = true;
    }
  }
  e.rho = transpose ? h->kappa : h->rho;
  e.kappa = transpose ? h->rho : h->kappa;
  e.x = P.alloc<T>(round_up(e.n, 8) + 64);
  e.z = P.alloc<T>(e.m + 64);
  e.b = P.alloc<T>(e.m + 64);
  e.q = P.alloc<T>(e.m + 64);
  e.r = P.alloc<T>(e.m + 64);
  e.g = P.alloc<T>(e.n + 64);
  e.eps_x = P.alloc<T>(e.m + 64);
  e.eps_z = P.alloc<T>(e.n + 64);
  e.off = P.alloc<T>(e.n + 64);
  e.U = P.alloc<int32_t>(e.kc + 64);
  if (e.tall_rows) {
    e.tall.d = P.alloc<T>(e.n + 64);
    e.tall.p = P.alloc<T>(e.n + 64);
    e.tall.s = P.alloc<T>(e.n + 64);
    e.tall.res = P.alloc<T>(e.kr + 64);
    e.tall.q = P.alloc<T>(e.kr + 64);
    if (!e.dense) e.tall.rhat = P.alloc<T>(e.m + 64);
  }
  e.J = P.alloc<int32_t>(e.kr + 64);
  const int64_t dmax = std::max(e.m, e.n);
  e.sel.keys = P.alloc<uint64_t>(dmax + 64, false);
  e.sel.pers = P.alloc<SelPersist>(1);
  e.sel.ncu = h->ncu;
  e.sel.hist = P.alloc<unsigned>(2048);
  e.sel.ckey = P.alloc<uint64_t>(4096);
  e.sel.cidx = P.alloc<int64_t>(4096);
  e.sel.blk = P.alloc<int32_t>(select_scratch_blocks(dmax) + 64);
  e.sel.gmax = P.alloc<double>(select_greedy_blocks(dmax) + 64);
  if (h->p.select_mode == RGDBEK_SELECT_BLOCK_LAW) {
    e.blw = P.alloc<double>(dmax + 64);
    e.bltmp = P.alloc<int32_t>(std::max(e.kc, e.kr) + 64);
  }
  if (h->p.select_mode == RGDBEK_SELECT_IID) {
    if (dmax > select_iid_max_d())
      throw ApiError{RGDBEK_ERR_UNSUPPORTED,
                     "draws with replacement take at most 16M rows/columns"};
    e.iid.ploc = P.alloc<uint64_t>(dmax + 64);
    e.iid.ctot = P.alloc<uint64_t>(select_iid_chunks(dmax) + 64);
    e.iid.flags = P.alloc<int32_t>(dmax + 64);
  }
  e.red.part = P.alloc<double>(1024);
  e.red.cap = 1024;
  if (h->nseg) {
    e.seltmp = P.alloc<int32_t>(std::max(e.kc, e.kr) + 64);
    e.selcnt = P.alloc<int64_t>(h->nseg + 1);
    e.segmax = P.alloc<double>(h->nseg + 1);
    for (const SegInfo &g : h->hseg) {
      const int64_t dc = transpose ? g.nrow : g.ncol;
      const int64_t dr = transpose ? g.ncol : g.nrow;
      e.seg_dmax[0] = std::max(e.seg_dmax[0], dc);
      e.seg_dmax[1] = std::max(e.seg_dmax[1], dr);
    }
    e.nseg = h->nseg;
    e.seg = transpose ? h->seg_t : h->seg;
  }
  {
    int64_t np = 2 * (dmax / 4 + 1024) +
                 2 * (h->csr_nlong + h->csc_nlong) * h->rep;
    if (!e.dense) {
      np = std::max(np, 2 * segdot_max_parts(h->bm, h->nnz, h->csr_mp.nchunk,
                                             h->csr_mp.ncross, h->csr_nlong,
                                             h->rep));
      np = std::max(np, 2 * segdot_max_parts(h->bn, h->nnz, h->csc_mp.nchunk,
                                             h->csc_mp.ncross, h->csc_nlong,
                                             h->rep));
    }
    e.part = P.alloc<double>(np);
  }
  e.ready = true;
}

// ------------------------------------------------------------ profiling
// With RGDBEK_FLAG_PROFILE every group of launches of an iteration (one
// region: a residual pass, a draw, a block solve, an update, the stop test)
// is bracketed by HIP events on the handle's stream, plus two tiny marks
// outside the events: whether the solve was still running when the region
// started, and the CG steps its block solve took.  Regions of iterations
// skipped after the stop test are not counted.
hipEvent_t prof_event(rgdbek_ctx *h) {
  if (h->prof_used_events == h->prof_events.size()) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    h->prof_events.push_back(e);
  }
  return h->prof_events[h->prof_used_events++];
}

struct ProfScope {
  rgdbek_ctx *h;
  int cat, ph;
  int64_t idx = -1;
  ProfScope(rgdbek_ctx *hh, int c, int phase = -1) : h(hh), cat(c), ph(phase) {
    if (!(h->p.flags & RGDBEK_FLAG_PROFILE) || !h->prof_log) return;
    if ((int64_t)h->prof_regions.size() >= h->prof_cap) return;
    idx = (int64_t)h->prof_regions.size();
    rgdbek_ctx::ProfRegion r;
    r.cat = cat;
    r.e0 = prof_event(h);
    r.e1 = prof_event(h);
    launch_prof_mark(h->ctrl, h->prof_log + idx, 0, ph, h->st);
    HIPCHK(hipEventRecord(r.e0, h->st));
    h->prof_regions.push_back(r);
  }
  ~ProfScope() {
    if (idx < 0) return;
    // an error here resurfaces at the solve's next HIP call
    (void)hipEventRecord(h->prof_regions[idx].e1, h->st);
    launch_prof_mark(h->ctrl, h->prof_log + idx, 1, ph, h->st);
  }
};

void prof_begin_solve(rgdbek_ctx *h) {
  if (!(h->p.flags & RGDBEK_FLAG_PROFILE)) return;
  if (!h->prof_log) {
    h->prof_cap = 1 << 16;
    h->prof_log = h->pool.alloc<ProfRec>(h->prof_cap);
  }
  h->prof_regions.clear();
  h->prof_used_events = 0;
  for (auto &p : h->prof) p = rgdbek_ctx::ProfSum{};
}

void prof_end_solve(rgdbek_ctx *h) {
  if (!(h->p.flags & RGDBEK_FLAG_PROFILE) || h->prof_regions.empty()) return;
  HIPCHK(hipStreamSynchronize(h->st));
  std::vector<ProfRec> log(h->prof_regions.size());
  HIPCHK(hipMemcpy(log.data(), h->prof_log, sizeof(ProfRec) * log.size(),
                   hipMemcpyDeviceToHost));
  for (size_t i = 0; i < log.size(); ++i) {
    if (!log[i].live) continue;
    const auto &r = h->prof_regions[i];
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, r.e0, r.e1));
    auto &sum = h->prof[r.cat];
    sum.launches += 1;
    sum.ms += ms;
    sum.steps += log[i].steps;
  }
}

// ------------------------------------------------------------ iteration
struct IterOpts {
  uint64_t key1 = 0;
  int stop = RGDBEK_STOP_NONE;
  const double *xref = nullptr;   // ERR_REF reference
  const double *xbase = nullptr;  // ERR_REF on xbase + x (mixed inner loop)
  bool use_off = false;           // column offset (refinement correction)
};

// Gram solve of a dense block projection: the persistent one-launch PCG when
// the block fits its LDS staging, else two launches per CG step.  With a
// precomputed full Gram F (leading dimension ldf) the block G is not yet
// gathered: the persistent PCG gathers it during its first step, the
// step-per-launch form after a gather launch.
template <typename T>
void pcg_solve(rgdbek_ctx *h, T *G, int64_t cap, const int64_t *cnt,
               const T *hsrc, const int32_t *hl, T *y, CgWork<T> &w, int maxs,
               double itol, int ph, const T *F = nullptr, int64_t ldf = 0) {
  const bool f64 = std::is_same<T, double>::value;
  if (cap <= pcg_persist_cap(f64)) {
    launch_pcg_persist<T>(G, cap, cnt, hsrc, hl, y, w,
                          pcg_persist_grid(cap, h->ncu), maxs, itol, h->ctrl,
                          ph, 1, h->st, F, ldf);
    return;
  }
  if (F) launch_gram_gather<T>(F, ldf, hl, cnt, cap, G, h->ctrl, 1, h->st);
  launch_pcg_gram_init<T>(G, cap, cnt, hsrc, hl, y, w, h->ctrl, ph, 1, h->st);
  for (int k = 0; k < maxs; ++k)
    launch_pcg_gram_step<T>(G, cap, cnt, y, w, k, itol, h->ctrl, ph, 1, h->st);
}

template <typename T>
void enqueue_iteration(rgdbek_ctx *h, Engine<T> &e, const IterOpts &o) {
  hipStream_t st = h->st;
  Ctrl *c = h->ctrl;
  const rgdbek_params &p = h->p;
  const int maxs = p.inner_max > 0 ? p.inner_max : 64;
  const bool f64 = std::is_same<T, double>::value;
  const double itol = p.inner_tol > 0 ? p.inner_tol : (f64 ? 1e-14 : 1e-7);
  const int64_t cnt0_off = offsetof(Ctrl, sel_count);
  const int64_t *cntU = (const int64_t *)((const char *)c + cnt0_off);
  const int64_t *cntJ = cntU + 1;
  const T *off = o.use_off ? e.off : nullptr;

  const int ns = e.nseg;
  if (o.stop == RGDBEK_STOP_ERR_REF) {
    ProfScope ps(h, RGDBEK_PROF_STOP);
    if (ns) {
      launch_seg_err_ref<T>(e.x, o.xref, o.xbase, e.seg, ns, c, 1, st);
      launch_seg_fold(e.seg, ns, c, 0, p.max_iter, 0, st);
    } else {
      launch_err_ref<T>(e.n, e.x, o.xref, o.xbase, e.red, c, 1, st);
    }
  }
  // ---- column phase: g = A^T z (+ t), eps^z, select U, project z
  {
  ProfScope ps(h, RGDBEK_PROF_COL_RESIDUAL);
  if (e.dense) {
    launch_dense_fused<T>(e.arm, e.x, e.z, e.dw, off, e.kappa, e.g, e.eps_z,
                          e.q, c, 1, st);
  } else {
    SegArgs<T> a;
    a.v = e.z; a.g = e.g; a.off = off; a.eps = e.eps_z; a.nrm = e.kappa;
    launch_segdot<T>(e.csc, EPI_COLRES, a, c, 1, st);
  }
  }
  {
  ProfScope ps(h, RGDBEK_PROF_COL_DRAW);
  if (ns)
    launch_select_seg<T>(e.eps_z, e.seg, ns, 0, e.seg_dmax[0], e.floor, p.seed,
                         o.key1, 0, e.sel.keys, e.segmax, e.seltmp, e.selcnt,
                         e.U, c, 1, st);
  else if (p.select_mode == RGDBEK_SELECT_GREEDY)
    launch_select_greedy<T>(e.eps_z, e.n, p.eta, e.kc, 0, e.sel, e.U, c, 1, st);
  else if (p.select_mode == RGDBEK_SELECT_BLOCK_LAW)
    launch_select_block_law<T>(e.eps_z, e.n, e.kc, e.floor, p.seed, o.key1, 0,
                               0, 0, e.sel, e.blw, e.bltmp, e.U, c, 1, st);
  else if (p.select_mode == RGDBEK_SELECT_IID)
    launch_select_iid<T>(e.eps_z, e.n, e.kc, e.floor, p.seed, o.key1, 0, 0, 0,
                         e.sel, e.iid, e.U, c, 1, st);
  else
    launch_select<T>(e.eps_z, e.n, e.kc, e.floor, p.seed, o.key1, 0, 0, 0,
                     e.sel, e.U, c, 1, st);
  }
  const bool chol_c = p.solver == RGDBEK_SOLVER_CHOL ||
                      (p.solver == RGDBEK_SOLVER_AUTO && e.kc <= 256);
  const bool chol_r = p.solver == RGDBEK_SOLVER_CHOL ||
                      (p.solver == RGDBEK_SOLVER_AUTO && e.kr <= 256);
  const bool cg_c = !(chol_c && e.kc <= CHOL_MAX);
  const bool cg_r = !(chol_r && e.kr <= CHOL_MAX);
  if (e.dense) {
    {
    ProfScope ps(h, RGDBEK_PROF_COL_SOLVE, 0);
    if (cg_c && e.ata) {
      pcg_solve<T>(h, e.GU, e.kc, cntU, e.g, e.U, e.y, e.cgc, maxs, itol, 0,
                   e.ata, e.n);
    } else {
      if (e.ata)
        launch_gram_gather<T>(e.ata, e.n, e.U, cntU, e.kc, e.GU, c, 1, st);
      else
        launch_gram_rows<T>(e.acm.a, e.acm.ld, e.m, e.U, cntU, e.kc, e.GU, c,
                            1, st);
      if (cg_c)
        pcg_solve<T>(h, e.GU, e.kc, cntU, e.g, e.U, e.y, e.cgc, maxs, itol, 0);
      else
        launch_chol_solve<T>(e.GU, e.kc, cntU, e.g, e.U, e.y, 1, c, 0, 1, st);
    }
    }
    ProfScope pu(h, RGDBEK_PROF_COL_UPDATE);
    launch_col_update<T>(e.acm.a, e.acm.ld, e.m, e.U, cntU, e.kc, e.y, e.z,
                         e.upd, c, 1, st);
  } else if (e.sgram) {
    {
    ProfScope ps(h, RGDBEK_PROF_COL_SOLVE, 0);
    if (cg_c) {
      pcg_solve<T>(h, e.GU, e.kc, cntU, e.g, e.U, e.y, e.cgc, maxs, itol, 0,
                   e.ata, e.n);
    } else {
      launch_gram_gather<T>(e.ata, e.n, e.U, cntU, e.kc, e.GU, c, 1, st);
      launch_chol_solve<T>(e.GU, e.kc, cntU, e.g, e.U, e.y, 1, c, 0, 1, st);
    }
    }
    ProfScope pu(h, RGDBEK_PROF_COL_UPDATE);
    launch_sparse_block_update<T>(e.csr, e.U, cntU, e.kc, e.y, -1, e.scc.phat,
                                  e.z, c, 1, st);
  } else {
    ProfScope ps(h, RGDBEK_PROF_COL_SOLVE, 0);
    const Csr<T> wcsr = e.subc.idx ? launch_sub_matrix<T>(e.csr, e.U, cntU, e.kc,
                                                          e.subc, c, st)
                                   : e.csr;
    launch_sparse_colproj<T>(wcsr, e.csc, e.U, cntU, e.kc, e.g, e.z, e.scc,
                             maxs, itol, c, 1, st);
  }
  // ---- row phase: r = b - z - A x, eps^x, stop test, select J, project x
  int nparts;
  {
  ProfScope ps(h, RGDBEK_PROF_ROW_RESIDUAL);
  if (e.dense) {
    nparts = launch_rowres_dense<T>(e.m, e.b, e.z, e.q, e.rho, e.r, e.eps_x,
                                    e.part, c, 1, st);
  } else {
    SegArgs<T> a;
    a.v = e.x; a.b = e.b; a.z = e.z; a.r = e.r; a.eps = e.eps_x;
    a.nrm = e.rho; a.part = e.part;
    nparts = launch_segdot<T>(e.csr, EPI_ROWRES, a, c, 1, st);
  }
  }
  if (o.stop == RGDBEK_STOP_RSE || o.stop == RGDBEK_STOP_RES_EXT) {
    ProfScope ps(h, RGDBEK_PROF_STOP);
    if (ns) {
      launch_seg_stop_rowres<T>(e.r, e.z, e.seg, ns, o.stop, c, 1, st);
      launch_seg_fold(e.seg, ns, c, 0, p.max_iter, 0, st);
    } else {
      launch_stop_rowres(e.part, nparts, c, st);
    }
  }
  {
  ProfScope ps(h, RGDBEK_PROF_ROW_DRAW);
  if (ns)
    launch_select_seg<T>(e.eps_x, e.seg, ns, 1, e.seg_dmax[1], e.floor, p.seed,
                         o.key1, 1, e.sel.keys, e.segmax, e.seltmp, e.selcnt,
                         e.J, c, 1, st);
  else if (p.select_mode == RGDBEK_SELECT_GREEDY)
    launch_select_greedy<T>(e.eps_x, e.m, p.eta, e.kr, 1, e.sel, e.J, c, 1, st);
  else if (p.select_mode == RGDBEK_SELECT_BLOCK_LAW)
    launch_select_block_law<T>(e.eps_x, e.m, e.kr, e.floor, p.seed, o.key1, 1,
                               0, 1, e.sel, e.blw, e.bltmp, e.J, c, 1, st);
  else if (p.select_mode == RGDBEK_SELECT_IID)
    launch_select_iid<T>(e.eps_x, e.m, e.kr, e.floor, p.seed, o.key1, 1, 0, 1,
                         e.sel, e.iid, e.J, c, 1, st);
  else
    launch_select<T>(e.eps_x, e.m, e.kr, e.floor, p.seed, o.key1, 1, 0, 1,
                     e.sel, e.J, c, 1, st);
  }
  if (e.tall_rows) {
    ProfScope ps(h, RGDBEK_PROF_ROW_SOLVE, 1);
    if (e.dense)
      launch_tall_rowproj_dense<T>(e.arm, e.J, cntJ, e.kr, e.r, e.x, e.tall,
                                   e.upd, maxs, itol, c, st);
    else
      launch_tall_rowproj_sparse<T>(e.csr, e.csc, e.J, cntJ, e.kr, e.r, e.x,
                                    e.tall, maxs, itol, c, st);
  } else if (e.dense) {
    {
    ProfScope ps(h, RGDBEK_PROF_ROW_SOLVE, 1);
    if (!cg_r || !e.aat) {
      if (e.aat)
        launch_gram_gather<T>(e.aat, e.m, e.J, cntJ, e.kr, e.GJ, c, 1, st);
      else
        launch_gram_rows<T>(e.arm.a, e.arm.ld, e.n, e.J, cntJ, e.kr, e.GJ, c,
                            1, st);
    }
    if (!cg_r) {
      launch_chol_solve<T>(e.GJ, e.kr, cntJ, e.r, e.J, e.w, 1, c, 1, 1, st);
    } else {
      pcg_solve<T>(h, e.GJ, e.kr, cntJ, e.r, e.J, e.w, e.cgr, maxs, itol, 1,
                   e.aat, e.m);
    }
    }
    ProfScope pu(h, RGDBEK_PROF_ROW_UPDATE);
    if (!cg_r) {
      launch_row_update<T>(e.arm.a, e.arm.ld, e.n, e.J, cntJ, e.kr, e.w, e.x,
                           e.upd, c, 1, st);
      // corrected semi-normal equations: one sweep with the residual of the
      // projected equations recomputed from A^J itself
      launch_list_resid<T>(e.arm.a, e.arm.ld, e.n, e.J, cntJ, e.kr, e.b, e.z,
                           e.x, e.s, c, 1, st);
      launch_chol_solve<T>(e.GJ, e.kr, cntJ, e.s, nullptr, e.w, 0, c, 1, 1,
                           st);
      launch_row_update<T>(e.arm.a, e.arm.ld, e.n, e.J, cntJ, e.kr, e.w, e.x,
                           e.upd, c, 1, st);
    } else {
      launch_row_update<T>(e.arm.a, e.arm.ld, e.n, e.J, cntJ, e.kr, e.w, e.x,
                           e.upd, c, 1, st);
    }
  } else if (e.sgram) {
    {
    ProfScope ps(h, RGDBEK_PROF_ROW_SOLVE, 1);
    if (cg_r) {
      pcg_solve<T>(h, e.GJ, e.kr, cntJ, e.r, e.J, e.w, e.cgr, maxs, itol, 1,
                   e.aat, e.m);
    } else {
      launch_gram_gather<T>(e.aat, e.m, e.J, cntJ, e.kr, e.GJ, c, 1, st);
      launch_chol_solve<T>(e.GJ, e.kr, cntJ, e.r, e.J, e.w, 1, c, 1, 1, st);
    }
    }
    ProfScope pu(h, RGDBEK_PROF_ROW_UPDATE);
    launch_sparse_block_update<T>(e.csc, e.J, cntJ, e.kr, e.w, 1, e.scr.phat,
                                  e.x, c, 1, st);
  } else {
    ProfScope ps(h, RGDBEK_PROF_ROW_SOLVE, 1);
    const Csr<T> wcsc = e.subr.idx ? launch_sub_matrix<T>(e.csc, e.J, cntJ, e.kr,
                                                          e.subr, c, st)
                                   : e.csc;
    launch_sparse_rowproj<T>(e.csr, wcsc, e.J, cntJ, e.kr, e.r, e.rho, e.x,
                             e.scr, maxs, itol, c, 1, st);
  }
  ProfScope ps(h, RGDBEK_PROF_STOP);
  if (ns) launch_seg_fold(e.seg, ns, c, 1, p.max_iter, 0, st);
  else launch_end_iter(c, st);
}

int graph_iters(const rgdbek_ctx *h) {
  return h->p.graph_iters > 0 ? h->p.graph_iters : 8;
}

template <typename T>
hipGraphExec_t get_graph(rgdbek_ctx *h, Engine<T> &e, int which,
                         const IterOpts &o) {
  for (auto &g : h->graphs)
    if (g.which == which && g.key1 == o.key1 && g.stop == o.stop &&
        g.use_xref == (o.xref != nullptr) && g.with_base == (o.xbase != nullptr))
      return g.exec;
  rgdbek_ctx::GraphEntry ge;
  ge.which = which;
  ge.key1 = o.key1;
  ge.stop = o.stop;
  ge.use_xref = o.xref != nullptr;
  ge.with_base = o.xbase != nullptr;
  HIPCHK(hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal));
  for (int i = 0; i < graph_iters(h); ++i) enqueue_iteration<T>(h, e, o);
  HIPCHK(hipStreamEndCapture(h->st, &ge.graph));
  HIPCHK(hipGraphInstantiate(&ge.exec, ge.graph, nullptr, nullptr, 0));
  h->graphs.push_back(ge);
  return ge.exec;
}

// Make `later` wait for the work enqueued so far on `earlier` (no host
// synchronisation; nothing to do for one stream).
void stream_after(hipStream_t later, hipStream_t earlier) {
  if (later == earlier) return;
  hipEvent_t ev;
  HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  HIPCHK(hipEventRecord(ev, earlier));
  HIPCHK(hipStreamWaitEvent(later, ev, 0));
  HIPCHK(hipEventDestroy(ev));
}

void ctrl_reset(rgdbek_ctx *h, int64_t it0, int64_t max_iter, int stop,
                double tol) {
  Ctrl &c = *h->hctrl;
  std::memset(&c, 0, sizeof(Ctrl));
  c.it = it0;
  c.it_end = max_iter;
  c.stop_mode = stop;
  c.tol = tol;
  c.done = max_iter <= 0 ? 1 : 0;
  HIPCHK(hipMemcpyAsync(h->ctrl, &c, sizeof(Ctrl), hipMemcpyHostToDevice,
                        h->st));
}

void ctrl_fetch(rgdbek_ctx *h) {
  HIPCHK(hipMemcpyAsync(h->hctrl, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost,
                        h->st));
  HIPCHK(hipStreamSynchronize(h->st));
}

// Run iterations until done; the host looks at the device flag once per graph.
template <typename T>
void run_loop(rgdbek_ctx *h, Engine<T> &e, int which, const IterOpts &o) {
  const bool use_graph = (h->p.flags & RGDBEK_FLAG_GRAPH) != 0 &&
                         !(h->p.flags & RGDBEK_FLAG_PROFILE);
  hipGraphExec_t ge = use_graph ? get_graph<T>(h, e, which, o) : nullptr;
  while (true) {
    if (use_graph) {
      HIPCHK(hipGraphLaunch(ge, h->st));
    } else {
      for (int i = 0; i < graph_iters(h); ++i) enqueue_iteration<T>(h, e, o);
    }
    HIPCHK(hipMemcpyAsync(&h->hctrl->done, &h->ctrl->done, sizeof(int32_t),
                          hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    if (h->hctrl->done) break;
  }
  HIPCHK(hipGetLastError());
}

rgdbek_status finish_status(rgdbek_ctx *h, rgdbek_info *info, double secs,
                            int64_t outer) {
  Ctrl &c = *h->hctrl;
  rgdbek_status s = RGDBEK_OK;
  if (c.sync_fail) {
    s = RGDBEK_ERR_DEVICE;
    set_err(h, "a grid-barrier wait of the block solver timed out (the "
               "workgroups of one launch were not all resident)");
  } else if (c.numeric) {
    s = RGDBEK_ERR_NUMERIC;
    set_err(h, "NaN, negative or infinite residual weight during the solve");
  } else if (!c.converged && h->p.stop != RGDBEK_STOP_NONE) {
    s = RGDBEK_ERR_NOT_CONVERGED;
    set_err(h, "max_iter reached before the stopping test held");
  }
  if (info) {
    info->iterations = c.iters_run;
    info->outer_iterations = outer;
    info->final_metric = c.metric;
    info->converged = (h->p.stop == RGDBEK_STOP_NONE) ? (c.numeric ? 0 : 1)
                                                      : c.converged;
    info->status = (int32_t)s;
    info->seconds = secs;
  }
  return s;
}

// Check that b (device) is finite.
void check_b(rgdbek_ctx *h, const double *b, int64_t len) {
  int *flag = h->pool.alloc<int>(1);
  launch_check_finite<double>(b, len, flag, h->st);
  int hv = 0;
  HIPCHK(hipMemcpyAsync(&hv, flag, sizeof(int), hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  HIPCHK(hipFree(flag));
  h->pool.ptrs.pop_back();
  if (hv) throw ApiError{RGDBEK_ERR_NUMERIC, "right-hand side has NaN/Inf"};
}

// ------------------------------------------------------------ FP64 solve
rgdbek_status solve64(rgdbek_ctx *h, Engine<double> &e, int which,
                      uint64_t key1, int stop, const double *b, double *x,
                      double *z_io, int64_t it0, bool resume,
                      const double *x_ref_user, rgdbek_info *info) {
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = h->st;
  const double *x_ref = nullptr;
  if (x_ref_user) {
    HIPCHK(hipMemcpyAsync(h->xref, x_ref_user, sizeof(double) * e.n,
                          hipMemcpyDeviceToDevice, st));
    x_ref = h->xref;
  }
  check_b(h, b, e.m);
  prof_begin_solve(h);
  HIPCHK(hipMemcpyAsync(e.b, b, sizeof(double) * e.m, hipMemcpyDeviceToDevice, st));
  if (resume) {
    HIPCHK(hipMemcpyAsync(e.x, x, sizeof(double) * e.n, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(e.z, z_io, sizeof(double) * e.m, hipMemcpyDeviceToDevice, st));
  } else {
    launch_axpby<double, double>(e.n, 0.0, e.x, 0.0, (const double *)nullptr, st);
    HIPCHK(hipMemcpyAsync(e.z, b, sizeof(double) * e.m, hipMemcpyDeviceToDevice, st));
  }
  ctrl_reset(h, it0, h->p.max_iter, stop, h->p.tol);
  if (stop == RGDBEK_STOP_ERR_REF) launch_set_ref2<double>(e.n, x_ref, h->ctrl, st);
  else launch_set_ref2<double>(e.m, e.b, h->ctrl, st);
  if (e.nseg) {
    launch_seg_reset(e.seg, e.nseg, it0, 0, nullptr, st);
    if (stop == RGDBEK_STOP_ERR_REF) launch_seg_ref2<double>(x_ref, e.seg, e.nseg, 1, st);
    else launch_seg_ref2<double>(e.b, e.seg, e.nseg, 0, st);
  }
  IterOpts o;
  o.key1 = key1;
  o.stop = stop;
  o.xref = stop == RGDBEK_STOP_ERR_REF ? x_ref : nullptr;
  run_loop<double>(h, e, which, o);
  if (stop == RGDBEK_STOP_ERR_REF) {
    if (e.nseg) {
      launch_seg_err_ref<double>(e.x, x_ref, nullptr, e.seg, e.nseg, h->ctrl,
                                 0, st);
      launch_seg_fold(e.seg, e.nseg, h->ctrl, 0, h->p.max_iter, 1, st);
    } else {
      launch_err_ref<double>(e.n, e.x, x_ref, nullptr, e.red, h->ctrl, 0, st);
    }
  }
  HIPCHK(hipMemcpyAsync(x, e.x, sizeof(double) * e.n, hipMemcpyDeviceToDevice, st));
  if (z_io)
    HIPCHK(hipMemcpyAsync(z_io, e.z, sizeof(double) * e.m, hipMemcpyDeviceToDevice, st));
  ctrl_fetch(h);
  const double secs = std::chrono::duration<double>(
                          std::chrono::steady_clock::now() - t0).count();
  prof_end_solve(h);
  return finish_status(h, info, secs, 1);
}

// ------------------------------------------------------------ mixed solve
// Refinement with FP32 inner RGDBEK.  FP64 state (x, z); each pass:
//   stop test in FP64 on the state (ERR_REF on x; RSE on b - A x; RES_EXT on
//   b - z - A x with the carried z, from the second pass on)
//   z = b - A x                        (FP64, so z - b stays in range(A))
//   t = A^T z                          (FP64, the normal-equation residual)
//   FP32 RGDBEK on the correction (dx, dz) from (0, 0): column residual
//   A^T dz + t, row residual -dz - A dx (right-hand side s = b - z - A x = 0)
//   x += dx, z += dz (FP64)
// The fixed point of a pass is x + dx = A^+ b exactly; FP32 only limits how
// far one pass contracts the error (about u_32 * cond).  Carrying z across
// passes instead would freeze FP32 rounding in its null(A^T) component and
// stall the refinement.  An inner pass ends on residuals only: its FP32
// extended residual ||dz + A dx|| (the extended residual b - z - A x of the
// refined state) falls to pass_drop (default 1e-5) times its first value in the pass
// (or to tol for an outer RES_EXT test), on an FP32 plateau (no 1% gain over
// 8 graphs once the residual is falling), or, after the first pass, at twice
// the first pass's length.  The outer loop ends when the FP64 test holds, or
// when a pass no longer cuts the FP64 metric by 10%.
constexpr double MIXED_PASS_DROP = 1e-5;   // default pass_drop

rgdbek_status solve_mixed(rgdbek_ctx *h, const double *b, double *x,
                          const double *x_ref_user, rgdbek_info *info) {
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = h->st;
  const double *x_ref = nullptr;
  if (x_ref_user) {
    HIPCHK(hipMemcpyAsync(h->xref, x_ref_user, sizeof(double) * h->n,
                          hipMemcpyDeviceToDevice, st));
    x_ref = h->xref;
  }
  Engine<double> &E = h->e64;
  Engine<float> &F = h->e32;
  const int stop = h->p.stop;
  check_b(h, b, E.m);
  prof_begin_solve(h);
  HIPCHK(hipMemcpyAsync(E.b, b, sizeof(double) * E.m, hipMemcpyDeviceToDevice, st));
  launch_axpby<double, double>(E.n, 0.0, h->x64, 0.0, (const double *)nullptr, st);
  HIPCHK(hipMemcpyAsync(h->z64, b, sizeof(double) * E.m, hipMemcpyDeviceToDevice, st));
  if (E.nseg) {
    HIPCHK(hipMemsetAsync(h->fixed, 0, sizeof(int32_t) * E.nseg, st));
    launch_seg_reset(E.seg, E.nseg, 0, 0, nullptr, st);
  }
  int64_t total_it = 0, outer = 0, pass1_its = -1;
  const int max_outer = 12;
  double metric = 0.0, prev_metric = 1e300;
  bool converged = false;
  int numeric = 0, sync_fail = 0;
  for (outer = 1; outer <= max_outer; ++outer) {
    // the FP64 stop test, then z = b - A x and t = A^T z (FP64 passes).
    // RES_EXT uses the carried z; before the first pass (x = 0, z = b) it
    // holds trivially, so it is first tested after one pass.
    const bool test_now = stop != RGDBEK_STOP_NONE &&
                          !(stop == RGDBEK_STOP_RES_EXT && outer == 1);
    ctrl_reset(h, 0, 1, test_now ? stop : RGDBEK_STOP_NONE, h->p.tol);
    int nparts;
    {
    ProfScope pr(h, RGDBEK_PROF_REFINE);
    if (E.dense) {
      launch_dense_fused<double>(E.arm, h->x64, h->z64, E.dw, nullptr, E.kappa,
                                 h->t64, E.eps_z, E.q, h->ctrl, 0, st);
      if (stop == RGDBEK_STOP_RES_EXT) {
        // r = b - z - A x with the carried z; then b - A x = r + z
        nparts = launch_rowres_dense<double>(E.m, E.b, h->z64, E.q, E.rho,
                                             E.r, E.eps_x, E.part, h->ctrl, 0,
                                             st);
        launch_axpby<double, double>(E.m, 1.0, h->z64, 1.0, E.r, st);
      } else {
        nparts = launch_rowres_dense<double>(E.m, E.b, h->zero64, E.q, E.rho,
                                             h->z64, E.eps_x, E.part, h->ctrl,
                                             0, st);
      }
      launch_dense_fused<double>(E.arm, h->x64, h->z64, E.dw, nullptr, E.kappa,
                                 h->t64, E.eps_z, E.q, h->ctrl, 0, st);
    } else {
      SegArgs<double> r;
      r.v = h->x64; r.b = E.b; r.eps = E.eps_x; r.nrm = E.rho; r.part = E.part;
      if (stop == RGDBEK_STOP_RES_EXT) {
        r.z = h->z64; r.r = E.r;
      } else {
        r.z = h->zero64; r.r = h->z64;
      }
      nparts = launch_segdot<double>(E.csr, EPI_ROWRES, r, h->ctrl, 0, st);
      if (stop == RGDBEK_STOP_RES_EXT)
        launch_axpby<double, double>(E.m, 1.0, h->z64, 1.0, E.r, st);
      SegArgs<double> a;
      a.v = h->z64; a.g = h->t64; a.eps = E.eps_z; a.nrm = E.kappa;
      launch_segdot<double>(E.csc, EPI_COLRES, a, h->ctrl, 0, st);
    }
    if (E.nseg && test_now) {
      launch_seg_reset(E.seg, E.nseg, 0, 1, nullptr, st);
      if (stop == RGDBEK_STOP_ERR_REF) {
        launch_seg_ref2<double>(x_ref, E.seg, E.nseg, 1, st);
        launch_seg_err_ref<double>(h->x64, x_ref, nullptr, E.seg, E.nseg,
                                   h->ctrl, 0, st);
      } else if (stop == RGDBEK_STOP_RES_EXT) {
        launch_seg_ref2<double>(E.b, E.seg, E.nseg, 0, st);
        launch_seg_stop_rowres<double>(E.r, h->zero64, E.seg, E.nseg, stop,
                                       h->ctrl, 0, st);
      } else {
        launch_seg_ref2<double>(E.b, E.seg, E.nseg, 0, st);
        launch_seg_stop_rowres<double>(h->z64, h->zero64, E.seg, E.nseg,
                                       stop, h->ctrl, 0, st);
      }
      launch_seg_fold(E.seg, E.nseg, h->ctrl, 0, h->p.max_iter, 1, st);
      launch_seg_converged(E.seg, E.nseg, h->fixed, st);
    } else if (test_now && stop == RGDBEK_STOP_ERR_REF) {
      launch_set_ref2<double>(E.n, x_ref, h->ctrl, st);
      launch_err_ref<double>(E.n, h->x64, x_ref, nullptr, E.red, h->ctrl, 0, st);
    } else if (test_now) {
      launch_set_ref2<double>(E.m, E.b, h->ctrl, st);
      launch_stop_rowres(E.part, nparts, h->ctrl, st);
    }
    }
    ctrl_fetch(h);
    metric = h->hctrl->metric;
    if (trace_on())
      std::fprintf(stderr, "[rgdbek] pass %lld fp64 metric %.3e (inner its so far %lld)\n",
                   (long long)outer, metric, (long long)total_it);
    if (test_now && h->hctrl->converged) {
      converged = true;
      break;
    }
    if (total_it >= h->p.max_iter) break;
    // refinement stalled: a pass that no longer cuts the metric by 10%
    if (test_now && outer > 2 && metric > 0.9 * prev_metric) break;
    if (test_now) prev_metric = metric;
    // FP32 pass on the correction system: s = 0, offset t
    launch_axpby<float, float>(F.m, 0.0, F.b, 0.0, (const float *)nullptr, st);
    launch_convert<float, double>(h->t64, F.off, E.n, st);
    launch_axpby<float, float>(F.n, 0.0, F.x, 0.0, (const float *)nullptr, st);
    launch_axpby<float, float>(F.m, 0.0, F.z, 0.0, (const float *)nullptr, st);
    const int istop = stop == RGDBEK_STOP_NONE ? RGDBEK_STOP_NONE
                                               : RGDBEK_STOP_RES_EXT;
    ctrl_reset(h, total_it, h->p.max_iter - total_it, istop,
               stop == RGDBEK_STOP_RES_EXT ? h->p.tol : 0.0);
    if (istop == RGDBEK_STOP_RES_EXT) {
      h->hctrl->pass_drop = h->p.pass_drop > 0.0 ? h->p.pass_drop
                                                 : MIXED_PASS_DROP;
      HIPCHK(hipMemcpyAsync(&h->ctrl->pass_drop, &h->hctrl->pass_drop,
                            sizeof(double), hipMemcpyHostToDevice, st));
    }
    launch_set_ref2<double>(E.m, E.b, h->ctrl, st);
    if (E.nseg) {
      launch_seg_reset(E.seg, E.nseg, 0, 1, h->fixed, st);
      launch_seg_ref2<double>(E.b, E.seg, E.nseg, 0, st);
    }
    IterOpts o;
    o.key1 = 0;
    o.stop = istop;
    o.use_off = true;
    {
      const bool use_graph = (h->p.flags & RGDBEK_FLAG_GRAPH) != 0 &&
                         !(h->p.flags & RGDBEK_FLAG_PROFILE);
      hipGraphExec_t ge = use_graph ? get_graph<float>(h, F, 2, o) : nullptr;
      // The extended residual of a pass that starts from a nonzero state
      // first grows (the column steps remove components of z faster than
      // the row steps let A x follow), then falls.  FP32 plateau: once it
      // has fallen below its first reading, the best value has not improved
      // by 1% over `window` graphs.  Passes after the first are also capped
      // at twice the first pass's length (each cuts the error by about the
      // same factor).
      double first = -1.0, best = 1e300;
      bool falling = false;
      int since_best = 0;
      const int window = 8;
      const int64_t cap = pass1_its > 0 ? 2 * pass1_its + graph_iters(h) : -1;
      while (true) {
        if (use_graph) HIPCHK(hipGraphLaunch(ge, st));
        else for (int i = 0; i < graph_iters(h); ++i) enqueue_iteration<float>(h, F, o);
        if (istop == RGDBEK_STOP_NONE) {
          HIPCHK(hipMemcpyAsync(&h->hctrl->done, &h->ctrl->done, sizeof(int32_t),
                                hipMemcpyDeviceToHost, st));
          HIPCHK(hipStreamSynchronize(st));
          if (h->hctrl->done) break;
          continue;
        }
        ctrl_fetch(h);
        if (trace_on())
          std::fprintf(stderr, "[rgdbek]   inner its %lld metric %.3e done %d\n",
                       (long long)h->hctrl->iters_run, h->hctrl->metric,
                       h->hctrl->done);
        if (h->hctrl->done) break;
        if (cap > 0 && h->hctrl->iters_run >= cap) break;
        const double mt = h->hctrl->metric;
        if (first < 0.0) first = mt;
        if (!falling && mt < first) falling = true;
        if (mt < 0.99 * best) { best = mt; since_best = 0; }
        else if (falling && ++since_best >= window) break;
      }
    }
    ctrl_fetch(h);
    if (pass1_its < 0) pass1_its = h->hctrl->iters_run;
    total_it += h->hctrl->iters_run;
    numeric |= h->hctrl->numeric;
    sync_fail |= h->hctrl->sync_fail;
    launch_axpby<double, float>(E.n, 1.0, h->x64, 1.0, F.x, st);
    launch_axpby<double, float>(E.m, 1.0, h->z64, 1.0, F.z, st);
    if (numeric || sync_fail || stop == RGDBEK_STOP_NONE) {
      if (stop == RGDBEK_STOP_NONE) converged = true;
      break;
    }
  }
  HIPCHK(hipMemcpyAsync(x, h->x64, sizeof(double) * E.n, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(E.z, h->z64, sizeof(double) * E.m, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  const double secs = std::chrono::duration<double>(
                          std::chrono::steady_clock::now() - t0).count();
  prof_end_solve(h);
  Ctrl &c = *h->hctrl;
  c.iters_run = total_it;
  c.metric = metric;
  c.converged = converged ? 1 : 0;
  c.numeric = numeric;
  c.sync_fail = sync_fail;
  return finish_status(h, info, secs, outer > max_outer ? max_outer : outer);
}

// ------------------------------------------------------------ validation
void validate_params(const rgdbek_params *p, int64_t m, int64_t n,
                     int64_t *kc, int64_t *kr) {
  if (!(p->eta >= 0.0) || p->eta > 1.0)
    throw ApiError{RGDBEK_ERR_INVALID_ARG, "eta must lie in [0, 1]"};
  auto from_eta = [&](int64_t d) -> int64_t {
    if (d <= 0) return 0;
    int64_t k = (int64_t)std::floor(p->eta * (double)d + 0.5);
    return std::min<int64_t>(d, std::max<int64_t>(1, k));
  };
  const bool greedy = p->select_mode == RGDBEK_SELECT_GREEDY;
  *kc = p->k_col > 0 ? p->k_col : (greedy ? n : from_eta(n));
  *kr = p->k_row > 0 ? p->k_row : (greedy ? m : from_eta(m));
  if (p->k_col < 0 || p->k_row < 0)
    throw ApiError{RGDBEK_ERR_INVALID_ARG, "k_col/k_row must be >= 0"};
  if (*kc > n || *kr > m)
    throw ApiError{RGDBEK_ERR_INVALID_ARG, "block size larger than the dimension"};
  if (*kc < 1 || *kr < 1)
    throw ApiError{RGDBEK_ERR_INVALID_ARG, "block sizes must be positive"};
  if (p->stop < RGDBEK_STOP_NONE || p->stop > RGDBEK_STOP_RES_EXT)
    throw ApiError{RGDBEK_ERR_INVALID_ARG, "unknown stop mode"};
  if (p->precision < RGDBEK_PREC_FP64 || p->precision > RGDBEK_PREC_MIXED_F32)
    throw ApiError{RGDBEK_ERR_INVALID_ARG, "unknown precision"};
  if (!(p->pass_drop >= 0.0) || p->pass_drop >= 1.0)
    throw ApiError{RGDBEK_ERR_INVALID_ARG, "pass_drop must lie in [0, 1)"};
  if (p->max_iter < 0 || !(p->tol >= 0.0))
    throw ApiError{RGDBEK_ERR_INVALID_ARG, "max_iter and tol must be >= 0"};
  if (p->solver < 0 || p->solver > RGDBEK_SOLVER_CG)
    throw ApiError{RGDBEK_ERR_INVALID_ARG, "unknown block solver"};
  if (p->inner_max < 0 || p->inner_max > 4096 || p->graph_iters < 0 ||
      p->graph_iters > 1024)
    throw ApiError{RGDBEK_ERR_INVALID_ARG, "inner_max/graph_iters out of range"};
  if (p->tile_rows < 0 || p->tile_rows > (1 << 20))
    throw ApiError{RGDBEK_ERR_INVALID_ARG, "tile_rows must lie in [0, 2^20]"};
  if (p->select_mode != RGDBEK_SELECT_RANDOM &&
      p->select_mode != RGDBEK_SELECT_GREEDY &&
      p->select_mode != RGDBEK_SELECT_BLOCK_LAW &&
      p->select_mode != RGDBEK_SELECT_IID)
    throw ApiError{RGDBEK_ERR_INVALID_ARG, "unknown select_mode"};
  if (p->select_mode == RGDBEK_SELECT_GREEDY && !(p->eta > 0.0))
    throw ApiError{RGDBEK_ERR_INVALID_ARG,
                   "the greedy threshold eta must lie in (0, 1]"};
}

// Compute units of the current device (sizes the dense pass grid).
int device_cus() {
  int dev = 0, ncu = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  return ncu > 0 ? ncu : 256;
}

// CSR structure check on the host (copies row_ptr and col_idx).
void validate_csr(const rgdbek_matrix *A) {
  std::vector<int64_t> rp(A->m + 1);
  HIPCHK(hipMemcpy(rp.data(), A->row_ptr, sizeof(int64_t) * (A->m + 1),
                   hipMemcpyDeviceToHost));
  if (rp[0] != 0 || rp[A->m] != A->nnz)
    throw ApiError{RGDBEK_ERR_INVALID_ARG, "row_ptr must start at 0 and end at nnz"};
  for (int64_t i = 0; i < A->m; ++i)
    if (rp[i + 1] < rp[i])
      throw ApiError{RGDBEK_ERR_INVALID_ARG, "row_ptr must be non-decreasing"};
  std::vector<int32_t> ci(A->nnz);
  if (A->nnz)
    HIPCHK(hipMemcpy(ci.data(), A->col_idx, sizeof(int32_t) * A->nnz,
                     hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < A->m; ++i)
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      if (ci[e] < 0 || ci[e] >= A->n)
        throw ApiError{RGDBEK_ERR_INVALID_ARG, "column index out of range"};
      if (e > rp[i] && ci[e] <= ci[e - 1])
        throw ApiError{RGDBEK_ERR_INVALID_ARG,
                       "column indices must increase within a row"};
    }
}

// long-segment lists (host-side from the pointer arrays)
void build_longs(rgdbek_ctx *h, const int64_t *ptr_dev, int64_t rows,
                 int64_t limit, int32_t **out, int64_t *count) {
  std::vector<int64_t> rp(rows + 1);
  HIPCHK(hipMemcpy(rp.data(), ptr_dev, sizeof(int64_t) * (rows + 1),
                   hipMemcpyDeviceToHost));
  std::vector<int32_t> longs;
  for (int64_t i = 0; i < rows; ++i)
    if (rp[i + 1] - rp[i] > limit) longs.push_back((int32_t)i);
  *count = (int64_t)longs.size();
  *out = h->pool.alloc<int32_t>(std::max<int64_t>(1, *count), false);
  if (*count)
    HIPCHK(hipMemcpy(*out, longs.data(), sizeof(int32_t) * longs.size(),
                     hipMemcpyHostToDevice));
}

// Chunk c holds nonzeros [c*MP_CH, (c+1)*MP_CH); it owns the rows whose
// first nonzero position lies in it (empty rows: the position of the next
// nonzero; trailing empty rows: the last chunk).  Rows running past their
// chunk are listed with their first and last chunk.
void build_merge_plan(rgdbek_ctx *h, const int64_t *ptr_dev, int64_t rows,
                      MergePlan *mp) {
  std::vector<int64_t> rp(rows + 1);
  HIPCHK(hipMemcpy(rp.data(), ptr_dev, sizeof(int64_t) * (rows + 1),
                   hipMemcpyDeviceToHost));
  const int64_t nnz = rp[rows];
  const int64_t nch = std::max<int64_t>(1, (nnz + MP_CH - 1) / MP_CH);
  std::vector<int32_t> rs(nch + 1);
  for (int64_t c = 0; c < nch; ++c)
    rs[c] = (int32_t)(std::lower_bound(rp.begin(), rp.begin() + rows,
                                       c * MP_CH) - rp.begin());
  rs[nch] = (int32_t)rows;
  std::vector<int32_t> xr, xs, xe;
  for (int64_t r = 0; r < rows; ++r) {
    if (rp[r + 1] == rp[r]) continue;
    const int64_t cs = rp[r] / MP_CH, ce = (rp[r + 1] - 1) / MP_CH;
    if (ce > cs) {
      xr.push_back((int32_t)r);
      xs.push_back((int32_t)cs);
      xe.push_back((int32_t)ce);
    }
  }
  mp->nchunk = nch;
  mp->ncross = (int64_t)xr.size();
  auto up = [&](const std::vector<int32_t> &v) {
    int32_t *d = h->pool.alloc<int32_t>(std::max<int64_t>(1, (int64_t)v.size()), false);
    if (!v.empty())
      HIPCHK(hipMemcpy(d, v.data(), sizeof(int32_t) * v.size(),
                       hipMemcpyHostToDevice));
    return d;
  };
  mp->rs = up(rs);
  mp->xrow = up(xr);
  mp->xcs = up(xs);
  mp->xce = up(xe);
}

void create_impl(rgdbek_ctx *h, const rgdbek_matrix *A) {
  hipStream_t st = h->st;
  Pool &P = h->pool;
  // Gram-based dense blocks are limited by the PCG's staging; row blocks
  // taller than A is wide go through CGLS and have no such limit (the
  // adjoint engine swaps the roles: its row blocks are the column blocks)
  if (h->dense && h->kc > pcg_cap_max())
    throw ApiError{RGDBEK_ERR_UNSUPPORTED,
                   "dense column blocks larger than " +
                       std::to_string(pcg_cap_max()) + " are not supported"};
  if (h->dense && (h->kr > pcg_cap_max() && h->kr <= h->n))
    throw ApiError{RGDBEK_ERR_UNSUPPORTED,
                   "dense row blocks larger than " +
                       std::to_string(pcg_cap_max()) +
                       " are not supported unless taller than A is wide"};
  h->ctrl = P.alloc<Ctrl>(1);
  HIPCHK(hipHostMalloc((void **)&h->hctrl, sizeof(Ctrl), hipHostMallocDefault));
  int *flag = P.alloc<int>(1);
  if (h->dense) {
    h->ld = round_up(std::max<int64_t>(h->n, 1), 8);
    h->ldc = round_up(std::max<int64_t>(h->m, 1), 8);
    h->a_rm = P.alloc<double>(h->m * h->ld, false);
    h->a_cm = P.alloc<double>(h->n * h->ldc, false);
    if (A->value_type == RGDBEK_F64) {
      launch_check_finite<double>((const double *)A->values, h->m * h->n, flag, st);
      launch_pack_dense<double, double>((const double *)A->values, h->m, h->n,
                                        h->n, h->a_rm, h->ld, h->a_cm, h->ldc, st);
    } else {
      launch_check_finite<float>((const float *)A->values, h->m * h->n, flag, st);
      launch_pack_dense<double, float>((const float *)A->values, h->m, h->n,
                                       h->n, h->a_rm, h->ld, h->a_cm, h->ldc, st);
    }
    h->rho = P.alloc<double>(h->m);
    h->kappa = P.alloc<double>(h->n);
    launch_sqnorms_dense<double>(h->a_rm, h->m, h->n, h->ld, h->a_cm, h->ldc,
                                 h->rho, h->kappa, st);
  } else {
    validate_csr(A);
    h->csr_ptr = P.alloc<int64_t>(h->m + 1, false);
    h->csr_idx = P.alloc<int32_t>(h->nnz, false);
    h->csr_val = P.alloc<double>(h->nnz, false);
    HIPCHK(hipMemcpyAsync(h->csr_ptr, A->row_ptr, 8 * (h->m + 1),
                          hipMemcpyDeviceToDevice, st));
    if (h->nnz)
      HIPCHK(hipMemcpyAsync(h->csr_idx, A->col_idx, 4 * h->nnz,
                            hipMemcpyDeviceToDevice, st));
    if (A->value_type == RGDBEK_F64) {
      launch_check_finite<double>((const double *)A->values, h->nnz, flag, st);
      launch_convert<double, double>((const double *)A->values, h->csr_val, h->nnz, st);
    } else {
      launch_check_finite<float>((const float *)A->values, h->nnz, flag, st);
      launch_convert<double, float>((const float *)A->values, h->csr_val, h->nnz, st);
    }
    h->csc_ptr = P.alloc<int64_t>(h->n + 1, false);
    h->csc_idx = P.alloc<int32_t>(h->nnz, false);
    h->csc_val = P.alloc<double>(h->nnz, false);
    int64_t *work = P.alloc<int64_t>(h->n + 1, false);
    launch_csr_to_csc<double>(h->m, h->n, h->nnz, h->csr_ptr, h->csr_idx,
                              h->csr_val, h->csc_ptr, h->csc_idx, h->csc_val,
                              work, st);
    HIPCHK(hipStreamSynchronize(st));
    const int gr = pick_group(h->m ? (double)h->nnz / h->m : 1.0);
    const int gc = pick_group(h->n ? (double)h->nnz / h->n : 1.0);
    build_longs(h, h->csr_ptr, h->m, 32LL * gr, &h->csr_longs, &h->csr_nlong);
    build_longs(h, h->csc_ptr, h->n, 32LL * gc, &h->csc_longs, &h->csc_nlong);
    build_merge_plan(h, h->csr_ptr, h->m, &h->csr_mp);
    build_merge_plan(h, h->csc_ptr, h->n, &h->csc_mp);
    h->rho = P.alloc<double>(h->m);
    h->kappa = P.alloc<double>(h->n);
    Csr<double> a, at;
    a.rows = h->m; a.ptr = h->csr_ptr; a.idx = h->csr_idx; a.val = h->csr_val;
    at.rows = h->n; at.ptr = h->csc_ptr; at.idx = h->csc_idx; at.val = h->csc_val;
    launch_sqnorms_csr<double>(a, h->rho, st);
    launch_sqnorms_csr<double>(at, h->kappa, st);
  }
  int hv = 0;
  HIPCHK(hipMemcpyAsync(&hv, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hv) throw ApiError{RGDBEK_ERR_NUMERIC, "matrix values contain NaN/Inf"};
  HIPCHK(hipStreamSynchronize(st));
}

// Work space and engines for the (virtual) dimensions h->m x h->n.
void build_engines(rgdbek_ctx *h) {
  Pool &P = h->pool;
  h->xref = P.alloc<double>(std::max(h->m, h->n) + 64);
  build_engine<double>(h, h->e64, false);
  if (h->p.precision == RGDBEK_PREC_MIXED_F32) {
    build_engine<float>(h, h->e32, false);
    h->x64 = P.alloc<double>(round_up(h->n, 8) + 64);
    h->z64 = P.alloc<double>(h->m + 64);
    h->zero64 = P.alloc<double>(h->m + 64);
    h->t64 = P.alloc<double>(h->n + 64);
  }
  HIPCHK(hipStreamSynchronize(h->st));
}

// Device copies of the per-system state (forward and adjoint orientation).
void upload_segments(rgdbek_ctx *h) {
  const int ns = h->nseg;
  h->seg = h->pool.alloc<SegInfo>(ns);
  h->seg_t = h->pool.alloc<SegInfo>(ns);
  h->fixed = h->pool.alloc<int32_t>(ns);
  std::vector<SegInfo> t(h->hseg);
  for (auto &g : t) {
    std::swap(g.row_off, g.col_off);
    std::swap(g.nrow, g.ncol);
    std::swap(g.kc, g.kr);
    std::swap(g.kc_off, g.kr_off);
  }
  // on the handle's stream, after the zero fills of the allocations above
  // (a plain hipMemcpy is not ordered after work on a non-blocking stream:
  // the fill could land after the copy and erase it)
  HIPCHK(hipMemcpyAsync(h->seg, h->hseg.data(), sizeof(SegInfo) * ns,
                        hipMemcpyHostToDevice, h->st));
  HIPCHK(hipMemcpyAsync(h->seg_t, t.data(), sizeof(SegInfo) * ns,
                        hipMemcpyHostToDevice, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
}

void destroy_impl(rgdbek_ctx *h) {
  if (h->st) (void)hipStreamSynchronize(h->st);
  for (auto &g : h->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  h->graphs.clear();
  for (hipEvent_t e : h->prof_events) (void)hipEventDestroy(e);
  h->prof_events.clear();
  h->pool.release();
  if (h->hctrl) (void)hipHostFree(h->hctrl);
  h->hctrl = nullptr;
  if (h->st && h->own_stream) (void)hipStreamDestroy(h->st);
  h->st = nullptr;
}

template <typename F>
rgdbek_status guarded(rgdbek_ctx *h, F &&f) {
  try {
    return f();
  } catch (const ApiError &e) {
    set_err(h, e.msg);
    return e.s;
  } catch (const HipError &e) {
    set_err(h, std::string("HIP error ") + hipGetErrorString(e.e) + " in " +
                   e.what);
    return RGDBEK_ERR_DEVICE;
  } catch (const std::bad_alloc &) {
    set_err(h, "host allocation failed");
    return RGDBEK_ERR_OUT_OF_MEMORY;
  } catch (...) {
    set_err(h, "unexpected internal error");
    return RGDBEK_ERR_DEVICE;
  }
}

}  // namespace

// ------------------------------------------------ allocation-free draw
// rgdbek_select_noalloc works in one static device array instead of
// hipMalloc'ed scratch.  Layout (byte offsets, each 256-aligned): the
// control block, the persistent draw's histograms and candidates, the
// multi-launch pipeline's histogram, candidates and per-chunk counts, then
// the d keys.  Every region but the keys is cleared at each call.
constexpr size_t na_align(size_t v) { return (v + 255) / 256 * 256; }
constexpr int64_t NA_BLK_N = RGDBEK_NOALLOC_MAX_D / 256 + 64;
constexpr size_t NA_CTRL = 0;
constexpr size_t NA_PERS = na_align(NA_CTRL + sizeof(Ctrl));
constexpr size_t NA_HIST = na_align(NA_PERS + sizeof(SelPersist));
constexpr size_t NA_CKEY = na_align(NA_HIST + 2048 * sizeof(unsigned));
constexpr size_t NA_CIDX = na_align(NA_CKEY + 4096 * sizeof(uint64_t));
constexpr size_t NA_BLK = na_align(NA_CIDX + 4096 * sizeof(int64_t));
constexpr size_t NA_KEYS = na_align(NA_BLK + NA_BLK_N * sizeof(int32_t));
constexpr size_t NA_BYTES =
    na_align(NA_KEYS + (RGDBEK_NOALLOC_MAX_D + 64) * sizeof(uint64_t));

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

__global__ void __launch_bounds__(256)
noalloc_zero_kernel(uint4 *p, int64_t n16) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16;
       i += (int64_t)gridDim.x * 256)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

namespace {
// Device address of `scratch` on the current device, looked up once per
// device: the host-side name is only a stand-in for the symbol.
unsigned char *noalloc_scratch_ptr() {
  static std::mutex mu;
  static std::vector<unsigned char *> addr;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw ApiError{RGDBEK_ERR_DEVICE, "no address for the static work space"};
    addr[dev] = (unsigned char *)p;
  }
  return addr[dev];
}
}  // namespace

// ============================================================ C-ABI
extern "C" {

rgdbek_status rgdbek_params_default(rgdbek_params *p) {
  if (!p) return RGDBEK_ERR_INVALID_ARG;
  std::memset(p, 0, sizeof(*p));
  p->eta = 0.5;
  p->tol = 1e-8;
  p->stop = RGDBEK_STOP_ERR_REF;
  p->precision = RGDBEK_PREC_FP64;
  p->max_iter = 10000;
  p->seed = 0;
  p->flags = RGDBEK_FLAG_GRAPH;
  return RGDBEK_OK;
}

rgdbek_status rgdbek_create(const rgdbek_matrix *A, const rgdbek_params *p,
                            void *stream, rgdbek_handle *out) {
  g_global_err.clear();
  if (!out) { set_err(nullptr, "out is NULL"); return RGDBEK_ERR_INVALID_ARG; }
  *out = nullptr;
  if (!A || !p) { set_err(nullptr, "A or p is NULL"); return RGDBEK_ERR_INVALID_ARG; }
  if (A->m <= 0 || A->n <= 0 || A->m > INT32_MAX || A->n > INT32_MAX) {
    set_err(nullptr, "m and n must lie in [1, 2^31)");
    return RGDBEK_ERR_INVALID_ARG;
  }
  if (A->layout != RGDBEK_DENSE_ROW_MAJOR && A->layout != RGDBEK_CSR) {
    set_err(nullptr, "unknown layout");
    return RGDBEK_ERR_INVALID_ARG;
  }
  if (A->value_type != RGDBEK_F64 && A->value_type != RGDBEK_F32) {
    set_err(nullptr, "unknown value type");
    return RGDBEK_ERR_INVALID_ARG;
  }
  if (!A->values) { set_err(nullptr, "values is NULL"); return RGDBEK_ERR_INVALID_ARG; }
  if (A->layout == RGDBEK_CSR) {
    if (!A->row_ptr || (!A->col_idx && A->nnz > 0) || A->nnz < 0 ||
        A->nnz > INT32_MAX) {
      set_err(nullptr, "CSR needs row_ptr, col_idx and 0 <= nnz < 2^31");
      return RGDBEK_ERR_INVALID_ARG;
    }
  } else if (A->row_ptr || A->col_idx) {
    set_err(nullptr, "dense layout takes no row_ptr/col_idx");
    return RGDBEK_ERR_INVALID_ARG;
  }
  rgdbek_ctx *h = new (std::nothrow) rgdbek_ctx();
  if (!h) { set_err(nullptr, "host allocation failed"); return RGDBEK_ERR_OUT_OF_MEMORY; }
  h->m = A->m;
  h->n = A->n;
  h->dense = A->layout == RGDBEK_DENSE_ROW_MAJOR;
  h->nnz = h->dense ? A->m * A->n : A->nnz;
  h->p = *p;
  h->user_st = (hipStream_t)stream;
  rgdbek_status s = guarded(nullptr, [&]() {
    validate_params(p, h->m, h->n, &h->kc, &h->kr);
    // HIP graphs cannot be captured on the legacy default stream: a NULL
    // stream gets a private non-blocking stream (default priority)
    if (h->user_st) {
      h->st = h->user_st;
    } else {
      HIPCHK(hipStreamCreateWithFlags(&h->st, hipStreamNonBlocking));
      h->own_stream = true;
    }
    h->pool.st = h->st;
    HIPCHK(hipStreamSynchronize(h->user_st));
    h->ncu = device_cus();
    h->bm = h->m;
    h->bn = h->n;
    create_impl(h, A);
    build_engines(h);
    return RGDBEK_OK;
  });
  if (s != RGDBEK_OK) {
    destroy_impl(h);
    delete h;
    return s;
  }
  *out = h;
  return RGDBEK_OK;
}

rgdbek_status rgdbek_create_batched(const rgdbek_matrix *A, int64_t nsys,
                                    const int64_t *row_off,
                                    const int64_t *col_off,
                                    const rgdbek_params *p, void *stream,
                                    rgdbek_handle *out) {
  g_global_err.clear();
  if (!out) { set_err(nullptr, "out is NULL"); return RGDBEK_ERR_INVALID_ARG; }
  *out = nullptr;
  if (!A || !p || !row_off || !col_off || nsys < 1 || nsys > (1 << 20)) {
    set_err(nullptr, "A, p, row_off, col_off required and 1 <= nsys <= 2^20");
    return RGDBEK_ERR_INVALID_ARG;
  }
  if (A->layout != RGDBEK_CSR) {
    set_err(nullptr, "batched systems are stored block-diagonally in CSR");
    return RGDBEK_ERR_UNSUPPORTED;
  }
  if (row_off[0] != 0 || col_off[0] != 0 || row_off[nsys] != A->m ||
      col_off[nsys] != A->n) {
    set_err(nullptr, "row_off/col_off must start at 0 and end at m/n");
    return RGDBEK_ERR_INVALID_ARG;
  }
  for (int64_t s = 0; s < nsys; ++s)
    if (row_off[s + 1] <= row_off[s] || col_off[s + 1] <= col_off[s]) {
      set_err(nullptr, "every system needs at least one row and one column");
      return RGDBEK_ERR_INVALID_ARG;
    }
  rgdbek_params q = *p;
  std::vector<SegInfo> segs(nsys);
  int64_t kc_tot = 0, kr_tot = 0;
  auto bs = [&](int64_t kfix, int64_t d) -> int64_t {
    if (kfix > 0) return std::min<int64_t>(kfix, d);
    int64_t k = (int64_t)std::floor(p->eta * (double)d + 0.5);
    return std::min<int64_t>(d, std::max<int64_t>(1, k));
  };
  for (int64_t s = 0; s < nsys; ++s) {
    SegInfo g{};
    g.row_off = row_off[s];
    g.nrow = row_off[s + 1] - row_off[s];
    g.col_off = col_off[s];
    g.ncol = col_off[s + 1] - col_off[s];
    g.kc = bs(p->k_col, g.ncol);
    g.kr = bs(p->k_row, g.nrow);
    g.kc_off = kc_tot;
    g.kr_off = kr_tot;
    kc_tot += g.kc;
    kr_tot += g.kr;
    segs[s] = g;
  }
  q.k_col = kc_tot;
  q.k_row = kr_tot;
  rgdbek_ctx *h = new (std::nothrow) rgdbek_ctx();
  if (!h) { set_err(nullptr, "host allocation failed"); return RGDBEK_ERR_OUT_OF_MEMORY; }
  h->m = A->m;
  h->n = A->n;
  h->dense = false;
  h->nnz = A->nnz;
  h->p = q;
  h->user_st = (hipStream_t)stream;
  h->nseg = (int)nsys;
  h->hseg = segs;
  rgdbek_status st = guarded(nullptr, [&]() {
    int64_t kc, kr;
    validate_params(&q, h->m, h->n, &kc, &kr);
    if (q.select_mode != RGDBEK_SELECT_RANDOM)
      throw ApiError{RGDBEK_ERR_UNSUPPORTED,
                     "greedy and block-law rules: single systems only"};
    h->kc = kc_tot;
    h->kr = kr_tot;
    if (!A->row_ptr || (!A->col_idx && A->nnz > 0) || !A->values || A->nnz < 0 ||
        A->nnz > INT32_MAX || A->m > INT32_MAX || A->n > INT32_MAX)
      throw ApiError{RGDBEK_ERR_INVALID_ARG, "CSR arrays and sizes required"};
    // block-diagonal structure: every row's columns inside its system
    std::vector<int64_t> rp(A->m + 1);
    std::vector<int32_t> ci(A->nnz);
    HIPCHK(hipMemcpy(rp.data(), A->row_ptr, 8 * (A->m + 1), hipMemcpyDeviceToHost));
    if (A->nnz)
      HIPCHK(hipMemcpy(ci.data(), A->col_idx, 4 * A->nnz, hipMemcpyDeviceToHost));
    for (int64_t s = 0; s < nsys; ++s)
      for (int64_t i = row_off[s]; i < row_off[s + 1]; ++i)
        for (int64_t e = rp[i]; e < rp[i + 1] && e < A->nnz; ++e)
          if (ci[e] < col_off[s] || ci[e] >= col_off[s + 1])
            throw ApiError{RGDBEK_ERR_INVALID_ARG,
                           "row " + std::to_string(i) + " leaves its system's columns"};
    if (h->user_st) {
      h->st = h->user_st;
    } else {
      HIPCHK(hipStreamCreateWithFlags(&h->st, hipStreamNonBlocking));
      h->own_stream = true;
    }
    h->pool.st = h->st;
    HIPCHK(hipStreamSynchronize(h->user_st));
    h->ncu = device_cus();
    h->bm = h->m;
    h->bn = h->n;
    create_impl(h, A);
    upload_segments(h);
    build_engines(h);
    return RGDBEK_OK;
  });
  if (st != RGDBEK_OK) {
    destroy_impl(h);
    delete h;
    return st;
  }
  *out = h;
  return RGDBEK_OK;
}

rgdbek_status rgdbek_create_multirhs(const rgdbek_matrix *A, int64_t nrhs,
                                     const rgdbek_params *p, void *stream,
                                     rgdbek_handle *out) {
  g_global_err.clear();
  if (!out) { set_err(nullptr, "out is NULL"); return RGDBEK_ERR_INVALID_ARG; }
  *out = nullptr;
  if (!A || !p || nrhs < 1 || nrhs > 4096) {
    set_err(nullptr, "A and p required, 1 <= nrhs <= 4096");
    return RGDBEK_ERR_INVALID_ARG;
  }
  if (A->layout != RGDBEK_CSR) {
    set_err(nullptr, "right-hand-side batches share a CSR matrix");
    return RGDBEK_ERR_UNSUPPORTED;
  }
  if (A->m <= 0 || A->n <= 0 || A->m * nrhs > INT32_MAX ||
      A->n * nrhs > INT32_MAX || !A->values || !A->row_ptr ||
      (!A->col_idx && A->nnz > 0) || A->nnz < 0 || A->nnz > INT32_MAX) {
    set_err(nullptr, "CSR arrays required; nrhs * m and nrhs * n < 2^31");
    return RGDBEK_ERR_INVALID_ARG;
  }
  auto bs = [&](int64_t kfix, int64_t d) -> int64_t {
    if (kfix > 0) return std::min<int64_t>(kfix, d);
    int64_t k = (int64_t)std::floor(p->eta * (double)d + 0.5);
    return std::min<int64_t>(d, std::max<int64_t>(1, k));
  };
  const int64_t kc = bs(p->k_col, A->n), kr = bs(p->k_row, A->m);
  std::vector<SegInfo> segs(nrhs);
  for (int64_t s = 0; s < nrhs; ++s) {
    SegInfo g{};
    g.row_off = s * A->m; g.nrow = A->m;
    g.col_off = s * A->n; g.ncol = A->n;
    g.kc = kc; g.kr = kr;
    g.kc_off = s * kc; g.kr_off = s * kr;
    segs[s] = g;
  }
  rgdbek_params q = *p;
  q.k_col = kc;
  q.k_row = kr;
  rgdbek_ctx *h = new (std::nothrow) rgdbek_ctx();
  if (!h) { set_err(nullptr, "host allocation failed"); return RGDBEK_ERR_OUT_OF_MEMORY; }
  h->m = A->m;
  h->n = A->n;
  h->bm = A->m;
  h->bn = A->n;
  h->dense = false;
  h->nnz = A->nnz;
  h->p = q;
  h->user_st = (hipStream_t)stream;
  h->nseg = (int)nrhs;
  h->rep = nrhs;
  h->hseg = segs;
  rgdbek_status st = guarded(nullptr, [&]() {
    int64_t k1, k2;
    validate_params(&q, A->m, A->n, &k1, &k2);
    if (q.select_mode != RGDBEK_SELECT_RANDOM)
      throw ApiError{RGDBEK_ERR_UNSUPPORTED,
                     "greedy and block-law rules: single systems only"};
    if (h->user_st) {
      h->st = h->user_st;
    } else {
      HIPCHK(hipStreamCreateWithFlags(&h->st, hipStreamNonBlocking));
      h->own_stream = true;
    }
    h->pool.st = h->st;
    HIPCHK(hipStreamSynchronize(h->user_st));
    h->ncu = device_cus();
    create_impl(h, A);
    // the batch sees I_nrhs (x) A: replicate the norms, widen the dimensions
    double *rho = h->pool.alloc<double>(A->m * nrhs, false);
    double *kap = h->pool.alloc<double>(A->n * nrhs, false);
    launch_replicate(h->rho, A->m, nrhs, rho, h->st);
    launch_replicate(h->kappa, A->n, nrhs, kap, h->st);
    h->rho = rho;
    h->kappa = kap;
    h->m = A->m * nrhs;
    h->n = A->n * nrhs;
    h->kc = kc * nrhs;
    h->kr = kr * nrhs;
    upload_segments(h);
    build_engines(h);
    return RGDBEK_OK;
  });
  if (st != RGDBEK_OK) {
    destroy_impl(h);
    delete h;
    return st;
  }
  *out = h;
  return RGDBEK_OK;
}

rgdbek_status rgdbek_batch_info(rgdbek_handle h, int64_t *iterations,
                                double *metric, int32_t *converged) {
  if (!h) return RGDBEK_ERR_INVALID_ARG;
  if (!h->nseg) {
    set_err(h, "not a batched handle");
    return RGDBEK_ERR_INVALID_ARG;
  }
  return guarded(h, [&]() {
    std::vector<SegInfo> g(h->nseg);
    HIPCHK(hipMemcpyAsync(g.data(), h->seg, sizeof(SegInfo) * h->nseg,
                          hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    for (int s = 0; s < h->nseg; ++s) {
      if (iterations) iterations[s] = g[s].iters_run;
      if (metric) metric[s] = g[s].metric;
      if (converged) converged[s] = g[s].converged;
    }
    return RGDBEK_OK;
  });
}

rgdbek_status rgdbek_solve(rgdbek_handle h, const void *b, void *x,
                           const void *x_ref, rgdbek_info *info) {
  if (!h) return RGDBEK_ERR_INVALID_ARG;
  h->err.clear();
  if (!b || !x) { set_err(h, "b and x are required"); return RGDBEK_ERR_INVALID_ARG; }
  if (h->p.stop == RGDBEK_STOP_ERR_REF && !x_ref) {
    set_err(h, "STOP_ERR_REF needs x_ref");
    return RGDBEK_ERR_INVALID_ARG;
  }
  return guarded(h, [&]() {
    HIPCHK(hipStreamSynchronize(h->user_st));
    if (h->p.precision == RGDBEK_PREC_MIXED_F32)
      return solve_mixed(h, (const double *)b, (double *)x,
                         (const double *)x_ref, info);
    return solve64(h, h->e64, 0, 0, h->p.stop, (const double *)b, (double *)x,
                   nullptr, 0, false, (const double *)x_ref, info);
  });
}

rgdbek_status rgdbek_solve_resume(rgdbek_handle h, const void *b, void *x,
                                  void *z, int64_t it0, const void *x_ref,
                                  rgdbek_info *info) {
  if (!h) return RGDBEK_ERR_INVALID_ARG;
  h->err.clear();
  if (!b || !x || !z || it0 < 0) {
    set_err(h, "b, x, z are required and it0 must be >= 0");
    return RGDBEK_ERR_INVALID_ARG;
  }
  if (h->p.stop == RGDBEK_STOP_ERR_REF && !x_ref) {
    set_err(h, "STOP_ERR_REF needs x_ref");
    return RGDBEK_ERR_INVALID_ARG;
  }
  if (h->p.precision != RGDBEK_PREC_FP64) {
    set_err(h, "resume is defined for the FP64 form");
    return RGDBEK_ERR_UNSUPPORTED;
  }
  return guarded(h, [&]() {
    HIPCHK(hipStreamSynchronize(h->user_st));
    return solve64(h, h->e64, 0, 0, h->p.stop, (const double *)b, (double *)x,
                   (double *)z, it0, true, (const double *)x_ref, info);
  });
}

rgdbek_status rgdbek_get_z(rgdbek_handle h, void *z) {
  if (!h || !z) return RGDBEK_ERR_INVALID_ARG;
  return guarded(h, [&]() {
    HIPCHK(hipStreamSynchronize(h->user_st));
    HIPCHK(hipMemcpyAsync(z, h->e64.z, sizeof(double) * h->m,
                          hipMemcpyDeviceToDevice, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    return RGDBEK_OK;
  });
}

rgdbek_status rgdbek_solve_adjoint(rgdbek_handle h, const void *g, void *w,
                                   rgdbek_info *info) {
  if (!h) return RGDBEK_ERR_INVALID_ARG;
  h->err.clear();
  if (!g || !w) { set_err(h, "g and w are required"); return RGDBEK_ERR_INVALID_ARG; }
  return guarded(h, [&]() {
    HIPCHK(hipStreamSynchronize(h->user_st));
    // the adjoint's column blocks are the forward row blocks: a tall row
    // block above the Gram limit has no column projection on A^T
    if (h->dense && h->kr > pcg_cap_max())
      throw ApiError{RGDBEK_ERR_UNSUPPORTED,
                     "adjoint solve: dense row blocks larger than " +
                         std::to_string(pcg_cap_max()) + " are not supported"};
    if (!h->e64t.ready) build_engine<double>(h, h->e64t, true);
    int stop = h->p.stop == RGDBEK_STOP_ERR_REF ? RGDBEK_STOP_RES_EXT : h->p.stop;
    return solve64(h, h->e64t, 1, 1, stop, (const double *)g, (double *)w,
                   nullptr, 0, false, nullptr, info);
  });
}

rgdbek_status rgdbek_grad_pattern(rgdbek_handle h, const void *r,
                                  const void *lam, const void *w,
                                  const void *x, void *dA_values) {
  if (!h) return RGDBEK_ERR_INVALID_ARG;
  h->err.clear();
  if (!w || !x || !dA_values || (lam && !r)) {
    set_err(h, "w, x and dA_values are required (and r with lam)");
    return RGDBEK_ERR_INVALID_ARG;
  }
  return guarded(h, [&]() {
    HIPCHK(hipStreamSynchronize(h->user_st));
    if (h->dense)
      launch_grad_pattern_dense(h->m, h->n, (const double *)r,
                                (const double *)lam, (const double *)w,
                                (const double *)x, (double *)dA_values, h->st);
    else
      launch_grad_pattern_csr(h->bm, h->bn, h->rep, h->csr_ptr, h->csr_idx,
                              (const double *)r,
                              (const double *)lam, (const double *)w,
                              (const double *)x, (double *)dA_values, h->st);
    HIPCHK(hipStreamSynchronize(h->st));
    return RGDBEK_OK;
  });
}

rgdbek_status rgdbek_apply(rgdbek_handle h, int32_t precision, const void *x,
                           const void *z, void *ax, void *atz) {
  if (!h) return RGDBEK_ERR_INVALID_ARG;
  h->err.clear();
  if (!x || !z || !ax || !atz) {
    set_err(h, "x, z, ax and atz are required");
    return RGDBEK_ERR_INVALID_ARG;
  }
  if (precision != RGDBEK_F64 && precision != RGDBEK_F32) {
    set_err(h, "precision must be RGDBEK_F64 or RGDBEK_F32");
    return RGDBEK_ERR_INVALID_ARG;
  }
  if (precision == RGDBEK_F32 && !h->e32.ready) {
    set_err(h, "FP32 storage exists only for a MIXED_F32 handle");
    return RGDBEK_ERR_UNSUPPORTED;
  }
  return guarded(h, [&]() {
    // no host synchronisation: stream order when the handle runs on the
    // caller's stream, an event dependency in both directions otherwise
    stream_after(h->st, h->user_st);
    auto run = [&](auto &e, auto *xv, auto *zv, auto *axv, auto *atzv) {
      using T = typename std::remove_pointer<decltype(axv)>::type;
      if (e.dense) {
        // the fused pass reads x up to the padded leading dimension: stage
        // it when padding exists
        const T *xp = xv;
        if (e.arm.ld != e.n) {
          HIPCHK(hipMemcpyAsync(e.x, xv, sizeof(T) * e.n, hipMemcpyDeviceToDevice, h->st));
          xp = e.x;
        }
        launch_dense_fused<T>(e.arm, xp, zv, e.dw, nullptr, e.kappa, atzv,
                              e.eps_z, axv, h->ctrl, 0, h->st);
      } else {
        SegArgs<T> a;
        a.v = xv; a.out = axv;
        launch_segdot<T>(e.csr, EPI_STORE, a, h->ctrl, 0, h->st);
        SegArgs<T> c;
        c.v = zv; c.out = atzv;
        launch_segdot<T>(e.csc, EPI_STORE, c, h->ctrl, 0, h->st);
      }
    };
    if (precision == RGDBEK_F64)
      run(h->e64, (const double *)x, (const double *)z, (double *)ax, (double *)atz);
    else
      run(h->e32, (const float *)x, (const float *)z, (float *)ax, (float *)atz);
    HIPCHK(hipGetLastError());
    stream_after(h->user_st, h->st);
    return RGDBEK_OK;
  });
}

rgdbek_status rgdbek_select(const double *eps, int64_t d, int64_t k,
                            double floor, uint64_t seed, uint64_t key1,
                            uint64_t it,
                            uint32_t phase, uint32_t sys, int32_t *out_idx,
                            int64_t *out_count, void *stream) {
  g_global_err.clear();
  if (!eps || !out_idx || !out_count || d <= 0 || k < 0 || d > INT32_MAX) {
    set_err(nullptr, "eps, out_idx, out_count required; 0 < d < 2^31, k >= 0");
    return RGDBEK_ERR_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  Pool P;
  P.st = st;
  rgdbek_status s = guarded(nullptr, [&]() {
    SelectScratch sc;
    sc.pers = P.alloc<SelPersist>(1);
    sc.ncu = device_cus();
    sc.keys = P.alloc<uint64_t>(d + 64, false);
    sc.hist = P.alloc<unsigned>(2048);
    sc.ckey = P.alloc<uint64_t>(4096);
    sc.cidx = P.alloc<int64_t>(4096);
    sc.blk = P.alloc<int32_t>(select_scratch_blocks(d) + 64);
    Ctrl *c = P.alloc<Ctrl>(1);
    launch_fill_ctrl_it(c, (int64_t)it, st);
    launch_select<double>(eps, d, k, floor, seed, key1, phase, sys, 0, sc,
                          out_idx, c, 0, st);
    Ctrl hc;
    HIPCHK(hipMemcpyAsync(&hc, c, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipGetLastError());
    *out_count = hc.sel_count[0];
    if (hc.sync_fail)
      throw ApiError{RGDBEK_ERR_DEVICE, "a grid-barrier wait timed out"};
    if (hc.numeric)
      throw ApiError{RGDBEK_ERR_NUMERIC, "weights must be finite and >= 0"};
    return RGDBEK_OK;
  });
  P.release();
  return s;
}

rgdbek_status rgdbek_select_block_law(const double *eps, int64_t d, int64_t s,
                                      double floor, uint64_t seed,
                                      uint64_t key1, uint64_t it,
                                      uint32_t phase, uint32_t sys,
                                      int32_t *out_idx, int64_t *out_count,
                                      void *stream) {
  if (!eps || !out_idx || !out_count || d <= 0 || s <= 0 || d > INT32_MAX) {
    set_err(nullptr, "invalid arguments to rgdbek_select_block_law");
    return RGDBEK_ERR_INVALID_ARG;
  }
  if (s > d) s = d;
  hipStream_t st = (hipStream_t)stream;
  Pool P;
  P.st = st;
  rgdbek_status r = guarded(nullptr, [&]() {
    SelectScratch sc;
    sc.pers = P.alloc<SelPersist>(1);
    sc.ncu = device_cus();
    sc.keys = P.alloc<uint64_t>(d + 64, false);
    sc.hist = P.alloc<unsigned>(2048);
    sc.ckey = P.alloc<uint64_t>(4096);
    sc.cidx = P.alloc<int64_t>(4096);
    sc.blk = P.alloc<int32_t>(select_scratch_blocks(d) + 64);
    double *w = P.alloc<double>(d + 64);
    int32_t *tmp = P.alloc<int32_t>(s + 64);
    Ctrl *c = P.alloc<Ctrl>(1);
    launch_fill_ctrl_it(c, (int64_t)it, st);
    launch_select_block_law<double>(eps, d, s, floor, seed, key1, phase, sys, 0,
                                    sc, w, tmp, out_idx, c, 0, st);
    Ctrl hc;
    HIPCHK(hipMemcpyAsync(&hc, c, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipGetLastError());
    *out_count = hc.sel_count[0];
    if (hc.sync_fail)
      throw ApiError{RGDBEK_ERR_DEVICE, "a grid-barrier wait timed out"};
    if (hc.numeric)
      throw ApiError{RGDBEK_ERR_NUMERIC, "weights must be finite and >= 0"};
    return RGDBEK_OK;
  });
  P.release();
  return r;
}

rgdbek_status rgdbek_select_iid(const double *eps, int64_t d, int64_t k,
                                double floor, uint64_t seed, uint64_t key1,
                                uint64_t it, uint32_t phase, uint32_t sys,
                                int32_t *out_idx, int64_t *out_count,
                                void *stream) {
  if (!eps || !out_idx || !out_count || d <= 0 || k <= 0 ||
      d > select_iid_max_d()) {
    set_err(nullptr, "invalid arguments to rgdbek_select_iid");
    return RGDBEK_ERR_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  Pool P;
  P.st = st;
  rgdbek_status r = guarded(nullptr, [&]() {
    SelectScratch sc;
    sc.blk = P.alloc<int32_t>(select_iid_chunks(d) + 64);
    sc.gmax = P.alloc<double>(select_iid_chunks(d) + 64);
    IidScratch w;
    w.ploc = P.alloc<uint64_t>(d + 64);
    w.ctot = P.alloc<uint64_t>(select_iid_chunks(d) + 64);
    w.flags = P.alloc<int32_t>(d + 64);
    Ctrl *c = P.alloc<Ctrl>(1);
    launch_fill_ctrl_it(c, (int64_t)it, st);
    launch_select_iid<double>(eps, d, k, floor, seed, key1, phase, sys, 0, sc,
                              w, out_idx, c, 0, st);
    Ctrl hc;
    HIPCHK(hipMemcpyAsync(&hc, c, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipGetLastError());
    *out_count = hc.sel_count[0];
    if (hc.numeric)
      throw ApiError{RGDBEK_ERR_NUMERIC, "weights must be finite and >= 0"};
    return RGDBEK_OK;
  });
  P.release();
  return r;
}

rgdbek_status rgdbek_select_threshold(const double *eps, int64_t d, double eta,
                                      int64_t cap, int32_t *out_idx,
                                      int64_t *out_count, void *stream) {
  if (!eps || !out_count || d < 0 || cap < 0 || (cap > 0 && !out_idx) ||
      !(eta > 0.0) || eta > 1.0) {
    set_err(nullptr, "invalid arguments to rgdbek_select_threshold");
    return RGDBEK_ERR_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  Pool P;
  P.st = st;
  rgdbek_status s = guarded(nullptr, [&]() {
    *out_count = 0;
    if (d == 0) return RGDBEK_OK;
    SelectScratch sc;
    sc.blk = P.alloc<int32_t>(select_greedy_blocks(d) + 64);
    sc.gmax = P.alloc<double>(select_greedy_blocks(d) + 64);
    int32_t *o = out_idx ? out_idx : P.alloc<int32_t>(1);
    Ctrl *c = P.alloc<Ctrl>(1);
    launch_select_greedy<double>(eps, d, eta, cap, 0, sc, o, c, 0, st);
    Ctrl hc;
    HIPCHK(hipMemcpyAsync(&hc, c, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipGetLastError());
    *out_count = hc.sel_count[0];
    if (hc.numeric)
      throw ApiError{RGDBEK_ERR_NUMERIC, "weights must be finite and >= 0"};
    return RGDBEK_OK;
  });
  P.release();
  return s;
}

rgdbek_status rgdbek_select_noalloc(const double *eps, int64_t d, int64_t k,
                                    double floor, uint64_t seed, uint64_t key1,
                                    uint64_t it, uint32_t phase, uint32_t sys,
                                    int32_t *out_idx, int64_t *out_count,
                                    void *stream) {
  g_global_err.clear();
  if (!eps || !out_idx || !out_count || d <= 0 || k < 0) {
    set_err(nullptr, "eps, out_idx, out_count required; d > 0, k >= 0");
    return RGDBEK_ERR_INVALID_ARG;
  }
  if (d > RGDBEK_NOALLOC_MAX_D) {
    set_err(nullptr, "rgdbek_select_noalloc: d = " + std::to_string(d) +
                         " exceeds its static work space (at most " +
                         std::to_string((long long)RGDBEK_NOALLOC_MAX_D) +
                         " weights); use rgdbek_select");
    return RGDBEK_ERR_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  return guarded(nullptr, [&]() {
    unsigned char *base = noalloc_scratch_ptr();
    if (select_scratch_blocks(d) + 64 > NA_BLK_N)
      throw ApiError{RGDBEK_ERR_INVALID_ARG, "block count exceeds the work space"};
    SelectScratch sc;
    sc.pers = (SelPersist *)(base + NA_PERS);
    sc.ncu = device_cus();
    sc.keys = (uint64_t *)(base + NA_KEYS);
    sc.hist = (unsigned *)(base + NA_HIST);
    sc.ckey = (uint64_t *)(base + NA_CKEY);
    sc.cidx = (int64_t *)(base + NA_CIDX);
    sc.blk = (int32_t *)(base + NA_BLK);
    Ctrl *c = (Ctrl *)(base + NA_CTRL);
    // the previous call's contents stay in the array: clear everything but
    // the keys (which every draw writes before reading) with a kernel
    hipLaunchKernelGGL(noalloc_zero_kernel, dim3(64), dim3(256), 0, st,
                       (uint4 *)base, (int64_t)(NA_KEYS / sizeof(uint4)));
    launch_fill_ctrl_it(c, (int64_t)it, st);
    launch_select<double>(eps, d, k, floor, seed, key1, phase, sys, 0, sc,
                          out_idx, c, 0, st);
    Ctrl hc;
    HIPCHK(hipMemcpyAsync(&hc, c, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipGetLastError());
    *out_count = hc.sel_count[0];
    if (hc.sync_fail)
      throw ApiError{RGDBEK_ERR_DEVICE, "a grid-barrier wait timed out"};
    if (hc.numeric)
      throw ApiError{RGDBEK_ERR_NUMERIC, "weights must be finite and >= 0"};
    return RGDBEK_OK;
  });
}

rgdbek_status rgdbek_profile_read(rgdbek_handle h, int32_t region,
                                  int64_t *launches, double *ms,
                                  int64_t *steps) {
  if (!h) return RGDBEK_ERR_INVALID_ARG;
  if (region < 0 || region >= RGDBEK_PROF_COUNT) {
    set_err(h, "unknown profile region");
    return RGDBEK_ERR_INVALID_ARG;
  }
  if (!(h->p.flags & RGDBEK_FLAG_PROFILE)) {
    set_err(h, "the handle was created without RGDBEK_FLAG_PROFILE");
    return RGDBEK_ERR_UNSUPPORTED;
  }
  const auto &r = h->prof[region];
  if (launches) *launches = r.launches;
  if (ms) *ms = r.ms;
  if (steps) *steps = r.steps;
  return RGDBEK_OK;
}

rgdbek_status rgdbek_destroy(rgdbek_handle h) {
  if (!h) return RGDBEK_OK;
  destroy_impl(h);
  delete h;
  return RGDBEK_OK;
}

const char *rgdbek_status_string(rgdbek_status s) {
  switch (s) {
    case RGDBEK_OK: return "ok";
    case RGDBEK_ERR_INVALID_ARG: return "invalid argument";
    case RGDBEK_ERR_NUMERIC: return "numeric error (NaN/Inf)";
    case RGDBEK_ERR_NOT_CONVERGED: return "not converged within max_iter";
    case RGDBEK_ERR_OUT_OF_MEMORY: return "out of device memory";
    case RGDBEK_ERR_DEVICE: return "device (HIP) error";
    case RGDBEK_ERR_UNSUPPORTED: return "unsupported request";
  }
  return "unknown status";
}

const char *rgdbek_last_error(rgdbek_handle h) {
  return h ? h->err.c_str() : g_global_err.c_str();
}

}  // extern "C"
