// solver.hip -- CG solvers on even sites: plain FP64 CG and mixed-precision
// CG with reliable updates (the paper's inverter does most of its arithmetic
// in single precision, section "GTX Titan Black"; the QUDA CG it moves to is
// mixed precision as well, section "CPS & QUDA").
//
// One iteration, all columns at once, all scalars on the device:
//   p   = r + beta p, |p|^2            (vector kernel, into the other p buffer)
//   t   = D_oe p, |t|^2                (sloppy Dslash)
//   alpha = rr / (4m^2 |p|^2 + |t|^2)  (= rr / <p, A p>, since D_eo = -D_oe^dag)
//   Ap = 4m^2 p - D_eo t in registers; r -= alpha Ap, x += alpha p, |r|^2
//                                      (sloppy Dslash, update epilogue)
//   beta = |r|^2 / rr; triggers; p buffer swap
// The sums are fixed-order FP64 reductions in one-block-per-column scalar
// kernels.  Every `poll` iterations the reliable update runs for the columns
// that asked for it: the FP32 x accumulator is folded into the FP64 x, and
// r = b - A x is recomputed with the FP64 operator, which also decides
// convergence on the true residual.  The host only polls the column flags
// between blocks (one block ahead, so the GPU never waits on the host); a
// block can be captured once into a hipGraph and replayed.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <string>
#include <vector>

#include "asq_internal.h"
#include "asq_solver.h"
#include "asq_batch.h"

namespace asq {

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string& msg) { g_last_error = msg; }

bool log_enabled() {
  static int on = -1;
  if (on < 0) {
    const char* e = getenv("ASQ_LOG");
    on = (e && *e && *e != '0') ? 1 : 0;
  }
  return on == 1;
}

bool env_flag(const char* name, bool dflt) {
  const char* e = getenv(name);
  if (!e || !*e) return dflt;
  return *e != '0';
}

int mode_pt(int mode) { return mode == ASQ_MODE_F64 ? VEC_F64 : (mode == ASQ_MODE_MIXED32 ? VEC_F32 : VEC_F16); }
int mode_rt(int mode) { return mode == ASQ_MODE_F64 ? VEC_F64 : VEC_F32; }

int sloppy_link(const asq_gauge* g, int mode) {
  if (mode == ASQ_MODE_F64) return LINK_F64_R18;
  if (mode == ASQ_MODE_MIXED32) return g->sloppy_link32;
  return g->sloppy_link16;
}

size_t batch_bytes(const asq_gauge* g, int ncol, int mode, bool with_bx) {
  const size_t half = (size_t)g->geom.half;
  const int pt = mode_pt(mode), rt = mode_rt(mode);
  size_t n = 0;
  n += 2 * align_up((size_t)ncol * sizeof(ColState), 256);  // states (two copies)
  n += 3 * align_up((size_t)ncol * g->nblk * sizeof(double), 256);  // partials (three sets)
  n += align_up((size_t)ncol * half * vec_site_bytes(rt), 256);      // r
  n += 3 * align_up((size_t)ncol * half * vec_site_bytes(pt), 256);  // p, p_alt, t
  if (mode != ASQ_MODE_F64) n += align_up((size_t)ncol * half * 48, 256);  // t64
  if (mode != ASQ_MODE_F64) n += align_up((size_t)ncol * half * 24, 256);  // x_s
  if (with_bx) n += 2 * align_up((size_t)ncol * half * 48, 256);         // b, x
  return n;
}

int next_mode(int mode) {
  return mode == ASQ_MODE_MIXED16 ? ASQ_MODE_MIXED32 : (mode == ASQ_MODE_MIXED32 ? ASQ_MODE_F64 : -1);
}

static size_t chain_bytes(const asq_gauge* g, int ncol, int mode) {
  size_t n = 0;
  for (int m = mode; m >= 0; m = next_mode(m)) n = std::max(n, batch_bytes(g, ncol, m, false));
  return n;
}

// The gathered b and x of each escalation level sit at the end of the
// workspace, the later levels' below the earlier ones.
size_t solve_bytes(const asq_gauge* g, int ncol, int mode) {
  int levels = 0;
  for (int m = next_mode(mode); m >= 0; m = next_mode(m)) ++levels;
  return chain_bytes(g, ncol, mode) + levels * 2 * align_up((size_t)ncol * g->geom.half * 48, 256);
}

int batch_carve(Batch& B, const asq_gauge* g, int ncol, int mode, void* work, size_t bytes, const double* b,
                double* x) {
  const size_t need = batch_bytes(g, ncol, mode, b == nullptr);
  if (bytes < need) return ASQ_ENOMEM;
  const size_t half = (size_t)g->geom.half;
  const int pt = mode_pt(mode), rt = mode_rt(mode);
  char* q = (char*)work;
  auto take = [&](size_t n) {
    char* r = q;
    q += align_up(n, 256);
    return (void*)r;
  };
  B.g = g;
  B.ncol = ncol;
  B.mode = mode;
  B.pt = pt;
  B.rt = rt;
  B.st = (ColState*)take((size_t)ncol * sizeof(ColState));
  B.partials = (double*)take((size_t)ncol * g->nblk * sizeof(double));
  B.partials_p = (double*)take((size_t)ncol * g->nblk * sizeof(double));
  B.partials_t = (double*)take((size_t)ncol * g->nblk * sizeof(double));
  B.r = take((size_t)ncol * half * vec_site_bytes(rt));
  B.p = take((size_t)ncol * half * vec_site_bytes(pt));
  B.p_alt = take((size_t)ncol * half * vec_site_bytes(pt));
  B.t = take((size_t)ncol * half * vec_site_bytes(pt));
  B.t64 = mode == ASQ_MODE_F64 ? B.t : take((size_t)ncol * half * 48);
  B.xs = mode == ASQ_MODE_F64 ? nullptr : take((size_t)ncol * half * 24);
  if (b == nullptr) {
    B.b = (double*)take((size_t)ncol * half * 48);
    B.x = (double*)take((size_t)ncol * half * 48);
  } else {
    B.b = const_cast<double*>(b);
    B.x = x;
  }
  B.st2 = (ColState*)take((size_t)ncol * sizeof(ColState));
  B.link = sloppy_link(g, mode);
  B.sweep = env_flag("ASQ_SWEEP", true);
  // Each D_eo block re-sums 2 x nblk partials per column of its tile, which is
  // cheap next to the Dslash only for narrow batches on lattices of at most
  // kFoldMaxBlocks site blocks.
  B.fold_alpha = ncol <= kFoldAlphaCols && g->nblk <= kFoldMaxBlocks && env_flag("ASQ_FOLD_ALPHA", true);
  // Likewise each direction-update block re-sums nblk partials of its column.
  B.fold_beta = ncol <= kFoldAlphaCols && g->nblk <= kFoldMaxBlocks && env_flag("ASQ_FOLD_BETA", true);
  batch_pick_tiles(B);
  return ASQ_OK;
}

void batch_pick_tiles(Batch& B) {
  const asq_gauge* g = B.g;
  B.rt_sloppy_norm = tuned_rtile(g, B.link, B.pt, B.pt, EPI_NORM, B.ncol);
  B.rt_sloppy_update = tuned_rtile(g, B.link, B.pt, B.rt, EPI_UPDATE, B.ncol);
  B.rt64_plain = tuned_rtile(g, LINK_F64_R18, VEC_F64, VEC_F64, EPI_PLAIN, B.ncol);
  B.rt64_resid = tuned_rtile(g, LINK_F64_R18, VEC_F64, B.rt, EPI_RESID, B.ncol);
}

// Autotune the batch's Dslash launches on its own buffers (p -> t, x -> t64),
// before the buffers hold solver data.
int batch_tune(Batch& B, hipStream_t s, bool trial_b) {
  // The trial launches read the sources, and the sloppy ones the sources
  // converted to the direction tier in the direction buffer (the start of the
  // solve overwrites it).  A fresh workspace often holds zeros, on which a
  // many-column Dslash draws less power and runs faster than on a solve's data
  // (about 9 % at 96 columns), which biased the timings and the choice.
  const size_t n = (size_t)B.ncol * B.g->geom.half;
  const bool lo = tune_pending(B.g, B.link, B.pt, B.ncol);
  const bool hi = tune_pending(B.g, LINK_F64_R18, VEC_F64, B.ncol);
  int rc;
  if ((lo || hi) && trial_b && (rc = fill_trial_values(B.b, n * 6, s))) return rc;
  const void* lo_in = B.b;
  if (lo && B.pt != VEC_F64) {
    if ((rc = asq_vec_convert(n, ASQ_F64, B.b, B.pt == VEC_F32 ? ASQ_F32 : ASQ_F16, B.p, s))) return rc;
    lo_in = B.p;
  }
  if ((rc = tune_dslash(B.g, B.link, B.pt, B.ncol, lo_in, B.t, s))) return rc;
  if ((rc = tune_dslash(B.g, LINK_F64_R18, VEC_F64, B.ncol, B.b, B.t64, s))) return rc;
  batch_pick_tiles(B);
  return ASQ_OK;
}

static DslashArgs dargs(const Batch& B, int out_parity, const void* in, void* out, int mask) {
  DslashArgs a;
  memset(&a, 0, sizeof(a));
  a.g = B.g->geom;
  a.out_parity = out_parity;
  a.ncol = B.ncol;
  a.in = in;
  a.out = out;
  a.st = B.st;
  a.mask = mask;
  a.partials = B.partials;
  a.nblk = B.g->nblk;
  a.coeff_fat = B.g->desc.fat_scale;
  a.coeff_long = B.g->desc.long_scale;
  return a;
}

static VecArgs vargs(const Batch& B, int c0) {
  VecArgs v;
  const size_t half = (size_t)B.g->geom.half;
  v.half = (int)half;
  v.nblk = B.g->nblk;
  // column offset c0: shift every per-column pointer
  v.b = B.b + (size_t)c0 * half * 6;
  v.x = B.x + (size_t)c0 * half * 6;
  v.xs = B.xs ? (char*)B.xs + (size_t)c0 * half * 24 : nullptr;
  v.r = (char*)B.r + (size_t)c0 * half * vec_site_bytes(B.rt);
  v.p = (char*)B.p + (size_t)c0 * half * vec_site_bytes(B.pt);
  v.p_alt = (char*)B.p_alt + (size_t)c0 * half * vec_site_bytes(B.pt);
  v.st = B.st + c0;
  v.partials = B.partials + (size_t)c0 * B.g->nblk;
  return v;
}

int enqueue_init(const Batch& B, int c0, int n, hipStream_t s) {
  VecArgs v = vargs(B, c0);
  int rc = launch_vec_kernel(VK_INIT, B.pt, B.rt, v, n, s);
  if (rc) return rc;
  return launch_reduce(OP_INIT, v.st, nullptr, v.partials, v.nblk, n, s);
}

// Start from the x in place: x_s = 0, p = 0, r = b - A x with the FP64 operator
// (stored in the r tier), then bb, rr and the convergence check per column.
int enqueue_init_guess(const Batch& B, hipStream_t s) {
  const Gauge_t* g = B.g;
  const void* L = g->links[LINK_F64_R18];
  VecArgs v = vargs(B, 0);
  v.partials = B.partials_p;
  int rc = launch_vec_kernel(VK_GUESS, B.pt, B.rt, v, B.ncol, s);
  if (rc) return rc;
  DslashArgs d1 = dargs(B, 1, B.x, B.t64, MASK_ALL);
  d1.links = L;
  rc = launch_dslash(LINK_F64_R18, VEC_F64, VEC_F64, EPI_PLAIN, B.rt64_plain, d1, s);
  if (rc) return rc;
  DslashArgs d2 = dargs(B, 0, B.t64, B.r, MASK_ALL);
  d2.links = L;
  d2.y = B.x;
  d2.b = B.b;
  rc = launch_dslash(LINK_F64_R18, VEC_F64, B.rt, EPI_RESID, B.rt64_resid, d2, s);
  if (rc) return rc;
  return launch_reduce(OP_INIT_GUESS, B.st, B.partials_p, B.partials, g->nblk, B.ncol, s);
}

// One CG iteration.  The direction update reads the column states from `in`;
// the rest of the iteration uses `out`.  in == out: beta was formed by the
// scalar launch at the end of the previous iteration.  in != out: the direction
// update forms it from the |r|^2 partials and writes the finalised states to
// out (the two copies alternate, so no kernel writes the copy it reads).  With
// defer_beta this iteration's own beta is left to the next direction update,
// or to the scalar launch at the end of the block.
int enqueue_iteration(const Batch& B, hipStream_t s, ColState* in, ColState* out, bool defer_beta) {
  const Gauge_t* g = B.g;
  const void* L = g->links[B.link];
  // p_new = r + beta p, partials of |p_new|^2
  VecArgs v = vargs(B, 0);
  v.st = in;
  v.partials = B.partials_p;
  if (in != out) {
    v.st_out = out;
    v.beta_partials = B.partials;
  }
  int rc = launch_vec_kernel(VK_P, B.pt, B.rt, v, B.ncol, s);
  if (rc) return rc;
  // t = D_oe p_new, partials of |t|^2
  DslashArgs d1 = dargs(B, 1, B.p, B.t, MASK_ACTIVE);
  d1.st = out;
  d1.links = L;
  d1.in_alt = B.p_alt;
  d1.in_sel = 1;
  d1.partials = B.partials_t;
  rc = launch_dslash(B.link, B.pt, B.pt, EPI_NORM, B.rt_sloppy_norm, d1, s);
  if (rc) return rc;
  // alpha = rr / (a |p|^2 + |t|^2): a scalar launch, or inside D_eo
  if (!B.fold_alpha) {
    rc = launch_reduce(OP_ALPHA, out, B.partials_p, B.partials_t, g->nblk, B.ncol, s);
    if (rc) return rc;
  }
  // Ap = a p - D_eo t; r -= alpha Ap; x += alpha p; partials of |r|^2 (backward sweep)
  DslashArgs d2 = dargs(B, 0, B.t, nullptr, MASK_ACTIVE);
  d2.st = out;
  if (B.fold_alpha) {
    d2.apa = B.partials_p;
    d2.apb = B.partials_t;
  }
  d2.links = L;
  d2.y = B.p;
  d2.y_alt = B.p_alt;
  d2.y_sel = 1;
  d2.r = B.r;
  d2.x = B.xs ? B.xs : (void*)B.x;
  d2.reverse = B.sweep ? 1 : 0;
  rc = launch_dslash(B.link, B.pt, B.rt, EPI_UPDATE, B.rt_sloppy_update, d2, s);
  if (rc) return rc;
  if (defer_beta) return ASQ_OK;
  // beta, triggers, p buffer swap
  return launch_reduce(OP_BETA, out, nullptr, B.partials, g->nblk, B.ncol, s);
}

int enqueue_iteration(const Batch& B, hipStream_t s) { return enqueue_iteration(B, s, B.st, B.st, false); }

// r = b - A x with FP64 links and vectors for the columns that asked for it,
// then the decision on the true residual.
int enqueue_reliable(const Batch& B, int mask, int op, hipStream_t s) {
  const Gauge_t* g = B.g;
  const void* L = g->links[LINK_F64_R18];
  if (B.xs) {
    // fold the segment's FP32 accumulator into the FP64 solution first
    VecArgs v = vargs(B, 0);
    v.st = B.st;
    const int rc0 = launch_vec_kernel(VK_FLUSH, B.pt, B.rt, v, B.ncol, s);
    if (rc0) return rc0;
  }
  DslashArgs d1 = dargs(B, 1, B.x, B.t64, mask);
  d1.links = L;
  int rc = launch_dslash(LINK_F64_R18, VEC_F64, VEC_F64, EPI_PLAIN, B.rt64_plain, d1, s);
  if (rc) return rc;
  DslashArgs d2 = dargs(B, 0, B.t64, B.r, mask);
  d2.links = L;
  d2.y = B.x;
  d2.b = B.b;
  d2.reverse = B.sweep ? 1 : 0;
  rc = launch_dslash(LINK_F64_R18, VEC_F64, B.rt, EPI_RESID, B.rt64_resid, d2, s);
  if (rc) return rc;
  return launch_reduce(op, B.st, nullptr, B.partials, g->nblk, B.ncol, s);
}

// `iters` iterations, then the reliable update of the columns that asked for
// one.  With fold_beta, every iteration after the first takes the previous
// beta inside its direction update, the states alternating between st and st2,
// and one scalar launch finalises the last beta back into st, so the block
// starts and ends with the states in st.
int enqueue_block(const Batch& B, int iters, hipStream_t s) {
  ColState* cur = B.st;
  for (int k = 0; k < iters; ++k) {
    ColState* next = (B.fold_beta && k > 0) ? (cur == B.st ? B.st2 : B.st) : cur;
    const int rc = enqueue_iteration(B, s, cur, next, B.fold_beta);
    if (rc) return rc;
    cur = next;
  }
  if (B.fold_beta && iters > 0) {
    const int rc = cur == B.st ? launch_reduce(OP_BETA, B.st, nullptr, B.partials, B.g->nblk, B.ncol, s)
                               : launch_reduce(OP_BETA, cur, nullptr, B.partials, B.g->nblk, B.ncol, s, B.st);
    if (rc) return rc;
  }
  return enqueue_reliable(B, MASK_RELIABLE, OP_RU, s);
}

// Thread-local host resources: pinned state mirrors, events, a capture stream.
struct HostRes {
  int device = -1;
  ColState* pinned = nullptr;
  size_t pinned_cols = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipStream_t cap = nullptr;
  ~HostRes() {
    if (pinned) (void)hipHostFree(pinned);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    if (cap) (void)hipStreamDestroy(cap);
  }
  int ensure(size_t cols) {
    int dev = 0;
    ASQ_HIP_TRY(hipGetDevice(&dev));
    if (dev != device) {
      if (pinned) (void)hipHostFree(pinned);
      for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
      if (cap) (void)hipStreamDestroy(cap);
      pinned = nullptr;
      pinned_cols = 0;
      ev[0] = ev[1] = nullptr;
      cap = nullptr;
      device = dev;
      ASQ_HIP_TRY(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
      ASQ_HIP_TRY(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
      ASQ_HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    }
    if (pinned_cols < 2 * cols) {
      if (pinned) (void)hipHostFree(pinned);
      pinned = nullptr;
      ASQ_HIP_TRY(hipHostMalloc((void**)&pinned, 2 * cols * sizeof(ColState), hipHostMallocDefault));
      pinned_cols = 2 * cols;
    }
    return ASQ_OK;
  }
};

static HostRes& host_res() {
  thread_local HostRes r;
  return r;
}

int capture_block(const Batch& B, int iters, hipStream_t cap, hipGraphExec_t* exec) {
  hipGraph_t graph = nullptr;
  ASQ_HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  int rc = enqueue_block(B, iters, cap);
  hipError_t e = hipStreamEndCapture(cap, &graph);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  ASQ_HIP_TRY(e);
  e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  ASQ_HIP_TRY(e);
  return ASQ_OK;
}

void fill_stats(const Batch& B, const ColState* S, double seconds, asq_cg_stats* out, int* worst) {
  const double half = (double)B.g->geom.half;
  double flops = 0;
  for (int c = 0; c < B.ncol; ++c)
    flops += half * ((2.0 * 1146 + 72) * S[c].iters + (2.0 * 1146 + 36) * S[c].n_ru);
  for (int c = 0; c < B.ncol; ++c) {
    asq_cg_stats& o = out[c];
    o.iters = S[c].iters;
    o.reliable_updates = S[c].n_ru;
    o.converged = S[c].converged;
    o.true_resid = S[c].bb > 0 ? sqrt(S[c].true_rr / S[c].bb) : 0.0;
    o.seconds = seconds;
    o.gflops = seconds > 0 ? flops / seconds * 1e-9 : 0.0;
    o.escalations = 0;
    o.final_mode = B.mode;
    int st = S[c].status;
    if (st == 0 && !S[c].converged) st = ASQ_ENOCONV;
    o.status = st;
    if (st == ASQ_ENAN) *worst = ASQ_ENAN;
    else if (st == ASQ_ENOCONV && *worst == ASQ_OK) *worst = ASQ_ENOCONV;
  }
}

int check_params(const asq_gauge* g, const asq_cg_params* p) {
  if (!p) return ASQ_EINVAL;
  if (!(p->tol > 0) || !isfinite(p->tol) || p->maxiter <= 0) return ASQ_EINVAL;
  if (p->mode < ASQ_MODE_F64 || p->mode > ASQ_MODE_MIXED16) return ASQ_EINVAL;
  if (!(p->delta >= 0 && p->delta < 1)) return ASQ_EINVAL;
  if (p->poll_iters < 0 || p->poll_iters > 4096) return ASQ_EINVAL;
  if (!g->links[LINK_F64_R18]) return ASQ_EINVAL;  // true residuals need the FP64 links
  if (p->mode == ASQ_MODE_MIXED32 && !g->links[g->sloppy_link32]) return ASQ_EINVAL;
  if (p->mode == ASQ_MODE_MIXED16 && !g->links[g->sloppy_link16]) return ASQ_EINVAL;
  return ASQ_OK;
}

void init_states(const Batch& B, const double* masses, const asq_cg_params* p, ColState* host, const double* tols) {
  for (int c = 0; c < B.ncol; ++c) {
    memset(&host[c], 0, sizeof(ColState));
    host[c].a = 4.0 * masses[c] * masses[c];
    host[c].tol = tols ? tols[c] : p->tol;
    host[c].delta = p->mode == ASQ_MODE_F64 ? 0.0 : p->delta;
    host[c].maxiter = p->maxiter;
  }
}

// Stagnation rule of the mixed tiers: ASQ_STALL_UPDATES (default 3) reliable
// updates in a row without the true residual falling by ASQ_STALL_DROP (default
// 10) hand the column to the next tier; 0 updates switches it off.  FP64 is the
// last tier and never hands on.
static void set_stall(ColState* host, int ncol, int mode) {
  const char* eu = getenv("ASQ_STALL_UPDATES");
  const int updates = eu && *eu ? atoi(eu) : 3;
  const char* ed = getenv("ASQ_STALL_DROP");
  double drop = ed && *ed ? atof(ed) : 10.0;
  if (!(drop > 1.0) || !isfinite(drop)) drop = 10.0;
  for (int c = 0; c < ncol; ++c) {
    host[c].stall_updates = next_mode(mode) >= 0 ? std::max(0, updates) : 0;
    host[c].stall_fac = 1.0 / (drop * drop);  // on |r|^2
  }
}

}  // namespace asq

using namespace asq;

int asq::solve_batch(const asq_gauge* g, int nrhs, const double* masses, const double* tols, const double* b_dev,
                     double* x_dev, void* work_dev, size_t work_bytes, const asq_cg_params* params,
                     asq_cg_stats* stats, void* hip_stream, bool guess) {
  if (!g || nrhs <= 0 || !masses || !b_dev || !x_dev || !work_dev || !stats) {
    set_last_error("cg_solve_batch: null pointer or nrhs <= 0");
    return ASQ_EINVAL;
  }
  if (check_params(g, params)) {
    set_last_error("cg_solve_batch: invalid parameters (tol > 0, maxiter > 0, mode, 0 <= delta < 1, link tiers)");
    return ASQ_EINVAL;
  }
  for (int c = 0; c < nrhs; ++c)
    if (!(masses[c] > 0) || !isfinite(masses[c]) || (tols && !(tols[c] > 0 && isfinite(tols[c])))) {
      set_last_error("cg_solve_batch: masses (and tolerances) must be positive and finite");
      return ASQ_EINVAL;
    }
  if (((uintptr_t)b_dev & 15) || ((uintptr_t)x_dev & 15) || ((uintptr_t)work_dev & 255)) {
    set_last_error("cg_solve_batch: b/x must be 16-byte and work 256-byte aligned");
    return ASQ_EINVAL;
  }
  const size_t vbytes = (size_t)nrhs * g->geom.half * 48;
  if (ranges_overlap(b_dev, vbytes, x_dev, vbytes) || ranges_overlap(b_dev, vbytes, work_dev, work_bytes) ||
      ranges_overlap(x_dev, vbytes, work_dev, work_bytes)) {
    set_last_error("cg_solve_batch: b, x and the workspace must not overlap");
    return ASQ_EINVAL;
  }
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = (hipStream_t)hip_stream;
  Batch B;
  int rc = batch_carve(B, g, nrhs, params->mode, work_dev, work_bytes, b_dev, x_dev);
  if (rc) {
    set_last_error("cg_solve_batch: workspace smaller than asq_workspace_bytes()");
    return rc;
  }
  if ((rc = batch_tune(B, s))) return rc;
  HostRes& H = host_res();
  if ((rc = H.ensure((size_t)nrhs))) return rc;
  ColState* mirror[2] = {H.pinned, H.pinned + nrhs};
  init_states(B, masses, params, mirror[0], tols);
  set_stall(mirror[0], nrhs, params->mode);
  ASQ_HIP_TRY(hipMemcpyAsync(B.st, mirror[0], nrhs * sizeof(ColState), hipMemcpyHostToDevice, s));
  if ((rc = guess ? enqueue_init_guess(B, s) : enqueue_init(B, 0, nrhs, s))) return rc;
  // the mirror is reused below: make sure the upload has consumed it
  ASQ_HIP_TRY(hipStreamSynchronize(s));

  const int poll = params->poll_iters > 0 ? params->poll_iters : 8;
  hipGraphExec_t exec = nullptr;
  if (params->use_graph) {
    rc = capture_block(B, poll, H.cap, &exec);
    if (rc) return rc;
  }
  int slot = 0, pending = -1, last = -1;
  long blocks = 0;
  const long max_blocks = (long)params->maxiter / poll + 4;
  for (;;) {
    if (exec) {
      hipError_t e = hipGraphLaunch(exec, s);
      if (e != hipSuccess) {
        (void)hipGraphExecDestroy(exec);
        set_last_error(hipGetErrorString(e));
        return ASQ_EHIP;
      }
    } else if ((rc = enqueue_block(B, poll, s))) {
      return rc;
    }
    ++blocks;
    ASQ_HIP_TRY(hipMemcpyAsync(mirror[slot], B.st, nrhs * sizeof(ColState), hipMemcpyDeviceToHost, s));
    ASQ_HIP_TRY(hipEventRecord(H.ev[slot], s));
    last = slot;
    if (pending >= 0) {
      ASQ_HIP_TRY(hipEventSynchronize(H.ev[pending]));
      bool any = false;
      for (int c = 0; c < nrhs; ++c) any |= mirror[pending][c].active != 0;
      if (!any) break;
    }
    if (blocks > max_blocks + 2) break;  // the device enforces maxiter; this only bounds the loop
    pending = slot;
    slot ^= 1;
  }
  ASQ_HIP_TRY(hipStreamSynchronize(s));
  if (exec) (void)hipGraphExecDestroy(exec);
  int worst = ASQ_OK;
  const ColState* fin = mirror[last];
  std::vector<int> esc;
  for (int c = 0; c < nrhs; ++c)
    if (fin[c].escalate) esc.push_back(c);
  double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  fill_stats(B, fin, secs, stats, &worst);
  if (!esc.empty()) {
    // Columns whose true residual stalled continue from their x in the next tier.
    // The states mirror is reused by the nested solve: copy what is needed first.
    std::vector<double> m_e, tol_e;
    std::vector<int> it_e, ru_e;
    for (int c : esc) {
      m_e.push_back(masses[c]);
      tol_e.push_back(tols ? tols[c] : params->tol);
      it_e.push_back(fin[c].iters);
      ru_e.push_back(fin[c].n_ru);
    }
    if ((rc = escalate(g, esc, m_e, tol_e, it_e, ru_e, b_dev, x_dev, work_dev, work_bytes, params, stats,
                       hip_stream)))
      return rc;
    worst = ASQ_OK;
    for (int c = 0; c < nrhs; ++c) {
      const int st = stats[c].status;
      if (st == ASQ_ENAN) worst = ASQ_ENAN;
      else if (st == ASQ_ENOCONV && worst == ASQ_OK) worst = ASQ_ENOCONV;
    }
    secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int c = 0; c < nrhs; ++c) stats[c].seconds = secs;
  }
  if (log_enabled())
    fprintf(stderr, "[asq] cg_solve_batch ncol=%d mode=%d iters0=%d ru0=%d resid0=%.3e esc=%zu %.3f s\n", nrhs,
            params->mode, stats[0].iters, stats[0].reliable_updates, stats[0].true_resid, esc.size(), secs);
  return worst;
}

// The stalled columns `cols` of a batch continue in the next precision tier:
// their b and x are gathered after the batch region of the workspace, solved
// from x (FP64 residual first) by a nested solve_batch, and x is scattered
// back.  Per-column counters add up; the nested solve may hand on again.
int asq::escalate(const asq_gauge* g, const std::vector<int>& cols, const std::vector<double>& masses,
                  const std::vector<double>& tols, const std::vector<int>& iters, const std::vector<int>& rus,
                  const double* b_dev, double* x_dev, void* work_dev, size_t work_bytes,
                  const asq_cg_params* params, asq_cg_stats* stats, void* hip_stream) {
  const int k = (int)cols.size();
  const int mode = next_mode(params->mode);
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t vcol = (size_t)g->geom.half * 48;
  // this level's gathered b and x take the end of the workspace; the nested solve
  // (and its own escalations) the rest: solve_bytes(ncol, mode) covers every level
  const size_t gather = 2 * align_up((size_t)k * vcol, 256);
  if (work_bytes < gather || work_bytes - gather < solve_bytes(g, k, mode)) return ASQ_ENOMEM;
  const size_t region = work_bytes - gather;
  double* bk = (double*)((char*)work_dev + region);
  double* xk = (double*)((char*)bk + align_up((size_t)k * vcol, 256));
  for (int j = 0; j < k; ++j) {
    ASQ_HIP_TRY(hipMemcpyAsync((char*)bk + j * vcol, (const char*)b_dev + cols[j] * vcol, vcol,
                               hipMemcpyDeviceToDevice, s));
    ASQ_HIP_TRY(hipMemcpyAsync((char*)xk + j * vcol, (const char*)x_dev + cols[j] * vcol, vcol,
                               hipMemcpyDeviceToDevice, s));
  }
  asq_cg_params p = *params;
  p.mode = mode;
  int budget = params->maxiter;
  for (int j = 0; j < k; ++j) budget = std::min(budget, std::max(1, params->maxiter - iters[j]));
  p.maxiter = budget;
  std::vector<asq_cg_stats> sub(k);
  const int rc = solve_batch(g, k, masses.data(), tols.data(), bk, xk, work_dev, region, &p, sub.data(), hip_stream,
                             true);
  if (rc != ASQ_OK && rc != ASQ_ENOCONV && rc != ASQ_ENAN) return rc;
  for (int j = 0; j < k; ++j)
    ASQ_HIP_TRY(hipMemcpyAsync((char*)x_dev + cols[j] * vcol, (char*)xk + j * vcol, vcol, hipMemcpyDeviceToDevice,
                               s));
  ASQ_HIP_TRY(hipStreamSynchronize(s));
  for (int j = 0; j < k; ++j) {
    asq_cg_stats& o = stats[cols[j]];
    const asq_cg_stats& t = sub[j];
    o.iters = iters[j] + t.iters;
    o.reliable_updates = rus[j] + t.reliable_updates;
    o.converged = t.converged;
    o.status = t.status;
    o.true_resid = t.true_resid;
    o.escalations = 1 + t.escalations;
    o.final_mode = t.final_mode;
  }
  return ASQ_OK;
}

// Shared by asqtad_dslash_eo, asqtad_dslash_eo_variant and the solvers'
// own FP64 operator calls: variant < 0 takes the tuned launch variant;
// canonical selects the C ABI's layouts, else the solvers' native ones.
int asq::dslash_run(const char* who, const asq_gauge* g, int out_parity, int prec, int nrhs, const void* in_dev,
                    void* out_dev, int variant, bool canonical, hipStream_t stream) {
  if (!g || !in_dev || !out_dev || nrhs <= 0 || (out_parity != 0 && out_parity != 1)) {
    set_last_error(std::string(who) + ": null pointer, nrhs <= 0 or parity not 0/1");
    return ASQ_EINVAL;
  }
  int link;
  if (prec == ASQ_F64) link = LINK_F64_R18;
  else if (prec == ASQ_F32) link = g->sloppy_link32;
  else if (prec == ASQ_F16) link = g->sloppy_link16;
  else {
    set_last_error(std::string(who) + ": prec must be ASQ_F64, ASQ_F32 or ASQ_F16");
    return ASQ_EINVAL;
  }
  if (!g->links[link]) {
    set_last_error(std::string(who) + ": the gauge field keeps no links for this precision");
    return ASQ_EINVAL;
  }
  if (((uintptr_t)in_dev & 15) || ((uintptr_t)out_dev & 15)) {
    set_last_error(std::string(who) + ": vectors must be 16-byte aligned");
    return ASQ_EINVAL;
  }
  const int vk = prec == ASQ_F64 ? VEC_F64 : (prec == ASQ_F32 ? VEC_F32 : VEC_F16);
  const size_t vbytes = (size_t)nrhs * g->geom.half * vec_site_bytes(vk);
  if (ranges_overlap(in_dev, vbytes, out_dev, vbytes)) {
    set_last_error(std::string(who) + ": input and output must not overlap");
    return ASQ_EINVAL;
  }
  DslashArgs a;
  memset(&a, 0, sizeof(a));
  a.g = g->geom;
  a.out_parity = out_parity;
  a.ncol = nrhs;
  a.links = g->links[link];
  a.in = in_dev;
  a.out = out_dev;
  a.st = nullptr;
  a.mask = MASK_ALL;
  a.nblk = g->nblk;
  a.coeff_fat = g->desc.fat_scale;
  a.coeff_long = g->desc.long_scale;
  // successive calls walk the lattice in alternate directions, so each starts on
  // the links the previous one read last, which the memory-side cache still
  // holds (as D_oe and D_eo do inside the solver); the result does not depend
  // on the direction
  static std::atomic<unsigned> calls{0};
  static const bool sweep = env_flag("ASQ_SWEEP", true);
  a.reverse = sweep && (calls.fetch_add(1, std::memory_order_relaxed) & 1) ? 1 : 0;
  const int epi = canonical ? EPI_CANON : EPI_PLAIN;
  int rt = variant;
  if (variant < 0) {
    const int rc0 = tune_dslash(g, link, vk, nrhs, in_dev, out_dev, stream, epi);
    if (rc0) return rc0;
    rt = tuned_rtile(g, link, vk, vk, epi, nrhs);
  }
  const int rc = launch_dslash(link, vk, vk, epi, rt, a, stream);
  if (rc == ASQ_EHIP) set_last_error(hipGetErrorString(hipGetLastError()));
  if (rc == ASQ_EINVAL) set_last_error(std::string(who) + ": launch variant not available for this tier");
  return rc;
}

extern "C" int asqtad_dslash_eo(const asq_gauge* g, int out_parity, int prec, int nrhs, const void* in_dev,
                                void* out_dev, void* hip_stream) {
  return dslash_run("asqtad_dslash_eo", g, out_parity, prec, nrhs, in_dev, out_dev, -1, true,
                    (hipStream_t)hip_stream);
}

extern "C" int asqtad_dslash_eo_variant(const asq_gauge* g, int out_parity, int prec, int nrhs, const void* in_dev,
                                        void* out_dev, int variant, void* hip_stream) {
  if (variant < 0) {
    set_last_error("asqtad_dslash_eo_variant: variant must be >= 0");
    return ASQ_EINVAL;
  }
  const bool native = (variant & ASQ_VARIANT_NATIVE) != 0;
  int v = variant & ~ASQ_VARIANT_NATIVE;
  if (native && v == 0) v = -1;  // the tuned variant on native vectors
  if (!native && (v & kMfmaBit)) {
    set_last_error("asqtad_dslash_eo_variant: the matrix-core form takes the native layout only");
    return ASQ_EINVAL;
  }
  return dslash_run("asqtad_dslash_eo_variant", g, out_parity, prec, nrhs, in_dev, out_dev, v, !native,
                    (hipStream_t)hip_stream);
}

extern "C" const char* asq_strerror(int code) {
  switch (code) {
    case ASQ_OK: return "ok";
    case ASQ_PENDING: return "pending";
    case ASQ_EINVAL: return "invalid argument";
    case ASQ_ENOMEM: return "caller storage, workspace or arena too small";
    case ASQ_ENOCONV: return "not converged within maxiter";
    case ASQ_ENOTSU3: return "links are not SU(3) times the given scale";
    case ASQ_EHIP: return "HIP runtime error";
    case ASQ_ENAN: return "non-finite or non-positive reduction";
    case ASQ_EAGAIN: return "queue full, try again";
  }
  return "unknown error";
}

extern "C" const char* asq_last_error(void) { return g_last_error.c_str(); }
