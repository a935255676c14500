// asq_internal.h -- host-side objects shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "../../include/asqtad.h"
#include "asq_device.h"

#define ASQ_HIP_TRY(expr)                          \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) {                        \
      asq::set_last_error(hipGetErrorString(e_));  \
      return ASQ_EHIP;                             \
    }                                              \
  } while (0)

namespace asq {

void set_last_error(const std::string& msg);
bool log_enabled();

inline size_t align_up(size_t n, size_t a) { return (n + a - 1) / a * a; }

FastDiv make_fastdiv(uint32_t d);
Geom make_geom(const int dims[4]);

// Bytes per site of one link slot for each storage tier.
size_t link_slot_bytes(int kind);
// Bytes per site of one colour vector for each storage tier.
size_t vec_site_bytes(int kind);

}  // namespace asq

// The opaque gauge handle: resident link copies inside caller-owned storage.
struct asq_gauge {
  asq_gauge_desc desc;
  asq::Geom geom;
  int device;
  void* base;                    // caller's storage
  size_t bytes;
  void* links[asq::LINK_KINDS];  // nullptr when the tier is not kept
  int sloppy_link32;             // link kind used by F32 vectors (LINK_F32_R18 or LINK_F32_R12, or
                                 // LINK_F64_F32 when only FP64 links are kept)
  int sloppy_link16;             // link kind used by F16 vectors
  int nblk;                      // site blocks of kBlock covering one parity
};

namespace asq {

// Dslash epilogues.
//   PLAIN   out = D in
//   NORM    out = D in, block partials of |out|^2 (as stored)
//   UPDATE  Ap = a y - D in in registers; r -= alpha Ap, x += alpha y; partials of |r|^2
//   RESID   out = b - a y + D in in FP64, stored in the output tier; partials of |out|^2
//   CANON   out = D in, both in the canonical layouts of the C ABI (the public operator)
enum Epi { EPI_PLAIN = 0, EPI_NORM = 1, EPI_UPDATE = 2, EPI_RESID = 3, EPI_CANON = 4 };
// Column masks (read from the per-column solver state).
enum Mask { MASK_ALL = 0, MASK_ACTIVE = 1, MASK_RELIABLE = 2 };

// Per-column solver state, resident in device memory.
struct alignas(128) ColState {
  double a;        // 4 m^2
  double bb;       // |b|^2
  double rr;       // |r|^2 of the iterated residual
  double rr_old;   // the previous rr (denominator of beta)
  double alpha;
  double beta;     // applied by the next iteration's fused p = r + beta p
  double maxr;     // max |r| since the last reliable update
  double true_rr;  // |b - A x|^2 from the last FP64 residual
  double pAp;
  double tol;      // relative tolerance on the FP64 true residual
  double delta;    // reliable-update trigger (0: only at convergence)
  int maxiter;
  int active;      // 1 while the column iterates
  int iters;
  int want_ru;     // reliable update requested
  int n_ru;        // reliable updates done
  int converged;
  int frozen;      // sloppy residual met tol: skip iterations until the FP64 check
  int status;      // 0 ok, ASQ_ENAN on a non-finite or non-positive reduction
  int pbuf;        // which of the two p buffers holds the current direction
  int sloppy_stop; // stop at the iterated residual, without an FP64 decision (shifted CG's first phase)
  // stagnation: stall_updates reliable updates in a row whose true |r|^2 is not below
  // stall_fac * ref_rr (ref_rr: |r|^2 at the last update that was) stop the column with
  // escalate = 1, and the host continues it from its x in the next precision tier
  double ref_rr;
  double stall_fac;
  int stall_updates;  // 0: never escalate
  int n_stall;
  int escalate;
};
static_assert(sizeof(ColState) == 256, "ColState layout");

// Scalar updates applied to a column from its reduced sums (see asq_reduce.h).
enum ReduceOp { OP_INIT = 0, OP_ALPHA = 1, OP_BETA = 2, OP_RU = 3, OP_INIT_GUESS = 5 };

struct DslashArgs {
  Geom g;
  int out_parity;
  int ncol;
  int ntiles;
  const void* links;
  const void* in;       // input vector (other parity)
  const void* in_alt;   // second p buffer: in_sel = 1 reads the column's new direction
  int in_sel;           // (in_alt if pbuf == 0, else in)
  void* out;            // PLAIN / NORM / RESID output
  const void* y;        // UPDATE / RESID: the vector multiplied by a = 4 m^2
  const void* y_alt;    // with y_sel = 1: y is the column's new direction (y_alt if pbuf == 0)
  int y_sel;
  const double* b;      // RESID: right-hand side (F64)
  void* r;              // UPDATE: iterated residual (r tier), read and written
  void* x;              // UPDATE: solution accumulator (F32 segment sum, or the F64 x in FP64 mode)
  ColState* st;         // per-column a, alpha and masks (nullptr: all columns)
  int mask;
  double* partials;     // [ncol][nblk] FP64 block partials (NORM, UPDATE, RESID)
  int nblk;
  const double* apa;    // UPDATE, when set: every block forms alpha = rr / (a sum(apa) + sum(apb))
  const double* apb;    // from the [ncol][nblk] partials of |p|^2 and |D_oe p|^2 itself
  int sgroup;           // block order: 0 site block by site block, else tile by tile in groups of sgroup
  double coeff_fat;     // 12-real tiers: fat / long coefficients re-applied in-kernel
  double coeff_long;
  int reverse;          // walk the lattice from the last site block to the first
  int sweep_chunk;      // 0: a contiguous slab per XCD; k >= 1: one sweep, each XCD taking runs of k blocks
};

// Launch one Dslash.  link_kind / in_kind select the template; out_kind is the
// output tier (PLAIN, NORM, RESID) or the residual tier (UPDATE).
int launch_dslash(int link_kind, int in_kind, int out_kind, int epi, int rtile, const DslashArgs& a,
                  hipStream_t s);
// The same, one function per link tier (one translation unit each).
int launch_dslash_f64(int out_kind, int epi, int rtile, const DslashArgs& a, hipStream_t s);
int launch_dslash_f32r18(int in_kind, int epi, int rtile, const DslashArgs& a, hipStream_t s);
int launch_dslash_f32r12(int in_kind, int epi, int rtile, const DslashArgs& a, hipStream_t s);
int launch_dslash_i16r12(int in_kind, int epi, int rtile, const DslashArgs& a, hipStream_t s);
int launch_dslash_f64f32(int in_kind, int epi, int rtile, const DslashArgs& a, hipStream_t s);
// (each also takes epi = EPI_CANON: the PLAIN operator on canonical layouts)
// Launch variant code: columns per thread (1, 2, 4, 6, 8, 12) in the low byte,
// kPipeBit for the software-pipelined hop loop, and the block order << kOrderShift:
// 0 the tiles of a site block adjacent; 1, 2, 3 tile by tile inside groups of
// 16, 64 or all site blocks.
constexpr int kPipeBit = 0x100;
// One-column launches of the FP32 and 16-bit link tiers: links read with
// non-temporal loads (the FP64-stored tiers always stream at one column).
constexpr int kStreamBit = 0x200;
constexpr int kOrderShift = 12;
// Pipelined launches on the solvers' native layouts: each block first copies
// the input records of its columns within three y-rows of its sites into LDS
// (the window every x hop and every non-wrapping y hop reads), and those hops
// read LDS instead of the caches.
constexpr int kLdsBit = 0x4000;
// Records per column in a block's window (its kBlock sites and three y-rows of
// xh checkerboard sites on either side), and the most LDS a window may take.
__host__ __device__ inline int lds_window(int xh) { return kBlock + 6 * xh; }
constexpr size_t kLdsWindowMax = 65536;
// Global sweep: blocks go to the XCDs round-robin in dispatch order instead of
// each XCD walking a contiguous slab, so the eight XCDs advance through the
// lattice together and the far-hop (t) neighbour records of the shared front
// stay in the memory-side cache instead of eight separate fronts.
constexpr int kGlobalSweepBit = 0x8000;
// With the global sweep, the XCDs can take runs of k consecutive blocks in turn
// instead of single blocks (k = 16, 64, 256 for chunk codes 1..3 << kChunkShift):
// the front still advances through the lattice together, and neighbours a few
// rows or planes away stay in one XCD's L2.
constexpr int kChunkShift = 10;
inline int sweep_chunk_of(int rtile) {
  if (!(rtile & kGlobalSweepBit)) return 0;
  const int code = (rtile >> kChunkShift) & 3;
  return code == 0 ? 1 : (code == 1 ? 16 : (code == 2 ? 64 : 256));
}
// The matrix-core form (FP32 18-real links with FP16-with-norm vectors only):
// kMfmaBit | kMfmaTile | order << kOrderShift, 32 columns per block of sites.
constexpr int kMfmaBit = 0x10000;
constexpr int kMfmaTile = 32;
inline int rtile_order(int rtile) { return (rtile >> kOrderShift) & 3; }
inline int order_group(int order, int nblk) { return order == 0 ? 0 : (order == 1 ? 16 : (order == 2 ? 64 : nblk)); }
// Whether the library builds launch variant rtile (for any link and vector tier).
bool variant_built(int link_kind, int in_kind, int rtile);
// Whether a built variant can launch on this lattice: an LDS window of the
// tile's columns must fit in kLdsWindowMax bytes.
bool variant_fits(const Geom& g, int in_kind, int rtile);
inline int make_rtile(int cols, bool pipe, int order, bool global_sweep = false, int chunk_code = 0,
                      bool stream = false, bool lds = false) {
  return cols | (pipe ? kPipeBit : 0) | (stream ? kStreamBit : 0) | (lds ? kLdsBit : 0) | (order << kOrderShift) |
         (global_sweep ? kGlobalSweepBit | (chunk_code << kChunkShift) : 0);
}
// Widest column tile whose UPDATE launch may form alpha itself (DslashArgs::apa).
constexpr int kFoldAlphaMaxTile = 2;

// Tuned launch variant for a Dslash configuration.
int tuned_rtile(const asq_gauge* g, int link_kind, int in_kind, int out_kind, int epi, int ncol);
// Time the candidate tiles once per configuration (in_buf read, out_buf scratch).
// epi_timed: EPI_PLAIN (the solvers' layouts; the winner serves every epilogue)
// or EPI_CANON (the public operator); persist: also write the ASQ_TUNE_CACHE file.
int tune_dslash(const asq_gauge* g, int link_kind, int in_kind, int ncol, const void* in_buf, void* out_buf,
                hipStream_t s, int epi_timed = EPI_PLAIN, bool persist = true);

}  // namespace asq
