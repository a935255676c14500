// asq_batch.h -- a batch of CG columns sharing one gauge field and one set of
// device buffers; used by cg_solve_batch and by the serving loop.
#pragma once
#include <vector>

#include "asq_internal.h"

namespace asq {

using Gauge_t = asq_gauge;

// Whether the byte ranges [a, a + na) and [b, b + nb) intersect (argument checks
// of the entry points: an output may not alias an input or the workspace).
inline bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
  return na && nb && pa < pb + nb && pb < pa + na;
}

// Widest batch whose D_eo launch forms alpha itself instead of a scalar launch
// (its tiles are then at most kFoldAlphaMaxTile columns wide).
constexpr int kFoldAlphaCols = kFoldAlphaMaxTile;
// Most site blocks for which the launches fold alpha and beta in: every block
// re-reads all nblk partials of its columns, which costs nblk^2 partial reads per
// launch; up to 4 kBlock blocks a thread loads at most four of them, issued before
// the hop loop (at 48^3 x 96, 20 736 blocks, a fold would re-read 6.9 GB).
constexpr int kFoldMaxBlocks = 4 * kBlock;

struct Batch {
  const asq_gauge* g = nullptr;
  int ncol = 0;
  int mode = 0;
  int pt = 0, rt = 0;  // storage tiers of p and t, and of r
  int link = 0;        // link tier of the iterated Dslash
  int rt_sloppy_norm = 1, rt_sloppy_update = 1, rt64_plain = 1, rt64_resid = 1;
  bool sweep = true;   // D_eo walks the lattice backwards (MALL reuse of the links)
  bool fold_alpha = false;  // D_eo forms alpha itself (few columns): no scalar launch between the Dslashes
  bool fold_beta = false;   // the direction update forms beta itself: no scalar launch after D_eo
  ColState* st = nullptr;   // the column states between blocks of iterations
  ColState* st2 = nullptr;  // second copy: with fold_beta, iterations alternate between st and st2
  double* partials = nullptr;    // [ncol][nblk] partials of |r|^2 (D_eo update, residual, init)
  double* partials_p = nullptr;  // [ncol][nblk] partials of |p|^2 (direction update)
  double* partials_t = nullptr;  // [ncol][nblk] partials of |D_oe p|^2
  double* b = nullptr;  // F64 [ncol][3][half][2]
  double* x = nullptr;
  void* xs = nullptr;  // F32 accumulator of x between reliable updates (mixed modes)
  void* r = nullptr;
  void* p = nullptr;      // two direction buffers; ColState::pbuf selects the current one
  void* p_alt = nullptr;

  void* t = nullptr;
  void* t64 = nullptr;
};

int mode_pt(int mode);
int mode_rt(int mode);
size_t batch_bytes(const asq_gauge* g, int ncol, int mode, bool with_bx);
// Workspace of solve_batch: the batch of `mode` or of any tier a stalled column
// escalates to (mixed16 -> mixed32 -> f64), then room to gather the escalated
// columns' b and x.
size_t solve_bytes(const asq_gauge* g, int ncol, int mode);
// The tier a stalled column of `mode` continues in (-1: none).
int next_mode(int mode);
// Lay the batch out in `work`; b == nullptr puts b and x in the workspace too.
int batch_carve(Batch& B, const asq_gauge* g, int ncol, int mode, void* work, size_t bytes, const double* b,
                double* x);
void batch_pick_tiles(Batch& B);
// Whether tune_dslash (tune.hip) would time this configuration (false once a
// winner is recorded, or with timing off).
bool tune_pending(const asq_gauge* g, int link_kind, int in_kind, int ncol, int epi_timed = EPI_PLAIN);
// Tune the batch's Dslash launches (trial data: B.b, which trial_b first fills
// with hashed values for a batch whose b holds nothing yet).
int batch_tune(Batch& B, hipStream_t s, bool trial_b = false);
int enqueue_init(const Batch& B, int c0, int n, hipStream_t s);
int enqueue_iteration(const Batch& B, hipStream_t s);
int enqueue_iteration(const Batch& B, hipStream_t s, ColState* in, ColState* out, bool defer_beta);
int enqueue_reliable(const Batch& B, int mask, int op, hipStream_t s);
int enqueue_block(const Batch& B, int iters, hipStream_t s);
int capture_block(const Batch& B, int iters, hipStream_t cap, hipGraphExec_t* exec);
void init_states(const Batch& B, const double* masses, const asq_cg_params* p, ColState* host, const double* tols);
// cg_solve_batch with optional per-column tolerances (host, or nullptr) and,
// with guess, the solution's initial values taken from x_dev instead of 0.
int solve_batch(const asq_gauge* g, int nrhs, const double* masses, const double* tols, const double* b_dev,
                double* x_dev, void* work_dev, size_t work_bytes, const asq_cg_params* params, asq_cg_stats* stats,
                void* hip_stream, bool guess = false);
int enqueue_init_guess(const Batch& B, hipStream_t s);
int escalate(const asq_gauge* g, const std::vector<int>& cols, const std::vector<double>& masses,
             const std::vector<double>& tols, const std::vector<int>& iters, const std::vector<int>& rus,
             const double* b_dev, double* x_dev, void* work_dev, size_t work_bytes, const asq_cg_params* params,
             asq_cg_stats* stats, void* hip_stream);
// One Dslash on caller buffers (the public operator, and the solvers' FP64
// operator on native layouts): variant < 0 takes the tuned launch variant.
int dslash_run(const char* who, const asq_gauge* g, int out_parity, int prec, int nrhs, const void* in_dev,
               void* out_dev, int variant, bool canonical, hipStream_t stream);
// The solvers on native layouts (b and x as structures of arrays); the C ABI
// entry points relayout canonical vectors around them.
size_t multishift_native_bytes(const asq_gauge* g, int nsrc, int nmass, int mode);
int solve_multishift_native(const asq_gauge* g, int nsrc, int nmass, const double* masses, const double* b_dev,
                            double* x_dev, void* work_dev, size_t work_bytes, const asq_cg_params* params,
                            asq_cg_stats* stats, void* hip_stream);
size_t full_native_bytes(const asq_gauge* g, int nrhs, int mode);
int solve_full_native(const asq_gauge* g, int nrhs, const double* masses, const double* b_dev, double* x_dev,
                      void* work_dev, size_t work_bytes, const asq_cg_params* params, asq_cg_stats* stats,
                      void* hip_stream);
// Canonical <-> native relayout of nrhs colour vectors of one parity (tier kind).
int relayout(int kind, bool to_native, int nrhs, int half, const void* src, void* dst, hipStream_t s);
void fill_stats(const Batch& B, const ColState* S, double seconds, asq_cg_stats* out, int* worst);
int check_params(const asq_gauge* g, const asq_cg_params* p);

}  // namespace asq
