// multishift.hip -- CG for one source and several masses at once (the shifted
// systems (K + sigma_j) x_j = b, K = -D_eo D_oe, sigma_j = 4 m_j^2, share the
// Krylov space of the smallest shift), followed by per-column refinement.
//
// Phase 1 runs CG on the smallest shift sigma_0 for every source (FP32 Dslash
// and vectors, no reliable updates) and carries each heavier shift along with
// vector updates only: with zeta_j the ratio of the shifted residual to the
// base residual,
//   zeta_{k+1} = zeta_k zeta_{k-1} a_{k-1} /
//                (a_k b_k (zeta_{k-1} - zeta_k) + zeta_{k-1} a_{k-1} (1 + (sigma_j - sigma_0) a_k))
//   alpha_j = a_k zeta_{k+1} / zeta_k,  beta_j = b_{k+1} (zeta_{k+1} / zeta_k)^2
//   x_j += alpha_j p_j,  p_j = zeta_{k+1} r_{k+1} + beta_j p_j
// (a_k, b_k: the base CG's alpha and beta; the shifted residual is zeta_j r).
// Phase 1 stops a column when its iterated residual meets the sloppy target.
// Phase 2 refines every (mass, source) column with the reliable-update CG from
// the phase-1 solution, to the requested FP64 true residual.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "asq_batch.h"
#include "asq_reduce.h"
#include "asq_solver.h"

namespace asq {
namespace {

struct alignas(64) ShiftState {
  double ds;          // sigma_j - sigma_0
  double zeta, zeta_prev;
  double a_prev;      // the base alpha of the previous iteration (1 before the first)
  double b_prev;      // the base beta that built the current base direction (0 before the first)
  double alpha, beta; // this iteration's shifted alpha and the next shifted beta
  double tol;         // stop when |zeta| |r| <= tol |b|
  int src;            // base column (source) of this shift
  int upd;            // apply this iteration's vector update
  int active;
  int base_iters;     // base iterations already accounted for
  int iters;
  int status;
};

// After the base's beta reduction: the shifted scalars of every shift column.
__global__ void shift_scalars_kernel(ShiftState* sh, const ColState* st, int nsh) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nsh) return;
  ShiftState T = sh[j];
  const ColState& S = st[T.src];
  T.upd = 0;
  if (T.active && S.iters != T.base_iters) {
    T.base_iters = S.iters;
    const double ak = S.alpha, bk = T.b_prev, bk1 = S.beta;
    const double z = T.zeta, zp = T.zeta_prev;
    const double den = ak * bk * (zp - z) + zp * T.a_prev * (1.0 + T.ds * ak);
    const double zn = z * zp * T.a_prev / den;
    const double q = zn / z;
    if (!isfinite(zn) || !isfinite(q)) {
      T.active = 0;
      T.status = ASQ_ENAN;
    } else {
      T.alpha = ak * q;
      T.beta = bk1 * q * q;
      T.zeta_prev = z;
      T.zeta = zn;
      T.a_prev = ak;
      T.b_prev = bk1;
      T.upd = 1;
      T.iters += 1;
      if (fabs(zn) * sqrt(S.rr) <= T.tol * sqrt(S.bb) || !S.active) T.active = 0;
    }
  }
  sh[j] = T;
}

// x_j += alpha_j p_j; p_j = zeta r_base + beta_j p_j (x_j, p_j FP32; r in the RT tier).
template <class RT>
__global__ void __launch_bounds__(kBlock) shift_update_kernel(const ShiftState* sh, float* xs, float* ps,
                                                              const void* r, int half) {
  const int j = blockIdx.y;
  const ShiftState& T = sh[j];
  if (!T.upd) return;
  const int i = blockIdx.x * kBlock + (int)threadIdx.x;
  if (i >= half) return;
  const Vec3<float> rv = convert<float>(RT::load(r, half, T.src, i));
  Vec3<float> p = VecF32::load(ps, half, j, i);
  Vec3<float> x = VecF32::load(xs, half, j, i);
  const float al = (float)T.alpha, be = (float)T.beta, ze = (float)T.zeta;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    x.c[a].re = fmaR(al, p.c[a].re, x.c[a].re);
    x.c[a].im = fmaR(al, p.c[a].im, x.c[a].im);
    p.c[a].re = fmaR(be, p.c[a].re, ze * rv.c[a].re);
    p.c[a].im = fmaR(be, p.c[a].im, ze * rv.c[a].im);
  }
  VecF32::store(xs, half, j, i, x);
  VecF32::store(ps, half, j, i, p);
}

// p_j = b (FP32), x_j = 0 for every shift column.
__global__ void __launch_bounds__(kBlock) shift_init_kernel(const ShiftState* sh, const double* b, float* xs,
                                                            float* ps, int half) {
  const int j = blockIdx.y;
  const int i = blockIdx.x * kBlock + (int)threadIdx.x;
  if (i >= half) return;
  const Vec3<double> bv = VecF64::load(b, half, sh[j].src, i);
  VecF32::store(ps, half, j, i, convert<float>(bv));
  Vec3<float> z;
#pragma unroll
  for (int a = 0; a < 3; ++a) z.c[a].re = z.c[a].im = 0.f;
  VecF32::store(xs, half, j, i, z);
}

// FP64 solution column dst_col of x from an FP32 column src_col of xs.
__global__ void __launch_bounds__(kBlock) widen_kernel(double* x, int dst_col, const float* xs, int src_col,
                                                       int half) {
  const int i = blockIdx.x * kBlock + (int)threadIdx.x;
  if (i >= half) return;
  VecF64::store(x, half, dst_col, i, convert<double>(VecF32::load(xs, half, src_col, i)));
}

size_t shift_bytes(const asq_gauge* g, int nsh) {
  const size_t half = (size_t)g->geom.half;
  return align_up((size_t)nsh * sizeof(ShiftState), 256) + 2 * align_up((size_t)nsh * half * 24, 256);
}

// The phase-1 block: poll_iters base iterations, each followed by the shift updates.
int enqueue_ms_block(const Batch& B, ShiftState* sh, int nsh, float* xs, float* ps, int iters, hipStream_t s) {
  const int half = B.g->geom.half;
  for (int k = 0; k < iters; ++k) {
    int rc = enqueue_iteration(B, s);
    if (rc) return rc;
    if (nsh > 0) {
      shift_scalars_kernel<<<(unsigned)((nsh + 63) / 64), 64, 0, s>>>(sh, B.st, nsh);
      const dim3 grid((unsigned)B.g->nblk, (unsigned)nsh);
      if (B.rt == VEC_F64) shift_update_kernel<VecF64><<<grid, kBlock, 0, s>>>(sh, xs, ps, B.r, half);
      else shift_update_kernel<VecF32><<<grid, kBlock, 0, s>>>(sh, xs, ps, B.r, half);
      ASQ_HIP_TRY(hipGetLastError());
    }
  }
  return ASQ_OK;
}

}  // namespace
}  // namespace asq

using namespace asq;

size_t asq::multishift_native_bytes(const asq_gauge* g, int nsrc, int nmass, int mode) {
  if (!g || nsrc <= 0 || nmass <= 0 || mode < ASQ_MODE_F64 || mode > ASQ_MODE_MIXED16) return 0;
  const size_t half = (size_t)g->geom.half;
  const int ncol = nsrc * nmass;
  const size_t phase1 = batch_bytes(g, nsrc, ASQ_MODE_MIXED32, false) + shift_bytes(g, nsrc * (nmass - 1));
  const size_t phase2 = solve_bytes(g, ncol, mode);
  return std::max(phase1, phase2) + align_up((size_t)ncol * half * 48, 256);
}

int asq::solve_multishift_native(const asq_gauge* g, int nsrc, int nmass, const double* masses,
                                 const double* b_dev, double* x_dev, void* work_dev, size_t work_bytes,
                                 const asq_cg_params* params, asq_cg_stats* stats, void* hip_stream) {
  if (!g || nsrc <= 0 || nmass <= 0 || !masses || !b_dev || !x_dev || !work_dev || !stats || !params) {
    set_last_error("cg_solve_multishift: null pointer, nsrc <= 0 or nmass <= 0");
    return ASQ_EINVAL;
  }
  if (check_params(g, params) || !g->links[g->sloppy_link32]) {
    set_last_error("cg_solve_multishift: invalid parameters, or no FP32 links for the shifted phase");
    return ASQ_EINVAL;
  }
  for (int j = 0; j < nmass; ++j)
    if (!(masses[j] > 0) || !isfinite(masses[j])) {
      set_last_error("cg_solve_multishift: masses must be positive and finite");
      return ASQ_EINVAL;
    }
  if (((uintptr_t)b_dev & 15) || ((uintptr_t)x_dev & 15) || ((uintptr_t)work_dev & 255)) {
    set_last_error("cg_solve_multishift: b/x must be 16-byte and work 256-byte aligned");
    return ASQ_EINVAL;
  }
  const size_t bbytes = (size_t)nsrc * g->geom.half * 48, xbytes = bbytes * nmass;
  if (ranges_overlap(b_dev, bbytes, x_dev, xbytes) || ranges_overlap(b_dev, bbytes, work_dev, work_bytes) ||
      ranges_overlap(x_dev, xbytes, work_dev, work_bytes)) {
    set_last_error("cg_solve_multishift: b, x and the workspace must not overlap");
    return ASQ_EINVAL;
  }
  if (work_bytes < multishift_native_bytes(g, nsrc, nmass, params->mode)) {
    set_last_error("cg_solve_multishift: workspace smaller than asq_multishift_workspace_bytes()");
    return ASQ_ENOMEM;
  }
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t half = (size_t)g->geom.half;
  const int ncol = nsrc * nmass;
  const int j0 = (int)(std::min_element(masses, masses + nmass) - masses);  // the base (smallest) shift
  const int nsh = nsrc * (nmass - 1);
  const size_t region = multishift_native_bytes(g, nsrc, nmass, params->mode) -
                        align_up((size_t)ncol * half * 48, 256);
  double* brep = (double*)((char*)work_dev + region);  // b of every (mass, source) column

  // ---- phase 1: shifted CG on the smallest mass, FP32, no reliable updates
  const double tol1 = std::max(params->tol, 1e-7);
  asq_cg_params p1 = *params;
  p1.mode = ASQ_MODE_MIXED32;
  p1.delta = 0;
  Batch B;
  int rc = batch_carve(B, g, nsrc, ASQ_MODE_MIXED32, work_dev, batch_bytes(g, nsrc, ASQ_MODE_MIXED32, false),
                       b_dev, brep);  // the base x goes to brep's first columns, overwritten later
  if (rc) return rc;
  char* q = (char*)work_dev + batch_bytes(g, nsrc, ASQ_MODE_MIXED32, false);
  ShiftState* sh = (ShiftState*)q;
  q += align_up((size_t)nsh * sizeof(ShiftState), 256);
  float* xs = (float*)q;
  q += align_up((size_t)nsh * half * 24, 256);
  float* ps = (float*)q;
  if ((rc = batch_tune(B, s))) return rc;
  std::vector<ColState> st0(nsrc);
  std::vector<double> m0(nsrc, masses[j0]), tols(nsrc, tol1);
  init_states(B, m0.data(), &p1, st0.data(), tols.data());
  for (auto& c : st0) c.sloppy_stop = 1;
  ASQ_HIP_TRY(hipMemcpyAsync(B.st, st0.data(), nsrc * sizeof(ColState), hipMemcpyHostToDevice, s));
  if ((rc = enqueue_init(B, 0, nsrc, s))) return rc;
  std::vector<ShiftState> sh0(nsh);
  std::vector<int> shift_mass(nsh);
  for (int j = 0, k = 0; j < nmass; ++j) {
    if (j == j0) continue;
    for (int src = 0; src < nsrc; ++src, ++k) {
      ShiftState& T = sh0[k];
      memset(&T, 0, sizeof(T));
      T.ds = 4.0 * (masses[j] * masses[j] - masses[j0] * masses[j0]);
      T.zeta = T.zeta_prev = 1.0;
      T.a_prev = 1.0;
      T.tol = tol1;
      T.src = src;
      T.active = 1;
      shift_mass[k] = j;
    }
  }
  if (nsh > 0) {
    ASQ_HIP_TRY(hipMemcpyAsync(sh, sh0.data(), nsh * sizeof(ShiftState), hipMemcpyHostToDevice, s));
    shift_init_kernel<<<dim3((unsigned)g->nblk, (unsigned)nsh), kBlock, 0, s>>>(sh, b_dev, xs, ps, (int)half);
    ASQ_HIP_TRY(hipGetLastError());
  }
  const int poll = params->poll_iters > 0 ? params->poll_iters : 8;
  std::vector<ColState> mirror(nsrc);
  const long max_blocks = (long)params->maxiter / poll + 2;
  for (long blk = 0; blk < max_blocks; ++blk) {
    if ((rc = enqueue_ms_block(B, sh, nsh, xs, ps, poll, s))) return rc;
    ASQ_HIP_TRY(hipMemcpyAsync(mirror.data(), B.st, nsrc * sizeof(ColState), hipMemcpyDeviceToHost, s));
    ASQ_HIP_TRY(hipStreamSynchronize(s));
    bool any = false;
    for (auto& c : mirror) any |= c.active != 0;
    if (!any) break;
  }
  std::vector<int> it1(ncol, 0);
  if (nsh > 0) ASQ_HIP_TRY(hipMemcpyAsync(sh0.data(), sh, nsh * sizeof(ShiftState), hipMemcpyDeviceToHost, s));
  ASQ_HIP_TRY(hipStreamSynchronize(s));
  // phase-1 solutions into x_dev (FP64): the base from its FP32 accumulator, the shifts from theirs
  const unsigned nb = (unsigned)g->nblk;
  for (int src = 0; src < nsrc; ++src) {
    widen_kernel<<<nb, kBlock, 0, s>>>(x_dev, j0 * nsrc + src, (const float*)B.xs, src, (int)half);
    it1[j0 * nsrc + src] = mirror[src].iters;
  }
  for (int k = 0; k < nsh; ++k) {
    const int c = shift_mass[k] * nsrc + sh0[k].src;
    widen_kernel<<<nb, kBlock, 0, s>>>(x_dev, c, xs, k, (int)half);
    it1[c] = sh0[k].iters;
  }
  ASQ_HIP_TRY(hipGetLastError());
  // ---- phase 2: every (mass, source) column refined from its phase-1 solution
  for (int j = 0; j < nmass; ++j)
    ASQ_HIP_TRY(hipMemcpyAsync(brep + (size_t)j * nsrc * half * 6, b_dev, (size_t)nsrc * half * 48,
                               hipMemcpyDeviceToDevice, s));
  std::vector<double> mcol(ncol);
  for (int j = 0; j < nmass; ++j)
    for (int src = 0; src < nsrc; ++src) mcol[j * nsrc + src] = masses[j];
  rc = solve_batch(g, ncol, mcol.data(), nullptr, brep, x_dev, work_dev, region, params, stats, hip_stream, true);
  for (int c = 0; c < ncol; ++c) stats[c].iters += it1[c];
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (int c = 0; c < ncol; ++c) stats[c].seconds = secs;
  if (log_enabled())
    fprintf(stderr, "[asq] multishift nsrc=%d nmass=%d phase-1 iters %d, total %.3f s\n", nsrc, nmass,
            it1[j0 * nsrc], secs);
  return rc;
}
