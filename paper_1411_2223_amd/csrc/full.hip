// full.hip -- the full-lattice system M x = b, M = 2m + D on both parities,
// through the even-odd reduction that the CG works on:
//   b' = 2m b_e - D_eo b_o,   (4m^2 - D_eo D_oe) x_e = b',   x_o = (b_o - D_oe x_e) / (2m).
// The odd equations hold by construction, so |b - M x| = |b' - A x_e| / (2m)
// and the even solve runs to tol' = 2m tol |b| / |b'|.  The returned residual
// is recomputed from M in FP64 after the reconstruction.
#include <math.h>
#include <string.h>

#include <vector>

#include "asq_batch.h"
#include "asq_reduce.h"

namespace asq {
namespace {

constexpr int kPer = 8;                     // doubles per thread in the norm kernels
constexpr size_t kChunk = (size_t)kBlock * kPer;

// out = a x + b y over n doubles (one column of one parity).
__global__ void __launch_bounds__(kBlock) combine_kernel(double* out, const double* x, const double* y, size_t n,
                                                          double a, double b) {
  const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = __builtin_fma(a, x[i], b * y[i]);
}

// Block partials of |b - a x - t|^2 (x, t may be null: terms dropped), each
// thread summing kPer consecutive entries in order, then the block tree.
__global__ void __launch_bounds__(kBlock) resid_partials_kernel(const double* b, const double* x, const double* t,
                                                                 size_t n, double a, double* partials) {
  const size_t i0 = (size_t)blockIdx.x * kChunk + (size_t)threadIdx.x * kPer;
  double v = 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const size_t i = i0 + k;
    if (i < n) {
      double r = b[i];
      if (x) r = __builtin_fma(-a, x[i], r);
      if (t) r -= t[i];
      v = __builtin_fma(r, r, v);
    }
  }
  __shared__ double sh[kBlock / 64];
  const double s = block_sum(v, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

size_t nparts(size_t n) { return (n + kChunk - 1) / kChunk; }

int combine(double* out, const double* x, const double* y, size_t n, double a, double b, hipStream_t s) {
  combine_kernel<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(out, x, y, n, a, b);
  return hipGetLastError() == hipSuccess ? ASQ_OK : ASQ_EHIP;
}

// |b - a x - t|^2 summed in a fixed order on the host (synchronizes s).
int resid2(const double* b, const double* x, const double* t, size_t n, double a, double* dev_parts,
           std::vector<double>& host_parts, double* out, hipStream_t s) {
  const size_t np = nparts(n);
  resid_partials_kernel<<<(unsigned)np, kBlock, 0, s>>>(b, x, t, n, a, dev_parts);
  ASQ_HIP_TRY(hipGetLastError());
  host_parts.resize(np);
  ASQ_HIP_TRY(hipMemcpyAsync(host_parts.data(), dev_parts, np * sizeof(double), hipMemcpyDeviceToHost, s));
  ASQ_HIP_TRY(hipStreamSynchronize(s));
  double acc = 0;
  for (size_t k = 0; k < np; ++k) acc += host_parts[k];
  *out = acc;
  return ASQ_OK;
}

}  // namespace
}  // namespace asq

using namespace asq;

size_t asq::full_native_bytes(const asq_gauge* g, int nrhs, int mode) {
  if (!g || nrhs <= 0 || mode < ASQ_MODE_F64 || mode > ASQ_MODE_MIXED16) return 0;
  const size_t n = (size_t)6 * g->geom.half;
  return solve_bytes(g, nrhs, mode) + align_up((size_t)nrhs * n * sizeof(double), 256) +
         align_up(nparts(n) * sizeof(double), 256);
}

int asq::solve_full_native(const asq_gauge* g, int nrhs, const double* masses, const double* b_dev, double* x_dev,
                           void* work_dev, size_t work_bytes, const asq_cg_params* params, asq_cg_stats* stats,
                           void* hip_stream) {
  if (!g || nrhs <= 0 || !masses || !b_dev || !x_dev || !work_dev || !stats || !params) {
    set_last_error("cg_solve_full: null pointer or nrhs <= 0");
    return ASQ_EINVAL;
  }
  for (int c = 0; c < nrhs; ++c)
    if (!(masses[c] > 0) || !isfinite(masses[c])) {
      set_last_error("cg_solve_full: masses must be positive and finite");
      return ASQ_EINVAL;
    }
  if (!(params->tol > 0)) {
    set_last_error("cg_solve_full: tol must be positive");
    return ASQ_EINVAL;
  }
  if (((uintptr_t)b_dev & 15) || ((uintptr_t)x_dev & 15) || ((uintptr_t)work_dev & 255)) {
    set_last_error("cg_solve_full: b/x must be 16-byte and work 256-byte aligned");
    return ASQ_EINVAL;
  }
  const size_t vbytes = (size_t)nrhs * 2 * g->geom.half * 48;  // both parities
  if (ranges_overlap(b_dev, vbytes, x_dev, vbytes) || ranges_overlap(b_dev, vbytes, work_dev, work_bytes) ||
      ranges_overlap(x_dev, vbytes, work_dev, work_bytes)) {
    set_last_error("cg_solve_full: b, x and the workspace must not overlap");
    return ASQ_EINVAL;
  }
  if (work_bytes < full_native_bytes(g, nrhs, params->mode)) {
    set_last_error("cg_solve_full: workspace smaller than asq_full_workspace_bytes()");
    return ASQ_ENOMEM;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t n = (size_t)6 * g->geom.half;  // doubles per column and parity
  const size_t cg_bytes = solve_bytes(g, nrhs, params->mode);
  double* bp = (double*)((char*)work_dev + cg_bytes);  // b', later D x
  double* parts = (double*)((char*)bp + align_up((size_t)nrhs * n * sizeof(double), 256));
  const double* b_e = b_dev;
  const double* b_o = b_dev + (size_t)nrhs * n;
  double* x_e = x_dev;
  double* x_o = x_dev + (size_t)nrhs * n;
  std::vector<double> hp;
  int rc;

  // b' = 2m b_e - D_eo b_o
  if ((rc = dslash_run("cg_solve_full", g, 0, ASQ_F64, nrhs, b_o, bp, -1, false, s))) return rc;
  for (int c = 0; c < nrhs; ++c)
    if ((rc = combine(bp + c * n, b_e + c * n, bp + c * n, n, 2.0 * masses[c], -1.0, s))) return rc;
  // per-column even tolerance from |b| and |b'|
  std::vector<double> bb(nrhs), tols(nrhs);
  for (int c = 0; c < nrhs; ++c) {
    double be2, bo2, bp2;
    if ((rc = resid2(b_e + c * n, nullptr, nullptr, n, 0.0, parts, hp, &be2, s))) return rc;
    if ((rc = resid2(b_o + c * n, nullptr, nullptr, n, 0.0, parts, hp, &bo2, s))) return rc;
    if ((rc = resid2(bp + c * n, nullptr, nullptr, n, 0.0, parts, hp, &bp2, s))) return rc;
    bb[c] = be2 + bo2;
    tols[c] = bp2 > 0 ? 2.0 * masses[c] * params->tol * sqrt(bb[c] / bp2) : params->tol;
  }
  // the even system
  asq_cg_params p = *params;
  rc = solve_batch(g, nrhs, masses, tols.data(), bp, x_e, work_dev, cg_bytes, &p, stats, hip_stream);
  if (rc != ASQ_OK && rc != ASQ_ENOCONV) return rc;
  // x_o = (b_o - D_oe x_e) / (2m)
  if ((rc = dslash_run("cg_solve_full", g, 1, ASQ_F64, nrhs, x_e, bp, -1, false, s))) return rc;
  for (int c = 0; c < nrhs; ++c) {
    const double inv = 0.5 / masses[c];
    if ((rc = combine(x_o + c * n, b_o + c * n, bp + c * n, n, inv, -inv, s))) return rc;
  }
  // |b - M x| / |b| in FP64: even part b_e - 2m x_e - D_eo x_o, odd part b_o - 2m x_o - D_oe x_e
  std::vector<double> r2(nrhs, 0.0);
  if ((rc = dslash_run("cg_solve_full", g, 0, ASQ_F64, nrhs, x_o, bp, -1, false, s))) return rc;
  for (int c = 0; c < nrhs; ++c) {
    double v;
    if ((rc = resid2(b_e + c * n, x_e + c * n, bp + c * n, n, 2.0 * masses[c], parts, hp, &v, s))) return rc;
    r2[c] += v;
  }
  if ((rc = dslash_run("cg_solve_full", g, 1, ASQ_F64, nrhs, x_e, bp, -1, false, s))) return rc;
  int worst = ASQ_OK;
  for (int c = 0; c < nrhs; ++c) {
    double v;
    if ((rc = resid2(b_o + c * n, x_o + c * n, bp + c * n, n, 2.0 * masses[c], parts, hp, &v, s))) return rc;
    r2[c] += v;
    const double res = bb[c] > 0 ? sqrt(r2[c] / bb[c]) : 0.0;
    stats[c].true_resid = res;
    if (stats[c].status == ASQ_OK && !(res <= params->tol)) {
      // the even solve met tol' but rounding in the reconstruction left more
      stats[c].status = ASQ_ENOCONV;
      stats[c].converged = 0;
    }
    if (stats[c].status == ASQ_ENAN || (worst == ASQ_OK && stats[c].status != ASQ_OK)) worst = stats[c].status;
  }
  return worst;
}
