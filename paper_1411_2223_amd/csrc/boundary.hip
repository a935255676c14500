// boundary.hip -- the canonical layouts of the C ABI.
//
// Callers hand the library colour vectors in the canonical checkerboard layout
// [col][V/2][3] of interleaved complex numbers (FP16-with-norm: the binary16
// values of every column, then every site's norm).  The kernels keep their
// own site-fastest structures of arrays ("native" layouts), so this file
//   * relayouts canonical <-> native vectors (pure data movement),
//   * converts canonical vectors between precisions (FP64, FP32, FP16 with a
//     per-site norm: the storage tiers of the paper's mixed-precision CG),
//   * and implements the public solver entry points, which stage b and x in
//     the native layout inside the caller's workspace around the solvers.
#include <math.h>
#include <string.h>

#include <chrono>
#include <string>

#include "asq_batch.h"
#include "asq_internal.h"

namespace asq {
namespace {

// One thread per (column, site): blockIdx.y is the column.
template <class NT, class CT, bool TO_NATIVE>
__global__ void __launch_bounds__(kBlock) relayout_kernel(const void* __restrict__ src, void* __restrict__ dst,
                                                          int half, int ncol) {
  const int c = blockIdx.y;
  const int i = blockIdx.x * kBlock + (int)threadIdx.x;
  if (i >= half) return;
  if constexpr (NT::kind == VEC_F16) {
    if constexpr (TO_NATIVE) {
      reinterpret_cast<uint4*>(dst)[(size_t)c * half + i] = VecF16C::load_rec(src, half, ncol, c, i);
    } else {
      VecF16C::store_rec(dst, half, ncol, c, i, VecF16::load_rec(src, half, c, i));
    }
  } else {
    if constexpr (TO_NATIVE) NT::store(dst, half, c, i, CT::load(src, half, c, i));
    else CT::store(dst, half, c, i, NT::load(src, half, c, i));
  }
}

// Canonical record k (of n) of a tier as exact FP64 values (FP16: nu * h, exact).
template <int SK>
__device__ __forceinline__ Vec3<double> load_canon(const void* base, size_t n, size_t k) {
  Vec3<double> v;
  if constexpr (SK == VEC_F64) {
    const double2* q = reinterpret_cast<const double2*>(base) + k * 3;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double2 w = q[a];
      v.c[a].re = w.x;
      v.c[a].im = w.y;
    }
  } else if constexpr (SK == VEC_F32) {
    const float2* q = reinterpret_cast<const float2*>(base) + k * 3;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float2 w = q[a];
      v.c[a].re = w.x;
      v.c[a].im = w.y;
    }
  } else {
    const uint32_t* q = reinterpret_cast<const uint32_t*>(base) + k * 3;
    const double nu = (double)reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + n * 12)[k];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const uint32_t w = q[a];
      v.c[a].re = (double)VecF16::h2f(w & 0xffffu) * nu;
      v.c[a].im = (double)VecF16::h2f(w >> 16) * nu;
    }
  }
  return v;
}

template <int DK>
__device__ __forceinline__ void store_canon(void* base, size_t n, size_t k, const Vec3<double>& v) {
  if constexpr (DK == VEC_F64) {
    double2* q = reinterpret_cast<double2*>(base) + k * 3;
#pragma unroll
    for (int a = 0; a < 3; ++a) q[a] = make_double2(v.c[a].re, v.c[a].im);
  } else if constexpr (DK == VEC_F32) {
    float2* q = reinterpret_cast<float2*>(base) + k * 3;
#pragma unroll
    for (int a = 0; a < 3; ++a) q[a] = make_float2((float)v.c[a].re, (float)v.c[a].im);
  } else {
    // the FP16 tier encodes the FP32-rounded values (as the solvers' FP32 arithmetic does)
    const uint4 w = VecF16::encode(convert<float>(v));
    uint32_t* q = reinterpret_cast<uint32_t*>(base) + k * 3;
    q[0] = w.x;
    q[1] = w.y;
    q[2] = w.z;
    reinterpret_cast<float*>(reinterpret_cast<char*>(base) + n * 12)[k] = __uint_as_float(w.w);
  }
}

// dst = src record by record, n records, between canonical tiers.
template <int SK, int DK>
__global__ void __launch_bounds__(kBlock) convert_kernel(const void* __restrict__ src, void* __restrict__ dst,
                                                         size_t n) {
  const size_t k = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  store_canon<DK>(dst, n, k, load_canon<SK>(src, n, k));
}

template <int SK>
int launch_convert(int dk, const void* src, void* dst, size_t n, hipStream_t s) {
  const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
  if (dk == VEC_F64) convert_kernel<SK, VEC_F64><<<nb, kBlock, 0, s>>>(src, dst, n);
  else if (dk == VEC_F32) convert_kernel<SK, VEC_F32><<<nb, kBlock, 0, s>>>(src, dst, n);
  else convert_kernel<SK, VEC_F16><<<nb, kBlock, 0, s>>>(src, dst, n);
  return hipGetLastError() == hipSuccess ? ASQ_OK : ASQ_EHIP;
}

int prec_kind(int prec) {
  return prec == ASQ_F64 ? VEC_F64 : (prec == ASQ_F32 ? VEC_F32 : (prec == ASQ_F16 ? VEC_F16 : -1));
}

bool misaligned(const void* p) { return ((uintptr_t)p & 15) != 0; }

}  // namespace

int relayout(int kind, bool to_native, int nrhs, int half, const void* src, void* dst, hipStream_t s) {
  if (nrhs <= 0 || half <= 0) return ASQ_OK;
  const dim3 grid((unsigned)((half + kBlock - 1) / kBlock), (unsigned)nrhs);
  if (kind == VEC_F64) {
    if (to_native) relayout_kernel<VecF64, VecF64C, true><<<grid, kBlock, 0, s>>>(src, dst, half, nrhs);
    else relayout_kernel<VecF64, VecF64C, false><<<grid, kBlock, 0, s>>>(src, dst, half, nrhs);
  } else if (kind == VEC_F32) {
    if (to_native) relayout_kernel<VecF32, VecF32C, true><<<grid, kBlock, 0, s>>>(src, dst, half, nrhs);
    else relayout_kernel<VecF32, VecF32C, false><<<grid, kBlock, 0, s>>>(src, dst, half, nrhs);
  } else if (kind == VEC_F16) {
    if (to_native) relayout_kernel<VecF16, VecF16C, true><<<grid, kBlock, 0, s>>>(src, dst, half, nrhs);
    else relayout_kernel<VecF16, VecF16C, false><<<grid, kBlock, 0, s>>>(src, dst, half, nrhs);
  } else {
    return ASQ_EINVAL;
  }
  return hipGetLastError() == hipSuccess ? ASQ_OK : ASQ_EHIP;
}

}  // namespace asq

using namespace asq;

// ---- vectors -----------------------------------------------------------------

extern "C" size_t asq_vec_bytes(int prec, size_t nsites) {
  const int k = prec_kind(prec);
  return k < 0 ? 0 : nsites * vec_site_bytes(k);
}

extern "C" int asq_vec_convert(size_t nsites, int src_prec, const void* src_dev, int dst_prec, void* dst_dev,
                               void* hip_stream) {
  const int sk = prec_kind(src_prec), dk = prec_kind(dst_prec);
  if (sk < 0 || dk < 0 || !src_dev || !dst_dev || misaligned(src_dev) || misaligned(dst_dev) ||
      nsites >= ((size_t)1 << 40)) {
    set_last_error("asq_vec_convert: bad precision, null or misaligned pointer");
    return ASQ_EINVAL;
  }
  if (ranges_overlap(src_dev, nsites * vec_site_bytes(sk), dst_dev, nsites * vec_site_bytes(dk))) {
    set_last_error("asq_vec_convert: source and destination must not overlap");
    return ASQ_EINVAL;
  }
  if (nsites == 0) return ASQ_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  int rc;
  if (sk == VEC_F64) rc = launch_convert<VEC_F64>(dk, src_dev, dst_dev, nsites, s);
  else if (sk == VEC_F32) rc = launch_convert<VEC_F32>(dk, src_dev, dst_dev, nsites, s);
  else rc = launch_convert<VEC_F16>(dk, src_dev, dst_dev, nsites, s);
  if (rc) set_last_error("asq_vec_convert: launch failed");
  return rc;
}

static int vec_native_call(const char* who, const asq_gauge* g, int prec, int nrhs, const void* src, void* dst,
                           bool to_native, void* hip_stream) {
  const int k = prec_kind(prec);
  if (!g || k < 0 || nrhs <= 0 || !src || !dst || misaligned(src) || misaligned(dst)) {
    set_last_error(std::string(who) + ": bad precision, nrhs <= 0, null or misaligned pointer");
    return ASQ_EINVAL;
  }
  const size_t n = (size_t)nrhs * g->geom.half * vec_site_bytes(k);
  if (ranges_overlap(src, n, dst, n)) {
    set_last_error(std::string(who) + ": source and destination must not overlap");
    return ASQ_EINVAL;
  }
  const int rc = relayout(k, to_native, nrhs, g->geom.half, src, dst, (hipStream_t)hip_stream);
  if (rc) set_last_error(std::string(who) + ": launch failed");
  return rc;
}

extern "C" int asq_vec_to_native(const asq_gauge* g, int prec, int nrhs, const void* canon_dev, void* native_dev,
                                 void* hip_stream) {
  return vec_native_call("asq_vec_to_native", g, prec, nrhs, canon_dev, native_dev, true, hip_stream);
}

extern "C" int asq_vec_from_native(const asq_gauge* g, int prec, int nrhs, const void* native_dev, void* canon_dev,
                                   void* hip_stream) {
  return vec_native_call("asq_vec_from_native", g, prec, nrhs, native_dev, canon_dev, false, hip_stream);
}

// ---- solvers: canonical b and x staged in the native layout inside the workspace

namespace {

// The native copies of b (nb columns) and x (nx columns) after a solver region.
struct Stage2 {
  double* b;
  double* x;
};

size_t stage_bytes(const asq_gauge* g, long nb, long nx) {
  const size_t v = (size_t)g->geom.half * 48;
  return align_up(v * nb, 256) + align_up(v * nx, 256);
}

Stage2 stage_at(const asq_gauge* g, void* work, size_t region, long nb) {
  Stage2 st;
  st.b = (double*)((char*)work + region);
  st.x = (double*)((char*)st.b + align_up((size_t)g->geom.half * 48 * nb, 256));
  return st;
}

// Checks shared by the public solvers: pointers, alignment, disjointness.
int check_io(const char* who, const void* b, size_t bbytes, const void* x, size_t xbytes, const void* work,
             size_t work_bytes) {
  if (misaligned(b) || misaligned(x) || ((uintptr_t)work & 255)) {
    set_last_error(std::string(who) + ": b/x must be 16-byte and work 256-byte aligned");
    return ASQ_EINVAL;
  }
  if (ranges_overlap(b, bbytes, x, xbytes) || ranges_overlap(b, bbytes, work, work_bytes) ||
      ranges_overlap(x, xbytes, work, work_bytes)) {
    set_last_error(std::string(who) + ": b, x and the workspace must not overlap");
    return ASQ_EINVAL;
  }
  return ASQ_OK;
}

// x (canonical) from the native solution, then wait: the public solvers return
// with x written.  An earlier solver error is kept.
int finish_x(int rc, const asq_gauge* g, int ncol, const double* x_native, double* x, hipStream_t s) {
  if (rc != ASQ_OK && rc != ASQ_ENOCONV && rc != ASQ_ENAN) return rc;
  const int rc2 = relayout(VEC_F64, false, ncol, g->geom.half, x_native, x, s);
  if (rc2) return rc2;
  ASQ_HIP_TRY(hipStreamSynchronize(s));
  return rc;
}

}  // namespace

extern "C" size_t asq_workspace_bytes(const asq_gauge* g, int nrhs, int mode) {
  if (!g || nrhs <= 0 || mode < ASQ_MODE_F64 || mode > ASQ_MODE_MIXED16) return 0;
  return solve_bytes(g, nrhs, mode) + stage_bytes(g, nrhs, nrhs);
}

extern "C" int cg_solve_batch(const asq_gauge* g, int nrhs, const double* masses, const double* b_dev,
                              double* x_dev, void* work_dev, size_t work_bytes, const asq_cg_params* params,
                              asq_cg_stats* stats, void* hip_stream) {
  const char* who = "cg_solve_batch";
  if (!g || nrhs <= 0 || !masses || !b_dev || !x_dev || !work_dev || !stats || !params) {
    set_last_error("cg_solve_batch: null pointer or nrhs <= 0");
    return ASQ_EINVAL;
  }
  const size_t vbytes = (size_t)nrhs * g->geom.half * 48;
  int rc = check_io(who, b_dev, vbytes, x_dev, vbytes, work_dev, work_bytes);
  if (rc) return rc;
  if (params->mode < ASQ_MODE_F64 || params->mode > ASQ_MODE_MIXED16) {
    set_last_error("cg_solve_batch: invalid mode");
    return ASQ_EINVAL;
  }
  if (work_bytes < asq_workspace_bytes(g, nrhs, params->mode)) {
    set_last_error("cg_solve_batch: workspace smaller than asq_workspace_bytes()");
    return ASQ_ENOMEM;
  }
  const size_t region = solve_bytes(g, nrhs, params->mode);
  const Stage2 st = stage_at(g, work_dev, region, nrhs);
  hipStream_t s = (hipStream_t)hip_stream;
  if ((rc = relayout(VEC_F64, true, nrhs, g->geom.half, b_dev, st.b, s))) return rc;
  rc = solve_batch(g, nrhs, masses, nullptr, st.b, st.x, work_dev, region, params, stats, hip_stream);
  return finish_x(rc, g, nrhs, st.x, x_dev, s);
}

extern "C" int cg_solve(const asq_gauge* g, double mass, const double* b_dev, double* x_dev, void* work_dev,
                        size_t work_bytes, const asq_cg_params* params, asq_cg_stats* stats, void* hip_stream) {
  return cg_solve_batch(g, 1, &mass, b_dev, x_dev, work_dev, work_bytes, params, stats, hip_stream);
}

extern "C" size_t asq_multishift_workspace_bytes(const asq_gauge* g, int nsrc, int nmass, int mode) {
  const size_t r = multishift_native_bytes(g, nsrc, nmass, mode);
  return r ? r + stage_bytes(g, nsrc, (long)nsrc * nmass) : 0;
}

extern "C" int cg_solve_multishift(const asq_gauge* g, int nsrc, int nmass, const double* masses, const double* b_dev,
                                   double* x_dev, void* work_dev, size_t work_bytes, const asq_cg_params* params,
                                   asq_cg_stats* stats, void* hip_stream) {
  const char* who = "cg_solve_multishift";
  if (!g || nsrc <= 0 || nmass <= 0 || !masses || !b_dev || !x_dev || !work_dev || !stats || !params) {
    set_last_error("cg_solve_multishift: null pointer, nsrc <= 0 or nmass <= 0");
    return ASQ_EINVAL;
  }
  const size_t bbytes = (size_t)nsrc * g->geom.half * 48, xbytes = bbytes * nmass;
  int rc = check_io(who, b_dev, bbytes, x_dev, xbytes, work_dev, work_bytes);
  if (rc) return rc;
  if (params->mode < ASQ_MODE_F64 || params->mode > ASQ_MODE_MIXED16) {
    set_last_error("cg_solve_multishift: invalid mode");
    return ASQ_EINVAL;
  }
  if (work_bytes < asq_multishift_workspace_bytes(g, nsrc, nmass, params->mode)) {
    set_last_error("cg_solve_multishift: workspace smaller than asq_multishift_workspace_bytes()");
    return ASQ_ENOMEM;
  }
  const size_t region = multishift_native_bytes(g, nsrc, nmass, params->mode);
  const Stage2 st = stage_at(g, work_dev, region, nsrc);
  hipStream_t s = (hipStream_t)hip_stream;
  if ((rc = relayout(VEC_F64, true, nsrc, g->geom.half, b_dev, st.b, s))) return rc;
  rc = solve_multishift_native(g, nsrc, nmass, masses, st.b, st.x, work_dev, region, params, stats, hip_stream);
  return finish_x(rc, g, nsrc * nmass, st.x, x_dev, s);
}

extern "C" size_t asq_full_workspace_bytes(const asq_gauge* g, int nrhs, int mode) {
  const size_t r = full_native_bytes(g, nrhs, mode);
  return r ? r + stage_bytes(g, 2L * nrhs, 2L * nrhs) : 0;
}

extern "C" int cg_solve_full(const asq_gauge* g, int nrhs, const double* masses, const double* b_dev, double* x_dev,
                             void* work_dev, size_t work_bytes, const asq_cg_params* params, asq_cg_stats* stats,
                             void* hip_stream) {
  const char* who = "cg_solve_full";
  if (!g || nrhs <= 0 || !masses || !b_dev || !x_dev || !work_dev || !stats || !params) {
    set_last_error("cg_solve_full: null pointer or nrhs <= 0");
    return ASQ_EINVAL;
  }
  const size_t vbytes = (size_t)nrhs * 2 * g->geom.half * 48;  // both parities
  int rc = check_io(who, b_dev, vbytes, x_dev, vbytes, work_dev, work_bytes);
  if (rc) return rc;
  if (params->mode < ASQ_MODE_F64 || params->mode > ASQ_MODE_MIXED16) {
    set_last_error("cg_solve_full: invalid mode");
    return ASQ_EINVAL;
  }
  if (work_bytes < asq_full_workspace_bytes(g, nrhs, params->mode)) {
    set_last_error("cg_solve_full: workspace smaller than asq_full_workspace_bytes()");
    return ASQ_ENOMEM;
  }
  const size_t region = full_native_bytes(g, nrhs, params->mode);
  const Stage2 st = stage_at(g, work_dev, region, 2L * nrhs);
  hipStream_t s = (hipStream_t)hip_stream;
  // the even halves of every column, then the odd halves: 2 nrhs vectors of one parity each
  if ((rc = relayout(VEC_F64, true, 2 * nrhs, g->geom.half, b_dev, st.b, s))) return rc;
  rc = solve_full_native(g, nrhs, masses, st.b, st.x, work_dev, region, params, stats, hip_stream);
  return finish_x(rc, g, 2 * nrhs, st.x, x_dev, s);
}
