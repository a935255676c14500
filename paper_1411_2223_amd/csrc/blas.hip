// blas.hip -- CG vector updates and deterministic FP64 reductions.
//
// Every vector kernel runs on a (site block, column) grid and writes one FP64
// partial per block and column; the reduction kernels sum the partials of a
// column in a fixed order and update that column's scalars on the device
// (alpha, beta, reliable-update and convergence decisions), so no scalar ever
// travels to the host inside the iteration and a column's arithmetic never
// depends on the other columns of the batch.
#include <math.h>

#include "asq_internal.h"
#include "asq_solver.h"

namespace asq {
namespace {

__device__ __forceinline__ bool state_on(const ColState& s, int mask) {
  if (mask == MASK_ALL) return true;
  if (mask == MASK_ACTIVE) return s.active != 0 && s.frozen == 0;
  return s.active != 0 && s.want_ru != 0;
}

template <class R>
__device__ __forceinline__ Vec3<R> zero3() {
  Vec3<R> v;
#pragma unroll
  for (int a = 0; a < 3; ++a) v.c[a].re = v.c[a].im = 0;
  return v;
}

// x = 0, r = b, p = b; partial |b|^2.
template <class PT, class RT>
__global__ void __launch_bounds__(kBlock) init_kernel(const VecArgs A) {
  const int c = blockIdx.y, sblk = blockIdx.x;
  const int half = A.half;
  const int i = sblk * kBlock + (int)threadIdx.x;
  double d = 0;
  if (i < half) {
    const Vec3<double> b = VecF64::load(A.b, half, c, i);
    VecF64::store(A.x, half, c, i, zero3<double>());
    RT::store(A.r, half, c, i, convert<typename RT::real>(b));
    PT::store(A.p, half, c, i, convert<typename PT::real>(b));
    d = norm2_d(b);
  }
  __shared__ double sh[kBlock / 64];
  const double tot = block_sum(d, sh);
  if (threadIdx.x == 0) A.partials[(size_t)c * A.nblk + sblk] = tot;
}

// x += alpha p (FP64); r -= alpha A p; partial |r|^2 of the stored r.
template <class PT, class RT>
__global__ void __launch_bounds__(kBlock) update_xr_kernel(const VecArgs A) {
  const int c = blockIdx.y, sblk = blockIdx.x;
  if (!state_on(A.st[c], MASK_ACTIVE)) return;
  using rr = typename RT::real;
  const int half = A.half;
  const int i = sblk * kBlock + (int)threadIdx.x;
  double d = 0;
  if (i < half) {
    const double alpha = A.st[c].alpha;
    const Vec3<double> p = convert<double>(PT::load(A.p, half, c, i));
    const Vec3<rr> ap = convert<rr>(PT::load(A.Ap, half, c, i));
    Vec3<double> x = VecF64::load(A.x, half, c, i);
    Vec3<rr> r = RT::load(A.r, half, c, i);
    const rr ar = (rr)alpha;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      x.c[a].re = __builtin_fma(alpha, p.c[a].re, x.c[a].re);
      x.c[a].im = __builtin_fma(alpha, p.c[a].im, x.c[a].im);
      r.c[a].re = fmaR(-ar, ap.c[a].re, r.c[a].re);
      r.c[a].im = fmaR(-ar, ap.c[a].im, r.c[a].im);
    }
    VecF64::store(A.x, half, c, i, x);
    d = norm2_d(RT::store(A.r, half, c, i, r));
  }
  __shared__ double sh[kBlock / 64];
  const double tot = block_sum(d, sh);
  if (threadIdx.x == 0) A.partials[(size_t)c * A.nblk + sblk] = tot;
}

// p = r + beta p.
template <class PT, class RT>
__global__ void __launch_bounds__(kBlock) update_p_kernel(const VecArgs A) {
  const int c = blockIdx.y, sblk = blockIdx.x;
  if (!state_on(A.st[c], MASK_ACTIVE)) return;
  using pr = typename PT::real;
  const int half = A.half;
  const int i = sblk * kBlock + (int)threadIdx.x;
  if (i >= half) return;
  const pr beta = (pr)A.st[c].beta;
  const Vec3<pr> r = convert<pr>(RT::load(A.r, half, c, i));
  Vec3<pr> p = PT::load(A.p, half, c, i);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    p.c[a].re = fmaR(beta, p.c[a].re, r.c[a].re);
    p.c[a].im = fmaR(beta, p.c[a].im, r.c[a].im);
  }
  PT::store(A.p, half, c, i, p);
}

// Fixed-order sum of a column's block partials, then the scalar update.
__global__ void __launch_bounds__(kBlock) reduce_kernel(ColState* st, const double* partials, int nblk, int op) {
  const int c = blockIdx.x;
  ColState& S = st[c];
  const int mask = op == OP_ALPHA || op == OP_BETA ? MASK_ACTIVE : (op == OP_RU ? MASK_RELIABLE : MASK_ALL);
  if (!state_on(S, mask)) return;
  double v = 0;
  for (int k = (int)threadIdx.x; k < nblk; k += kBlock) v += partials[(size_t)c * nblk + k];
  __shared__ double sh[kBlock / 64];
  const double s = block_sum(v, sh);
  if (threadIdx.x != 0) return;
  const bool finite = isfinite(s);
  switch (op) {
    case OP_INIT:
      S.bb = s;
      S.rr = s;
      S.true_rr = s;
      S.maxr = sqrt(s);
      S.iters = 0;
      S.n_ru = 0;
      S.want_ru = 0;
      S.frozen = 0;
      S.status = finite ? 0 : ASQ_ENAN;
      S.converged = finite && s == 0;
      S.active = finite && s > 0;
      break;
    case OP_ALPHA:
      S.pAp = s;
      if (!finite || !(s > 0)) {
        S.status = ASQ_ENAN;
        S.active = 0;
      } else {
        S.alpha = S.rr / s;
      }
      break;
    case OP_BETA: {
      S.iters += 1;
      if (!finite) {
        S.status = ASQ_ENAN;
        S.active = 0;
        break;
      }
      S.beta = s / S.rr;
      S.rr = s;
      const double r = sqrt(s);
      if (r <= S.tol * sqrt(S.bb) || S.iters >= S.maxiter) {
        // iterated residual met tol (or the budget is spent): check in FP64
        S.frozen = 1;
        S.want_ru = 1;
      } else if (S.delta > 0 && r < S.delta * S.maxr) {
        S.want_ru = 1;
      }
      S.maxr = fmax(S.maxr, r);
      break;
    }
    case OP_RU:
      S.true_rr = s;
      S.n_ru += 1;
      if (!finite) {
        S.status = ASQ_ENAN;
        S.active = 0;
      } else if (sqrt(s) <= S.tol * sqrt(S.bb)) {
        S.converged = 1;
        S.active = 0;
      } else if (S.iters >= S.maxiter) {
        S.status = ASQ_ENOCONV;
        S.active = 0;
      } else {
        S.rr = s;
        S.maxr = sqrt(s);
        S.want_ru = 0;
        S.frozen = 0;
      }
      break;
    case OP_FINAL:
      S.true_rr = s;
      break;
  }
}

__global__ void copy_kernel(uint4* __restrict__ dst, const uint4* __restrict__ src, size_t n) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
    dst[k] = src[k];
}

template <class PT, class RT>
int launch_vec(int which, const VecArgs& a, int ncol, hipStream_t s) {
  const dim3 grid((unsigned)a.nblk, (unsigned)ncol);
  if (which == VK_INIT) init_kernel<PT, RT><<<grid, kBlock, 0, s>>>(a);
  else if (which == VK_XR) update_xr_kernel<PT, RT><<<grid, kBlock, 0, s>>>(a);
  else update_p_kernel<PT, RT><<<grid, kBlock, 0, s>>>(a);
  return hipGetLastError() == hipSuccess ? ASQ_OK : ASQ_EHIP;
}

}  // namespace

int launch_vec_kernel(int which, int pt, int rt, const VecArgs& a, int ncol, hipStream_t s) {
  if (pt == VEC_F64 && rt == VEC_F64) return launch_vec<VecF64, VecF64>(which, a, ncol, s);
  if (pt == VEC_F32 && rt == VEC_F32) return launch_vec<VecF32, VecF32>(which, a, ncol, s);
  if (pt == VEC_F16 && rt == VEC_F32) return launch_vec<VecF16, VecF32>(which, a, ncol, s);
  return ASQ_EINVAL;
}

int launch_reduce(int op, ColState* st, const double* partials, int nblk, int ncol, hipStream_t s) {
  reduce_kernel<<<(unsigned)ncol, kBlock, 0, s>>>(st, partials, nblk, op);
  return hipGetLastError() == hipSuccess ? ASQ_OK : ASQ_EHIP;
}

size_t vec_site_bytes(int kind) {
  switch (kind) {
    case VEC_F64: return 48;
    case VEC_F32: return 24;
    case VEC_F16: return 16;
  }
  return 0;
}

}  // namespace asq

extern "C" int asq_copy_probe(void* dst_dev, const void* src_dev, size_t n, void* hip_stream) {
  if (!dst_dev || !src_dev || (n & 15) || ((uintptr_t)dst_dev & 15) || ((uintptr_t)src_dev & 15))
    return ASQ_EINVAL;
  const size_t n16 = n / 16;
  if (n16 == 0) return ASQ_OK;
  size_t blocks = (n16 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  asq::copy_kernel<<<(unsigned)blocks, 256, 0, (hipStream_t)hip_stream>>>((uint4*)dst_dev, (const uint4*)src_dev, n16);
  ASQ_HIP_TRY(hipGetLastError());
  return ASQ_OK;
}
