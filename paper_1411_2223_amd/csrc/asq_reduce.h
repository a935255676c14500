// asq_reduce.h -- deterministic per-column reductions and the scalar updates
// of CG.  Producers write one FP64 partial per (column, site block); a
// consumer sums a column's partials in block order with a fixed tree, so the
// result is bitwise reproducible and independent of the other columns.  No
// block waits on another inside a kernel: on a multi-XCD part that would need
// device-scope release/acquire fences, which write back and invalidate the
// XCD's L2 and with it the cached neighbour vectors of every other block.
#pragma once
#include <math.h>

#include "asq_internal.h"

namespace asq {

// Scalar update of one column from its reduced sum s (thread 0 of one block).
__device__ inline void finalize_column(ColState& S, double s, int op) {
  const bool finite = isfinite(s);
  switch (op) {
    case OP_INIT:
      S.bb = s;
      S.rr = s;
      S.rr_old = s;
      S.true_rr = s;
      S.maxr = sqrt(s);
      S.alpha = 0;
      S.beta = 0;
      S.iters = 0;
      S.n_ru = 0;
      S.want_ru = 0;
      S.frozen = 0;
      S.pbuf = 0;
      S.status = finite ? 0 : ASQ_ENAN;
      S.converged = finite && s == 0;
      S.active = finite && s > 0;
      S.ref_rr = s;
      S.n_stall = 0;
      S.escalate = 0;
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
      if (!S.active) break;  // stopped by OP_ALPHA
      S.iters += 1;
      S.pbuf ^= 1;  // the new direction becomes current
      if (!finite) {
        S.status = ASQ_ENAN;
        S.active = 0;
        break;
      }
      S.rr_old = S.rr;
      S.rr = s;
      S.beta = s / S.rr_old;
      const double r = sqrt(s);
      if (r <= S.tol * sqrt(S.bb) || S.iters >= S.maxiter) {
        if (S.sloppy_stop) {
          S.active = 0;  // the caller decides on the solution
        } else {
          // iterated residual met tol (or the budget is spent): decide on the FP64 residual
          S.frozen = 1;
          S.want_ru = 1;
        }
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
      } else if (S.stall_updates > 0 && !(s < S.stall_fac * S.ref_rr) && ++S.n_stall >= S.stall_updates) {
        // the true residual stopped falling in this precision: hand the column on
        S.escalate = 1;
        S.active = 0;
      } else {
        if (s < S.stall_fac * S.ref_rr) {
          S.ref_rr = s;
          S.n_stall = 0;
        }
        // r was replaced by the true residual: restart the norm history from it
        S.rr = s;
        S.beta = s / S.rr_old;
        S.maxr = sqrt(s);
        S.want_ru = 0;
        S.frozen = 0;
      }
      break;
  }
}

// Start from a given x: bb = |b|^2, rr = |b - A x|^2 (FP64).  With b = 0 the
// relative tolerance cannot be met unless r = 0 as well.
__device__ inline void finalize_guess(ColState& S, double bb, double rr) {
  const bool finite = isfinite(bb) && isfinite(rr);
  S.bb = bb;
  S.rr = rr;
  S.rr_old = rr;
  S.true_rr = rr;
  S.maxr = sqrt(rr);
  S.alpha = 0;
  S.beta = 0;
  S.iters = 0;
  S.n_ru = 0;
  S.want_ru = 0;
  S.frozen = 0;
  S.pbuf = 0;
  S.status = finite ? 0 : ASQ_ENAN;
  S.converged = finite && (rr == 0 || (bb > 0 && sqrt(rr) <= S.tol * sqrt(bb)));
  S.active = finite && !S.converged;
  S.ref_rr = rr;
  S.n_stall = 0;
  S.escalate = 0;
}

// This thread's share of a fixed-order sum of partials[0..n): elements
// threadIdx.x, threadIdx.x + kBlock, ... added in increasing order.  Every
// group of four loads, the last partial one included, is issued before its adds
// (the same adds in the same order, so the same bits), so a sum of n partials
// costs about n / (4 kBlock) memory round trips instead of n / kBlock.
__device__ inline double strided_sum(const double* partials, int n) {
  double v = 0;
  for (int k = (int)threadIdx.x; k < n; k += 4 * kBlock) {
    const bool h1 = k + kBlock < n, h2 = k + 2 * kBlock < n, h3 = k + 3 * kBlock < n;
    const double a = partials[k];
    const double b = h1 ? partials[k + kBlock] : 0.0;
    const double c = h2 ? partials[k + 2 * kBlock] : 0.0;
    const double d = h3 ? partials[k + 3 * kBlock] : 0.0;
    v += a;
    if (h1) v += b;
    if (h2) v += c;
    if (h3) v += d;
  }
  return v;
}

// Sums of u and v over the block, valid in every thread (each the bits of
// block_sum).  sh: 2 (kBlock/64 + 1) doubles of LDS.
__device__ inline void block_sum2_all(double& u, double& v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    u += __shfl_xor(u, o, 64);
    v += __shfl_xor(v, o, 64);
  }
  constexpr int W = kBlock / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    sh[w] = u;
    sh[W + 1 + w] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double su = 0, sv = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      su += sh[k];
      sv += sh[W + 1 + k];
    }
    sh[W] = su;
    sh[2 * W + 1] = sv;
  }
  __syncthreads();
  u = sh[W];
  v = sh[2 * W + 1];
}

}  // namespace asq
