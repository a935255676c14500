// dslash_impl.h -- the single-parity asqtad hopping term on gfx950 (kernel
// templates; each dslash_*.hip file instantiates one link tier).
//
//   out(x) = sum_mu eta_mu(x) [ F_mu(x) in(x+mu) - F_mu(x-mu)^dag in(x-mu)
//                             + L_mu(x) in(x+3mu) - L_mu(x-3mu)^dag in(x-3mu) ]
// for x of the output parity (the operator whose cost dominates the paper's
// CG inverter; the paper gives no formula, this is the standard asqtad form).
//
// One thread per output site and R columns: every link is loaded once and
// applied to R colour vectors.  Links and vectors are site-fastest structures
// of arrays, so each wavefront load is one contiguous run; neighbour vectors
// come through L2 (blocks are remapped so each XCD walks a contiguous slab).
//
// Epilogues (the CG arithmetic that touches the same output sites):
//   EPI_PLAIN   out = D in
//   EPI_NORM    out = D in and block partials of |out|^2: with t = D_oe p this
//               gives <p, A p> = a |p|^2 + |t|^2, since D_eo = -D_oe^dag
//   EPI_UPDATE  Ap = a p - D_eo t kept in registers; r -= alpha Ap and
//               x += alpha p at the site; block partials of |r|^2.  With few
//               columns every block sums the <p, A p> partials itself (same
//               order and tree as the scalar kernel, so the same alpha) and the
//               scalar launch between the two Dslash launches disappears
//   EPI_RESID   out = b - a y + D in in FP64 (the true residual), stored in the
//               output tier as the new iterated r; block partials of |out|^2
#pragma once
#include <type_traits>

#include "asq_reduce.h"

// The dynamic LDS of a Dslash launch: the block's window of neighbour records
// (launch variant kLdsBit).  Declared here, at file scope, so that the helpers
// that read and write it address it as LDS.
extern __shared__ __align__(16) unsigned char dslash_window[];

namespace asq {
namespace {

__device__ __forceinline__ bool col_on(const DslashArgs& A, int c) {
  if (c >= A.ncol) return false;
  if (A.mask == MASK_ALL || A.st == nullptr) return true;
  const ColState& s = A.st[c];
  if (A.mask == MASK_ACTIVE) return s.active != 0 && s.frozen == 0;
  return s.active != 0 && s.want_ru != 0;
}

// Raw neighbour record of one column: FP16 keeps the 16-byte record (halves and
// norm), the other tiers the colour vector.
template <class InT>
__device__ __forceinline__ typename InT::raw fetch(const void* in, int half, int ncol, int c, int j) {
  if constexpr (InT::kind == VEC_F16) return load_rec_any<InT>(in, half, ncol, c, j);
  else return InT::load(in, half, c, j);
}

// acc += sgn * (U or U^dag) v for one column.  Folded 18-real links carry their
// sign (add or subtract); 12-real links pass their full scale.  FP16 records
// keep the norm out of the product, acc += (sgn nu) (U h), so the binary16
// values feed mixed-precision FMAs directly.
template <class Link, class InT, bool ADJ>
__device__ __forceinline__ void term(const typename InT::raw& w, const Mat3<typename InT::real>& U,
                                     typename InT::real scale, bool neg, Vec3<typename InT::real>& acc) {
  using real = typename InT::real;
  if constexpr (InT::kind == VEC_F16) {
    const float nu = __uint_as_float(w.w);
    const Vec3<float> h = VecF16::halves(w);
    const Vec3<float> u = ADJ ? mul_adj(U, h) : mul(U, h);
    float sc = Link::folded ? nu : nu * scale;
    if (neg) sc = -sc;
    axpy3(acc, sc, u);
  } else {
    const Vec3<real> u = ADJ ? mul_adj(U, w) : mul(U, w);
    if constexpr (Link::folded) {
      if (neg) sub3(acc, u);
      else add3(acc, u);
    } else {
      axpy3(acc, neg ? -scale : scale, u);
    }
  }
}

// The link of a term.  One-column FP64 launches stream their links (measured:
// FP64 CG at 20^3 x 64 104 instead of 110 ms); with several columns the tiles of
// a site block share each link through L2, and the FP32 tiers reuse theirs
// through the memory-side cache across launches, so they load normally.
template <class Link, int R>
__device__ __forceinline__ Mat3<typename Link::real> load_link(const void* base, int half, int p, int slot, int i) {
  if constexpr (R == 1 && (std::is_same<Link, LinkF64R18>::value || std::is_same<Link, LinkF64F32>::value))
    return Link::load_streaming(base, half, p, slot, i);
  else return Link::load(base, half, p, slot, i);
}

// One link term for R columns: all R neighbour loads are issued together
// (columns past the batch read its last column, so no branch is needed), then
// each active column accumulates under its own uniform branch.
template <class Link, class InT, int R, bool ADJ>
__device__ __forceinline__ void link_term(const DslashArgs& A, int p, int slot, int site, int j, int half,
                                          const bool (&on)[R], const int (&col)[R], const void* const (&in)[R],
                                          typename InT::real scale, bool neg, Vec3<typename InT::real> (&acc)[R]) {
  using real = typename InT::real;
  const Mat3<real> U = load_link<Link, R>(A.links, half, p, slot, site);
  typename InT::raw w[R];
#pragma unroll
  for (int r = 0; r < R; ++r) w[r] = fetch<InT>(in[r], half, A.ncol, col[r], j);
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (on[r]) term<Link, InT, ADJ>(w[r], U, scale, neg, acc[r]);
}

// The four terms of direction MU for output site i, accumulated into R columns.
template <class Link, class InT, int R, int MU>
__device__ __forceinline__ void hop_dir(const DslashArgs& A, int i, const Site& s, const bool (&on)[R],
                                        const int (&col)[R], const void* const (&in)[R],
                                        Vec3<typename InT::real> (&acc)[R]) {
  using real = typename InT::real;
  static_assert(std::is_same<typename Link::real, real>::value, "link and vector arithmetic must match");
  const Geom& g = A.g;
  const int p = A.out_parity;
  const int half = g.half;
  const int jf1 = neighbour<MU>(g, i, s, +1);
  const int jb1 = neighbour<MU>(g, i, s, -1);
  const int jf3 = neighbour<MU>(g, i, s, +3);
  const int jb3 = neighbour<MU>(g, i, s, -3);
  // 12-real tiers: coefficient * eta * time-boundary sign, applied to U psi.
  real sf1 = 1, sb1 = 1, sf3 = 1, sb3 = 1;
  if constexpr (!Link::folded) {
    const real e = (real)eta_sign<MU>(s);
    const real cf = (real)A.coeff_fat, cl = (real)A.coeff_long;
    sf1 = e * cf;
    sb1 = e * cf;
    sf3 = e * cl;
    sb3 = e * cl;
    if constexpr (MU == 3) {
      if (s.t == g.T - 1) sf1 = -sf1;
      if (s.t == 0) sb1 = -sb1;
      if (s.t >= g.T - 3) sf3 = -sf3;
      if (s.t < 3) sb3 = -sb3;
    }
  }
  link_term<Link, InT, R, false>(A, p, MU, i, jf1, half, on, col, in, sf1, false, acc);
  link_term<Link, InT, R, true>(A, 1 - p, MU, jb1, jb1, half, on, col, in, sb1, true, acc);
  link_term<Link, InT, R, false>(A, p, 4 + MU, i, jf3, half, on, col, in, sf3, false, acc);
  link_term<Link, InT, R, true>(A, 1 - p, 4 + MU, jb3, jb3, half, on, col, in, sb3, true, acc);
}

// The LDS window of a block (launch variant kLdsBit): the input records
// [lo, lo + n) of each of its R columns, kept word-major per column (word k of
// record q of column r at (r * kWords + k) * stride + q) so that the lanes of a
// wave read consecutive words.  The window spans the block's sites and three
// y-rows on either side, which holds every x neighbour and every y neighbour
// that does not wrap round the lattice.
template <class InT, int R>
struct LdsWin {
  using raw = typename InT::raw;
  static constexpr bool kRecord = InT::kind == VEC_F16;  // FP16: one 16-byte word per record
  using word = typename std::conditional<kRecord, uint4, typename InT::real>::type;
  static constexpr int kWords = kRecord ? 1 : 6;
  int lo = 0, n = 0, stride = 0;
  __device__ __forceinline__ static word* words() { return reinterpret_cast<word*>(dslash_window); }
  __device__ __forceinline__ void put(int r, int q, const raw& v) const {
    const int b = r * kWords * stride + q;
    if constexpr (kRecord) {
      words()[b] = v;
    } else {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        words()[b + (2 * a) * stride] = v.c[a].re;
        words()[b + (2 * a + 1) * stride] = v.c[a].im;
      }
    }
  }
  __device__ __forceinline__ raw get(int r, int q) const {
    const int b = r * kWords * stride + q;
    if constexpr (kRecord) {
      return words()[b];
    } else {
      raw v;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        v.c[a].re = words()[b + (2 * a) * stride];
        v.c[a].im = words()[b + (2 * a + 1) * stride];
      }
      return v;
    }
  }
};

// Software-pipelined form of the 16 terms: the link and the R neighbour records
// of term K+1 are loaded before the arithmetic of term K, so each wave keeps
// loads in flight while it computes (two stages of registers).
template <class Link, class InT, int R>
struct Stage {
  Mat3<typename InT::real> U;
  typename InT::raw w[R];
};

template <int K>
struct TermK {
  static constexpr int MU = K / 4;
  static constexpr int kind = K % 4;  // +1, -1, +3, -3 hops
  static constexpr int hop = kind == 0 ? 1 : (kind == 1 ? -1 : (kind == 2 ? 3 : -3));
  static constexpr int slot = (kind < 2 ? 0 : 4) + MU;
  static constexpr bool back = (kind & 1) != 0;
};

template <class Link, class InT, int R, int K, bool LDS>
__device__ __forceinline__ void stage_load(const DslashArgs& A, int i, const Site& s, const int (&col)[R],
                                           const void* const (&in)[R], const LdsWin<InT, R>& win,
                                           Stage<Link, InT, R>& st) {
  using T = TermK<K>;
  const int half = A.g.half;
  const int p = A.out_parity;
  const int j = neighbour<T::MU>(A.g, i, s, T::hop);
  st.U = load_link<Link, R>(A.links, half, T::back ? 1 - p : p, T::slot, T::back ? j : i);
  if constexpr (LDS && T::MU < 2) {
    // y hops that wrap round the lattice leave the window: those lanes load as usual
    const int q = j - win.lo;
    if ((unsigned)q < (unsigned)win.n) {
#pragma unroll
      for (int r = 0; r < R; ++r) st.w[r] = win.get(r, q);
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) st.w[r] = fetch<InT>(in[r], half, A.ncol, col[r], j);
    }
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) st.w[r] = fetch<InT>(in[r], half, A.ncol, col[r], j);
  }
}

template <class Link, class InT, int R, int K>
__device__ __forceinline__ void stage_compute(const DslashArgs& A, const Site& s, const bool (&on)[R],
                                              const Stage<Link, InT, R>& st, Vec3<typename InT::real> (&acc)[R]) {
  using T = TermK<K>;
  using real = typename InT::real;
  real sc = 1;
  if constexpr (!Link::folded) {
    sc = (real)eta_sign<T::MU>(s) * (real)(T::kind < 2 ? A.coeff_fat : A.coeff_long);
    if constexpr (T::MU == 3) {
      const int t = s.t, Tn = A.g.T;
      const bool flip = T::kind == 0 ? (t == Tn - 1) : T::kind == 1 ? (t == 0) : T::kind == 2 ? (t >= Tn - 3) : (t < 3);
      if (flip) sc = -sc;
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (on[r]) term<Link, InT, T::back>(st.w[r], st.U, sc, T::back, acc[r]);
}

template <class Link, class InT, int R, int K, bool LDS>
__device__ __forceinline__ void pipe_run(const DslashArgs& A, int i, const Site& s, const bool (&on)[R],
                                         const int (&col)[R], const void* const (&in)[R], const LdsWin<InT, R>& win,
                                         Stage<Link, InT, R> (&st)[2], Vec3<typename InT::real> (&acc)[R]) {
  if constexpr (K + 1 < 16) stage_load<Link, InT, R, K + 1, LDS>(A, i, s, col, in, win, st[(K + 1) & 1]);
  stage_compute<Link, InT, R, K>(A, s, on, st[K & 1], acc);
  if constexpr (K + 1 < 16) pipe_run<Link, InT, R, K + 1, LDS>(A, i, s, on, col, in, win, st, acc);
}

// alpha of column c from its reduced |p|^2 and |t|^2 partial sums: false (and
// the column stopped, by one block) when <p, A p> is not positive and finite.
// Block 0 also leaves the record the scalar kernel would have left; no block of
// the launch reads those fields.
__device__ __forceinline__ bool fold_alpha(const DslashArgs& A, int c, int sblk, double pp, double tt,
                                           double& alpha) {
  ColState& S = A.st[c];
  const double pAp = S.a * pp + tt;
  const bool ok = isfinite(pAp) && pAp > 0;
  alpha = ok ? S.rr / pAp : 0.0;
  if (sblk == 0 && threadIdx.x == 0) {
    S.pAp = pAp;
    if (ok) {
      S.alpha = alpha;
    } else {
      S.status = ASQ_ENAN;
      S.active = 0;
    }
  }
  return ok;
}

// The column's new direction buffer (pbuf == 0: the alternate one).
__device__ __forceinline__ const void* pick_new(const DslashArgs& A, const void* base, const void* alt, int c) {
  return A.st[c].pbuf ? base : alt;
}

// One block covers kBlock sites and one tile of R columns.  The order in which
// blocks walk (site block, tile) pairs is a launch choice (Order): with the
// tiles of a site block adjacent, a link leaves HBM once for all tiles; with
// all site blocks of a tile adjacent (inside groups of site blocks), a column's
// far neighbours (the t and z hops) are re-read while still in L2.
template <class Link, class InT, class OutT, int R, int EPI, bool PIPE, bool LDS = false>
__global__ void __launch_bounds__(kBlock) dslash_kernel(const DslashArgs A) {
  using real = typename InT::real;
  int lin = A.sweep_chunk > 0 ? sweep_remap((int)blockIdx.x, (int)gridDim.x, A.sweep_chunk)
                              : xcd_remap((int)blockIdx.x, (int)gridDim.x);
  // Alternate sweeps start on the links the previous sweep read last, which the
  // memory-side cache (MALL) still holds.
  if (A.reverse) lin = (int)gridDim.x - 1 - lin;
  int tile, sblk;
  if (A.sgroup <= 0) {
    tile = lin % A.ntiles;  // the tiles of a site block are neighbours in dispatch order
    sblk = lin / A.ntiles;
  } else {
    // groups of sgroup site blocks; inside a group, tile by tile
    const int per = A.sgroup * A.ntiles;
    const int grp = lin / per, w = lin % per;
    const int gsz = min(A.sgroup, A.nblk - grp * A.sgroup);  // the last group may be short
    tile = w / gsz;
    sblk = grp * A.sgroup + w % gsz;
  }
  const int tid = (int)threadIdx.x;
  const int c0 = tile * R;
  bool on[R];
  int col[R];
  const void* in[R];
  bool any = false;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int c = c0 + r;
    on[r] = col_on(A, c);
    any |= on[r];
    col[r] = c < A.ncol ? c : A.ncol - 1;  // in-bounds column for the unconditional loads
    in[r] = (on[r] && A.in_sel) ? pick_new(A, A.in, A.in_alt, c) : A.in;
  }
  if (!any) return;  // uniform over the block
  // alpha of each column for the UPDATE epilogue, formed in this launch from the
  // partials for the narrow tiles of small batches (same order and tree as the
  // scalar kernel): up to 4 kBlock partials per column (the launch refuses more),
  // loaded here and summed after the hop loop, which hides their latency.
  [[maybe_unused]] double alpha[R];
  [[maybe_unused]] double qa[R][4], qb[R][4];
  [[maybe_unused]] bool fold = false;
  if constexpr (EPI == EPI_UPDATE && R <= kFoldAlphaMaxTile) {
    fold = A.apa != nullptr;
    if (fold) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double* pa = A.apa + (size_t)(c0 + r) * A.nblk;
        const double* pb = A.apb + (size_t)(c0 + r) * A.nblk;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int k = tid + q * kBlock;
          const bool in = on[r] && k < A.nblk;
          qa[r][q] = in ? pa[k] : 0.0;
          qb[r][q] = in ? pb[k] : 0.0;
        }
      }
    }
  }
  const int half = A.g.half;
  const int i = sblk * kBlock + tid;
  const bool valid = i < half;

  LdsWin<InT, R> win;
  if constexpr (LDS) {
    // every thread of the block, in range or not, helps fill the window (the
    // columns past the batch, or not active, are read as the hop loop reads them)
    win.stride = lds_window(A.g.Xh);
    const int i0 = sblk * kBlock;
    win.lo = max(0, i0 - 3 * A.g.Xh);
    win.n = min(half, i0 + kBlock + 3 * A.g.Xh) - win.lo;
    for (int q = tid; q < win.n; q += kBlock) {
#pragma unroll
      for (int r = 0; r < R; ++r) win.put(r, q, fetch<InT>(in[r], half, A.ncol, col[r], win.lo + q));
    }
    __syncthreads();
  }

  Vec3<real> acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int a = 0; a < 3; ++a) acc[r].c[a].re = acc[r].c[a].im = 0;

  if (valid) {
    const Site s = decode(A.g, i, A.out_parity);
    if constexpr (PIPE) {
      Stage<Link, InT, R> st[2];
      stage_load<Link, InT, R, 0, LDS>(A, i, s, col, in, win, st[0]);
      pipe_run<Link, InT, R, 0, LDS>(A, i, s, on, col, in, win, st, acc);
    } else {
      hop_dir<Link, InT, R, 0>(A, i, s, on, col, in, acc);
      hop_dir<Link, InT, R, 1>(A, i, s, on, col, in, acc);
      hop_dir<Link, InT, R, 2>(A, i, s, on, col, in, acc);
      hop_dir<Link, InT, R, 3>(A, i, s, on, col, in, acc);
    }
  }

  if constexpr (EPI == EPI_PLAIN) {
    if (valid) {
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (on[r]) store_any<OutT>(A.out, half, A.ncol, c0 + r, i, convert<typename OutT::real>(acc[r]));
    }
  } else {
    if constexpr (EPI == EPI_UPDATE && R <= kFoldAlphaMaxTile) {
      if (fold) {
        // the sums of the partials loaded before the hop loop (strided_sum's order)
        __shared__ double sa[2 * (kBlock / 64 + 1)];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          alpha[r] = 0;
          if (!on[r]) continue;  // uniform over the block
          double pp = 0, tt = 0;
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (tid + q * kBlock < A.nblk) {
              pp += qa[r][q];
              tt += qb[r][q];
            }
          block_sum2_all(pp, tt, sa);
          on[r] = fold_alpha(A, c0 + r, sblk, pp, tt, alpha[r]);
        }
      }
    }
    // Block partials of |out|^2 per column over the kBlock sites: a wave tree,
    // then the four wave sums in order (the tree and order of block_sum).
    __shared__ double sh[R][kBlock / 64];
    const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int c = c0 + r;
      double d = 0;
      if (valid && on[r]) {
        if constexpr (EPI == EPI_NORM) {
          d = norm2_d(OutT::store(A.out, half, c, i, convert<typename OutT::real>(acc[r])));
        } else if constexpr (EPI == EPI_UPDATE) {
          // OutT is the residual tier.  Ap = a p - D t; r -= alpha Ap; x += alpha p
          using rr = typename OutT::real;
          const ColState& S = A.st[c];
          const void* pb = A.y_sel ? pick_new(A, A.y, A.y_alt, c) : A.y;
          const Vec3<real> y = InT::load(pb, half, c, i);
          const real a = (real)S.a;
          Vec3<rr> ap;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            ap.c[k].re = (rr)fmaR(a, y.c[k].re, -acc[r].c[k].re);
            ap.c[k].im = (rr)fmaR(a, y.c[k].im, -acc[r].c[k].im);
          }
          Vec3<rr> rv = OutT::load(A.r, half, c, i);
          const double al64 = (R <= kFoldAlphaMaxTile && A.apa) ? alpha[r] : S.alpha;
          const rr ar = (rr)al64;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            rv.c[k].re = fmaR(-ar, ap.c[k].re, rv.c[k].re);
            rv.c[k].im = fmaR(-ar, ap.c[k].im, rv.c[k].im);
          }
          d = norm2_d(OutT::store(A.r, half, c, i, rv));
          if constexpr (InT::kind == VEC_F64) {
            // FP64 mode: x itself
            Vec3<double> x = VecF64::load(A.x, half, c, i);
            const double al = al64;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              x.c[k].re = __builtin_fma(al, (double)y.c[k].re, x.c[k].re);
              x.c[k].im = __builtin_fma(al, (double)y.c[k].im, x.c[k].im);
            }
            VecF64::store(A.x, half, c, i, x);
          } else {
            // FP32 accumulator of the reliable-update segment
            Vec3<float> x = VecF32::load(A.x, half, c, i);
            const float al = (float)al64;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              x.c[k].re = fmaR(al, (float)y.c[k].re, x.c[k].re);
              x.c[k].im = fmaR(al, (float)y.c[k].im, x.c[k].im);
            }
            VecF32::store(A.x, half, c, i, x);
          }
        } else {
          // out = b - a y + D in  (FP64);  d = |out|^2
          const double a = A.st[c].a;
          const Vec3<double> y = VecF64::load(A.y, half, c, i);
          const Vec3<double> b = VecF64::load(A.b, half, c, i);
          Vec3<double> o;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            o.c[k].re = __builtin_fma(-a, y.c[k].re, b.c[k].re) + (double)acc[r].c[k].re;
            o.c[k].im = __builtin_fma(-a, y.c[k].im, b.c[k].im) + (double)acc[r].c[k].im;
          }
          OutT::store(A.out, half, c, i, convert<typename OutT::real>(o));
          d = norm2_d(o);
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
      if (lane == 0) sh[r][wv] = d;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (tid == r && on[r]) {
        double tot = 0;
#pragma unroll
        for (int k = 0; k < kBlock / 64; ++k) tot += sh[r][k];
        A.partials[(size_t)(c0 + r) * A.nblk + sblk] = tot;
      }
    }
  }
}

template <class Link, class InT, class OutT, int R, int EPI, bool PIPE, bool LDS = false>
int go(const DslashArgs& a0, int order, int sweep_chunk, hipStream_t s) {
  // alpha is formed in-kernel only by narrow tiles, from at most 4 kBlock partials
  if (a0.apa && (R > kFoldAlphaMaxTile || a0.nblk > 4 * kBlock)) return ASQ_EINVAL;
  DslashArgs a = a0;
  a.ntiles = (a.ncol + R - 1) / R;
  a.sgroup = order_group(order, a.nblk);
  a.sweep_chunk = sweep_chunk;
  const long nb = (long)a.nblk * a.ntiles;
  if (nb <= 0) return ASQ_OK;
  if (nb >= (1L << 31)) return ASQ_EINVAL;
  size_t lds = 0;
  if constexpr (LDS) {
    lds = (size_t)R * lds_window(a.g.Xh) * sizeof(typename InT::raw);
    if (lds > kLdsWindowMax) return ASQ_EINVAL;  // rows too long, or too many columns, for the window
  }
  dslash_kernel<Link, InT, OutT, R, EPI, PIPE, LDS><<<(unsigned)nb, kBlock, lds, s>>>(a);
  return hipGetLastError() == hipSuccess ? ASQ_OK : ASQ_EHIP;
}

// rtile encodes the launch variant (see kPipeBit, kOrderShift): columns per
// thread, the software-pipelined hop loop, the block order.
template <class Link, class InT, class OutT, int EPI>
int pick_r(int rtile, const DslashArgs& a, hipStream_t s) {
  const bool pipe = (rtile & kPipeBit) != 0;
  const int ord = rtile_order(rtile);
  const int gs = sweep_chunk_of(rtile);
  if (rtile & kLdsBit) {
    // the LDS window: pipelined loop, native layouts; one column with ordinary
    // or streamed links, or a tile of 2 to 12 columns
    constexpr bool canon = std::is_same<InT, VecF64C>::value || std::is_same<InT, VecF32C>::value ||
                           std::is_same<InT, VecF16C>::value;
    constexpr bool f64_links = std::is_same<Link, LinkF64R18>::value || std::is_same<Link, LinkF64F32>::value;
    if constexpr (canon) {
      return ASQ_EINVAL;
    } else {
      if (!pipe) return ASQ_EINVAL;
      if (rtile & kStreamBit) {
        if constexpr (f64_links) return ASQ_EINVAL;
        else return (rtile & 0xff) == 1 ? go<Streamed<Link>, InT, OutT, 1, EPI, true, true>(a, ord, gs, s) : ASQ_EINVAL;
      }
      switch (rtile & 0xff) {
        case 1: return go<Link, InT, OutT, 1, EPI, true, true>(a, ord, gs, s);
        case 2: return go<Link, InT, OutT, 2, EPI, true, true>(a, ord, gs, s);
        case 4: return go<Link, InT, OutT, 4, EPI, true, true>(a, ord, gs, s);
        case 6: return go<Link, InT, OutT, 6, EPI, true, true>(a, ord, gs, s);
        case 8: return go<Link, InT, OutT, 8, EPI, true, true>(a, ord, gs, s);
        case 12:
          if constexpr (InT::kind == VEC_F64) return ASQ_EINVAL;
          else return go<Link, InT, OutT, 12, EPI, true, true>(a, ord, gs, s);
      }
      return ASQ_EINVAL;
    }
  }
  if (rtile & kStreamBit) {
    // links streamed past the caches: one column, FP32 and 16-bit tiers (the
    // FP64-stored tiers always stream at one column)
    if constexpr (std::is_same<Link, LinkF64R18>::value || std::is_same<Link, LinkF64F32>::value) {
      return ASQ_EINVAL;
    } else {
      if ((rtile & 0xff) != 1) return ASQ_EINVAL;
      return pipe ? go<Streamed<Link>, InT, OutT, 1, EPI, true>(a, ord, gs, s)
                  : go<Streamed<Link>, InT, OutT, 1, EPI, false>(a, ord, gs, s);
    }
  }
  switch (rtile & 0xff) {
    case 1: return pipe ? go<Link, InT, OutT, 1, EPI, true>(a, ord, gs, s) : go<Link, InT, OutT, 1, EPI, false>(a, ord, gs, s);
    case 2: return pipe ? go<Link, InT, OutT, 2, EPI, true>(a, ord, gs, s) : go<Link, InT, OutT, 2, EPI, false>(a, ord, gs, s);
    case 4: return pipe ? go<Link, InT, OutT, 4, EPI, true>(a, ord, gs, s) : go<Link, InT, OutT, 4, EPI, false>(a, ord, gs, s);
    case 6: return pipe ? go<Link, InT, OutT, 6, EPI, true>(a, ord, gs, s) : go<Link, InT, OutT, 6, EPI, false>(a, ord, gs, s);
    case 8: return pipe ? go<Link, InT, OutT, 8, EPI, true>(a, ord, gs, s) : go<Link, InT, OutT, 8, EPI, false>(a, ord, gs, s);
    case 12:
      // twelve FP64 columns would spill the accumulators: not built
      if constexpr (InT::kind == VEC_F64) return ASQ_EINVAL;
      else return pipe ? go<Link, InT, OutT, 12, EPI, true>(a, ord, gs, s) : go<Link, InT, OutT, 12, EPI, false>(a, ord, gs, s);
  }
  return ASQ_EINVAL;
}

// The public operator on the canonical layouts of the C ABI (PLAIN epilogue).
template <class Link, class V>
int pick_canon(int rtile, const DslashArgs& a, hipStream_t s) {
  return pick_r<Link, V, V, EPI_PLAIN>(rtile, a, s);
}

// Iterated tiers: PLAIN and NORM write the input tier; UPDATE takes the residual tier.
template <class Link, class V, class RT>
int pick_iter(int epi, int rtile, const DslashArgs& a, hipStream_t s) {
  if (epi == EPI_PLAIN) return pick_r<Link, V, V, EPI_PLAIN>(rtile, a, s);
  if (epi == EPI_NORM) return pick_r<Link, V, V, EPI_NORM>(rtile, a, s);
  if (epi == EPI_UPDATE) return pick_r<Link, V, RT, EPI_UPDATE>(rtile, a, s);
  return ASQ_EINVAL;
}

}  // namespace
}  // namespace asq
