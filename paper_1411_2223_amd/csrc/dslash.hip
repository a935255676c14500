// dslash.hip -- the single-parity asqtad hopping term on gfx950.
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
// Fused CG work:
//   FUSEP        the input is the CG direction p = r + beta p_old, formed on the
//                fly at every neighbour; the thread of site x writes the new p of
//                its -x neighbour (each site of the other parity has exactly one
//                such owner) into the second p buffer.
//   EPI_PLAIN    out = D in
//   EPI_XPAY_DOT out = a_c y - D in, block partials of Re<y, out>   (A p and <p, A p>)
//   EPI_RESID    out = b - a_c y + D in (FP64), block partials of |out|^2 (the true
//                residual, also stored in the output tier as the new iterated r)
#include "asq_reduce.h"

namespace asq {
namespace {

__device__ __forceinline__ bool col_on(const DslashArgs& A, int c) {
  if (c >= A.ncol) return false;
  if (A.mask == MASK_ALL || A.st == nullptr) return true;
  const ColState& s = A.st[c];
  if (A.mask == MASK_ACTIVE) return s.active != 0 && s.frozen == 0;
  return s.active != 0 && s.want_ru != 0;
}

template <class InT, int R>
struct Cols {
  using real = typename InT::real;
  bool on[R];
  const void* in[R];  // input (or p_old) base of each column
  void* pnew[R];      // FUSEP: where the owner writes the new p
  real beta[R];
};

// Neighbour vector of column r at site j, with the fused direction update.
template <class InT, class RT, int R, bool FUSEP>
__device__ __forceinline__ Vec3<typename InT::real> fetch(const DslashArgs& A, const Cols<InT, R>& C, int r, int c,
                                                          int j) {
  using real = typename InT::real;
  const int half = A.g.half;
  if constexpr (!FUSEP) {
    return InT::load(C.in[r], half, c, j);
  } else {
    const Vec3<real> p = InT::load(C.in[r], half, c, j);
    const Vec3<real> rv = convert<real>(RT::load(A.rfuse, half, c, j));
    Vec3<real> v;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      v.c[a].re = fmaR(C.beta[r], p.c[a].re, rv.c[a].re);
      v.c[a].im = fmaR(C.beta[r], p.c[a].im, rv.c[a].im);
    }
    return InT::quantize(v);  // exactly the value the owner stores
  }
}

// acc += sgn * (U or U^dag) psi_r(j) for one column.  Folded links carry their
// sign (sgn = +-1 is applied by add/sub); 12-real links pass the full scale.
// FP16 inputs keep the norm out of the product, acc += (sgn nu) (U h), so the
// binary16 values feed the FMAs directly and the per-element rescale is saved.
template <class Link, class InT, class RT, int R, bool FUSEP, bool ADJ>
__device__ __forceinline__ void term(const DslashArgs& A, const Cols<InT, R>& C, int r, int c, int j,
                                     const Mat3<typename InT::real>& U, typename InT::real scale, bool neg,
                                     Vec3<typename InT::real>& acc, void* owner_out) {
  using real = typename InT::real;
  if constexpr (InT::kind == VEC_F16 && !FUSEP) {
    float nu;
    const Vec3<float> h = VecF16::load_raw(C.in[r], A.g.half, c, j, &nu);
    const Vec3<float> u = ADJ ? mul_adj(U, h) : mul(U, h);
    float sc = Link::folded ? nu : nu * scale;
    if (neg) sc = -sc;
    axpy3(acc, sc, u);
  } else {
    const Vec3<real> v = fetch<InT, RT, R, FUSEP>(A, C, r, c, j);
    if (owner_out) InT::store(owner_out, A.g.half, c, j, v);
    const Vec3<real> u = ADJ ? mul_adj(U, v) : mul(U, v);
    if constexpr (Link::folded) {
      if (neg) sub3(acc, u);
      else add3(acc, u);
    } else {
      axpy3(acc, neg ? -scale : scale, u);
    }
  }
}

// The four terms of direction MU for output site i, accumulated into R columns.
template <class Link, class InT, class RT, int R, bool FUSEP, int MU>
__device__ __forceinline__ void hop_dir(const DslashArgs& A, int i, const Site& s, int c0, const Cols<InT, R>& C,
                                        Vec3<typename InT::real> (&acc)[R]) {
  using real = typename InT::real;
  static_assert(sizeof(typename Link::real) == sizeof(real), "link and vector arithmetic must match");
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
  {
    const Mat3<real> U = Link::load(A.links, half, p, MU, i);
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (C.on[r]) term<Link, InT, RT, R, FUSEP, false>(A, C, r, c0 + r, jf1, U, sf1, false, acc[r], nullptr);
  }
  {
    const Mat3<real> U = Link::load(A.links, half, 1 - p, MU, jb1);
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (C.on[r]) {
        // owner of site x - x^: writes the new direction there (fused update only)
        void* own = (FUSEP && MU == 0) ? C.pnew[r] : nullptr;
        term<Link, InT, RT, R, FUSEP, true>(A, C, r, c0 + r, jb1, U, sb1, true, acc[r], own);
      }
  }
  {
    const Mat3<real> U = Link::load(A.links, half, p, 4 + MU, i);
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (C.on[r]) term<Link, InT, RT, R, FUSEP, false>(A, C, r, c0 + r, jf3, U, sf3, false, acc[r], nullptr);
  }
  {
    const Mat3<real> U = Link::load(A.links, half, 1 - p, 4 + MU, jb3);
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (C.on[r]) term<Link, InT, RT, R, FUSEP, true>(A, C, r, c0 + r, jb3, U, sb3, true, acc[r], nullptr);
  }
}

template <class Link, class InT, class OutT, class RT, int R, int EPI, bool FUSEP>
__global__ void __launch_bounds__(kBlock) dslash_kernel(const DslashArgs A) {
  using real = typename InT::real;
  int lin = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  // Alternate sweeps start on the links the previous sweep read last, which the
  // memory-side cache (MALL) still holds.
  if (A.reverse) lin = (int)gridDim.x - 1 - lin;
  const int tile = lin % A.ntiles;  // column tiles of the same sites are neighbours in dispatch order
  const int sblk = lin / A.ntiles;
  const int c0 = tile * R;
  Cols<InT, R> C;
  bool any = false;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int c = c0 + r;
    C.on[r] = col_on(A, c);
    any |= C.on[r];
    int pb = (C.on[r] && A.in_sel) ? A.st[c].pbuf : 0;
    if (A.in_sel == 2) pb ^= 1;
    C.in[r] = pb ? A.in_alt : A.in;
    C.pnew[r] = const_cast<void*>(pb ? A.in : A.in_alt);
    C.beta[r] = (FUSEP && C.on[r]) ? (real)A.st[c].beta : (real)0;
  }
  if (!any) return;  // uniform over the block
  const int half = A.g.half;
  const int i = sblk * kBlock + (int)threadIdx.x;
  const bool valid = i < half;

  Vec3<real> acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int a = 0; a < 3; ++a) acc[r].c[a].re = acc[r].c[a].im = 0;

  if (valid) {
    const Site s = decode(A.g, i, A.out_parity);
    hop_dir<Link, InT, RT, R, FUSEP, 0>(A, i, s, c0, C, acc);
    hop_dir<Link, InT, RT, R, FUSEP, 1>(A, i, s, c0, C, acc);
    hop_dir<Link, InT, RT, R, FUSEP, 2>(A, i, s, c0, C, acc);
    hop_dir<Link, InT, RT, R, FUSEP, 3>(A, i, s, c0, C, acc);
  }

  if constexpr (EPI == EPI_PLAIN) {
    if (valid) {
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (C.on[r]) OutT::store(A.out, half, c0 + r, i, convert<typename OutT::real>(acc[r]));
    }
  } else {
    __shared__ double sh[kBlock / 64];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!C.on[r]) continue;  // uniform over the block
      const int c = c0 + r;
      double d = 0;
      if (valid) {
        if constexpr (EPI == EPI_XPAY_DOT) {
          // out = a y - D in;  d = Re<y, out>
          const real a = (real)A.st[c].a;
          const void* yb = A.y;
          if (A.y_sel) yb = A.st[c].pbuf ? A.y : A.y_alt;
          const Vec3<real> y = InT::load(yb, half, c, i);
          Vec3<real> o;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            o.c[k].re = fmaR(a, y.c[k].re, -acc[r].c[k].re);
            o.c[k].im = fmaR(a, y.c[k].im, -acc[r].c[k].im);
          }
          // the dot uses the stored (possibly 16-bit) A p, the value the update reads back
          const Vec3<real> os = OutT::store(A.out, half, c, i, convert<typename OutT::real>(o));
          d = redot_d(y, os);
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
      const double tot = block_sum(d, sh);
      if (threadIdx.x == 0) A.partials[(size_t)c * A.nblk + sblk] = tot;
      __syncthreads();
    }
  }
}

template <class Link, class InT, class OutT, class RT, int R, int EPI, bool FUSEP>
int go(const DslashArgs& a0, hipStream_t s) {
  DslashArgs a = a0;
  a.ntiles = (a.ncol + R - 1) / R;
  const long nb = (long)a.nblk * a.ntiles;
  if (nb <= 0) return ASQ_OK;
  if (nb >= (1L << 31)) return ASQ_EINVAL;
  dslash_kernel<Link, InT, OutT, RT, R, EPI, FUSEP><<<(unsigned)nb, kBlock, 0, s>>>(a);
  return hipGetLastError() == hipSuccess ? ASQ_OK : ASQ_EHIP;
}

template <class Link, class InT, class OutT, class RT, int EPI, bool FUSEP>
int pick_r(int rtile, const DslashArgs& a, hipStream_t s) {
  switch (rtile) {
    case 1: return go<Link, InT, OutT, RT, 1, EPI, FUSEP>(a, s);
    case 2: return go<Link, InT, OutT, RT, 2, EPI, FUSEP>(a, s);
    case 4: return go<Link, InT, OutT, RT, 4, EPI, FUSEP>(a, s);
    case 8: return go<Link, InT, OutT, RT, 8, EPI, FUSEP>(a, s);
  }
  return ASQ_EINVAL;
}

// Iterated tiers: PLAIN (optionally with the fused direction update) and XPAY_DOT.
template <class Link, class V, class RT>
int pick_sloppy(int epi, int rtile, const DslashArgs& a, hipStream_t s, bool fuse) {
  if (epi == EPI_PLAIN) {
    if (fuse) return pick_r<Link, V, V, RT, EPI_PLAIN, true>(rtile, a, s);
    return pick_r<Link, V, V, RT, EPI_PLAIN, false>(rtile, a, s);
  }
  if (epi == EPI_XPAY_DOT && !fuse) return pick_r<Link, V, V, RT, EPI_XPAY_DOT, false>(rtile, a, s);
  return ASQ_EINVAL;
}

}  // namespace

int launch_dslash(int link_kind, int in_kind, int out_kind, int epi, int rtile, const DslashArgs& a,
                  hipStream_t s, int fuse_rt) {
  const bool fuse = fuse_rt >= 0;
  if (fuse && !a.rfuse) return ASQ_EINVAL;
  if (link_kind == LINK_F64_R18) {
    if (in_kind != VEC_F64) return ASQ_EINVAL;
    if (epi == EPI_RESID) {
      if (fuse) return ASQ_EINVAL;
      if (out_kind == VEC_F64) return pick_r<LinkF64R18, VecF64, VecF64, VecF64, EPI_RESID, false>(rtile, a, s);
      if (out_kind == VEC_F32) return pick_r<LinkF64R18, VecF64, VecF32, VecF64, EPI_RESID, false>(rtile, a, s);
      return ASQ_EINVAL;
    }
    if (out_kind != VEC_F64 || (fuse && fuse_rt != VEC_F64)) return ASQ_EINVAL;
    return pick_sloppy<LinkF64R18, VecF64, VecF64>(epi, rtile, a, s, fuse);
  }
  if (epi == EPI_RESID || in_kind != out_kind) return ASQ_EINVAL;
  if (fuse && fuse_rt != VEC_F32) return ASQ_EINVAL;
  if (link_kind == LINK_F32_R18) {
    if (in_kind == VEC_F32) return pick_sloppy<LinkF32R18, VecF32, VecF32>(epi, rtile, a, s, fuse);
    if (in_kind == VEC_F16) return pick_sloppy<LinkF32R18, VecF16, VecF32>(epi, rtile, a, s, fuse);
  } else if (link_kind == LINK_F32_R12) {
    if (in_kind == VEC_F32) return pick_sloppy<LinkF32R12, VecF32, VecF32>(epi, rtile, a, s, fuse);
    if (in_kind == VEC_F16) return pick_sloppy<LinkF32R12, VecF16, VecF32>(epi, rtile, a, s, fuse);
  } else if (link_kind == LINK_I16_R12) {
    if (in_kind == VEC_F16) return pick_sloppy<LinkI16R12, VecF16, VecF32>(epi, rtile, a, s, fuse);
  }
  return ASQ_EINVAL;
}

}  // namespace asq
