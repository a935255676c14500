// dslash_mfma.h -- the many-column hopping term on the matrix cores: FP32
// 18-real links, FP16-with-norm input vectors, FP32 arithmetic.
//
// For one output site x and a set of columns the 16 link terms form one real
// contraction: out(x)[6 reals x columns] = sum over terms d of W_d [6 x 6] times
// in(x + d)[6 reals x columns], where W_d is the real form of the signed 3x3
// complex link of term d (U for forward hops, -U^dag for backward ones; the
// 18-real tier already carries eta, the time-boundary sign and the fat or long
// coefficient).  In the real form, for W = U or U^dag with entry w = (wr, wi)
// in row c and column c',
//     out_re[c] += wr in_re[c'] - wi in_im[c']      out_im[c] += wi in_re[c'] + wr in_im[c'].
//
// v_mfma_f32_4x4x1_16b_f32 does 16 independent 4x4x1 products per wave.  Block
// b of the instruction (lanes 4b..4b+3) is one output site; lane 4b+q supplies
// row q of the A operand (a row of W) and column q of the B operand (the input
// of column q).  The six output rows are two row tiles (rows 0-3 and 4-7, the
// last two zero), so 75 % of the products are useful, and each input real is one
// K step.  The accumulator of lane 4b+q holds rows 0-3 (and 4-7 in the second
// tile) of column q: the whole output vector of one (site, column) in one lane,
// which the epilogues (FP16 encoding, norms, the CG update) need.
//
// A block of kBlock threads covers kBlock sites: each of its 4 waves walks 4
// groups of 16 sites; the block's columns are a tile of kMfmaCols.  Partials of
// |out|^2 are per column and block of kBlock sites, like the other kernels',
// but summed in another order; the matrix-core sums also round differently, so
// this form is bitwise reproducible only against itself.
#pragma once

namespace asq {
namespace {

constexpr int kMfmaGroups = 8;                  // column groups of 4 per block
constexpr int kMfmaCols = 4 * kMfmaGroups;      // columns per block

typedef float mfma_v4 __attribute__((ext_vector_type(4)));

// The loads of one link term for the 16 sites of a wave and kMfmaGroups groups
// of 4 columns: two rows of the link (this lane's row of W and row 2) and the
// input record of each of the lane's columns.
struct MfmaStage {
  float2 w0[3], w2[3];
  uint4 rec[kMfmaGroups];
};

template <int K>
__device__ __forceinline__ void mfma_load(const DslashArgs& A, int i, const Site& s, int q,
                                          const int (&col)[kMfmaGroups], const void* const (&in)[kMfmaGroups],
                                          MfmaStage& st) {
  using T = TermK<K>;
  const int half = A.g.half;
  const int p = A.out_parity;
  const int j = neighbour<T::MU>(A.g, i, s, T::hop);
  const float2* L = reinterpret_cast<const float2*>(A.links) +
                    (size_t)(((T::back ? 1 - p : p) * 8 + T::slot) * LinkF32R18::NCH) * half + (T::back ? j : i);
  const int c0 = q >> 1;  // colour of this lane's row in the first row tile
#pragma unroll
  for (int cp = 0; cp < 3; ++cp) {
    // W[c][c'] = U[c][c'] forward, conj(U[c'][c]) backward (conjugated in mfma_compute)
    st.w0[cp] = T::back ? L[(size_t)(3 * cp + c0) * half] : L[(size_t)(3 * c0 + cp) * half];
    st.w2[cp] = T::back ? L[(size_t)(3 * cp + 2) * half] : L[(size_t)(6 + cp) * half];
  }
#pragma unroll
  for (int g = 0; g < kMfmaGroups; ++g) st.rec[g] = VecF16::load_rec(in[g], half, col[g], j);
}

template <int K>
__device__ __forceinline__ void mfma_compute(int q, const MfmaStage& st, mfma_v4 (&acc)[kMfmaGroups][2]) {
  using T = TermK<K>;
  const bool imrow = q & 1;  // the row is the imaginary part
  const float sgn = T::back ? -1.f : 1.f;
  const float z = q < 2 ? sgn : 0.f;  // rows 6 and 7 of the second tile are padding
  float a0[6], a1[6];
#pragma unroll
  for (int cp = 0; cp < 3; ++cp) {
    const float w0r = st.w0[cp].x, w0i = T::back ? -st.w0[cp].y : st.w0[cp].y;
    const float w2r = st.w2[cp].x, w2i = T::back ? -st.w2[cp].y : st.w2[cp].y;
    a0[2 * cp] = sgn * (imrow ? w0i : w0r);
    a0[2 * cp + 1] = sgn * (imrow ? w0r : -w0i);
    a1[2 * cp] = z * (imrow ? w2i : w2r);
    a1[2 * cp + 1] = z * (imrow ? w2r : -w2i);
  }
#pragma unroll
  for (int g = 0; g < kMfmaGroups; ++g) {
    const float nu = __uint_as_float(st.rec[g].w);
    const Vec3<float> h = VecF16::halves(st.rec[g]);
    const float bv[6] = {h.c[0].re * nu, h.c[0].im * nu, h.c[1].re * nu, h.c[1].im * nu, h.c[2].re * nu,
                         h.c[2].im * nu};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      acc[g][0] = __builtin_amdgcn_mfma_f32_4x4x1f32(a0[k], bv[k], acc[g][0], 0, 0, 0);
      acc[g][1] = __builtin_amdgcn_mfma_f32_4x4x1f32(a1[k], bv[k], acc[g][1], 0, 0, 0);
    }
  }
}

// The 16 terms, software-pipelined: the loads of term K+1 are issued before the
// products of term K.
template <int K>
__device__ __forceinline__ void mfma_terms(const DslashArgs& A, int i, const Site& s, int q,
                                           const int (&col)[kMfmaGroups], const void* const (&in)[kMfmaGroups],
                                           MfmaStage (&st)[2], mfma_v4 (&acc)[kMfmaGroups][2]) {
  if constexpr (K + 1 < 16) mfma_load<K + 1>(A, i, s, q, col, in, st[(K + 1) & 1]);
  mfma_compute<K>(q, st[K & 1], acc);
  if constexpr (K + 1 < 16) mfma_terms<K + 1>(A, i, s, q, col, in, st, acc);
}

// EPI_PLAIN / EPI_NORM (OutT = VecF16) and EPI_UPDATE (OutT = the FP32 residual tier).
template <class OutT, int EPI>
__global__ void __launch_bounds__(kBlock) dslash_mfma_kernel(const DslashArgs A) {
  int lin = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  if (A.reverse) lin = (int)gridDim.x - 1 - lin;
  int tile, sblk;
  if (A.sgroup <= 0) {
    tile = lin % A.ntiles;
    sblk = lin / A.ntiles;
  } else {
    const int per = A.sgroup * A.ntiles;
    const int grp = lin / per, w = lin % per;
    const int gsz = min(A.sgroup, A.nblk - grp * A.sgroup);
    tile = w / gsz;
    sblk = grp * A.sgroup + w % gsz;
  }
  const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int b = lane >> 2, q = lane & 3;
  const int half = A.g.half;
  const int c0 = tile * kMfmaCols;
  // the block leaves when none of its columns takes part (uniform: every lane checks them all)
  bool any = false;
  for (int c = c0; c < c0 + kMfmaCols; ++c) any |= col_on(A, c);
  if (!any) return;
  int col[kMfmaGroups];
  bool on[kMfmaGroups];
  const void* in[kMfmaGroups];
#pragma unroll
  for (int g = 0; g < kMfmaGroups; ++g) {
    const int c = c0 + 4 * g + q;
    on[g] = col_on(A, c);
    col[g] = c < A.ncol ? c : A.ncol - 1;  // in-bounds column for the unconditional loads
    in[g] = (on[g] && A.in_sel) ? pick_new(A, A.in, A.in_alt, c) : A.in;
  }
  [[maybe_unused]] double part[kMfmaGroups];
#pragma unroll
  for (int g = 0; g < kMfmaGroups; ++g) part[g] = 0;

#pragma unroll 1
  for (int sg = 0; sg < kBlock / 64; ++sg) {
    const int i_raw = sblk * kBlock + wave * 64 + sg * 16 + b;
    const bool valid = i_raw < half;
    const int i = valid ? i_raw : half - 1;  // lanes past the end compute a copy of the last site
    const Site s = decode(A.g, i, A.out_parity);
    mfma_v4 acc[kMfmaGroups][2];
#pragma unroll
    for (int g = 0; g < kMfmaGroups; ++g) acc[g][0] = acc[g][1] = (mfma_v4){0.f, 0.f, 0.f, 0.f};
    MfmaStage st[2];
    mfma_load<0>(A, i, s, q, col, in, st[0]);
    mfma_terms<0>(A, i, s, q, col, in, st, acc);
#pragma unroll
    for (int g = 0; g < kMfmaGroups; ++g) {
      if (!(valid && on[g])) continue;
      const int c = c0 + 4 * g + q;
      Vec3<float> o;
      o.c[0].re = acc[g][0][0];
      o.c[0].im = acc[g][0][1];
      o.c[1].re = acc[g][0][2];
      o.c[1].im = acc[g][0][3];
      o.c[2].re = acc[g][1][0];
      o.c[2].im = acc[g][1][1];
      if constexpr (EPI == EPI_PLAIN) {
        VecF16::store(A.out, half, c, i, o);
      } else if constexpr (EPI == EPI_NORM) {
        part[g] += norm2_d(VecF16::store(A.out, half, c, i, o));
      } else {
        // Ap = a p - D t; r -= alpha Ap; x_s += alpha p (FP32 segment accumulator)
        const ColState& S = A.st[c];
        const void* pb = A.y_sel ? pick_new(A, A.y, A.y_alt, c) : A.y;
        const Vec3<float> y = VecF16::load(pb, half, c, i);
        const float a = (float)S.a;
        Vec3<float> ap;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          ap.c[k].re = fmaR(a, y.c[k].re, -o.c[k].re);
          ap.c[k].im = fmaR(a, y.c[k].im, -o.c[k].im);
        }
        Vec3<float> rv = OutT::load(A.r, half, c, i);
        const float al = (float)S.alpha;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          rv.c[k].re = fmaR(-al, ap.c[k].re, rv.c[k].re);
          rv.c[k].im = fmaR(-al, ap.c[k].im, rv.c[k].im);
        }
        part[g] += norm2_d(OutT::store(A.r, half, c, i, rv));
        Vec3<float> x = VecF32::load(A.x, half, c, i);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          x.c[k].re = fmaR(al, y.c[k].re, x.c[k].re);
          x.c[k].im = fmaR(al, y.c[k].im, x.c[k].im);
        }
        VecF32::store(A.x, half, c, i, x);
      }
    }
  }

  if constexpr (EPI != EPI_PLAIN) {
    // per column: over the 16 sites of a wave (lanes of equal q), then the 4 waves in order
    __shared__ double sh[kMfmaCols][kBlock / 64];
#pragma unroll
    for (int g = 0; g < kMfmaGroups; ++g) {
      double d = part[g];
#pragma unroll
      for (int o = 4; o < 64; o <<= 1) d += __shfl_xor(d, o, 64);
      if (b == 0) sh[4 * g + q][wave] = d;
    }
    __syncthreads();
    if (tid < kMfmaCols && col_on(A, c0 + tid)) {
      double tot = 0;
#pragma unroll
      for (int w = 0; w < kBlock / 64; ++w) tot += sh[tid][w];
      A.partials[(size_t)(c0 + tid) * A.nblk + sblk] = tot;
    }
  }
}

template <class OutT, int EPI>
int go_mfma(const DslashArgs& a0, int order, hipStream_t s) {
  if (a0.apa) return ASQ_EINVAL;  // alpha comes from the column state here
  DslashArgs a = a0;
  a.ntiles = (a.ncol + kMfmaCols - 1) / kMfmaCols;
  a.sgroup = order_group(order, a.nblk);
  const long nb = (long)a.nblk * a.ntiles;
  if (nb <= 0) return ASQ_OK;
  if (nb >= (1L << 31)) return ASQ_EINVAL;
  dslash_mfma_kernel<OutT, EPI><<<(unsigned)nb, kBlock, 0, s>>>(a);
  return hipGetLastError() == hipSuccess ? ASQ_OK : ASQ_EHIP;
}

// PLAIN and NORM write FP16 records; UPDATE takes the FP32 residual tier.
inline int pick_mfma(int epi, int rtile, const DslashArgs& a, hipStream_t s) {
  const int ord = rtile_order(rtile);
  if (epi == EPI_PLAIN) return go_mfma<VecF16, EPI_PLAIN>(a, ord, s);
  if (epi == EPI_NORM) return go_mfma<VecF16, EPI_NORM>(a, ord, s);
  if (epi == EPI_UPDATE) return go_mfma<VecF32, EPI_UPDATE>(a, ord, s);
  return ASQ_EINVAL;
}

}  // namespace
}  // namespace asq
