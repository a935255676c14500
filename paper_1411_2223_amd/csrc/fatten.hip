// fatten.hip -- asqtad fat and long links from thin links, in FP64.
//
// The paper's lattices are MILC asqtad ensembles (CG benchmark, "GTX Titan
// Black" section); it gives no smearing formula, so the standard asqtad action
// is used.  For a direction mu, with nu, rho, sigma signed directions on
// pairwise different axes, none on mu's, and the staple map
//
//   T_d(X)(y) = W_d(y) X(y + d) W_d(y + mu)^dag,   W_d(y) = the thin link from y to y + d
//             (U_a(y) for d = +a, U_a(y - a)^dag for d = -a),
//
// the fat link is evaluated as nested staples
//
//   F_mu(x) = c1 U_mu(x) + sum_nu T_nu( c3 U_mu + cL T_nu(U_mu)
//                                       + sum_rho T_rho( c5 U_mu + c7 sum_sigma T_sigma(U_mu) ) )(x)
//
// which expands to the one-link, 6 three-staple, 24 five-staple, 48
// seven-staple and 6 Lepage paths, and the long link is
// L_mu(x) = cN U_mu(x) U_mu(x+mu) U_mu(x+2mu).  Coefficients: c1 = 5/8,
// c3 = 1/(16 u0^2), c5 = 1/(64 u0^4), c7 = 1/(384 u0^6), cL = -1/(16 u0^4),
// cN = -1/(24 u0^2); u0 is the tadpole factor.  Links are periodic in every
// direction (the time-boundary sign is applied when the links are imported).
//
// Three launches on the caller's stream:
//   1. a site-fastest copy of the thin links, written into the long-link output
//      (used as scratch, so the call needs no workspace);
//   2. the fat links: a block covers 64 sites (lane = site) for one mu, so mu is
//      uniform and the direction loops do not diverge, and every link load is a
//      coalesced 1 KB row; the four waves split the staple sums and meet in LDS;
//      nothing else is staged in global memory (staples are rebuilt from thin
//      links, which come from L2);
//   3. the long links from the canonical thin links, overwriting the copy.
// Per (site, mu) the fat link takes 12 x (4 + 2 x 4) + 6 x 2 = 156 SU(3)
// products (the two orders of a {nu, rho} group share their core) and the
// long link 2.
#include <math.h>

#include <map>
#include <mutex>

#include "asq_reduce.h"

namespace asq {
namespace {

using M3 = Mat3<double>;

struct FattenArgs {
  int d[4];
  long V;
  const double2* thin;  // canonical [V][4][9] complex
  const double2* soa;   // the same links site-fastest, [4][9][V] complex
  double2* fat;
  double2* lng;
  double c1, c3, c5, c7, cL, cN;
};

__device__ __forceinline__ long lex_of(const int d[4], const int c[4]) {
  return c[0] + (long)d[0] * (c[1] + (long)d[1] * (c[2] + (long)d[2] * c[3]));
}

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// U_mu at site c from the site-fastest copy: lanes on consecutive sites read
// consecutive 16-byte words.
__device__ __forceinline__ M3 load(const FattenArgs& A, const int c[4], int mu) {
  const double2* q = A.soa + (size_t)mu * 9 * A.V + lex_of(A.d, c);
  M3 U;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const double2 v = q[(size_t)k * A.V];
    U.e[k / 3][k % 3].re = v.x;
    U.e[k / 3][k % 3].im = v.y;
  }
  return U;
}

// U_mu at site c from the canonical array.
__device__ __forceinline__ M3 load_canonical(const FattenArgs& A, long lex, int mu) {
  const double2* q = A.thin + (lex * 4 + mu) * 9;
  M3 U;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const double2 v = q[k];
    U.e[k / 3][k % 3].re = v.x;
    U.e[k / 3][k % 3].im = v.y;
  }
  return U;
}

// C = A B, C = A^dag B, C += s A B^dag and C += s A B (s real), C = s X
__device__ __forceinline__ M3 mul_nn(const M3& A, const M3& B) {
  M3 C;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      cx<double> v{0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 3; ++k) cmac(v, A.e[a][k], B.e[k][b]);
      C.e[a][b] = v;
    }
  return C;
}

__device__ __forceinline__ M3 mul_dn(const M3& A, const M3& B) {
  M3 C;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      cx<double> v{0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 3; ++k) cmac_conj(v, A.e[k][a], B.e[k][b]);
      C.e[a][b] = v;
    }
  return C;
}

__device__ __forceinline__ void acc_nd(M3& C, double s, const M3& A, const M3& B) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      cx<double> v{0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 3; ++k) cmac_conj(v, B.e[b][k], A.e[a][k]);  // A[a][k] conj(B[b][k])
      C.e[a][b].re = fmaR(s, v.re, C.e[a][b].re);
      C.e[a][b].im = fmaR(s, v.im, C.e[a][b].im);
    }
}

__device__ __forceinline__ void acc_nn(M3& C, double s, const M3& A, const M3& B) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      cx<double> v{0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 3; ++k) cmac(v, A.e[a][k], B.e[k][b]);
      C.e[a][b].re = fmaR(s, v.re, C.e[a][b].re);
      C.e[a][b].im = fmaR(s, v.im, C.e[a][b].im);
    }
}

__device__ __forceinline__ M3 scaled(double s, const M3& X) {
  M3 C;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      C.e[a][b].re = s * X.e[a][b].re;
      C.e[a][b].im = s * X.e[a][b].im;
    }
  return C;
}

// C += s T_d(X)(y), with d = +(ax) or -(ax) given by (ax, neg) and X the matrix at y + d.
__device__ __forceinline__ void acc_staple(const FattenArgs& A, M3& C, double s, const int y[4], int mu, int ax,
                                           bool neg, const M3& X) {
  int w[4] = {y[0], y[1], y[2], y[3]};   // the site holding the first link
  if (neg) w[ax] = wrap(w[ax] - 1, A.d[ax]);
  const M3 P = neg ? mul_dn(load(A, w, ax), X) : mul_nn(load(A, w, ax), X);
  w[mu] = wrap(w[mu] + 1, A.d[mu]);       // the closing link starts at y + mu (or y + mu - d)
  if (neg) acc_nn(C, s, P, load(A, w, ax));
  else acc_nd(C, s, P, load(A, w, ax));
}

__device__ __forceinline__ void step(int c[4], int ax, bool neg, const int d[4]) {
  c[ax] = wrap(c[ax] + (neg ? -1 : 1), d[ax]);
}

// A block covers 64 consecutive sites (one per lane) for one mu.  The 24
// signed (nu, rho) pairs form 12 unordered groups {nu, rho}; both orders share
// the core c5 U_mu + c7 sum_sigma T_sigma(U_mu) at z = x + nu + rho (sigma runs
// over the one axis left), so a group costs one core and two chains
// T_nu(T_rho(core))(x) and T_rho(T_nu(core))(x).  Wave w takes the three groups
// whose signs are (w & 1, w >> 1), one per axis pair.  The once-per-direction
// term T_d(c3 U_mu + cL T_d(U_mu))(x) rides on a chain whose outer direction is
// d, in a wave fixed per d.  Each wave sums into its own LDS slice; the slices
// and c1 U_mu(x) are then added in a fixed order, so the result does not
// depend on scheduling.
constexpr int kFatSites = 64;

__global__ void __launch_bounds__(256) fatten_kernel(const FattenArgs A) {
  __shared__ double2 part[4][9][kFatSites];
  __shared__ double2 cores[4][9][kFatSites];  // each wave's current core, kept out of registers
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // the four directions of a site range are neighbouring blocks (same XCD, same
  // L2): they read the same neighbour links and write the same output lines
  const int lin = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int mu = lin & 3;
  const long site = (long)(lin >> 2) * kFatSites + lane;
  const bool valid = site < A.V;
  const long lex = valid ? site : A.V - 1;  // lanes past the end compute a copy of the last site
  int x[4];
  {
    long r = lex;
    x[0] = (int)(r % A.d[0]);
    r /= A.d[0];
    x[1] = (int)(r % A.d[1]);
    r /= A.d[1];
    x[2] = (int)(r % A.d[2]);
    x[3] = (int)(r / A.d[2]);
  }
  int others[3];
  for (int a = 0, n = 0; a < 4; ++a)
    if (a != mu) others[n++] = a;
  // the wave carrying the once-per-direction term of others[i] with sign bit g
  // (+a -> 2, -a -> 1, +b -> 0, -b -> 3, +c -> 1, -c -> 2): each has a chain
  // with that outer direction
  const int extra_wave[3][2] = {{2, 1}, {0, 3}, {1, 2}};
  const bool sgn1 = wave & 1, sgn2 = wave >> 1;

  bool first = true;
#pragma unroll 1
  for (int p = 0; p < 3; ++p) {
    // axis pair p: (a, b), (a, c), (b, c) with a, b, c = others[0..2]
    const int i1 = p == 2 ? 1 : 0, i2 = p == 0 ? 1 : 2;
    const int ax1 = others[i1], ax2 = others[i2];
    const int sax = 6 - mu - ax1 - ax2;
    int z[4] = {x[0], x[1], x[2], x[3]};
    step(z, ax1, sgn1, A.d);
    step(z, ax2, sgn2, A.d);
    M3 core = scaled(A.c5, load(A, z, mu));
#pragma unroll 1
    for (int sn = 0; sn < 2; ++sn) {
      int z2[4] = {z[0], z[1], z[2], z[3]};
      step(z2, sax, sn, A.d);
      acc_staple(A, core, A.c7, z, mu, sax, sn, load(A, z2, mu));
    }
#pragma unroll
    for (int k = 0; k < 9; ++k)
      cores[wave][k][lane] = make_double2(core.e[k / 3][k % 3].re, core.e[k / 3][k % 3].im);
#pragma unroll 1
    for (int ch = 0; ch < 2; ++ch) {
      // reread through a volatile pointer, so the core does not stay live in registers
      const volatile double2* cq = &cores[wave][0][lane];
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        core.e[k / 3][k % 3].re = cq[k * kFatSites].x;
        core.e[k / 3][k % 3].im = cq[k * kFatSites].y;
      }
      // chain ch: outer direction (oax, oneg), inner direction (iax, ineg)
      const int oax = ch ? ax2 : ax1, iax = ch ? ax1 : ax2;
      const bool oneg = ch ? sgn2 : sgn1, ineg = ch ? sgn1 : sgn2;
      const int oi = ch ? i2 : i1;
      int y[4] = {x[0], x[1], x[2], x[3]};
      step(y, oax, oneg, A.d);
      M3 v = scaled(0.0, core);
      acc_staple(A, v, 1.0, y, mu, iax, ineg, core);
      // the once-per-direction term goes with the first chain of its wave
      // whose outer direction it is (axis pair 0 or 1 for a, 0 or 2 for b, 1
      // or 2 for c: the first such pair in the loop)
      const bool first_pair = oi == 0 ? p == 0 : (oi == 1 ? p == 0 : p == 1);
      if (wave == extra_wave[oi][oneg] && first_pair) {
        int y2[4] = {y[0], y[1], y[2], y[3]};
        step(y2, oax, oneg, A.d);
        acc_staple(A, v, A.cL, y, mu, oax, oneg, load(A, y2, mu));  // Lepage
        const M3 Uy = load(A, y, mu);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b) {
            v.e[a][b].re = fmaR(A.c3, Uy.e[a][b].re, v.e[a][b].re);
            v.e[a][b].im = fmaR(A.c3, Uy.e[a][b].im, v.e[a][b].im);
          }
      }
      M3 out = scaled(0.0, v);
      acc_staple(A, out, 1.0, x, mu, oax, oneg, v);
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        double2 o = make_double2(out.e[k / 3][k % 3].re, out.e[k / 3][k % 3].im);
        if (!first) {
          const double2 q = part[wave][k][lane];
          o.x += q.x;
          o.y += q.y;
        }
        part[wave][k][lane] = o;
      }
      first = false;
    }
  }
  __syncthreads();

  if (wave < 3 && valid) {
    // waves 0-2 finish three of the nine entries each
    const double2* q = A.soa + (size_t)mu * 9 * A.V + lex;
    double2* qf = A.fat + (lex * 4 + mu) * 9;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int k = wave * 3 + j;
      const double2 u = q[(size_t)k * A.V];
      double re = A.c1 * u.x, im = A.c1 * u.y;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        re += part[w][k][lane].x;
        im += part[w][k][lane].y;
      }
      qf[k] = make_double2(re, im);
    }
  }
}

// Canonical thin links -> the site-fastest copy.  A block moves 64 sites: it
// reads their 36 complex entries each as one contiguous 36 KB run and writes 36
// rows of 64 entries, both coalesced, through LDS.
__global__ void __launch_bounds__(256) thin_soa_kernel(const double2* __restrict__ thin, double2* __restrict__ soa,
                                                       long V) {
  __shared__ double2 tile[36][kFatSites + 1];
  const long s0 = (long)blockIdx.x * kFatSites;
  const int n = (int)(V - s0 < kFatSites ? V - s0 : kFatSites);
  for (int e = threadIdx.x; e < n * 36; e += blockDim.x) tile[e % 36][e / 36] = thin[s0 * 36 + e];
  __syncthreads();
  for (int e = threadIdx.x; e < 36 * kFatSites; e += blockDim.x) {
    const int j = e / kFatSites, i = e % kFatSites;
    if (i < n) soa[(size_t)j * V + s0 + i] = tile[j][i];
  }
}

// L_mu(x) = cN U_mu(x) U_mu(x+mu) U_mu(x+2mu) from the canonical thin links
// (the site-fastest copy occupies the output until this kernel runs).
__global__ void __launch_bounds__(256) long_link_kernel(const FattenArgs A) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= A.V * 4) return;
  const long lex = gid >> 2;
  const int mu = (int)(gid & 3);
  int x[4];
  {
    long r = lex;
    x[0] = (int)(r % A.d[0]);
    r /= A.d[0];
    x[1] = (int)(r % A.d[1]);
    r /= A.d[1];
    x[2] = (int)(r % A.d[2]);
    x[3] = (int)(r / A.d[2]);
  }
  int x1[4] = {x[0], x[1], x[2], x[3]};
  step(x1, mu, false, A.d);
  int x2[4] = {x1[0], x1[1], x1[2], x1[3]};
  step(x2, mu, false, A.d);
  const M3 Ux = load_canonical(A, lex, mu);
  M3 L = scaled(0.0, Ux);
  acc_nn(L, A.cN, mul_nn(Ux, load_canonical(A, lex_of(A.d, x1), mu)), load_canonical(A, lex_of(A.d, x2), mu));
  double2* ql = A.lng + (lex * 4 + mu) * 9;
#pragma unroll
  for (int k = 0; k < 9; ++k) ql[k] = make_double2(L.e[k / 3][k % 3].re, L.e[k / 3][k % 3].im);
}

// Mean plaquette, first pass: one thread per site sums (1/3) Re tr over its six
// planes in a fixed order, then one partial per block (block_sum's tree).
// Re tr[U_mu(x) U_nu(x+mu) (U_nu(x) U_mu(x+nu))^dag] is the sum over the entries
// of M1 conj(M2), so the last product is not formed.
__global__ void __launch_bounds__(kBlock) plaquette_kernel(const FattenArgs A, double* partials) {
  const long lex = (long)blockIdx.x * kBlock + threadIdx.x;
  double v = 0;
  if (lex < A.V) {
    int x[4];
    long r = lex;
    x[0] = (int)(r % A.d[0]);
    r /= A.d[0];
    x[1] = (int)(r % A.d[1]);
    r /= A.d[1];
    x[2] = (int)(r % A.d[2]);
    x[3] = (int)(r / A.d[2]);
    for (int mu = 0; mu < 4; ++mu)
      for (int nu = mu + 1; nu < 4; ++nu) {
        int xm[4] = {x[0], x[1], x[2], x[3]}, xn[4] = {x[0], x[1], x[2], x[3]};
        step(xm, mu, false, A.d);
        step(xn, nu, false, A.d);
        const M3 m1 = mul_nn(load_canonical(A, lex, mu), load_canonical(A, lex_of(A.d, xm), nu));
        const M3 m2 = mul_nn(load_canonical(A, lex, nu), load_canonical(A, lex_of(A.d, xn), mu));
        double t = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b) {
            t = fmaR(m1.e[a][b].re, m2.e[a][b].re, t);
            t = fmaR(m1.e[a][b].im, m2.e[a][b].im, t);
          }
        v += t / 3.0;
      }
  }
  __shared__ double sh[kBlock / 64];
  const double tot = block_sum(v, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// Second pass: the partials in order, divided by the number of plaquettes.
__global__ void __launch_bounds__(kBlock) plaquette_final(double* partials, int n, double inv_count) {
  const double v = strided_sum(partials, n);
  __shared__ double sh[kBlock / 64];
  const double tot = block_sum(v, sh);
  if (threadIdx.x == 0) partials[n] = tot * inv_count;
}

bool valid_extents(const int dims[4]) {
  if (!dims) return false;
  for (int mu = 0; mu < 4; ++mu)
    if (dims[mu] < 4 || (dims[mu] & 1) || dims[mu] > (1 << 14)) return false;
  const long V = (long)dims[0] * dims[1] * dims[2] * dims[3];
  return V * 36 / 256 + 1 < (1L << 31);
}

bool overlaps(const void* a, const void* b, size_t n) {
  const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
  return pa < pb + n && pb < pa + n;
}

}  // namespace
}  // namespace asq

using namespace asq;

extern "C" int asqtad_build_links(const int dims[4], const double* thin_dev, double u0, double* fat_dev,
                                  double* long_dev, void* hip_stream) {
  if (!dims || !thin_dev || !fat_dev || !long_dev) {
    set_last_error("asqtad_build_links: null pointer");
    return ASQ_EINVAL;
  }
  if (!valid_extents(dims)) {
    set_last_error("asqtad_build_links: extents must be even and >= 4, the lattice not too large");
    return ASQ_EINVAL;
  }
  const long V = (long)dims[0] * dims[1] * dims[2] * dims[3];
  if (!(u0 > 0) || !isfinite(u0)) {
    set_last_error("asqtad_build_links: u0 must be positive and finite");
    return ASQ_EINVAL;
  }
  if (((uintptr_t)thin_dev & 15) || ((uintptr_t)fat_dev & 15) || ((uintptr_t)long_dev & 15)) {
    set_last_error("asqtad_build_links: link arrays must be 16-byte aligned");
    return ASQ_EINVAL;
  }
  const size_t bytes = (size_t)V * 4 * 18 * sizeof(double);
  if (overlaps(thin_dev, fat_dev, bytes) || overlaps(thin_dev, long_dev, bytes) ||
      overlaps(fat_dev, long_dev, bytes)) {
    set_last_error("asqtad_build_links: thin, fat and long arrays must not overlap");
    return ASQ_EINVAL;
  }
  FattenArgs a;
  for (int mu = 0; mu < 4; ++mu) a.d[mu] = dims[mu];
  a.V = V;
  a.thin = (const double2*)thin_dev;
  a.fat = (double2*)fat_dev;
  a.lng = (double2*)long_dev;
  const double u2 = u0 * u0, u4 = u2 * u2, u6 = u4 * u2;
  a.c1 = 5.0 / 8.0;
  a.c3 = 1.0 / (16.0 * u2);
  a.c5 = 1.0 / (64.0 * u4);
  a.c7 = 1.0 / (384.0 * u6);
  a.cL = -1.0 / (16.0 * u4);
  a.cN = -1.0 / (24.0 * u2);
  // The long-link output holds the site-fastest copy of the thin links while the
  // fat links are built; the long links overwrite it last.
  a.soa = (const double2*)long_dev;
  hipStream_t s = (hipStream_t)hip_stream;
  thin_soa_kernel<<<(unsigned)((V + kFatSites - 1) / kFatSites), 256, 0, s>>>(a.thin, (double2*)long_dev, V);
  ASQ_HIP_TRY(hipGetLastError());
  fatten_kernel<<<(unsigned)(4 * ((V + kFatSites - 1) / kFatSites)), 256, 0, s>>>(a);
  ASQ_HIP_TRY(hipGetLastError());
  long_link_kernel<<<(unsigned)((V * 4 + 255) / 256), 256, 0, s>>>(a);
  ASQ_HIP_TRY(hipGetLastError());
  return ASQ_OK;
}

extern "C" size_t asqtad_plaquette_workspace_bytes(const int dims[4]) {
  if (!valid_extents(dims)) return 0;
  const long V = (long)dims[0] * dims[1] * dims[2] * dims[3];
  return align_up((size_t)((V + kBlock - 1) / kBlock + 1) * sizeof(double), 256);
}

extern "C" int asqtad_plaquette(const int dims[4], const double* thin_dev, void* work_dev, size_t work_bytes,
                                double* plaq, void* hip_stream) {
  if (!thin_dev || !work_dev || !plaq || !valid_extents(dims)) {
    set_last_error("asqtad_plaquette: null pointer or invalid extents (even, >= 4)");
    return ASQ_EINVAL;
  }
  if (((uintptr_t)thin_dev & 15) || ((uintptr_t)work_dev & 7)) {
    set_last_error("asqtad_plaquette: thin links 16-byte and workspace 8-byte aligned");
    return ASQ_EINVAL;
  }
  if (work_bytes < asqtad_plaquette_workspace_bytes(dims)) {
    set_last_error("asqtad_plaquette: workspace smaller than asqtad_plaquette_workspace_bytes()");
    return ASQ_ENOMEM;
  }
  const size_t thin_bytes = (size_t)dims[0] * dims[1] * dims[2] * dims[3] * 4 * 18 * sizeof(double);
  const uintptr_t t0 = (uintptr_t)thin_dev, w0 = (uintptr_t)work_dev;
  if (t0 < w0 + work_bytes && w0 < t0 + thin_bytes) {
    set_last_error("asqtad_plaquette: workspace must not overlap the thin links");
    return ASQ_EINVAL;
  }
  FattenArgs a{};
  for (int mu = 0; mu < 4; ++mu) a.d[mu] = dims[mu];
  a.V = (long)dims[0] * dims[1] * dims[2] * dims[3];
  a.thin = (const double2*)thin_dev;
  const int nb = (int)((a.V + kBlock - 1) / kBlock);
  double* partials = (double*)work_dev;
  hipStream_t s = (hipStream_t)hip_stream;
  plaquette_kernel<<<(unsigned)nb, kBlock, 0, s>>>(a, partials);
  ASQ_HIP_TRY(hipGetLastError());
  plaquette_final<<<1, kBlock, 0, s>>>(partials, nb, 1.0 / (6.0 * (double)a.V));
  ASQ_HIP_TRY(hipGetLastError());
  ASQ_HIP_TRY(hipMemcpyAsync(plaq, partials + nb, sizeof(double), hipMemcpyDeviceToHost, s));
  ASQ_HIP_TRY(hipStreamSynchronize(s));
  return ASQ_OK;
}

// ---- the same without any allocation --------------------------------------
// For callers that cannot allocate (code under graph capture, tight serving
// loops): the partial sums live in a fixed device array of the library, one per
// GPU, found once per device with hipGetSymbolAddress.  Every call on a GPU
// shares that GPU's array, so calls that overlap on one GPU race.
namespace asq {
namespace {

constexpr size_t kNoAllocScratchDoubles = 262144;  // 2 MiB: V up to 67 108 608 sites
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_ptr;  // device -> address of its copy of `scratch`

// The device address of this device's scratch array (looked up once per device,
// with the device current).  nullptr and a message on failure.
double* scratch_ptr() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
  g_scratch_ptr[dev] = (double*)p;
  return (double*)p;
}

// The final pass writes P straight to the caller's device output.
__global__ void __launch_bounds__(kBlock) plaquette_final_to(const double* partials, int n, double inv_count,
                                                             double* out) {
  __shared__ double sh[kBlock / 64];
  const double tot = block_sum(strided_sum(partials, n), sh);
  if (threadIdx.x == 0) *out = tot * inv_count;
}

}  // namespace
}  // namespace asq

extern "C" int asqtad_plaquette_noalloc(const int dims[4], const double* thin_dev, double* plaq_dev,
                                        void* hip_stream) {
  if (!thin_dev || !plaq_dev || !valid_extents(dims)) {
    set_last_error("asqtad_plaquette_noalloc: null pointer or invalid extents (even, >= 4)");
    return ASQ_EINVAL;
  }
  if (((uintptr_t)thin_dev & 15) || ((uintptr_t)plaq_dev & 7)) {
    set_last_error("asqtad_plaquette_noalloc: thin links 16-byte and the output 8-byte aligned");
    return ASQ_EINVAL;
  }
  const long V = (long)dims[0] * dims[1] * dims[2] * dims[3];
  const long nb = (V + kBlock - 1) / kBlock;
  if ((size_t)nb > kNoAllocScratchDoubles) {
    set_last_error("asqtad_plaquette_noalloc: lattice too large for the fixed scratch (at most 67108608 sites)");
    return ASQ_ENOMEM;
  }
  const size_t thin_bytes = (size_t)V * 4 * 18 * sizeof(double);
  const uintptr_t t0 = (uintptr_t)thin_dev, o0 = (uintptr_t)plaq_dev;
  if (o0 < t0 + thin_bytes && t0 < o0 + sizeof(double)) {
    set_last_error("asqtad_plaquette_noalloc: the output must not overlap the thin links");
    return ASQ_EINVAL;
  }
  double* partials = scratch_ptr();
  if (!partials) {
    set_last_error("asqtad_plaquette_noalloc: hipGetSymbolAddress of the scratch array failed");
    return ASQ_EHIP;
  }
  FattenArgs a{};
  for (int mu = 0; mu < 4; ++mu) a.d[mu] = dims[mu];
  a.V = V;
  a.thin = (const double2*)thin_dev;
  hipStream_t s = (hipStream_t)hip_stream;
  // every partial the final pass reads is written by the first pass: nothing to clear
  plaquette_kernel<<<(unsigned)nb, kBlock, 0, s>>>(a, partials);
  ASQ_HIP_TRY(hipGetLastError());
  plaquette_final_to<<<1, kBlock, 0, s>>>(partials, (int)nb, 1.0 / (6.0 * (double)V), plaq_dev);
  ASQ_HIP_TRY(hipGetLastError());
  return ASQ_OK;
}
