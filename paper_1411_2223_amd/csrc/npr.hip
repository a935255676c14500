// npr.hip -- the one-colour four-fermion operator of the paper's NPR code
// (section "GTX Titan Black", Eq. (1)), in FP64 as the paper runs it.
//
// For every hypercube z (corners z_A = 2z + A, A a 4-bit mask) and operator
// I = (S1, F1, S2, F2):
//   V[a1][a2][a3][a4] = sum_{A,B,C,D} M1_AB M2_CD eps(z_A) eps(z_C)
//       (G1(z_A)^dag U_AD G4(z_D))_{a1 a4} (G3(z_C)^dag U_CB G2(z_B))_{a3 a2}
// M = (gamma_S (x) xi_F)bar, the spin-taste matrix (1/4) Tr[gamma_A^dag gamma_S
// gamma_B gamma_F^dag]; eps = (-1)^(x+y+z+t); U_AD the link product averaged
// over every shortest path from z_A to z_D; G_f the propagators (each chi by a
// propagator, each chibar by its staggered conjugate).  M has one nonzero per
// row, at B = A ^ S ^ F, so each operator is 16 x 16 terms (A, C).
//
// One workgroup per hypercube:
//   1. the 16 corners' propagators to LDS, and the 64 single steps of the
//      hypercube (from corner A along mu: the link U_mu(z_A) if bit mu of A is
//      clear, else the conjugate of the link arriving at z_A);
//   2. the 256 averages U_AD by the first step of each path, in rounds of
//      growing distance |A ^ D| (U_AD = (1/d) sum_mu step(A, mu) U_{A^mu, D});
//      the pairs are dealt to threads in order of distance, so the lanes of a
//      wave share a round;
//   3. X_AD = G1(A)^dag U_AD G4(D) and Y_AD = G3(A)^dag U_AD G2(D) to LDS;
//   4. the contraction: a lane owns one operator and one corner A, sums the 16
//      terms D and accumulates all 81 outputs; the 16 corners' partial sums of
//      an operator are added across lanes by halving exchanges, after which
//      each lane stores the outputs it ended with.
#include <math.h>
#include <string.h>

#include <string>

#include "asq_internal.h"

namespace asq {
namespace {

constexpr int kNprThreads = 256;
constexpr int kNprOpsPerLaunch = 32;
constexpr int kNprOpsPerPass = 16;  // 4 per wave, each over the 16 lanes of its corners A
// a matrix per pair (A, D) at A * kRow + 9 D complex entries: one spare entry per
// row A puts the 16 rows A that a wave reads at once in different LDS banks
constexpr int kRow = 16 * 9 + 1;
constexpr int kPairMats = 16 * kRow;

// the 256 pairs (A, D), 16 A + D, in order of distance |A ^ D| (then A, then D)
struct PairOrder {
  unsigned char p[256];
};
constexpr int popcount4(int m) { return (m & 1) + (m >> 1 & 1) + (m >> 2 & 1) + (m >> 3 & 1); }
constexpr PairOrder make_pair_order() {
  PairOrder t{};
  int n = 0;
  for (int d = 0; d <= 4; ++d)
    for (int a = 0; a < 16; ++a)
      for (int b = 0; b < 16; ++b)
        if (popcount4(a ^ b) == d) t.p[n++] = (unsigned char)(16 * a + b);
  return t;
}
__constant__ PairOrder kPairOrder = make_pair_order();

struct NprOp {
  unsigned char p1, p2;  // S1 ^ F1, S2 ^ F2: B = A ^ p1, D = C ^ p2
  unsigned short neg1;   // bit A: M1_{A, A^p1} eps(z_A) = -1 (else +1)
  unsigned short neg2;   // bit C: M2_{C, C^p2} eps(z_C) = -1
};

struct NprArgs {
  int X, Y, Z, T;
  int hx, hy, hz;  // hypercubes per direction (x, y, z)
  const double2* thin;
  const double2* g[4];
  double2* out;     // [nop_total][nz][81]
  long nz;
  int op0;          // index of this launch's first operator in the output
  int nop;
  NprOp ops[kNprOpsPerLaunch];
};

typedef double2 c64;

__device__ __forceinline__ c64 cmul(c64 a, c64 b) {
  return make_double2(__builtin_fma(a.x, b.x, -a.y * b.y), __builtin_fma(a.x, b.y, a.y * b.x));
}
// acc + conj(a) b
__device__ __forceinline__ c64 cmac_cj(c64 acc, c64 a, c64 b) {
  acc.x = __builtin_fma(a.x, b.x, acc.x);
  acc.x = __builtin_fma(a.y, b.y, acc.x);
  acc.y = __builtin_fma(a.x, b.y, acc.y);
  acc.y = __builtin_fma(-a.y, b.x, acc.y);
  return acc;
}
__device__ __forceinline__ c64 cmac(c64 acc, c64 a, c64 b) {
  acc.x = __builtin_fma(a.x, b.x, acc.x);
  acc.x = __builtin_fma(-a.y, b.y, acc.x);
  acc.y = __builtin_fma(a.x, b.y, acc.y);
  acc.y = __builtin_fma(a.y, b.x, acc.y);
  return acc;
}

// c = a b (3 x 3, row-major)
__device__ __forceinline__ void m3mul(const c64* a, const c64* b, c64* c) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      c64 s = cmul(a[3 * i], b[j]);
      s = cmac(s, a[3 * i + 1], b[3 + j]);
      s = cmac(s, a[3 * i + 2], b[6 + j]);
      c[3 * i + j] = s;
    }
}
// c = a^dag b
__device__ __forceinline__ void m3mul_dag(const c64* a, const c64* b, c64* c) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      c64 s = make_double2(0.0, 0.0);
      s = cmac_cj(s, a[i], b[j]);
      s = cmac_cj(s, a[3 + i], b[3 + j]);
      s = cmac_cj(s, a[6 + i], b[6 + j]);
      c[3 * i + j] = s;
    }
}
// c = a b^dag
__device__ __forceinline__ void m3mul_bdag(const c64* a, const c64* b, c64* c) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      c64 s = make_double2(0.0, 0.0);
      s = cmac_cj(s, b[3 * j], a[3 * i]);
      s = cmac_cj(s, b[3 * j + 1], a[3 * i + 1]);
      s = cmac_cj(s, b[3 * j + 2], a[3 * i + 2]);
      c[3 * i + j] = s;
    }
}

__global__ void __launch_bounds__(kNprThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) npr_kernel(const NprArgs P) {
  // LDS: 74 240 bytes, reused between phases.
  //   phases 1-2: propagators [f][A][9] at 0, steps [A][mu][9] at 576, U (pair layout) at kPairMats
  //   phases 3-4: X (pair layout) at 0, Y (pair layout) at kPairMats
  __shared__ c64 lds[2 * kPairMats];
  c64* Gs = lds;
  c64* Ls = lds + 576;
  c64* Us = lds + kPairMats;
  c64* Xs = lds;
  c64* Ys = lds + kPairMats;

  const int tid = (int)threadIdx.x;
  const long z = (long)blockIdx.x;
  int zc[4];
  {
    long r = z;
    zc[0] = (int)(r % P.hx);
    r /= P.hx;
    zc[1] = (int)(r % P.hy);
    r /= P.hy;
    zc[2] = (int)(r % P.hz);
    zc[3] = (int)(r / P.hz);
  }
  auto lex = [&](int A) -> long {
    const long x = 2 * zc[0] + (A & 1), y = 2 * zc[1] + (A >> 1 & 1);
    const long zz = 2 * zc[2] + (A >> 2 & 1), t = 2 * zc[3] + (A >> 3 & 1);
    return x + P.X * (y + P.Y * (zz + P.Z * t));
  };
  // 1. propagators of the 16 corners (4 x 16 x 9 complex), and the 32 links inside
  //    the hypercube, each stored as the forward step from its lower corner and,
  //    conjugated, as the backward step from its upper corner
  for (int k = tid; k < 576; k += kNprThreads) {
    const int f = k / 144, A = (k / 9) % 16, e = k % 9;
    Gs[k] = P.g[f][lex(A) * 9 + e];
  }
  for (int k = tid; k < 288; k += kNprThreads) {
    const int j = k / 9, e = k % 9;
    const int mu = j >> 3, lo = j & 7;
    const int A = ((lo >> mu) << (mu + 1)) | (lo & ((1 << mu) - 1));  // bit mu clear
    const c64 v = P.thin[(lex(A) * 4 + mu) * 9 + e];
    Ls[(A * 4 + mu) * 9 + e] = v;
    Ls[((A | 1 << mu) * 4 + mu) * 9 + 3 * (e % 3) + e / 3] = make_double2(v.x, -v.y);
  }
  // 2. U_AD for the pair this thread owns, in rounds of growing distance
  const int pr = kPairOrder.p[tid];
  const int A = pr >> 4, D = pr & 15;
  const int d = __popc(A ^ D);
  c64* const umine = Us + A * kRow + 9 * D;
  c64 u[9];
  if (d == 0) {
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = make_double2(e % 4 == 0 ? 1.0 : 0.0, 0.0);
#pragma unroll
    for (int e = 0; e < 9; ++e) umine[e] = u[e];
  }
  __syncthreads();
  if (d == 1) {
    const c64* st = Ls + (A * 4 + (__ffs(A ^ D) - 1)) * 9;
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = st[e];
#pragma unroll
    for (int e = 0; e < 9; ++e) umine[e] = u[e];
  }
  for (int round = 2; round <= 4; ++round) {
    __syncthreads();
    if (d == round) {
      c64 acc[9];
#pragma unroll
      for (int e = 0; e < 9; ++e) acc[e] = make_double2(0.0, 0.0);
      int m = A ^ D;
      for (int q = 0; q < round; ++q) {
        const int mu = __ffs(m) - 1;
        m &= m - 1;
        c64 t[9];
        m3mul(Ls + (A * 4 + mu) * 9, Us + (A ^ 1 << mu) * kRow + 9 * D, t);
#pragma unroll
        for (int e = 0; e < 9; ++e) {
          acc[e].x += t[e].x;
          acc[e].y += t[e].y;
        }
      }
      const double inv = 1.0 / (double)round;
#pragma unroll
      for (int e = 0; e < 9; ++e) {
        u[e] = make_double2(acc[e].x * inv, acc[e].y * inv);
        umine[e] = u[e];
      }
    }
  }
  __syncthreads();
  // 3. the bilinears' colour matrices of the pair (A, D)
  c64 xm[9], ym[9];
  {
    c64 t[9];
    m3mul_dag(Gs + (0 * 16 + A) * 9, u, t);  // G1(A)^dag U_AD
    m3mul(t, Gs + (3 * 16 + D) * 9, xm);    // ... G4(D)
    m3mul_dag(Gs + (2 * 16 + A) * 9, u, t);  // G3(A)^dag U_AD
    m3mul(t, Gs + (1 * 16 + D) * 9, ym);    // ... G2(D)
  }
  __syncthreads();  // everyone is done with the propagators, steps and U in LDS
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    Xs[A * kRow + 9 * D + e] = xm[e];
    Ys[A * kRow + 9 * D + e] = ym[e];
  }
  __syncthreads();
  // 4. contraction.  Lane l of wave w takes operator 4 w + (l >> 4) of the pass
  //    and corner A = l & 15.  With C = D ^ p2 and B = A ^ p1 it sums, over D,
  //    sign * X_AD[a1][a4] Y_CB[a3][a2] into out[a1][a2][a3][a4], one a3 at a
  //    time (27 outputs).  The 16 lanes of an operator read 16 rows A of X and
  //    16 entries B of a row C of Y, each in its own LDS banks.
  const int lane = tid & 63, wv = tid >> 6;
  const int Ak = lane & 15;
  for (int pass = 0; pass * kNprOpsPerPass < P.nop; ++pass) {
    const int opl = pass * kNprOpsPerPass + 4 * wv + (lane >> 4);
    const bool act = opl < P.nop;
    NprOp o = {0, 0, 0, 0};
    if (act) o = P.ops[opl];
    const int B = Ak ^ o.p1;
    const double s1 = (o.neg1 >> Ak & 1) ? -1.0 : 1.0;
    const c64* xrow = Xs + Ak * kRow;
    double* const out = (double*)(P.out + ((size_t)(P.op0 + (act ? opl : 0)) * P.nz + z) * 81);
#pragma unroll 1
    for (int a3 = 0; a3 < 3; ++a3) {
      double v[54];  // [a1][a2][a4] as (re, im) pairs
#pragma unroll
      for (int k = 0; k < 54; ++k) v[k] = 0.0;
      if (act) {
        const c64* ybase = Ys + 9 * B + 3 * a3;
#pragma unroll 2
        for (int Dk = 0; Dk < 16; ++Dk) {
          const int C = Dk ^ o.p2;
          const double s = (o.neg2 >> C & 1) ? -s1 : s1;
          c64 xv[9], yv[3];
#pragma unroll
          for (int e = 0; e < 9; ++e) xv[e] = xrow[9 * Dk + e];  // X_AD[a1][a4]
#pragma unroll
          for (int e = 0; e < 3; ++e) {                           // Y_CB[a3][a2]
            const c64 y = ybase[C * kRow + e];
            yv[e] = make_double2(s * y.x, s * y.y);
          }
#pragma unroll
          for (int a1 = 0; a1 < 3; ++a1)
#pragma unroll
            for (int a2 = 0; a2 < 3; ++a2)
#pragma unroll
              for (int a4 = 0; a4 < 3; ++a4) {
                const int k = 2 * (9 * a1 + 3 * a2 + a4);
                const c64 a = xv[3 * a1 + a4], b = yv[a2];
                v[k] = __builtin_fma(a.x, b.x, v[k]);
                v[k] = __builtin_fma(-a.y, b.y, v[k]);
                v[k + 1] = __builtin_fma(a.x, b.y, v[k + 1]);
                v[k + 1] = __builtin_fma(a.y, b.x, v[k + 1]);
              }
        }
      }
      // the 16 lanes of an operator (lane bits 0..3) add their partial sums by
      // halving: at each step a lane keeps the lower or upper part of its current
      // range (by one lane bit), adds the partner's copy of that part and hands
      // over the other part.  Ranges 54 -> 27 -> 14 -> 7 -> 4 (odd lengths padded
      // by a zero).
      const bool u3 = lane & 8, u2 = lane & 4, u1 = lane & 2, u0 = lane & 1;
#pragma unroll
      for (int k = 0; k < 27; ++k) {
        const double lo = v[k], hi = v[k + 27];
        v[k] = (u3 ? hi : lo) + __shfl_xor(u3 ? lo : hi, 8, 64);
      }
#pragma unroll
      for (int k = 0; k < 14; ++k) {
        const double lo = v[k], hi = k + 14 < 27 ? v[k + 14] : 0.0;
        v[k] = (u2 ? hi : lo) + __shfl_xor(u2 ? lo : hi, 4, 64);
      }
#pragma unroll
      for (int k = 0; k < 7; ++k) {
        const double lo = v[k], hi = k + 7 < 14 ? v[k + 7] : 0.0;
        v[k] = (u1 ? hi : lo) + __shfl_xor(u1 ? lo : hi, 2, 64);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double lo = v[k], hi = k + 4 < 7 ? v[k + 4] : 0.0;
        v[k] = (u0 ? hi : lo) + __shfl_xor(u0 ? lo : hi, 1, 64);
      }
      if (act) {
        // this lane's 4 entries start at 27 u3 + 14 u2 + 7 u1 + 4 u0 of the 54;
        // an entry is real where it lies inside every range it was cut from
        const int o3 = 4 * u0, o2 = 7 * u1 + o3, o1 = 14 * u2 + o2, base = 27 * u3 + o1;
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (o3 + k < 7 && o2 + k < 14 && o1 + k < 27) {
            const int q = base + k, jj = q >> 1;  // jj = 9 a1 + 3 a2 + a4
            const int a1 = jj / 9, a2 = jj / 3 % 3, a4 = jj % 3;
            out[2 * (27 * a1 + 9 * a2 + 3 * a3 + a4) + (q & 1)] = v[k];
          }
      }
    }
  }
}

// gamma_X gamma_Y = sigma(X, Y) gamma_{X ^ Y}: each gamma_nu of Y moves left past
// the gamma_mu of X with mu > nu, each exchange a sign (they anticommute).
int sigma(int X, int Y) {
  int n = 0;
  for (int mu = 0; mu < 4; ++mu)
    for (int nu = 0; nu < mu; ++nu) n += (X >> mu & 1) & (Y >> nu & 1);
  return (n & 1) ? -1 : 1;
}
// gamma_X^dag = reversed product = (-1)^(k(k-1)/2) gamma_X, k = |X|
int rev(int X) {
  const int k = __builtin_popcount(X);
  return ((k * (k - 1) / 2) & 1) ? -1 : 1;
}
// (1/4) Tr[gamma_A^dag gamma_S gamma_B gamma_F^dag] for B = A ^ S ^ F (the only
// nonzero entry of row A): the product is r(A) r(F) gamma_A gamma_S gamma_B gamma_F,
// which reduces to a sign times gamma_0 = 1.
int spin_taste_sign(int A, int S, int F) {
  const int B = A ^ S ^ F;
  return rev(A) * rev(F) * sigma(A, S) * sigma(A ^ S, B) * sigma(A ^ S ^ B, F);
}

}  // namespace
}  // namespace asq

using namespace asq;

extern "C" int asqtad_npr_fourfermion(const int dims[4], const double* thin_dev, const double* g1_dev,
                                      const double* g2_dev, const double* g3_dev, const double* g4_dev, int nop,
                                      const int* ops_host, double* out_dev, void* hip_stream) {
  const char* who = "asqtad_npr_fourfermion";
  if (!dims || !thin_dev || !g1_dev || !g2_dev || !g3_dev || !g4_dev || !ops_host || !out_dev || nop <= 0) {
    set_last_error(std::string(who) + ": null pointer or nop <= 0");
    return ASQ_EINVAL;
  }
  for (int mu = 0; mu < 4; ++mu)
    if (dims[mu] < 2 || (dims[mu] & 1) || dims[mu] > (1 << 14)) {
      set_last_error(std::string(who) + ": extents must be even, 2 .. 16384");
      return ASQ_EINVAL;
    }
  for (int k = 0; k < 4 * nop; ++k)
    if (ops_host[k] < 0 || ops_host[k] > 15) {
      set_last_error(std::string(who) + ": spin and taste labels are 4-bit masks (0 .. 15)");
      return ASQ_EINVAL;
    }
  const uintptr_t al = (uintptr_t)thin_dev | (uintptr_t)g1_dev | (uintptr_t)g2_dev | (uintptr_t)g3_dev |
                       (uintptr_t)g4_dev | (uintptr_t)out_dev;
  if (al & 15) {
    set_last_error(std::string(who) + ": links, propagators and output must be 16-byte aligned");
    return ASQ_EINVAL;
  }
  const long V = (long)dims[0] * dims[1] * dims[2] * dims[3];
  const long nz = V / 16;
  if (nz >= (1L << 31)) {
    set_last_error(std::string(who) + ": lattice too large");
    return ASQ_EINVAL;
  }
  // the output may not overlap an input
  const size_t ob = (size_t)nop * nz * 81 * 16;
  const void* ins[5] = {thin_dev, g1_dev, g2_dev, g3_dev, g4_dev};
  const size_t ib[5] = {(size_t)V * 4 * 9 * 16, (size_t)V * 9 * 16, (size_t)V * 9 * 16, (size_t)V * 9 * 16,
                        (size_t)V * 9 * 16};
  for (int k = 0; k < 5; ++k) {
    const uintptr_t a = (uintptr_t)ins[k], o = (uintptr_t)out_dev;
    if (o < a + ib[k] && a < o + ob) {
      set_last_error(std::string(who) + ": the output must not overlap the links or propagators");
      return ASQ_EINVAL;
    }
  }
  NprArgs P;
  memset(&P, 0, sizeof(P));
  P.X = dims[0];
  P.Y = dims[1];
  P.Z = dims[2];
  P.T = dims[3];
  P.hx = dims[0] / 2;
  P.hy = dims[1] / 2;
  P.hz = dims[2] / 2;
  P.thin = (const double2*)thin_dev;
  P.g[0] = (const double2*)g1_dev;
  P.g[1] = (const double2*)g2_dev;
  P.g[2] = (const double2*)g3_dev;
  P.g[3] = (const double2*)g4_dev;
  P.out = (double2*)out_dev;
  P.nz = nz;
  hipStream_t s = (hipStream_t)hip_stream;
  for (int op0 = 0; op0 < nop; op0 += kNprOpsPerLaunch) {
    P.op0 = op0;
    P.nop = nop - op0 < kNprOpsPerLaunch ? nop - op0 : kNprOpsPerLaunch;
    for (int k = 0; k < P.nop; ++k) {
      const int* o = ops_host + 4 * (op0 + k);
      NprOp& q = P.ops[k];
      q.p1 = (unsigned char)(o[0] ^ o[1]);
      q.p2 = (unsigned char)(o[2] ^ o[3]);
      q.neg1 = q.neg2 = 0;
      for (int A = 0; A < 16; ++A) {
        // eps(z_A) = (-1)^|A|: the hypercube origin 2z has even coordinates
        const int eps = (__builtin_popcount(A) & 1) ? -1 : 1;
        if (spin_taste_sign(A, o[0], o[1]) * eps < 0) q.neg1 |= (unsigned short)(1u << A);
        if (spin_taste_sign(A, o[2], o[3]) * eps < 0) q.neg2 |= (unsigned short)(1u << A);
      }
    }
    npr_kernel<<<(unsigned)nz, kNprThreads, 0, s>>>(P);
    ASQ_HIP_TRY(hipGetLastError());
  }
  return ASQ_OK;
}
