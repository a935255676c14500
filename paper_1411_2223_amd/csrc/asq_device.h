// asq_device.h -- device-side building blocks of the gfx950 asqtad path:
// lattice geometry on a checkerboard, complex arithmetic with explicit FMAs,
// SU(3) link loaders (18-real and 12-real), colour-vector loaders/stores for
// the three storage tiers, and deterministic FP64 block reductions.
//
// Conventions (the staggered operator of the paper's CG workload; the paper
// gives no formulas, so the standard MILC asqtad forms are used):
//   lex = x + X*(y + Y*(z + Z*t)); parity = (x+y+z+t) & 1; checkerboard index = lex >> 1
//   eta_x = 1, eta_y = (-1)^x, eta_z = (-1)^(x+y), eta_t = (-1)^(x+y+z)
//   fermions antiperiodic in t, links periodic.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace asq {

constexpr int kBlock = 256;  // sites per block and per reduction group (fixed: keeps sums batch-invariant)

// n / d for 32-bit n and 2 <= d < 2^32 with a 64-bit magic multiplier:
// m = floor(2^64 / d) + 1 gives floor(n*m / 2^64) = floor(n / d) exactly.
struct FastDiv {
  uint32_t d;
  uint64_t m;
  __device__ __forceinline__ uint32_t div(uint32_t n) const {
    return (uint32_t)__umul64hi((uint64_t)n, m);
  }
};

struct Geom {
  int X, Y, Z, T;
  int Xh;          // X / 2
  int half;        // V / 2 sites of one parity
  int sY, sZ, sT;  // checkerboard-index strides of y, z, t: Xh, Xh*Y, Xh*Y*Z
  FastDiv dXh, dY, dZ;
};

struct Site {
  int x, y, z, t;
};

// Coordinates of checkerboard site i of parity p.
__device__ __forceinline__ Site decode(const Geom& g, int i, int p) {
  const uint32_t r = g.dXh.div((uint32_t)i);
  const int xh = i - (int)r * g.Xh;
  const uint32_t r2 = g.dY.div(r);
  const int y = (int)r - (int)r2 * g.Y;
  const uint32_t t = g.dZ.div(r2);
  const int z = (int)r2 - (int)t * g.Z;
  Site s;
  s.y = y;
  s.z = z;
  s.t = (int)t;
  s.x = 2 * xh + ((y + z + (int)t + p) & 1);
  return s;
}

__device__ __forceinline__ int wrap(int v, int L) {
  return v < 0 ? v + L : (v >= L ? v - L : v);
}

// Checkerboard index of the site h steps (|h| = 1 or 3) from site (i, s) along mu.
template <int MU>
__device__ __forceinline__ int neighbour(const Geom& g, int i, const Site& s, int h) {
  if constexpr (MU == 0) {
    const int xn = wrap(s.x + h, g.X);
    return i - (s.x >> 1) + (xn >> 1);
  } else if constexpr (MU == 1) {
    return i + (wrap(s.y + h, g.Y) - s.y) * g.sY;
  } else if constexpr (MU == 2) {
    return i + (wrap(s.z + h, g.Z) - s.z) * g.sZ;
  } else {
    return i + (wrap(s.t + h, g.T) - s.t) * g.sT;
  }
}

// MILC staggered phase eta_mu at site s.
template <int MU>
__device__ __forceinline__ int eta_sign(const Site& s) {
  if (MU == 0) return 1;
  if (MU == 1) return (s.x & 1) ? -1 : 1;
  if (MU == 2) return ((s.x + s.y) & 1) ? -1 : 1;
  return ((s.x + s.y + s.z) & 1) ? -1 : 1;
}

// ---------------------------------------------------------------------------
// complex arithmetic (explicit FMAs so that every instance rounds identically)
// ---------------------------------------------------------------------------
template <class R>
struct cx {
  R re, im;
};

template <class R>
__device__ __forceinline__ R fmaR(R a, R b, R c);
template <>
__device__ __forceinline__ float fmaR<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <>
__device__ __forceinline__ double fmaR<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

// acc += a * b
template <class R>
__device__ __forceinline__ void cmac(cx<R>& acc, const cx<R>& a, const cx<R>& b) {
  acc.re = fmaR(a.re, b.re, acc.re);
  acc.re = fmaR(-a.im, b.im, acc.re);
  acc.im = fmaR(a.re, b.im, acc.im);
  acc.im = fmaR(a.im, b.re, acc.im);
}

// acc += conj(a) * b
template <class R>
__device__ __forceinline__ void cmac_conj(cx<R>& acc, const cx<R>& a, const cx<R>& b) {
  acc.re = fmaR(a.re, b.re, acc.re);
  acc.re = fmaR(a.im, b.im, acc.re);
  acc.im = fmaR(a.re, b.im, acc.im);
  acc.im = fmaR(-a.im, b.re, acc.im);
}

template <class R>
struct Mat3 {
  cx<R> e[3][3];
};

template <class R>
struct Vec3 {
  cx<R> c[3];
};

// y = U v
template <class R>
__device__ __forceinline__ Vec3<R> mul(const Mat3<R>& U, const Vec3<R>& v) {
  Vec3<R> y;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    y.c[a].re = U.e[a][0].re * v.c[0].re;
    y.c[a].im = U.e[a][0].re * v.c[0].im;
    y.c[a].re = fmaR(-U.e[a][0].im, v.c[0].im, y.c[a].re);
    y.c[a].im = fmaR(U.e[a][0].im, v.c[0].re, y.c[a].im);
    cmac(y.c[a], U.e[a][1], v.c[1]);
    cmac(y.c[a], U.e[a][2], v.c[2]);
  }
  return y;
}

// y = U^dagger v
template <class R>
__device__ __forceinline__ Vec3<R> mul_adj(const Mat3<R>& U, const Vec3<R>& v) {
  Vec3<R> y;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    y.c[a].re = U.e[0][a].re * v.c[0].re;
    y.c[a].im = U.e[0][a].re * v.c[0].im;
    y.c[a].re = fmaR(U.e[0][a].im, v.c[0].im, y.c[a].re);
    y.c[a].im = fmaR(-U.e[0][a].im, v.c[0].re, y.c[a].im);
    cmac_conj(y.c[a], U.e[1][a], v.c[1]);
    cmac_conj(y.c[a], U.e[2][a], v.c[2]);
  }
  return y;
}

// acc += s * v
template <class R>
__device__ __forceinline__ void axpy3(Vec3<R>& acc, R s, const Vec3<R>& v) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    acc.c[a].re = fmaR(s, v.c[a].re, acc.c[a].re);
    acc.c[a].im = fmaR(s, v.c[a].im, acc.c[a].im);
  }
}

template <class R>
__device__ __forceinline__ void add3(Vec3<R>& acc, const Vec3<R>& v) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    acc.c[a].re += v.c[a].re;
    acc.c[a].im += v.c[a].im;
  }
}

template <class R>
__device__ __forceinline__ void sub3(Vec3<R>& acc, const Vec3<R>& v) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    acc.c[a].re -= v.c[a].re;
    acc.c[a].im -= v.c[a].im;
  }
}

// Third row of an SU(3) matrix from the first two: row2 = conj(row0 x row1).
template <class R>
__device__ __forceinline__ void reconstruct_row2(Mat3<R>& U) {
  const cx<R>* a = U.e[0];
  const cx<R>* b = U.e[1];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
    // (a x b)_k = a_k1 b_k2 - a_k2 b_k1
    R re = a[k1].re * b[k2].re;
    re = fmaR(-a[k1].im, b[k2].im, re);
    re = fmaR(-a[k2].re, b[k1].re, re);
    re = fmaR(a[k2].im, b[k1].im, re);
    R im = a[k1].re * b[k2].im;
    im = fmaR(a[k1].im, b[k2].re, im);
    im = fmaR(-a[k2].re, b[k1].im, im);
    im = fmaR(-a[k2].im, b[k1].re, im);
    U.e[2][k].re = re;
    U.e[2][k].im = -im;
  }
}

// ---------------------------------------------------------------------------
// link storage tiers.  Per parity p and slot s (0..3 fat x,y,z,t; 4..7 long)
// the links are stored chunk-major: chunk k of site i at
// base[((p*8 + s)*NCH + k)*half + i]  (structure of arrays, site fastest).
// 18-real tiers hold the link with eta, the time-boundary sign and the fat /
// long coefficient folded in.  12-real tiers hold the first two rows of the
// SU(3) part (link / coefficient); the kernel rebuilds row 3 and applies
// coefficient * eta * boundary sign to the product.
// ---------------------------------------------------------------------------
// LINK_F64_F32 is no storage of its own: the FP64 18-real links read by an FP32
// Dslash, converted on load (a field kept in FP64 only still runs the mixed CG).
enum LinkKind {
  LINK_F64_R18 = 0,
  LINK_F32_R18 = 1,
  LINK_F32_R12 = 2,
  LINK_I16_R12 = 3,
  LINK_F64_F32 = 4,
  LINK_KINDS = 5
};

struct LinkF64R18 {
  using real = double;
  using chunk = double2;
  static constexpr int NCH = 9;
  static constexpr bool folded = true;
  __device__ __forceinline__ static Mat3<double> load(const void* base, int half, int p, int slot, int i) {
    const double2* q = reinterpret_cast<const double2*>(base) + (size_t)((p * 8 + slot) * NCH) * half + i;
    Mat3<double> U;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double2 v = q[(size_t)k * half];
      U.e[k / 3][k % 3].re = v.x;
      U.e[k / 3][k % 3].im = v.y;
    }
    return U;
  }
  // The same with non-temporal loads: the FP64 links of a lattice like 20^3 x 64
  // (590 MB) cannot stay in the memory-side cache between launches, so streaming
  // them past the caches leaves more room for the neighbour vectors.
  __device__ __forceinline__ static Mat3<double> load_streaming(const void* base, int half, int p, int slot,
                                                               int i) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2* q = reinterpret_cast<const d2*>(base) + (size_t)((p * 8 + slot) * NCH) * half + i;
    Mat3<double> U;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const d2 v = __builtin_nontemporal_load(q + (size_t)k * half);
      U.e[k / 3][k % 3].re = v.x;
      U.e[k / 3][k % 3].im = v.y;
    }
    return U;
  }
};

// FP64 18-real storage, FP32 arithmetic: each double is rounded to float on load.
struct LinkF64F32 {
  using real = float;
  using chunk = double2;
  static constexpr int NCH = 9;
  static constexpr bool folded = true;
  __device__ __forceinline__ static Mat3<float> load(const void* base, int half, int p, int slot, int i) {
    const double2* q = reinterpret_cast<const double2*>(base) + (size_t)((p * 8 + slot) * NCH) * half + i;
    Mat3<float> U;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double2 v = q[(size_t)k * half];
      U.e[k / 3][k % 3].re = (float)v.x;
      U.e[k / 3][k % 3].im = (float)v.y;
    }
    return U;
  }
  // non-temporal loads, as for the FP64 tier: these links do not stay in the
  // memory-side cache between launches either
  __device__ __forceinline__ static Mat3<float> load_streaming(const void* base, int half, int p, int slot, int i) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2* q = reinterpret_cast<const d2*>(base) + (size_t)((p * 8 + slot) * NCH) * half + i;
    Mat3<float> U;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const d2 v = __builtin_nontemporal_load(q + (size_t)k * half);
      U.e[k / 3][k % 3].re = (float)v.x;
      U.e[k / 3][k % 3].im = (float)v.y;
    }
    return U;
  }
};

struct LinkF32R18 {
  using real = float;
  using chunk = float2;
  static constexpr int NCH = 9;
  static constexpr bool folded = true;
  __device__ __forceinline__ static Mat3<float> load(const void* base, int half, int p, int slot, int i) {
    const float2* q = reinterpret_cast<const float2*>(base) + (size_t)((p * 8 + slot) * NCH) * half + i;
    Mat3<float> U;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const float2 v = q[(size_t)k * half];
      U.e[k / 3][k % 3].re = v.x;
      U.e[k / 3][k % 3].im = v.y;
    }
    return U;
  }
  __device__ __forceinline__ static Mat3<float> load_streaming(const void* base, int half, int p, int slot, int i) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    const f2* q = reinterpret_cast<const f2*>(base) + (size_t)((p * 8 + slot) * NCH) * half + i;
    Mat3<float> U;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const f2 v = __builtin_nontemporal_load(q + (size_t)k * half);
      U.e[k / 3][k % 3].re = v.x;
      U.e[k / 3][k % 3].im = v.y;
    }
    return U;
  }
};

struct LinkF32R12 {
  using real = float;
  using chunk = float4;
  static constexpr int NCH = 3;
  static constexpr bool folded = false;
  __device__ __forceinline__ static Mat3<float> load(const void* base, int half, int p, int slot, int i) {
    const float4* q = reinterpret_cast<const float4*>(base) + (size_t)((p * 8 + slot) * NCH) * half + i;
    Mat3<float> U;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float4 v = q[(size_t)k * half];
      const int e0 = 2 * k, e1 = 2 * k + 1;
      U.e[e0 / 3][e0 % 3].re = v.x;
      U.e[e0 / 3][e0 % 3].im = v.y;
      U.e[e1 / 3][e1 % 3].re = v.z;
      U.e[e1 / 3][e1 % 3].im = v.w;
    }
    reconstruct_row2(U);
    return U;
  }
  __device__ __forceinline__ static Mat3<float> load_streaming(const void* base, int half, int p, int slot, int i) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4* q = reinterpret_cast<const f4*>(base) + (size_t)((p * 8 + slot) * NCH) * half + i;
    Mat3<float> U;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const f4 v = __builtin_nontemporal_load(q + (size_t)k * half);
      const int e0 = 2 * k, e1 = 2 * k + 1;
      U.e[e0 / 3][e0 % 3].re = v.x;
      U.e[e0 / 3][e0 % 3].im = v.y;
      U.e[e1 / 3][e1 % 3].re = v.z;
      U.e[e1 / 3][e1 % 3].im = v.w;
    }
    reconstruct_row2(U);
    return U;
  }
};

// 16-bit fixed point: entries of an SU(3) matrix lie in [-1, 1]; value = q / 32767.
struct LinkI16R12 {
  using real = float;
  using chunk = short4;
  static constexpr int NCH = 3;
  static constexpr bool folded = false;
  __device__ __forceinline__ static Mat3<float> load(const void* base, int half, int p, int slot, int i) {
    const short4* q = reinterpret_cast<const short4*>(base) + (size_t)((p * 8 + slot) * NCH) * half + i;
    constexpr float inv = 1.0f / 32767.0f;
    Mat3<float> U;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const short4 v = q[(size_t)k * half];
      const int e0 = 2 * k, e1 = 2 * k + 1;
      U.e[e0 / 3][e0 % 3].re = (float)v.x * inv;
      U.e[e0 / 3][e0 % 3].im = (float)v.y * inv;
      U.e[e1 / 3][e1 % 3].re = (float)v.z * inv;
      U.e[e1 / 3][e1 % 3].im = (float)v.w * inv;
    }
    reconstruct_row2(U);
    return U;
  }
  __device__ __forceinline__ static Mat3<float> load_streaming(const void* base, int half, int p, int slot, int i) {
    typedef short s4 __attribute__((ext_vector_type(4)));
    const s4* q = reinterpret_cast<const s4*>(base) + (size_t)((p * 8 + slot) * NCH) * half + i;
    constexpr float inv = 1.0f / 32767.0f;
    Mat3<float> U;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const s4 v = __builtin_nontemporal_load(q + (size_t)k * half);
      const int e0 = 2 * k, e1 = 2 * k + 1;
      U.e[e0 / 3][e0 % 3].re = (float)v.x * inv;
      U.e[e0 / 3][e0 % 3].im = (float)v.y * inv;
      U.e[e1 / 3][e1 % 3].re = (float)v.z * inv;
      U.e[e1 / 3][e1 % 3].im = (float)v.w * inv;
    }
    reconstruct_row2(U);
    return U;
  }
};

// A link tier read with non-temporal loads (one-column launches on lattices whose
// links cannot stay in the memory-side cache: streaming them leaves it to the
// neighbour vectors).  Same values, same arithmetic.
template <class L>
struct Streamed : L {
  __device__ __forceinline__ static Mat3<typename L::real> load(const void* base, int half, int p, int slot, int i) {
    return L::load_streaming(base, half, p, slot, i);
  }
};

// ---------------------------------------------------------------------------
// colour-vector storage tiers (one parity, ncol columns):
//   F64: double2 [col][colour][half]       F32: float2 [col][colour][half]
//   F16: 16-byte record [col][half] = six binary16 values (c0re c0im c1re ...)
//        h = component x r rounded once to binary16 (nearest even), r = 1/nu in
//        float32, then nu as float32; nu = max |component|.  The product and the
//        rounding are one mixed-precision FMA (v_fma_mixlo_f16), so the product
//        is never rounded to float32 first.
// ---------------------------------------------------------------------------
enum VecKind { VEC_F64 = 0, VEC_F32 = 1, VEC_F16 = 2 };

struct VecF64 {
  using real = double;
  using raw = Vec3<double>;
  static constexpr int kind = VEC_F64;
  __device__ __forceinline__ static Vec3<double> load(const void* base, int half, int col, int i) {
    const double2* q = reinterpret_cast<const double2*>(base) + (size_t)col * 3 * half + i;
    Vec3<double> v;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double2 w = q[(size_t)a * half];
      v.c[a].re = w.x;
      v.c[a].im = w.y;
    }
    return v;
  }
  __device__ __forceinline__ static Vec3<double> quantize(const Vec3<double>& v) { return v; }
  // Stores v; returns the value a later load gives back.
  __device__ __forceinline__ static Vec3<double> store(void* base, int half, int col, int i, const Vec3<double>& v) {
    double2* q = reinterpret_cast<double2*>(base) + (size_t)col * 3 * half + i;
#pragma unroll
    for (int a = 0; a < 3; ++a) q[(size_t)a * half] = make_double2(v.c[a].re, v.c[a].im);
    return v;
  }
};

struct VecF32 {
  using real = float;
  using raw = Vec3<float>;
  static constexpr int kind = VEC_F32;
  __device__ __forceinline__ static Vec3<float> load(const void* base, int half, int col, int i) {
    const float2* q = reinterpret_cast<const float2*>(base) + (size_t)col * 3 * half + i;
    Vec3<float> v;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float2 w = q[(size_t)a * half];
      v.c[a].re = w.x;
      v.c[a].im = w.y;
    }
    return v;
  }
  __device__ __forceinline__ static Vec3<float> quantize(const Vec3<float>& v) { return v; }
  __device__ __forceinline__ static Vec3<float> store(void* base, int half, int col, int i, const Vec3<float>& v) {
    float2* q = reinterpret_cast<float2*>(base) + (size_t)col * 3 * half + i;
#pragma unroll
    for (int a = 0; a < 3; ++a) q[(size_t)a * half] = make_float2(v.c[a].re, v.c[a].im);
    return v;
  }
};

struct VecF16 {
  using real = float;
  using raw = uint4;
  static constexpr int kind = VEC_F16;
  __device__ __forceinline__ static uint4 load_rec(const void* base, int half, int col, int i) {
    return reinterpret_cast<const uint4*>(base)[(size_t)col * half + i];
  }
  // The six stored binary16 values as floats (without the norm) of a record.
  __device__ __forceinline__ static Vec3<float> halves(const uint4 w) {
    Vec3<float> h;
    h.c[0].re = h2f(w.x & 0xffffu);
    h.c[0].im = h2f(w.x >> 16);
    h.c[1].re = h2f(w.y & 0xffffu);
    h.c[1].im = h2f(w.y >> 16);
    h.c[2].re = h2f(w.z & 0xffffu);
    h.c[2].im = h2f(w.z >> 16);
    return h;
  }
  __device__ __forceinline__ static float h2f(unsigned short u) {
    return __half2float(__ushort_as_half(u));
  }
  __device__ __forceinline__ static Vec3<float> load(const void* base, int half, int col, int i) {
    return unpack(reinterpret_cast<const uint4*>(base)[(size_t)col * half + i]);
  }
  // The six stored binary16 values as floats, without the norm: psi = nu * h.
  __device__ __forceinline__ static Vec3<float> load_raw(const void* base, int half, int col, int i, float* nu) {
    const uint4 w = reinterpret_cast<const uint4*>(base)[(size_t)col * half + i];
    *nu = __uint_as_float(w.w);
    Vec3<float> h;
    h.c[0].re = h2f(w.x & 0xffffu);
    h.c[0].im = h2f(w.x >> 16);
    h.c[1].re = h2f(w.y & 0xffffu);
    h.c[1].im = h2f(w.y >> 16);
    h.c[2].re = h2f(w.z & 0xffffu);
    h.c[2].im = h2f(w.z >> 16);
    return h;
  }
  __device__ __forceinline__ static Vec3<float> unpack(const uint4 w) {
    const float nu = __uint_as_float(w.w);
    Vec3<float> v;
    v.c[0].re = h2f(w.x & 0xffffu) * nu;
    v.c[0].im = h2f(w.x >> 16) * nu;
    v.c[1].re = h2f(w.y & 0xffffu) * nu;
    v.c[1].im = h2f(w.y >> 16) * nu;
    v.c[2].re = h2f(w.z & 0xffffu) * nu;
    v.c[2].im = h2f(w.z >> 16) * nu;
    return v;
  }
  __device__ __forceinline__ static unsigned pack2(float a, float b) {
    const unsigned lo = __half_as_ushort(__float2half_rn(a));
    const unsigned hi = __half_as_ushort(__float2half_rn(b));
    return lo | (hi << 16);
  }
  __device__ __forceinline__ static uint4 encode(const Vec3<float>& v) {
    float nu = fabsf(v.c[0].re);
    nu = fmaxf(nu, fabsf(v.c[0].im));
    nu = fmaxf(nu, fabsf(v.c[1].re));
    nu = fmaxf(nu, fabsf(v.c[1].im));
    nu = fmaxf(nu, fabsf(v.c[2].re));
    nu = fmaxf(nu, fabsf(v.c[2].im));
    const float inv = nu > 0.f ? 1.0f / nu : 0.f;
    uint4 w;
    w.x = pack2(v.c[0].re * inv, v.c[0].im * inv);
    w.y = pack2(v.c[1].re * inv, v.c[1].im * inv);
    w.z = pack2(v.c[2].re * inv, v.c[2].im * inv);
    w.w = __float_as_uint(nu);
    return w;
  }
  // The value a store followed by a load gives back.
  __device__ __forceinline__ static Vec3<float> quantize(const Vec3<float>& v) { return unpack(encode(v)); }
  __device__ __forceinline__ static Vec3<float> store(void* base, int half, int col, int i, const Vec3<float>& v) {
    const uint4 w = encode(v);
    reinterpret_cast<uint4*>(base)[(size_t)col * half + i] = w;
    return unpack(w);
  }
};

// ---------------------------------------------------------------------------
// canonical colour-vector layouts of the C ABI (one parity, ncol columns):
//   F64: double2 [col][half][3]    F32: float2 [col][half][3]
//   F16: binary16 pairs [col][half][3] (psi / nu), then float nu [col][half]
// The public Dslash reads and writes these directly (PLAIN epilogue only);
// the solvers keep the structures of arrays above and relayout at entry/exit.
// ---------------------------------------------------------------------------
struct VecF64C {
  using real = double;
  using raw = Vec3<double>;
  static constexpr int kind = VEC_F64;
  __device__ __forceinline__ static Vec3<double> load(const void* base, int half, int col, int i) {
    const double2* q = reinterpret_cast<const double2*>(base) + ((size_t)col * half + i) * 3;
    Vec3<double> v;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double2 w = q[a];
      v.c[a].re = w.x;
      v.c[a].im = w.y;
    }
    return v;
  }
  __device__ __forceinline__ static Vec3<double> store(void* base, int half, int col, int i, const Vec3<double>& v) {
    double2* q = reinterpret_cast<double2*>(base) + ((size_t)col * half + i) * 3;
#pragma unroll
    for (int a = 0; a < 3; ++a) q[a] = make_double2(v.c[a].re, v.c[a].im);
    return v;
  }
};

struct VecF32C {
  using real = float;
  using raw = Vec3<float>;
  static constexpr int kind = VEC_F32;
  __device__ __forceinline__ static Vec3<float> load(const void* base, int half, int col, int i) {
    const float2* q = reinterpret_cast<const float2*>(base) + ((size_t)col * half + i) * 3;
    Vec3<float> v;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float2 w = q[a];
      v.c[a].re = w.x;
      v.c[a].im = w.y;
    }
    return v;
  }
  __device__ __forceinline__ static Vec3<float> store(void* base, int half, int col, int i, const Vec3<float>& v) {
    float2* q = reinterpret_cast<float2*>(base) + ((size_t)col * half + i) * 3;
#pragma unroll
    for (int a = 0; a < 3; ++a) q[a] = make_float2(v.c[a].re, v.c[a].im);
    return v;
  }
};

// The record of VecF16 gathered from the split canonical arrays: the three
// words of binary16 pairs, then the norm.  ncol: columns of the whole buffer
// (the norms follow all of them).
struct VecF16C {
  using real = float;
  using raw = uint4;
  static constexpr int kind = VEC_F16;
  __device__ __forceinline__ static const float* norms(const void* base, int half, int ncol) {
    return reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + (size_t)ncol * half * 12);
  }
  __device__ __forceinline__ static uint4 load_rec(const void* base, int half, int ncol, int col, int i) {
    const size_t k = (size_t)col * half + i;
    const uint32_t* q = reinterpret_cast<const uint32_t*>(base) + k * 3;
    uint4 w;
    w.x = q[0];
    w.y = q[1];
    w.z = q[2];
    w.w = __float_as_uint(norms(base, half, ncol)[k]);
    return w;
  }
  __device__ __forceinline__ static void store_rec(void* base, int half, int ncol, int col, int i, const uint4 w) {
    const size_t k = (size_t)col * half + i;
    uint32_t* q = reinterpret_cast<uint32_t*>(base) + k * 3;
    q[0] = w.x;
    q[1] = w.y;
    q[2] = w.z;
    const_cast<float*>(norms(base, half, ncol))[k] = __uint_as_float(w.w);
  }
  __device__ __forceinline__ static Vec3<float> store(void* base, int half, int ncol, int col, int i,
                                                      const Vec3<float>& v) {
    const uint4 w = VecF16::encode(v);
    store_rec(base, half, ncol, col, i, w);
    return VecF16::unpack(w);
  }
};

// Loads and stores by tier with the whole buffer's column count (only the
// canonical FP16 layout needs it: its norms follow every column's halves).
template <class T>
__device__ __forceinline__ uint4 load_rec_any(const void* base, int half, int ncol, int col, int i) {
  if constexpr (std::is_same<T, VecF16C>::value) return VecF16C::load_rec(base, half, ncol, col, i);
  else return VecF16::load_rec(base, half, col, i);
}
template <class T>
__device__ __forceinline__ Vec3<typename T::real> store_any(void* base, int half, int ncol, int col, int i,
                                                            const Vec3<typename T::real>& v) {
  if constexpr (std::is_same<T, VecF16C>::value) return VecF16C::store(base, half, ncol, col, i, v);
  else return T::store(base, half, col, i, v);
}

template <class RD, class RS>
__device__ __forceinline__ Vec3<RD> convert(const Vec3<RS>& v) {
  Vec3<RD> o;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    o.c[a].re = (RD)v.c[a].re;
    o.c[a].im = (RD)v.c[a].im;
  }
  return o;
}

template <class R>
__device__ __forceinline__ double norm2_d(const Vec3<R>& v) {
  double s = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    s = __builtin_fma((double)v.c[a].re, (double)v.c[a].re, s);
    s = __builtin_fma((double)v.c[a].im, (double)v.c[a].im, s);
  }
  return s;
}

template <class R>
__device__ __forceinline__ double redot_d(const Vec3<R>& u, const Vec3<R>& v) {
  double s = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    s = __builtin_fma((double)u.c[a].re, (double)v.c[a].re, s);
    s = __builtin_fma((double)u.c[a].im, (double)v.c[a].im, s);
  }
  return s;
}

// Deterministic sum over a kBlock-thread block; the result is valid in thread 0.
// `sh` holds kBlock/64 doubles; the caller separates successive uses with a barrier.
__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kBlock / 64; ++k) s += sh[k];
  }
  return s;
}

// Blocks are dealt to the 8 XCDs round-robin; remap so that each XCD walks a
// contiguous range of the lattice and neighbour vectors stay in its own L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int q = n >> 3, rem = n & 7, k = b & 7, j = b >> 3;
  return k * q + (k < rem ? k : rem) + j;
}

// One sweep of the whole lattice in which XCD x takes runs of k consecutive
// blocks: inside each group of 8 k blocks, block b (on XCD b mod 8) gets
// position (b mod 8) k + (b div 8) mod k; blocks past the last whole group keep
// their place.  A permutation of [0, n); k = 1 leaves every block in place.
__device__ __forceinline__ int sweep_remap(int b, int n, int k) {
  const int g = 8 * k;
  const int base = (b / g) * g;
  if (base + g > n) return b;
  const int r = b - base;
  return base + (r & 7) * k + (r >> 3);
}

}  // namespace asq
