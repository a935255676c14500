// gauge.hip -- link import: canonical FP64 links -> resident per-parity
// structure-of-arrays copies in each kept precision, with the staggered phases
// and the antiperiodic time-boundary sign folded in (18-real tiers) or left to
// the Dslash (12-real tiers, which keep the SU(3) part only).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>

#include "asq_internal.h"

namespace asq {

size_t link_slot_bytes(int kind) {
  switch (kind) {
    case LINK_F64_R18: return 18 * sizeof(double);
    case LINK_F32_R18: return 18 * sizeof(float);
    case LINK_F32_R12: return 12 * sizeof(float);
    case LINK_I16_R12: return 12 * sizeof(short);
    case LINK_F64_F32: return 0;  // reads the FP64 tier
  }
  return 0;
}

namespace {

struct ImportArgs {
  Geom g;
  long lex0, nsites;  // the canonical sites [lex0, lex0 + nsites) held at fat, lng
  const double* fat;
  const double* lng;
  double2* l64;   // LINK_F64_R18 or nullptr
  float2* l32f;   // LINK_F32_R18 or nullptr
  float4* l32c;   // LINK_F32_R12 or nullptr
  short4* l16c;   // LINK_I16_R12 or nullptr
  double fat_scale, long_scale;
  int* bad;       // set to 1 when a compressed copy is requested for a non-SU(3) link
};

__device__ inline short q16(double v) {
  double s = rint(v * 32767.0);
  s = fmin(32767.0, fmax(-32767.0, s));
  return (short)s;
}

// One thread per (site, slot); slot 0..3 fat x,y,z,t, 4..7 long x,y,z,t.
__global__ void __launch_bounds__(256) import_kernel(const ImportArgs a) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= a.nsites * 8) return;
  const long lex = a.lex0 + (gid >> 3);
  const int slot = (int)(gid & 7);
  const int mu = slot & 3;
  const bool is_long = slot >= 4;
  long r = lex;
  const int x = (int)(r % a.g.X); r /= a.g.X;
  const int y = (int)(r % a.g.Y); r /= a.g.Y;
  const int z = (int)(r % a.g.Z);
  const int t = (int)(r / a.g.Z);
  const int p = (x + y + z + t) & 1;
  const int i = (int)(lex >> 1);
  const int half = a.g.half;

  int eta = 1;
  if (mu == 1) eta = (x & 1) ? -1 : 1;
  if (mu == 2) eta = ((x + y) & 1) ? -1 : 1;
  if (mu == 3) eta = ((x + y + z) & 1) ? -1 : 1;
  const int hop = is_long ? 3 : 1;
  const int bc = (mu == 3 && t + hop >= a.g.T) ? -1 : 1;
  const double sign = (double)(eta * bc);

  const double* src = (is_long ? a.lng : a.fat) + ((lex - a.lex0) * 4 + mu) * 18;
  double u[18];
#pragma unroll
  for (int k = 0; k < 18; ++k) u[k] = src[k];

  const size_t base = (size_t)(p * 8 + slot);
  if (a.l64) {
    double2* q = a.l64 + base * 9 * half + i;
#pragma unroll
    for (int k = 0; k < 9; ++k) q[(size_t)k * half] = make_double2(sign * u[2 * k], sign * u[2 * k + 1]);
  }
  if (a.l32f) {
    float2* q = a.l32f + base * 9 * half + i;
#pragma unroll
    for (int k = 0; k < 9; ++k) q[(size_t)k * half] = make_float2((float)(sign * u[2 * k]), (float)(sign * u[2 * k + 1]));
  }
  if (a.l32c || a.l16c) {
    const double inv = 1.0 / (is_long ? a.long_scale : a.fat_scale);
    double w[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) w[k] = u[k] * inv;
    // unitarity |W W^dag - 1| and the row-3 identity row2 = conj(row0 x row1)
    double err = 0;
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int n = 0; n < 3; ++n) {
        double re = 0, im = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double ar = w[2 * (3 * m + c)], ai = w[2 * (3 * m + c) + 1];
          const double br = w[2 * (3 * n + c)], bi = w[2 * (3 * n + c) + 1];
          re += ar * br + ai * bi;  // a * conj(b)
          im += ai * br - ar * bi;
        }
        err = fmax(err, fabs(re - (m == n ? 1.0 : 0.0)));
        err = fmax(err, fabs(im));
      }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
      const double a1r = w[2 * k1], a1i = w[2 * k1 + 1], a2r = w[2 * k2], a2i = w[2 * k2 + 1];
      const double b1r = w[2 * (3 + k1)], b1i = w[2 * (3 + k1) + 1];
      const double b2r = w[2 * (3 + k2)], b2i = w[2 * (3 + k2) + 1];
      const double cr = (a1r * b2r - a1i * b2i) - (a2r * b1r - a2i * b1i);
      const double ci = (a1r * b2i + a1i * b2r) - (a2r * b1i + a2i * b1r);
      err = fmax(err, fabs(w[2 * (6 + k)] - cr));
      err = fmax(err, fabs(w[2 * (6 + k) + 1] + ci));
    }
    if (!(err <= 1e-6)) atomicOr(a.bad, 1);
    if (a.l32c) {
      float4* q = a.l32c + base * 3 * half + i;
#pragma unroll
      for (int k = 0; k < 3; ++k)
        q[(size_t)k * half] = make_float4((float)w[4 * k], (float)w[4 * k + 1], (float)w[4 * k + 2], (float)w[4 * k + 3]);
    }
    if (a.l16c) {
      short4* q = a.l16c + base * 3 * half + i;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        short4 v;
        v.x = q16(w[4 * k]);
        v.y = q16(w[4 * k + 1]);
        v.z = q16(w[4 * k + 2]);
        v.w = q16(w[4 * k + 3]);
        q[(size_t)k * half] = v;
      }
    }
  }
}

bool valid_desc(const asq_gauge_desc* d) {
  if (!d) return false;
  for (int mu = 0; mu < 4; ++mu)
    if (d->dims[mu] < 4 || (d->dims[mu] & 1) || d->dims[mu] > (1 << 14)) return false;
  const long V = (long)d->dims[0] * d->dims[1] * d->dims[2] * d->dims[3];
  if (V / 2 * 9 >= (1L << 31)) return false;
  if (d->prec_mask <= 0 || (d->prec_mask & ~7)) return false;
  if (d->recon != 18 && d->recon != 12) return false;
  const bool needs_scale = d->recon == 12 || (d->prec_mask & (1 << ASQ_F16));
  if (needs_scale) {
    if (!(fabs(d->fat_scale) > 0) || !isfinite(d->fat_scale)) return false;
    if (!(fabs(d->long_scale) > 0) || !isfinite(d->long_scale)) return false;
  }
  return true;
}

// Sites of canonical host links staged per copy by asq_gauge_create: at most
// 16 MB of FP64 fat and long links (1152 bytes per site).
long stage_sites(const asq_gauge_desc* d) {
  const long V = (long)d->dims[0] * d->dims[1] * d->dims[2] * d->dims[3];
  return std::min(V, (long)((16u << 20) / 1152));
}

// Offsets of each kept tier inside the storage, then the staging area of
// asq_gauge_create and a flag word; returns the total bytes.
size_t layout(const asq_gauge_desc* d, size_t off[LINK_KINDS], size_t* stage_off = nullptr) {
  const long half = (long)d->dims[0] * d->dims[1] * d->dims[2] * d->dims[3] / 2;
  size_t total = 0;
  for (int k = 0; k < LINK_KINDS; ++k) off[k] = (size_t)-1;
  auto take = [&](int kind) {
    off[kind] = total;
    total = align_up(total + (size_t)16 * half * link_slot_bytes(kind), 256);
  };
  if (d->prec_mask & (1 << ASQ_F64)) take(LINK_F64_R18);
  if (d->prec_mask & (1 << ASQ_F32)) take(d->recon == 12 ? LINK_F32_R12 : LINK_F32_R18);
  if (d->prec_mask & (1 << ASQ_F16)) take(LINK_I16_R12);
  if (stage_off) *stage_off = total;
  total = align_up(total + (size_t)stage_sites(d) * 1152, 256);
  return total + 256;  // flag word
}

}  // namespace

FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  // floor(2^64 / d) + 1 (d >= 2)
  const unsigned __int128 one = 1;
  f.m = (uint64_t)(((one << 64) / d) + 1);
  return f;
}

Geom make_geom(const int dims[4]) {
  Geom g;
  g.X = dims[0];
  g.Y = dims[1];
  g.Z = dims[2];
  g.T = dims[3];
  g.Xh = g.X / 2;
  g.half = g.Xh * g.Y * g.Z * g.T;
  g.sY = g.Xh;
  g.sZ = g.Xh * g.Y;
  g.sT = g.Xh * g.Y * g.Z;
  g.dXh = make_fastdiv(g.Xh);
  g.dY = make_fastdiv(g.Y);
  g.dZ = make_fastdiv(g.Z);
  return g;
}

}  // namespace asq

using namespace asq;

extern "C" size_t asq_gauge_bytes(const asq_gauge_desc* desc) {
  if (!valid_desc(desc)) return 0;
  size_t off[LINK_KINDS];
  return layout(desc, off);
}

// Import canonical links into a new handle.  host: fat/lng are host pointers,
// copied through the staging area of the storage a chunk of sites at a time;
// otherwise device pointers read in place.
static int gauge_import(const char* who, const asq_gauge_desc* desc, const double* fat, const double* lng,
                        bool host, void* storage_dev, size_t storage_bytes, void* hip_stream, asq_gauge** out) {
  if (!out) return ASQ_EINVAL;
  *out = nullptr;
  if (!valid_desc(desc)) {
    set_last_error(std::string(who) + ": invalid description (extents even >= 4, recon 18|12, prec_mask, scales)");
    return ASQ_EINVAL;
  }
  if (!fat || !lng || !storage_dev) {
    set_last_error(std::string(who) + ": null pointer");
    return ASQ_EINVAL;
  }
  if (((uintptr_t)storage_dev & 255) || (!host && (((uintptr_t)fat & 15) || ((uintptr_t)lng & 15)))) {
    set_last_error(std::string(who) + ": storage must be 256-byte aligned, device links 16-byte aligned");
    return ASQ_EINVAL;
  }
  size_t off[LINK_KINDS], stage_off = 0;
  const size_t need = layout(desc, off, &stage_off);
  if (storage_bytes < need) {
    set_last_error(std::string(who) + ": storage smaller than asq_gauge_bytes()");
    return ASQ_ENOMEM;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  asq_gauge* g = new asq_gauge();
  g->desc = *desc;
  g->geom = make_geom(desc->dims);
  g->base = storage_dev;
  g->bytes = storage_bytes;
  g->nblk = (g->geom.half + kBlock - 1) / kBlock;
  if (hipGetDevice(&g->device) != hipSuccess) {
    delete g;
    set_last_error(std::string(who) + ": no current HIP device");
    return ASQ_EHIP;
  }
  char* b = (char*)storage_dev;
  for (int k = 0; k < LINK_KINDS; ++k) g->links[k] = off[k] == (size_t)-1 ? nullptr : b + off[k];
  g->links[LINK_F64_F32] = g->links[LINK_F64_R18];  // no copy: converted on load
  if (desc->prec_mask & (1 << ASQ_F32)) g->sloppy_link32 = desc->recon == 12 ? LINK_F32_R12 : LINK_F32_R18;
  else g->sloppy_link32 = LINK_F64_F32;
  g->sloppy_link16 = g->links[LINK_I16_R12] ? LINK_I16_R12 : g->sloppy_link32;
  int* flag = (int*)(b + need - 256);

  ImportArgs a;
  a.g = g->geom;
  a.l64 = (double2*)g->links[LINK_F64_R18];
  a.l32f = (float2*)g->links[LINK_F32_R18];
  a.l32c = (float4*)g->links[LINK_F32_R12];
  a.l16c = (short4*)g->links[LINK_I16_R12];
  a.fat_scale = desc->fat_scale;
  a.long_scale = desc->long_scale;
  a.bad = flag;
  int bad = 0;
  const long V = 2L * g->geom.half;
  const long chunk = host ? stage_sites(desc) : V;
  double* st_fat = (double*)(b + stage_off);
  double* st_lng = st_fat + (size_t)chunk * 72;
  hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), s);
  for (long lex0 = 0; lex0 < V && e == hipSuccess; lex0 += chunk) {
    const long n = std::min(chunk, V - lex0);
    a.lex0 = lex0;
    a.nsites = n;
    if (host) {
      // the previous chunk's import has read the staging area when this copy runs (same stream)
      e = hipMemcpyAsync(st_fat, fat + (size_t)lex0 * 72, (size_t)n * 576, hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = hipMemcpyAsync(st_lng, lng + (size_t)lex0 * 72, (size_t)n * 576,
                                              hipMemcpyHostToDevice, s);
      a.fat = st_fat;
      a.lng = st_lng;
    } else {
      a.fat = fat + (size_t)lex0 * 72;
      a.lng = lng + (size_t)lex0 * 72;
    }
    if (e == hipSuccess) {
      import_kernel<<<(unsigned)((n * 8 + 255) / 256), 256, 0, s>>>(a);
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    set_last_error(hipGetErrorString(e));
    delete g;
    return ASQ_EHIP;
  }
  if (bad) {
    set_last_error(std::string(who) +
                   ": link/scale is not SU(3) to 1e-6; 12-real or 16-bit copies need SU(3) links");
    delete g;
    return ASQ_ENOTSU3;
  }
  *out = g;
  return ASQ_OK;
}

extern "C" int asq_gauge_create(const asq_gauge_desc* desc, const double* fat_host, const double* long_host,
                                void* storage_dev, size_t storage_bytes, void* hip_stream, asq_gauge** out) {
  return gauge_import("asq_gauge_create", desc, fat_host, long_host, true, storage_dev, storage_bytes, hip_stream,
                      out);
}

extern "C" int asq_gauge_create_device(const asq_gauge_desc* desc, const double* fat_dev, const double* long_dev,
                                       void* storage_dev, size_t storage_bytes, void* hip_stream, asq_gauge** out) {
  return gauge_import("asq_gauge_create_device", desc, fat_dev, long_dev, false, storage_dev, storage_bytes,
                      hip_stream, out);
}

extern "C" int asq_gauge_destroy(asq_gauge* g) {
  if (!g) return ASQ_EINVAL;
  delete g;
  return ASQ_OK;
}
