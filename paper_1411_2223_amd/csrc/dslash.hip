// dslash.hip -- tier checks and dispatch of the Dslash launches (the kernels
// are in dslash_impl.h, one translation unit per link tier).
#include "asq_internal.h"

namespace asq {

bool variant_built(int link_kind, int in_kind, int rtile) {
  const int cols = rtile & 0xff;
  if (rtile & kMfmaBit) {
    // matrix-core form: one tile width, no pipelined form
    if ((rtile & ~(kMfmaBit | 0xff | (3 << kOrderShift))) != 0) return false;
    return link_kind == LINK_F32_R18 && in_kind == VEC_F16 && cols == kMfmaTile;
  }
  if ((rtile & ~(0xff | kPipeBit | kStreamBit | kLdsBit | (3 << kOrderShift) | kGlobalSweepBit | (3 << kChunkShift))) !=
      0)
    return false;
  // the LDS window: pipelined loop, streamed links only at one column (native
  // layouts only: the public operator on canonical vectors refuses it)
  if ((rtile & kLdsBit) && (!(rtile & kPipeBit) || ((rtile & kStreamBit) && cols != 1))) return false;
  if ((rtile & (3 << kChunkShift)) && !(rtile & kGlobalSweepBit)) return false;  // runs only within a sweep
  // streamed links: one column, and not the FP64-stored tiers (which always stream there)
  if ((rtile & kStreamBit) && (cols != 1 || link_kind == LINK_F64_R18 || link_kind == LINK_F64_F32)) return false;
  return cols == 1 || cols == 2 || cols == 4 || cols == 6 || cols == 8 || (cols == 12 && in_kind != VEC_F64);
}

bool variant_fits(const Geom& g, int in_kind, int rtile) {
  if (!(rtile & kLdsBit)) return true;
  return (size_t)(rtile & 0xff) * lds_window(g.Xh) * vec_site_bytes(in_kind) <= kLdsWindowMax;
}

int launch_dslash(int link_kind, int in_kind, int out_kind, int epi, int rtile, const DslashArgs& a,
                  hipStream_t s) {
  if (!variant_built(link_kind, in_kind, rtile)) return ASQ_EINVAL;
  if (link_kind == LINK_F64_R18) {
    if (in_kind != VEC_F64) return ASQ_EINVAL;
    if (epi == EPI_CANON && out_kind != VEC_F64) return ASQ_EINVAL;
    return launch_dslash_f64(out_kind, epi, rtile, a, s);
  }
  if (epi == EPI_RESID) return ASQ_EINVAL;
  if (epi == EPI_CANON && (rtile & kMfmaBit)) return ASQ_EINVAL;
  // PLAIN / NORM / CANON write the input tier; UPDATE keeps r in FP32
  const int want_out = epi == EPI_UPDATE ? VEC_F32 : in_kind;
  if (out_kind != want_out) return ASQ_EINVAL;
  if (link_kind == LINK_F32_R18) return launch_dslash_f32r18(in_kind, epi, rtile, a, s);
  if (link_kind == LINK_F32_R12) return launch_dslash_f32r12(in_kind, epi, rtile, a, s);
  if (link_kind == LINK_I16_R12) return launch_dslash_i16r12(in_kind, epi, rtile, a, s);
  if (link_kind == LINK_F64_F32) return launch_dslash_f64f32(in_kind, epi, rtile, a, s);
  return ASQ_EINVAL;
}

}  // namespace asq
