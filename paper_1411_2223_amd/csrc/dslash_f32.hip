// dslash_f32.hip -- Dslash launches with FP32 18-real links with FP32 or FP16-with-norm vectors.
#include "dslash_impl.h"
#include "dslash_mfma.h"

namespace asq {

int launch_dslash_f32r18(int in_kind, int epi, int rtile, const DslashArgs& a, hipStream_t s) {
  if (rtile & kMfmaBit) return in_kind == VEC_F16 ? pick_mfma(epi, rtile, a, s) : ASQ_EINVAL;
  if (epi == EPI_CANON) {
    if (in_kind == VEC_F32) return pick_canon<LinkF32R18, VecF32C>(rtile, a, s);
    if (in_kind == VEC_F16) return pick_canon<LinkF32R18, VecF16C>(rtile, a, s);
    return ASQ_EINVAL;
  }
  if (in_kind == VEC_F32) return pick_iter<LinkF32R18, VecF32, VecF32>(epi, rtile, a, s);
  if (in_kind == VEC_F16) return pick_iter<LinkF32R18, VecF16, VecF32>(epi, rtile, a, s);
  return ASQ_EINVAL;
}

}  // namespace asq
