// dslash_r12.hip -- Dslash launches with FP32 12-real links with FP32 or FP16-with-norm vectors.
#include "dslash_impl.h"

namespace asq {

int launch_dslash_f32r12(int in_kind, int epi, int rtile, const DslashArgs& a, hipStream_t s) {
  if (epi == EPI_CANON) {
    if (in_kind == VEC_F32) return pick_canon<LinkF32R12, VecF32C>(rtile, a, s);
    if (in_kind == VEC_F16) return pick_canon<LinkF32R12, VecF16C>(rtile, a, s);
    return ASQ_EINVAL;
  }
  if (in_kind == VEC_F32) return pick_iter<LinkF32R12, VecF32, VecF32>(epi, rtile, a, s);
  if (in_kind == VEC_F16) return pick_iter<LinkF32R12, VecF16, VecF32>(epi, rtile, a, s);
  return ASQ_EINVAL;
}

}  // namespace asq
