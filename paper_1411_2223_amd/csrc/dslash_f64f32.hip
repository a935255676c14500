// dslash_f64f32.hip -- Dslash launches that read FP64 18-real links and compute
// in FP32 (FP32 or FP16-with-norm vectors): the sloppy tier of a field kept in FP64 only.
#include "dslash_impl.h"

namespace asq {

int launch_dslash_f64f32(int in_kind, int epi, int rtile, const DslashArgs& a, hipStream_t s) {
  if (epi == EPI_CANON) {
    if (in_kind == VEC_F32) return pick_canon<LinkF64F32, VecF32C>(rtile, a, s);
    if (in_kind == VEC_F16) return pick_canon<LinkF64F32, VecF16C>(rtile, a, s);
    return ASQ_EINVAL;
  }
  if (in_kind == VEC_F32) return pick_iter<LinkF64F32, VecF32, VecF32>(epi, rtile, a, s);
  if (in_kind == VEC_F16) return pick_iter<LinkF64F32, VecF16, VecF32>(epi, rtile, a, s);
  return ASQ_EINVAL;
}

}  // namespace asq
