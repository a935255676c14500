// dslash_i16.hip -- Dslash launches with 16-bit 12-real links with FP16-with-norm vectors (the three-level tier).
#include "dslash_impl.h"

namespace asq {

int launch_dslash_i16r12(int in_kind, int epi, int rtile, const DslashArgs& a, hipStream_t s) {
  if (in_kind != VEC_F16) return ASQ_EINVAL;
  if (epi == EPI_CANON) return pick_canon<LinkI16R12, VecF16C>(rtile, a, s);
  return pick_iter<LinkI16R12, VecF16, VecF32>(epi, rtile, a, s);
}

}  // namespace asq
