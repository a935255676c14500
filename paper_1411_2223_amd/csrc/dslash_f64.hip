// dslash_f64.hip -- Dslash launches with FP64 18-real links (the FP64 solver and the reliable update).
#include "dslash_impl.h"

namespace asq {

int launch_dslash_f64(int out_kind, int epi, int rtile, const DslashArgs& a, hipStream_t s) {
  if (epi == EPI_RESID) {
    if (out_kind == VEC_F64) return pick_r<LinkF64R18, VecF64, VecF64, EPI_RESID>(rtile, a, s);
    if (out_kind == VEC_F32) return pick_r<LinkF64R18, VecF64, VecF32, EPI_RESID>(rtile, a, s);
    return ASQ_EINVAL;
  }
  if (out_kind != VEC_F64) return ASQ_EINVAL;
  if (epi == EPI_CANON) return pick_canon<LinkF64R18, VecF64C>(rtile, a, s);
  return pick_iter<LinkF64R18, VecF64, VecF64>(epi, rtile, a, s);
}

}  // namespace asq
