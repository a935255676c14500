// asq_solver.h -- interfaces between the CG driver and its vector/reduction kernels.
#pragma once
#include "asq_internal.h"

namespace asq {

enum VecKernel { VK_INIT = 0, VK_P = 2, VK_FLUSH = 3, VK_GUESS = 4 };

struct VecArgs {
  int half;
  int nblk;
  const double* b;  // F64 right-hand sides
  double* x;        // F64 solutions
  void* xs;         // F32 accumulator of the current reliable-update segment (nullptr: update x)
  void* r;          // iterated residual (RT tier)
  void* p;          // search directions (PT tier): two buffers, ColState::pbuf picks
  void* p_alt;
  ColState* st;
  double* partials;  // this kernel's partials ([ncol][nblk])
};

int launch_vec_kernel(int which, int pt, int rt, const VecArgs& a, int ncol, hipStream_t s);
int launch_reduce(int op, ColState* st, const double* pa, const double* pb, int nblk, int ncol, hipStream_t s);

}  // namespace asq
