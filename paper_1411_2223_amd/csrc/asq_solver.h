// asq_solver.h -- interfaces between the CG host loop and its vector/reduction kernels.
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
  // direction update only: with st_out set, beta of the previous iteration is
  // formed from beta_partials (its |r|^2 partials) and the finalised state is
  // written to st_out (st itself is only read)
  ColState* st_out = nullptr;
  const double* beta_partials = nullptr;
};

int launch_vec_kernel(int which, int pt, int rt, const VecArgs& a, int ncol, hipStream_t s);
// x[0..n) = hashed values in [-1, 1) (trial data for the autotuner).
int fill_trial_values(double* x, size_t n, hipStream_t s);
int launch_reduce(int op, ColState* st, const double* pa, const double* pb, int nblk, int ncol, hipStream_t s,
                  ColState* dst = nullptr);

}  // namespace asq
