// asq_solver.h -- interfaces between the CG driver and its vector/reduction kernels.
#pragma once
#include "asq_internal.h"

namespace asq {

enum ReduceOp { OP_INIT = 0, OP_ALPHA = 1, OP_BETA = 2, OP_RU = 3, OP_FINAL = 4 };
enum VecKernel { VK_INIT = 0, VK_XR = 1, VK_P = 2 };

struct VecArgs {
  int half;
  int nblk;
  const double* b;  // F64 right-hand sides
  double* x;        // F64 solutions
  void* r;          // iterated residual (RT tier)
  void* p;          // search direction (PT tier)
  void* Ap;         // A p (PT tier)
  ColState* st;
  double* partials;
};

int launch_vec_kernel(int which, int pt, int rt, const VecArgs& a, int ncol, hipStream_t s);
int launch_reduce(int op, ColState* st, const double* partials, int nblk, int ncol, hipStream_t s);

}  // namespace asq
