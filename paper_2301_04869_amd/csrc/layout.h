// Layout of the per-line quantities shared by the symbolic layer (which builds
// gather lists into them) and the kernels (which write them).
#pragma once

#include <hip/hip_runtime.h>

namespace rkkt {

// per (scenario, line): end e in {0: from, 1: to} at offset 14*e holds
// P, Q, dP[4], dQ[4], d|S|^2[4] over the locals (th_f, th_t, v_f, v_t)
constexpr int kLVsize = 28;
constexpr int kLVP = 0, kLVQ = 1, kLVdP = 2, kLVdQ = 6, kLVdS = 10;
// per (scenario, line): upper triangle of the local 4x4 Hessian
constexpr int kLHsize = 10;

__host__ __device__ inline int lh_index(int a, int b) {  // a <= b
  return (a == 0 ? 0 : a == 1 ? 4 : a == 2 ? 7 : 9) + (b - a);
}

}  // namespace rkkt
