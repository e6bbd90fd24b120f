// Vector-ALU building blocks of the fp32 per-pixel kernels (forward and
// backward): one thread per pixel, per-pixel vectors streamed from planes.
#pragma once

#include "gn_internal.h"

namespace gn {
namespace valu {

__device__ __forceinline__ float relu(float x) { return fmaxf(x, 0.0f); }

// Weights are read through the constant address space: the kernel never
// writes them, and wave-uniform loads from it go through the scalar cache.
typedef const float __attribute__((address_space(4))) cfloat;

// acc[o] (o < NB) += sum_k Wt[col0+k][row0+o] * src[k] for k < NIN, where Wt is
// a layer's matrix stored transposed ([in][out]) and src is streamed from the
// per-thread scratch with the given stride, one block of 8 ahead.
template <int NB, int NIN>
__device__ __forceinline__ void acc_from_scratch(float (&acc)[NB], cfloat *Wt,
                                                 int ldo, int row0, int col0,
                                                 const float *__restrict__ src, int stride,
                                                 int tid) {
  static_assert(NIN % 8 == 0, "streamed inputs come in blocks of 8");
  float x[8], xn[8];
#pragma unroll
  for (int kk = 0; kk < 8; ++kk) x[kk] = src[(size_t)kk * stride + tid];
  for (int kb = 0; kb < NIN; kb += 8) {
    if (kb + 8 < NIN) {
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) xn[kk] = src[(size_t)(kb + 8 + kk) * stride + tid];
    }
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      cfloat *wr = Wt + (size_t)(col0 + kb + kk) * ldo + row0;
#pragma unroll
      for (int o = 0; o < NB; ++o) acc[o] = fmaf(wr[o], x[kk], acc[o]);
      // keep one input row's weights (NB scalars) live at a time
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) x[kk] = xn[kk];
  }
}

template <int NB, int NIN>
__device__ __forceinline__ void acc_from_regs(float (&acc)[NB], cfloat *Wt,
                                              int ldo, int row0, int col0,
                                              const float (&x)[NIN]) {
#pragma unroll
  for (int k = 0; k < NIN; ++k) {
    cfloat *wr = Wt + (size_t)(col0 + k) * ldo + row0;
#pragma unroll
    for (int o = 0; o < NB; ++o) acc[o] = fmaf(wr[o], x[k], acc[o]);
    __builtin_amdgcn_sched_barrier(0);
  }
}

}  // namespace valu
}  // namespace gn
