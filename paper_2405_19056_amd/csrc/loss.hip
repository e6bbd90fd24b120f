// L1 term of the training loss (Sec. 3.5): mean |y - t| and its subgradient.
// Deterministic two-pass reduction in fp32 (fixed partial count and order).
#include "gn_internal.h"

namespace gn {
namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void l1_partial_kernel(const float *__restrict__ y,
                                                              const float *__restrict__ t,
                                                              uint64_t n, float inv_n,
                                                              float *__restrict__ grad,
                                                              float *__restrict__ partials) {
  __shared__ float red[kThreads];
  float s = 0.0f;
  for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kThreads) {
    const float d = y[i] - t[i];
    s += fabsf(d);
    if (grad) grad[i] = d > 0.0f ? inv_n : (d < 0.0f ? -inv_n : 0.0f);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kThreads) void l1_final_kernel(const float *__restrict__ partials,
                                                            int npart, float inv_n,
                                                            float *__restrict__ loss) {
  __shared__ float red[kThreads];
  float s = 0.0f;
  for (int i = threadIdx.x; i < npart; i += kThreads) s += partials[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] * inv_n;
}

}  // namespace

hipError_t launch_l1(const float *out, const float *target, uint64_t count, float *loss,
                     float *grad, float *partials, int npart, hipStream_t stream) {
  const float inv_n = count ? 1.0f / (float)count : 0.0f;
  hipLaunchKernelGGL(l1_partial_kernel, dim3(npart), dim3(kThreads), 0, stream, out, target,
                     count, inv_n, grad, partials);
  hipLaunchKernelGGL(l1_final_kernel, dim3(1), dim3(kThreads), 0, stream, partials, npart, inv_n,
                     loss);
  return hipGetLastError();
}

}  // namespace gn
