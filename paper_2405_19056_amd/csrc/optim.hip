// Optimiser step of the training loop (Sec. 4: the networks are trained with
// Adam, Kingma & Ba, with a per-scene learning rate and weight decay).
// Weight decay enters as an L2 term added to the gradient before the moment
// updates.  Elementwise over the flat fp32 master vector (751 KB at W = 128):
// one grid-stride pass, HBM-bound and a few microseconds.
#include <algorithm>

#include "gn_internal.h"

namespace gn {
namespace {

constexpr int kThreads = 256;

// g' = g + wd w;  m = b1 m + (1 - b1) g';  v = b2 v + (1 - b2) g'^2;
// w -= lr (m c1) / (sqrt(v c2) + eps), with the bias corrections
// c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t).
__global__ __launch_bounds__(kThreads) void adam_kernel(float *__restrict__ w,
                                                        const float *__restrict__ g,
                                                        float *__restrict__ m,
                                                        float *__restrict__ v, int64_t n,
                                                        float lr, float b1, float b2, float eps,
                                                        float wd, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const float wi = w[i];
    const float gi = g[i] + wd * wi;
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] = wi - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  }
}

}  // namespace

hipError_t launch_adam(float *w, const float *g, float *m, float *v, int64_t n, float c1, float c2,
                       float lr, float b1, float b2, float eps, float wd, hipStream_t stream) {
  const int64_t blocks = std::min<int64_t>((n + kThreads - 1) / kThreads, 1024);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(kThreads), 0,
                     stream, w, g, m, v, n, lr, b1, b2, eps, wd, c1, c2);
  return hipGetLastError();
}

}  // namespace gn
