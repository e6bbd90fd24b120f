// L1 term of the training loss (Sec. 3.5): mean |y - t| and its subgradient.
// Deterministic two-pass reduction in fp32 (fixed partial count and order).
#include <cmath>

#include <mutex>

#include "gn_internal.h"

namespace gn {
namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void l1_partial_kernel(const float *__restrict__ y,
                                                              const float *__restrict__ t,
                                                              uint64_t n, float inv_n,
                                                              const float *__restrict__ gscale,
                                                              float *__restrict__ grad,
                                                              float *__restrict__ partials) {
  __shared__ float red[kThreads];
  float s = 0.0f;
  // the gradient's upstream factor (a device scalar) folded into 1 / n
  const float gn = gscale ? inv_n * *gscale : inv_n;
  for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kThreads) {
    const float d = y[i] - t[i];
    s += fabsf(d);
    if (grad) grad[i] = d > 0.0f ? gn : (d < 0.0f ? -gn : 0.0f);
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

// ---- structural dissimilarity (DSSIM) ----------------------------------------
// SSIM of Wang et al. (11 x 11 Gaussian window, every fully contained window)
// per channel; the loss term is (1 - mean SSIM) / 2.  A 16 x 16 tile of
// windows (or of pixels, for the gradient) per workgroup, its 26 x 26 input
// patch in LDS; the separable window is applied as two 11-tap passes.
constexpr int kWin = 11, kTile = 16, kPatch = kTile + kWin - 1;

struct Gauss {
  float g[kWin];     // 1-D weights, sum 1 (the window is their outer product)
};

// Per window p: S_p and its partial derivatives with respect to the local
// mean of x, of x^2 and of x y (a, b, c maps: [3][planes][hm][wm]); one
// partial sum of S per workgroup.
__global__ __launch_bounds__(256) void ssim_fwd_kernel(const float *__restrict__ x,
                                                       const float *__restrict__ y, int h, int w,
                                                       float C1, float C2, Gauss gs,
                                                       float *__restrict__ coef, int64_t plane_m,
                                                       float *__restrict__ partials) {
  __shared__ float px[kPatch][kPatch], py[kPatch][kPatch];
  __shared__ float hm[5][kPatch][kTile];
  __shared__ float red[256];
  const int hm_ = h - kWin + 1, wm = w - kWin + 1;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int c0 = blockIdx.x * kTile, r0 = blockIdx.y * kTile, pl = blockIdx.z;
  const float *X = x + (size_t)pl * h * w, *Y = y + (size_t)pl * h * w;
  for (int i = threadIdx.x; i < kPatch * kPatch; i += 256) {
    const int r = i / kPatch, c = i - r * kPatch, gr = r0 + r, gc = c0 + c;
    const bool in = gr < h && gc < w;
    px[r][c] = in ? X[(size_t)gr * w + gc] : 0.0f;
    py[r][c] = in ? Y[(size_t)gr * w + gc] : 0.0f;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kPatch * kTile; i += 256) {
    const int r = i / kTile, c = i - r * kTile;
    float s[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < kWin; ++j) {
      const float a = px[r][c + j], b = py[r][c + j], g = gs.g[j];
      s[0] += g * a;
      s[1] += g * b;
      s[2] += g * a * a;
      s[3] += g * b * b;
      s[4] += g * a * b;
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) hm[k][r][c] = s[k];
  }
  __syncthreads();
  float m[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < kWin; ++i)
#pragma unroll
    for (int k = 0; k < 5; ++k) m[k] += gs.g[i] * hm[k][ty + i][tx];
  const int pr = r0 + ty, pc = c0 + tx;
  float S = 0.0f;
  if (pr < hm_ && pc < wm) {
    const float mx = m[0], my = m[1];
    const float A1 = 2.0f * mx * my + C1, A2 = 2.0f * (m[4] - mx * my) + C2;
    const float B1 = mx * mx + my * my + C1, B2 = (m[2] - mx * mx) + (m[3] - my * my) + C2;
    S = (A1 * A2) / (B1 * B2);
    const size_t o = (size_t)pl * hm_ * wm + (size_t)pr * wm + pc;
    coef[o] = S * (2.0f * my / A1 - 2.0f * my / A2 - 2.0f * mx / B1 + 2.0f * mx / B2);
    coef[plane_m + o] = -S / B2;
    coef[2 * plane_m + o] = 2.0f * S / A2;
  }
  red[threadIdx.x] = S;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    partials[((size_t)pl * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = red[0];
}

// grad[q] (+)= scale (A_q + 2 x_q B_q + y_q C_q), where A, B, C are the a, b,
// c maps spread back over each window's pixels by its weights:
// A_q = sum_{i,j} G[i][j] a_{q - (i, j)} over windows inside the map.
__global__ __launch_bounds__(256) void ssim_bwd_kernel(const float *__restrict__ x,
                                                       const float *__restrict__ y, int h, int w,
                                                       Gauss gs, const float *__restrict__ coef,
                                                       int64_t plane_m, float scale,
                                                       float *__restrict__ grad, int accumulate) {
  __shared__ float pc_[3][kPatch][kPatch];
  __shared__ float hs[3][kPatch][kTile];
  const int hm_ = h - kWin + 1, wm = w - kWin + 1;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int c0 = blockIdx.x * kTile, r0 = blockIdx.y * kTile, pl = blockIdx.z;
  // map positions r0 - 10 .. r0 + 15 (rows) and c0 - 10 .. c0 + 15 (columns)
  for (int i = threadIdx.x; i < kPatch * kPatch; i += 256) {
    const int r = i / kPatch, c = i - r * kPatch;
    const int mr = r0 - (kWin - 1) + r, mc = c0 - (kWin - 1) + c;
    const bool in = mr >= 0 && mr < hm_ && mc >= 0 && mc < wm;
    const size_t o = (size_t)pl * hm_ * wm + (size_t)(in ? mr : 0) * wm + (in ? mc : 0);
#pragma unroll
    for (int k = 0; k < 3; ++k) pc_[k][r][c] = in ? coef[k * plane_m + o] : 0.0f;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kPatch * kTile; i += 256) {
    const int r = i / kTile, c = i - r * kTile;
    float s[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < kWin; ++j) {
      const float g = gs.g[j];
#pragma unroll
      for (int k = 0; k < 3; ++k) s[k] += g * pc_[k][r][c + kWin - 1 - j];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) hs[k][r][c] = s[k];
  }
  __syncthreads();
  float v[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < kWin; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] += gs.g[i] * hs[k][ty + kWin - 1 - i][tx];
  const int qr = r0 + ty, qc = c0 + tx;
  if (qr >= h || qc >= w) return;
  const size_t o = (size_t)pl * h * w + (size_t)qr * w + qc;
  const float d = scale * (v[0] + 2.0f * x[o] * v[1] + y[o] * v[2]);
  grad[o] = accumulate ? grad[o] + d : d;
}

// loss = (1 - sum(partials) / count) / 2, summed in fp32 in a fixed order
// (a strided sum per thread, then a tree): deterministic.
__global__ __launch_bounds__(256) void ssim_final_kernel(const float *__restrict__ partials,
                                                         int64_t npart, float inv_count,
                                                         float *__restrict__ loss) {
  __shared__ float red[256];
  float s = 0.0f;
  for (int64_t i = threadIdx.x; i < npart; i += 256) s += partials[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (1.0f - red[0] * inv_count) * 0.5f;
}

}  // namespace

size_t dssim_workspace_bytes(int planes, int h, int w) {
  const int64_t hm = h - kWin + 1, wm = w - kWin + 1;
  const int64_t blocks = (int64_t)planes * ((hm + kTile - 1) / kTile) * ((wm + kTile - 1) / kTile);
  return sizeof(float) * (size_t)(3 * planes * hm * wm + blocks);
}

hipError_t launch_dssim(const float *out, const float *target, int planes, int h, int w,
                        float *loss, float *grad, int accumulate, float *ws, hipStream_t stream) {
  Gauss gs;
  float e[kWin], z = 0.0f;
  for (int i = 0; i < kWin; ++i) {
    const float r = (float)i - (kWin - 1) / 2.0f;
    e[i] = std::exp(-r * r / (2.0f * 1.5f * 1.5f));
    z += e[i];
  }
  for (int i = 0; i < kWin; ++i) gs.g[i] = e[i] / z;
  const float C1 = 0.01f * 0.01f, C2 = 0.03f * 0.03f;     // (K L)^2 with L = 1
  const int hm = h - kWin + 1, wm = w - kWin + 1;
  const int64_t plane_m = (int64_t)planes * hm * wm;
  float *coef = ws, *partials = ws + 3 * plane_m;
  const dim3 gm((wm + kTile - 1) / kTile, (hm + kTile - 1) / kTile, planes);
  hipLaunchKernelGGL(ssim_fwd_kernel, gm, dim3(256), 0, stream, out, target, h, w, C1, C2, gs,
                     coef, plane_m, partials);
  const int64_t npart = (int64_t)gm.x * gm.y * gm.z;
  hipLaunchKernelGGL(ssim_final_kernel, dim3(1), dim3(256), 0, stream, partials, npart,
                     1.0f / (float)plane_m, loss);
  if (grad) {
    const dim3 gp((w + kTile - 1) / kTile, (h + kTile - 1) / kTile, planes);
    hipLaunchKernelGGL(ssim_bwd_kernel, gp, dim3(256), 0, stream, out, target, h, w, gs, coef,
                       plane_m, -0.5f / (float)plane_m, grad, accumulate);
  }
  return hipGetLastError();
}

// ---- the DSSIM term's allocation-free form ---------------------------------
// A fixed device array serves as the DSSIM workspace for callers that cannot
// allocate (graph capture, serving loops).  Each GPU holds its own copy for
// the life of the process; its device address is looked up once per device
// (host code never passes the array's name to a kernel).  Every call on a GPU
// shares that copy: calls that overlap on one GPU race.  Nothing in it needs
// clearing: each launch writes every coefficient and partial it reads.
static __device__ __align__(256) float scratch[kDssimScratchBytes / sizeof(float)];

namespace {
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t dssim_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = (float *)p;
  return hipSuccess;
}

float *dssim_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

hipError_t launch_l1(const float *out, const float *target, uint64_t count, float *loss,
                     float *grad, const float *grad_scale, float *partials, int npart,
                     hipStream_t stream) {
  const float inv_n = count ? 1.0f / (float)count : 0.0f;
  hipLaunchKernelGGL(l1_partial_kernel, dim3(npart), dim3(kThreads), 0, stream, out, target,
                     count, inv_n, grad_scale, grad, partials);
  hipLaunchKernelGGL(l1_final_kernel, dim3(1), dim3(kThreads), 0, stream, partials, npart, inv_n,
                     loss);
  return hipGetLastError();
}

}  // namespace gn
