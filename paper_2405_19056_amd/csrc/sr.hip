// x2 super-sampling network (Sec. 3.4, end; Sec. 4.1: GlassNet renders at the
// training resolution and a small CNN, fed by full-resolution G-buffers from
// the rasterizer, doubles it).  Layers: bilinear x2 of the render (half-pixel
// centres, clamped sources) joined with the 14 G-buffer planes, conv 3x3
// 17 -> 32 + ReLU, conv 3x3 32 -> 32 + ReLU, conv 1x1 32 -> 3, plus the
// upsampled render; 3x3 convs zero-padded to keep the size.
//
// One fused kernel per call, fp32 throughout.  A 256-thread block owns a
// 16 x 16 output tile: it stages the 17-channel input over the tile plus a
// two-pixel halo in LDS (upsampling on the fly), evaluates conv1 over the
// tile plus a one-pixel halo into LDS (zero outside the image, as conv2's
// padding requires), then each thread evaluates conv2, conv1x1 and the
// residual for its own pixel.  Weights are read at wave-uniform addresses
// (scalar loads, broadcast as instruction operands) from a copy re-laid so
// that the 32 output channels of one (input channel, tap) are contiguous.
#include <algorithm>

#include "gn_internal.h"

namespace gn {
namespace {

constexpr int kC = kSrWidth;          // hidden channels
constexpr int kIn = kSrIn;            // 3 upsampled + 14 G-buffer channels
constexpr int kT = 16;                // output tile edge
constexpr int kE0 = kT + 4;           // staged input edge (two-pixel halo)
constexpr int kE1 = kT + 2;           // conv1 output edge (one-pixel halo)
constexpr int kThreads = 256;
constexpr int kW1 = kIn * 9 * kC;     // re-laid conv1 weights [cin][tap][cout]
constexpr int kW2 = kC * 9 * kC;      // re-laid conv2 weights [cin][tap][cout]

static_assert(kT * kT == kThreads, "one output pixel per thread");

// packed [cout][cin][3][3] -> [cin][tap][cout] for both 3x3 convs; biases and
// the 1x1 head copied as they are.  Layout of wt: w1t, b1, w2t, b2, w3, b3.
__global__ __launch_bounds__(kThreads) void sr_relayout_kernel(const float *__restrict__ w,
                                                               float *__restrict__ wt) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= kSrParams) return;
  int dst = i;
  if (i < kW1) {
    const int o = i / (kIn * 9), r = i % (kIn * 9);  // r = cin * 9 + tap
    dst = r * kC + o;
  } else if (i >= kW1 + kC && i < kW1 + kC + kW2) {
    const int j = i - (kW1 + kC);
    const int o = j / (kC * 9), r = j % (kC * 9);
    dst = kW1 + kC + r * kC + o;
  }
  wt[dst] = w[i];
}

__global__ __launch_bounds__(kThreads, 2) void sr_forward_kernel(
    const float *__restrict__ wt, const float *__restrict__ lowres,
    const float *__restrict__ gbuf, float *__restrict__ out, int h, int w) {
  __shared__ float in_s[kIn * kE0 * kE0];   // 27.2 KB
  __shared__ float a1_s[kC * kE1 * kE1];    // 41.5 KB

  const int H = 2 * h, W = 2 * w;
  const int f = blockIdx.z;
  const int oy0 = blockIdx.y * kT, ox0 = blockIdx.x * kT;
  const int tid = threadIdx.x;
  const int64_t plane_lo = (int64_t)h * w, plane_hi = (int64_t)H * W;
  const float *lo_f = lowres + (int64_t)f * 3 * plane_lo;
  const float *g_f = gbuf + (int64_t)f * (kIn - 3) * plane_hi;

  // stage 0: the 17-channel input over the tile and a two-pixel halo
  for (int e = tid; e < kIn * kE0 * kE0; e += kThreads) {
    const int c = e / (kE0 * kE0), r = (e / kE0) % kE0, q = e % kE0;
    const int Y = oy0 - 2 + r, X = ox0 - 2 + q;
    float v = 0.0f;
    if (Y >= 0 && Y < H && X >= 0 && X < W) {
      if (c < 3) {
        // source position (Y + 0.5) / 2 - 0.5: row Y/2 - 1 at weight 1/4 for
        // even Y, row (Y-1)/2 at weight 3/4 for odd Y; likewise for columns
        const int y0 = (Y >> 1) - ((Y & 1) ? 0 : 1), x0 = (X >> 1) - ((X & 1) ? 0 : 1);
        const float fy = (Y & 1) ? 0.25f : 0.75f, fx = (X & 1) ? 0.25f : 0.75f;
        const int ya = max(y0, 0), yb = min(y0 + 1, h - 1);
        const int xa = max(x0, 0), xb = min(x0 + 1, w - 1);
        const float *p = lo_f + c * plane_lo;
        const float top = (1.0f - fx) * p[(int64_t)ya * w + xa] + fx * p[(int64_t)ya * w + xb];
        const float bot = (1.0f - fx) * p[(int64_t)yb * w + xa] + fx * p[(int64_t)yb * w + xb];
        v = (1.0f - fy) * top + fy * bot;
      } else {
        v = g_f[(c - 3) * plane_hi + (int64_t)Y * W + X];
      }
    }
    in_s[e] = v;
  }
  __syncthreads();

  // stage 1: conv1 + ReLU over the tile and a one-pixel halo (324 positions,
  // two passes of the block); zero where the position is outside the image
  const float *w1 = wt;
  const float *b1 = w1 + kW1;
  for (int q = tid; q < kE1 * kE1; q += kThreads) {
    const int qy = q / kE1, qx = q % kE1;
    float acc[kC];
#pragma unroll
    for (int o = 0; o < kC; ++o) acc[o] = b1[o];
    for (int c = 0; c < kIn; ++c) {
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const float v = in_s[c * kE0 * kE0 + (qy + t / 3) * kE0 + qx + t % 3];
        const float *wr = w1 + (c * 9 + t) * kC;
#pragma unroll
        for (int o = 0; o < kC; ++o) acc[o] = fmaf(wr[o], v, acc[o]);
      }
    }
    const int Y = oy0 - 1 + qy, X = ox0 - 1 + qx;
    const bool inside = Y >= 0 && Y < H && X >= 0 && X < W;
#pragma unroll
    for (int o = 0; o < kC; ++o) a1_s[o * kE1 * kE1 + q] = inside ? fmaxf(acc[o], 0.0f) : 0.0f;
  }
  __syncthreads();

  // stage 2: conv2 + ReLU, the 1x1 head and the residual, one pixel a thread
  const float *w2 = b1 + kC;
  const float *b2 = w2 + kW2;
  const float *w3 = b2 + kC;
  const float *b3 = w3 + kSrOut * kC;
  const int ty = tid / kT, tx = tid % kT;
  float acc[kC];
#pragma unroll
  for (int o = 0; o < kC; ++o) acc[o] = b2[o];
  for (int c = 0; c < kC; ++c) {
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const float v = a1_s[c * kE1 * kE1 + (ty + t / 3) * kE1 + tx + t % 3];
      const float *wr = w2 + (c * 9 + t) * kC;
#pragma unroll
      for (int o = 0; o < kC; ++o) acc[o] = fmaf(wr[o], v, acc[o]);
    }
  }
  const int Y = oy0 + ty, X = ox0 + tx;
  if (Y >= H || X >= W) return;
  float *out_f = out + (int64_t)f * kSrOut * plane_hi + (int64_t)Y * W + X;
#pragma unroll
  for (int k = 0; k < kSrOut; ++k) {
    float y = b3[k];
#pragma unroll
    for (int o = 0; o < kC; ++o) y = fmaf(w3[k * kC + o], fmaxf(acc[o], 0.0f), y);
    out_f[k * plane_hi] = in_s[k * kE0 * kE0 + (ty + 2) * kE0 + tx + 2] + y;
  }
}

}  // namespace

hipError_t launch_sr_forward(const float *w, float *wt, const float *lowres, const float *gbuf,
                             float *out, int n, int h, int w_lo, hipStream_t stream) {
  hipLaunchKernelGGL(sr_relayout_kernel, dim3((kSrParams + kThreads - 1) / kThreads),
                     dim3(kThreads), 0, stream, w, wt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)((2 * w_lo + kT - 1) / kT), (unsigned)((2 * h + kT - 1) / kT),
                  (unsigned)n);
  hipLaunchKernelGGL(sr_forward_kernel, grid, dim3(kThreads), 0, stream, wt, lowres, gbuf, out, h,
                     w_lo);
  return hipGetLastError();
}

}  // namespace gn
