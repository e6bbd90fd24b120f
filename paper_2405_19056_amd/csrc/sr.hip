// x2 super-sampling network (Sec. 3.4, end; Sec. 4.1: GlassNet renders at the
// training resolution and a small CNN, fed by full-resolution G-buffers from
// the rasterizer, doubles it).  Layers: bilinear x2 of the render (half-pixel
// centres, clamped sources) joined with the 14 G-buffer planes, conv 3x3
// 17 -> 32 + ReLU, conv 3x3 32 -> 32 + ReLU, conv 1x1 32 -> 3, plus the
// upsampled render; 3x3 convs zero-padded to keep the size.
//
// One fused kernel per call, fp32 throughout, both 3x3 convs on the fp32
// matrix cores (16x16x4 MFMA) as implicit GEMMs with the weights as the
// 16-row operand (two tiles of 16 output channels) and 16 pixels as the
// columns.  A 256-thread block owns a 16 x 16 output tile:
//   stage 0  the 17-channel input over the tile plus a two-pixel halo into
//            LDS (upsampling on the fly; three zero channels pad K to 20 per
//            tap);
//   stage 1  conv1 + ReLU over the tile plus a one-pixel halo (324 positions,
//            21 column tiles of 16) into LDS, zero outside the image as
//            conv2's padding requires;
//   stage 2  conv2 + ReLU, one output row of 16 pixels per column tile, then
//            the 1x1 head: each lane holds 8 of the 32 channels of its pixel,
//            and two cross-lane sums complete the 3 outputs; plus the
//            upsampled render.
// The K order is tap-major (k = tap * C + channel), so each 4-wide K step
// reads four channels of one tap: an LDS address per lane that is a constant
// offset from a per-tile base.  The weights are re-laid once per call into
// the operand order of the MFMA (K step, channel tile, lane) so that each
// wave loads its fragments with coalesced loads into registers.
#include <algorithm>

#include "gn_internal.h"

namespace gn {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kC = kSrWidth;          // hidden channels
constexpr int kIn = kSrIn;            // 3 upsampled + 14 G-buffer channels
constexpr int kInP = 20;              // input channels padded to a multiple of 4
constexpr int kT = 16;                // output tile edge
constexpr int kE0 = kT + 4;           // staged input edge (two-pixel halo)
constexpr int kE1 = kT + 2;           // conv1 output edge (one-pixel halo)
constexpr int kP1 = kE1 * kE1;        // conv1 positions per tile (324)
constexpr int kA1Stride = 336;        // LDS floats per conv1 output channel
constexpr int kThreads = 256;
constexpr int kS1 = 9 * kInP / 4;     // conv1 K steps (45)
constexpr int kS2 = 9 * kC / 4;       // conv2 K steps (72)
constexpr int kN1 = (kP1 + 15) / 16;  // conv1 column tiles (21)
// re-laid weights: A1 [kS1][2][64], b1 [32], A2 [kS2][2][64], b2 [32],
// w3 [3][32], b3 [3], then for the backward A2T [kS2][2][64]: conv2's
// transpose (input and output channels swapped, taps mirrored)
constexpr int kOffB1 = kS1 * 2 * 64;
constexpr int kOffA2 = kOffB1 + kC;
constexpr int kOffB2 = kOffA2 + kS2 * 2 * 64;
constexpr int kOffW3 = kOffB2 + kC;
constexpr int kOffB3 = kOffW3 + kSrOut * kC;
constexpr int kOffA2T = kOffB3 + kSrOut;
static_assert(kOffA2T + kS2 * 2 * 64 == kSrWtFloats, "re-laid weight size");
static_assert(kA1Stride >= kP1 && kA1Stride % 64 == 16, "conv1 output channel stride");

// packed weights -> MFMA operand order.  Fragment (s, mt, lane): output
// channel 16 mt + lane % 16, K index 4 s + lane / 16 = tap * C + channel.
__global__ __launch_bounds__(kThreads) void sr_relayout_kernel(const float *__restrict__ w,
                                                               float *__restrict__ wt) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= kSrWtFloats) return;
  const float *w1 = w, *b1 = w1 + kC * kIn * 9, *w2 = b1 + kC, *b2 = w2 + kC * kC * 9;
  const float *w3 = b2 + kC, *b3 = w3 + kSrOut * kC;
  float v;
  if (i < kOffB1) {
    const int s = i / 128, mt = (i / 64) % 2, l = i % 64;
    const int k = 4 * s + l / 16, tap = k / kInP, c = k % kInP, o = 16 * mt + l % 16;
    v = c < kIn ? w1[(o * kIn + c) * 9 + tap] : 0.0f;
  } else if (i < kOffA2) {
    v = b1[i - kOffB1];
  } else if (i < kOffB2) {
    const int j = i - kOffA2;
    const int s = j / 128, mt = (j / 64) % 2, l = j % 64;
    const int k = 4 * s + l / 16, tap = k / kC, c = k % kC, o = 16 * mt + l % 16;
    v = w2[(o * kC + c) * 9 + tap];
  } else if (i < kOffW3) {
    v = b2[i - kOffB2];
  } else if (i < kOffB3) {
    v = w3[i - kOffW3];
  } else if (i < kOffA2T) {
    v = b3[i - kOffB3];
  } else {
    // fragment (s, mt, lane): input channel c = 16 mt + lane % 16 of conv2
    // (the transpose's output), K index 4 s + lane / 16 = tap * C + o
    const int j = i - kOffA2T;
    const int s = j / 128, mt = (j / 64) % 2, l = j % 64;
    const int k = 4 * s + l / 16, tap = k / kC, o = k % kC, c = 16 * mt + l % 16;
    v = w2[(o * kC + c) * 9 + (8 - tap)];
  }
  wt[i] = v;
}

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// LDS staging with many loads in flight: element e < N of a block goes to
// dst(e) from byte offset off(e) of the buffer behind r (kOutside, past the
// buffer's bound, reads zero: the callers' zero padding).  Loads guarded by a
// branch or followed by a select on their value are each waited for before
// the next one issues; these are neither, so the compiler issues a group of
// them before the first store.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr uint32_t kOutside = 0x80000000u;   // past every bound (buffers stay under 2 GiB)
__device__ __forceinline__ rsrc_t make_rsrc(const void *base, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0,
                                           (int)std::min<int64_t>(bytes, kOutside), 0x00020000);
}

template <int N, class Off, class Dst>
__device__ __forceinline__ void stage(int tid, rsrc_t r, Off off, Dst dst) {
  constexpr int kIt = (N + kThreads - 1) / kThreads, kG = 8;
  // groups of kG loads, then their kG stores (in program order: the
  // compiler does not move a buffer load above an LDS store)
  for (int i0 = 0; i0 < kIt; i0 += kG) {
    float v[kG];
#pragma unroll
    for (int j = 0; j < kG; ++j) {
      const int e = min(tid + (i0 + j) * kThreads, N - 1);
      v[j] = i0 + j < kIt
                 ? __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off(e), 0, 0))
                 : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < kG; ++j) {
      const int e = tid + (i0 + j) * kThreads;
      if (i0 + j < kIt && (N % kThreads == 0 || e < N)) *dst(e) = v[j];
    }
  }
}

// The render's 3 channels upsampled x2 into LDS over a square window of edge
// E at (y0, x0) of the output image: element e < 3 E^2 is channel e / E^2,
// row (e / E) % E, column e % E.  Output pixel (Y, X) samples source
// position (Y + 0.5) / 2 - 0.5: rows Y/2 - 1 and Y/2 at weights 1/4 and 3/4
// for even Y, rows (Y-1)/2 and (Y+1)/2 at 3/4 and 1/4 for odd Y (clamped
// into the image); likewise for columns.  Outside the image
// the four source offsets are past the buffer's bound, so the loads read
// zeros and the blend is zero; groups of 4 elements issue their 16 loads
// before any store.
template <int E>
__device__ __forceinline__ void stage_up(int tid, rsrc_t rlo, int h, int w, int y0, int x0,
                                         float *dst) {
  constexpr int N = 3 * E * E, kIt = (N + kThreads - 1) / kThreads, kG = 4;
  const int H = 2 * h, W = 2 * w;
  for (int i0 = 0; i0 < kIt; i0 += kG) {
    float v[kG][4], fx[kG], fy[kG];
#pragma unroll
    for (int j = 0; j < kG; ++j) {
      const int e = min(tid + (i0 + j) * kThreads, N - 1);
      const int c = e / (E * E), Y = y0 + (e / E) % E, X = x0 + e % E;
      const bool ok = i0 + j < kIt && Y >= 0 && Y < H && X >= 0 && X < W;
      const int sy = (Y >> 1) - ((Y & 1) ? 0 : 1), sx = (X >> 1) - ((X & 1) ? 0 : 1);
      fy[j] = (Y & 1) ? 0.25f : 0.75f;
      fx[j] = (X & 1) ? 0.25f : 0.75f;
      const int ya = max(sy, 0), yb = min(sy + 1, h - 1), xa = max(sx, 0), xb = min(sx + 1, w - 1);
      const uint32_t base = (uint32_t)(c * h * w);
      const uint32_t o[4] = {base + ya * w + xa, base + ya * w + xb, base + yb * w + xa,
                             base + yb * w + xb};
#pragma unroll
      for (int k = 0; k < 4; ++k)
        v[j][k] = __builtin_bit_cast(
            float, __builtin_amdgcn_raw_buffer_load_b32(rlo, ok ? 4 * o[k] : kOutside, 0, 0));
    }
#pragma unroll
    for (int j = 0; j < kG; ++j) {
      const int e = tid + (i0 + j) * kThreads;
      if (i0 + j < kIt && (N % kThreads == 0 || e < N)) {
        const float top = (1.0f - fx[j]) * v[j][0] + fx[j] * v[j][1];
        const float bot = (1.0f - fx[j]) * v[j][2] + fx[j] * v[j][3];
        dst[e] = (1.0f - fy[j]) * top + fy[j] * bot;
      }
    }
  }
}

// SAVE (the backward's recompute): instead of the output, write relu(z1) and
// relu(z2) of the tile's own pixels to a1_out, a2_out [n][32][2h][2w].
template <bool SAVE>
__global__ __launch_bounds__(kThreads, 2) void sr_forward_kernel(
    const float *__restrict__ wt, const float *__restrict__ lowres,
    const float *__restrict__ gbuf, float *__restrict__ out, int h, int w,
    float *__restrict__ a1_out, float *__restrict__ a2_out) {
  __shared__ float in_s[kInP * kE0 * kE0];   // 32.0 KB
  __shared__ float a1_s[kC * kA1Stride];     // 43.0 KB

  const int H = 2 * h, W = 2 * w;
  const int f = blockIdx.z;
  const int oy0 = blockIdx.y * kT, ox0 = blockIdx.x * kT;
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int col = lane % 16, grp = lane / 16;
  const int64_t plane_lo = (int64_t)h * w, plane_hi = (int64_t)H * W;
  const float *lo_f = lowres + (int64_t)f * 3 * plane_lo;
  const float *g_f = gbuf + (int64_t)f * (kIn - 3) * plane_hi;

  // stage 0: the input over the tile and a two-pixel halo (zero outside the
  // image and in the three padding channels)
  {
    constexpr int E2 = kE0 * kE0;
    auto inside = [&](int e) {
      const int Y = oy0 - 2 + (e / kE0) % kE0, X = ox0 - 2 + e % kE0;
      return Y >= 0 && Y < H && X >= 0 && X < W;
    };
    auto pix = [&](int e) {
      return (int64_t)(oy0 - 2 + (e / kE0) % kE0) * W + ox0 - 2 + e % kE0;
    };
    // the 14 G-buffer channels, the upsampled render, the padding channels
    const rsrc_t rg = make_rsrc(g_f, 4 * (kIn - 3) * plane_hi);
    stage<(kIn - 3) * E2>(
        tid, rg,
        [&](int e) {
          return inside(e) ? (uint32_t)(4 * ((e / E2) * plane_hi + pix(e))) : kOutside;
        },
        [&](int e) { return in_s + 3 * E2 + e; });
    stage_up<kE0>(tid, make_rsrc(lo_f, 4 * 3 * plane_lo), h, w, oy0 - 2, ox0 - 2, in_s);
    for (int e = tid; e < (kInP - kIn) * E2; e += kThreads) in_s[kIn * E2 + e] = 0.0f;
  }

  // stage 1: conv1 + ReLU over the tile and a one-pixel halo
  {
    float a[kS1][2];
#pragma unroll
    for (int s = 0; s < kS1; ++s) {
      a[s][0] = wt[(2 * s) * 64 + lane];
      a[s][1] = wt[(2 * s + 1) * 64 + lane];
    }
    float bias[2][4];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) bias[mt][i] = wt[kOffB1 + 16 * mt + 4 * grp + i];
    __syncthreads();
    for (int j = wave; j < kN1; j += kThreads / 64) {
      const int q = 16 * j + col;
      const int qq = min(q, kP1 - 1);  // the 12 columns past the last position are discarded
      const float *src = in_s + grp * kE0 * kE0 + (qq / kE1) * kE0 + qq % kE1;
      f32x4 acc0 = {0.0f, 0.0f, 0.0f, 0.0f}, acc1 = acc0;
#pragma unroll
      for (int s = 0; s < kS1; ++s) {
        const int tap = s / (kInP / 4), c4 = 4 * (s % (kInP / 4));
        const float b = src[c4 * kE0 * kE0 + (tap / 3) * kE0 + tap % 3];
        acc0 = mfma4(a[s][0], b, acc0);
        acc1 = mfma4(a[s][1], b, acc1);
      }
      if (q < kP1) {
        const int Y = oy0 - 1 + q / kE1, X = ox0 - 1 + q % kE1;
        const bool inside = Y >= 0 && Y < H && X >= 0 && X < W;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          a1_s[(4 * grp + i) * kA1Stride + q] = inside ? fmaxf(acc0[i] + bias[0][i], 0.0f) : 0.0f;
          a1_s[(16 + 4 * grp + i) * kA1Stride + q] =
              inside ? fmaxf(acc1[i] + bias[1][i], 0.0f) : 0.0f;
        }
      }
    }
  }
  __syncthreads();
  if (SAVE) {
    for (int e = tid; e < kC * kT * kT; e += kThreads) {
      const int o = e / (kT * kT), p = e % (kT * kT);
      const int Y = oy0 + p / kT, X = ox0 + p % kT;
      if (Y < H && X < W)
        a1_out[((int64_t)f * kC + o) * plane_hi + (int64_t)Y * W + X] =
            a1_s[o * kA1Stride + (p / kT + 1) * kE1 + p % kT + 1];
    }
  }

  // stage 2: conv2 + ReLU, the 1x1 head and the residual; one row per tile
  float a[kS2][2];
#pragma unroll
  for (int s = 0; s < kS2; ++s) {
    a[s][0] = wt[kOffA2 + (2 * s) * 64 + lane];
    a[s][1] = wt[kOffA2 + (2 * s + 1) * 64 + lane];
  }
  float bias[2][4], w3[kSrOut][2][4];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int o = 16 * mt + 4 * grp + i;
      bias[mt][i] = wt[kOffB2 + o];
#pragma unroll
      for (int k = 0; k < kSrOut; ++k) w3[k][mt][i] = wt[kOffW3 + k * kC + o];
    }
  const int kout = min(grp, kSrOut - 1);
  const float b3 = wt[kOffB3 + kout];
  for (int ty = wave; ty < kT; ty += kThreads / 64) {
    const float *src = a1_s + grp * kA1Stride + ty * kE1 + col;
    f32x4 acc0 = {0.0f, 0.0f, 0.0f, 0.0f}, acc1 = acc0;
#pragma unroll
    for (int s = 0; s < kS2; ++s) {
      const int tap = s / (kC / 4), c4 = 4 * (s % (kC / 4));
      const float b = src[c4 * kA1Stride + (tap / 3) * kE1 + tap % 3];
      acc0 = mfma4(a[s][0], b, acc0);
      acc1 = mfma4(a[s][1], b, acc1);
    }
    if (SAVE) {
      const int Y = oy0 + ty, X = ox0 + col;
      if (Y < H && X < W) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float *dst = a2_out + ((int64_t)f * kC + 4 * grp + i) * plane_hi + (int64_t)Y * W + X;
          dst[0] = fmaxf(acc0[i] + bias[0][i], 0.0f);
          dst[16 * plane_hi] = fmaxf(acc1[i] + bias[1][i], 0.0f);
        }
      }
      continue;
    }
    float y[kSrOut];
#pragma unroll
    for (int k = 0; k < kSrOut; ++k) {
      float p = 0.0f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        p = fmaf(w3[k][0][i], fmaxf(acc0[i] + bias[0][i], 0.0f), p);
        p = fmaf(w3[k][1][i], fmaxf(acc1[i] + bias[1][i], 0.0f), p);
      }
      p += __shfl_xor(p, 16);
      p += __shfl_xor(p, 32);
      y[k] = p;
    }
    // lanes of group k < 3 write output channel k of pixel col
    const int Y = oy0 + ty, X = ox0 + col;
    if (grp < kSrOut && Y < H && X < W) {
      const float yk = grp == 0 ? y[0] : (grp == 1 ? y[1] : y[2]);
      out[(int64_t)f * kSrOut * plane_hi + kout * plane_hi + (int64_t)Y * W + X] =
          in_s[kout * kE0 * kE0 + (ty + 2) * kE0 + col + 2] + b3 + yk;
    }
  }
}

// ---------------------------------------------------------------- backward
// The weight gradient of sum(dy * out), after a recompute of the forward that
// saves a1 = relu(z1) and a2 = relu(z2) (the masks z > 0 are a > 0):
//   dz2 = [a2 > 0] W3^T dy                       per pixel
//   dz1 = [a1 > 0] (conv2's transpose of dz2)    per pixel, 3x3 neighbourhood
//   dW3 = sum dy a2^T, dW2 = sum dz2 (a1 window)^T, dW1 = sum dz1 (x window)^T
// per persistent workgroup into one row of fp32 partials, then fp32 sums of
// those rows, in groups and then over the groups, each in a fixed order
// (deterministic).  The transposed conv and the two conv weight
// gradients run on the fp32 matrix cores; the rest is per-pixel vector work.

__global__ __launch_bounds__(kThreads) void sr_bwd_dz2_kernel(
    const float *__restrict__ w, const float *__restrict__ dy, const float *__restrict__ a2,
    float *__restrict__ dz2, int n, int64_t plane) {
  const float *w3 = w + kC * kIn * 9 + kC + kC * kC * 9 + kC;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n * plane;
       i += (int64_t)gridDim.x * kThreads) {
    const int64_t f = i / plane, p = i % plane;
    const float *d = dy + f * kSrOut * plane + p;
    const float d0 = d[0], d1 = d[plane], d2 = d[2 * plane];
#pragma unroll 4
    for (int o = 0; o < kC; ++o) {
      const int64_t at = (f * kC + o) * plane + p;
      const float g = fmaf(w3[o], d0, fmaf(w3[kC + o], d1, w3[2 * kC + o] * d2));
      dz2[at] = a2[at] > 0.0f ? g : 0.0f;
    }
  }
}

// dz1[c][Y][X] = [a1 > 0] sum_o sum_tap W2[o][c][tap] dz2[o][Y + 1 - ty][X + 1 - tx]:
// a zero-padded 3x3 correlation of dz2 with conv2's transpose (taps
// mirrored), on the matrix cores exactly as the forward's conv2: dz2 over the
// tile and a one-pixel halo in LDS, one output row per 16-pixel column tile.
__global__ __launch_bounds__(kThreads, 2) void sr_bwd_dz1_kernel(
    const float *__restrict__ wt, const float *__restrict__ dz2, const float *__restrict__ a1,
    float *__restrict__ dz1, int H, int W) {
  __shared__ float d_s[kC * kA1Stride];
  const int f = blockIdx.z, oy0 = blockIdx.y * kT, ox0 = blockIdx.x * kT;
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int col = lane % 16, grp = lane / 16;
  const int64_t plane = (int64_t)H * W;
  {
    const rsrc_t rd = make_rsrc(dz2 + (int64_t)f * kC * plane, 4 * kC * plane);
    stage<kC * kP1>(
        tid, rd,
        [&](int e) {
          const int o = e / kP1, q = e % kP1, Y = oy0 - 1 + q / kE1, X = ox0 - 1 + q % kE1;
          return Y >= 0 && Y < H && X >= 0 && X < W
                     ? (uint32_t)(4 * (o * plane + (int64_t)Y * W + X)) : kOutside;
        },
        [&](int e) { return d_s + (e / kP1) * kA1Stride + e % kP1; });
  }
  float a[kS2][2];
#pragma unroll
  for (int s = 0; s < kS2; ++s) {
    a[s][0] = wt[kOffA2T + (2 * s) * 64 + lane];
    a[s][1] = wt[kOffA2T + (2 * s + 1) * 64 + lane];
  }
  __syncthreads();
  for (int ty = wave; ty < kT; ty += kThreads / 64) {
    const float *src = d_s + grp * kA1Stride + ty * kE1 + col;
    f32x4 acc0 = {0.0f, 0.0f, 0.0f, 0.0f}, acc1 = acc0;
#pragma unroll
    for (int s = 0; s < kS2; ++s) {
      const int tap = s / (kC / 4), c4 = 4 * (s % (kC / 4));
      const float b = src[c4 * kA1Stride + (tap / 3) * kE1 + tap % 3];
      acc0 = mfma4(a[s][0], b, acc0);
      acc1 = mfma4(a[s][1], b, acc1);
    }
    const int Y = oy0 + ty, X = ox0 + col;
    if (Y < H && X < W) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t at = ((int64_t)f * kC + 4 * grp + i) * plane + (int64_t)Y * W + X;
        dz1[at] = a1[at] > 0.0f ? acc0[i] : 0.0f;
        dz1[at + 16 * plane] = a1[at + 16 * plane] > 0.0f ? acc1[i] : 0.0f;
      }
    }
  }
}

// Per-tile partial sums of every weight's gradient, in the packed order.
// The two conv gradients are GEMMs over the tile's 256 pixels on the matrix
// cores: dW[o][(c, tap)] = sum_p dz[o][p] act[c][p + tap], with dz (32 x 256)
// as the 16-row operand, held in registers, and the activation windows
// (columns (c, tap) in packed order, c * 9 + tap) gathered from LDS.  One
// more column reads a plane of ones: its sums are the bias gradients
// sum_p dz[o][p].
constexpr int kDzStride = kT * kT + 4;   // LDS row of dz: rows land in distinct banks
// floats: dz rows, the activation windows, the plane of ones (two workgroups per CU)
constexpr int kWgLds = kC * kDzStride + kC * kP1 + kP1;

// dz_s rows (32 x 256, stride kDzStride) against the windows of act_s
// (channels of kP1 floats, the tile plus a one-pixel halo) and, as column
// ncol, against ones_s, added to acc: column tile j = wave + 4 jj of 16.
template <int NJ>
__device__ __forceinline__ void wgrad_gemm(const float *dz_s, const float *act_s,
                                           const float *ones_s, int ncol, f32x4 (&acc)[NJ][2],
                                           int lane, int wave) {
  const int col = lane % 16, grp = lane / 16;
  // the wave's column tiles; a tile past the last column repeats the ones
  // column (its sums are never stored)
  const float *src[NJ];
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) {
    const int n = min(16 * (wave + (kThreads / 64) * jj) + col, ncol);
    const int c = n / 9, tap = n % 9;
    src[jj] = n == ncol ? ones_s + grp : act_s + c * kP1 + (tap / 3) * kE1 + tap % 3 + grp;
  }
#pragma unroll 4
  for (int s = 0; s < kT * kT / 4; ++s) {
    // pixel p = 4 s + grp: row s / 4, column 4 (s % 4) + grp
    const float a0 = dz_s[col * kDzStride + 4 * s + grp];
    const float a1 = dz_s[(16 + col) * kDzStride + 4 * s + grp];
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
      const float b = src[jj][(s / 4) * kE1 + 4 * (s % 4)];
      acc[jj][0] = mfma4(a0, b, acc[jj][0]);
      acc[jj][1] = mfma4(a1, b, acc[jj][1]);
    }
  }
}

// Column n < ncol to out[row * ncol + n], the ones column to bias[row].
template <int NJ>
__device__ __forceinline__ void wgrad_store(const f32x4 (&acc)[NJ][2], int ncol,
                                            float *__restrict__ out, float *__restrict__ bias,
                                            int lane, int wave) {
  const int col = lane % 16, grp = lane / 16;
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) {
    const int n = 16 * (wave + (kThreads / 64) * jj) + col;
    if (n > ncol) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float *d0 = n < ncol ? out + (4 * grp + i) * ncol + n : bias + 4 * grp + i;
      float *d1 = n < ncol ? out + (16 + 4 * grp + i) * ncol + n : bias + 16 + 4 * grp + i;
      *d0 = acc[jj][0][i];
      *d1 = acc[jj][1][i];
    }
  }
}

constexpr int kNJ2 = (kC * 9 / 16 + 1 + 3) / 4;    // conv2 column tiles (19) per wave (5)
constexpr int kNJ1 = (kIn * 9 + 1 + 15) / 16;      // conv1 column tiles (10)
constexpr int kNJ1w = (kNJ1 + 3) / 4;              // per wave (3)
static_assert((kC * 9 + 1 + 15) / 16 <= 4 * kNJ2, "conv2 columns and the ones column");

// Persistent: workgroup b takes tiles b, b + gridDim.x, ... (in that order)
// and keeps its running sums of every weight gradient in registers, written
// once to partial[b].
__global__ __launch_bounds__(kThreads, 2) void sr_bwd_wgrad_kernel(
    const float *__restrict__ lowres, const float *__restrict__ gbuf, const float *__restrict__ dy,
    const float *__restrict__ a1, const float *__restrict__ a2, const float *__restrict__ dz1,
    const float *__restrict__ dz2, float *__restrict__ partial, int n, int h, int w) {
  __shared__ float buf[kWgLds];   // 76.1 KB
  const int H = 2 * h, W = 2 * w;
  const int tx_n = (W + kT - 1) / kT, ty_n = (H + kT - 1) / kT;
  const int ntiles = n * tx_n * ty_n;
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int col = lane % 16, grp = lane / 16;
  const int64_t plane = (int64_t)H * W, plane_lo = (int64_t)h * w;
  constexpr int kOffW2 = kC * kIn * 9 + kC, kOffB2p = kOffW2 + kC * kC * 9;
  constexpr int kOffW3p = kOffB2p + kC, kOffB3p = kOffW3p + kSrOut * kC;
  f32x4 acc2[kNJ2][2] = {}, acc1[kNJ1w][2] = {};
  // the head on waves 0..2: column tile `wave` of [a2^T | 1] against dy
  f32x4 acc_h = {0.f, 0.f, 0.f, 0.f};
  float *dz_s = buf, *ones_s = buf + kC * kDzStride + kC * kP1;
  for (int e = tid; e < kP1; e += kThreads) ones_s[e] = 1.0f;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int f = t / (tx_n * ty_n), oy0 = ((t / tx_n) % ty_n) * kT, ox0 = (t % tx_n) * kT;
    // plane offsets of the tile's own pixel p and of halo position q (clamped
    // into the image), and whether they lie inside it
    // byte offsets of channel c at the tile's own pixel p and at halo
    // position q within frame f's planes; kOutside outside the image
    auto own = [&](int c, int p) {
      const int Y = oy0 + p / kT, X = ox0 + p % kT;
      return Y < H && X < W ? (uint32_t)(4 * (c * plane + (int64_t)Y * W + X)) : kOutside;
    };
    auto halo = [&](int c, int q) {
      const int Y = oy0 - 1 + q / kE1, X = ox0 - 1 + q % kE1;
      return Y >= 0 && Y < H && X >= 0 && X < W ? (uint32_t)(4 * (c * plane + (int64_t)Y * W + X))
                                                : kOutside;
    };
    const int64_t fb = 4 * kC * plane;   // bytes of one frame's 32 planes
    // phase 0: the head, dW3[k][o] = sum_p dy[k][p] a2[o][p] and b3[k] =
    // sum_p dy[k][p] on the matrix cores: dy (3 rows of 16) the row operand,
    // [a2^T | 1] (33 of 48 columns) the column operand, over the tile's own
    // pixels (zero outside the image).  a2_s [32][256], dy_s [3][256].
    {
      float *a2_s = buf, *dy_s = buf + kC * kT * kT;
      constexpr int P = kT * kT;
      stage<kC * P>(tid, make_rsrc(a2 + (int64_t)f * kC * plane, fb),
                    [&](int e) { return own(e / P, e % P); }, [&](int e) { return a2_s + e; });
      stage<kSrOut * P>(tid, make_rsrc(dy + (int64_t)f * kSrOut * plane, 4 * kSrOut * plane),
                        [&](int e) { return own(e / P, e % P); }, [&](int e) { return dy_s + e; });
      __syncthreads();
      if (wave < 3) {
        const int nc = 16 * wave + col;            // column: a2 channel, 32 = ones
#pragma unroll 8
        for (int s = 0; s < kT * kT / 4; ++s) {
          const int p = 4 * s + grp;
          const float av = col < kSrOut ? dy_s[col * kT * kT + p] : 0.0f;
          const float bv = nc < kC ? a2_s[nc * kT * kT + p] : (nc == kC ? 1.0f : 0.0f);
          acc_h = mfma4(av, bv, acc_h);
        }
      }
      __syncthreads();
    }
    // phase A: conv2.  dz_s [32][256] = dz2 over the tile's own pixels and
    // act_s [32][18][18] = a1 over the tile and a one-pixel halo; zero
    // outside the image.
    float *act_s = buf + kC * kDzStride;
    constexpr int P = kT * kT;
    stage<kC * P>(tid, make_rsrc(dz2 + (int64_t)f * kC * plane, fb),
                  [&](int e) { return own(e / P, e % P); },
                  [&](int e) { return dz_s + (e / P) * kDzStride + e % P; });
    stage<kC * kP1>(tid, make_rsrc(a1 + (int64_t)f * kC * plane, fb),
                    [&](int e) { return halo(e / kP1, e % kP1); }, [&](int e) { return act_s + e; });
    __syncthreads();
    wgrad_gemm<kNJ2>(dz_s, act_s, ones_s, kC * 9, acc2, lane, wave);
    __syncthreads();
    // phase B: conv1.  dz_s = dz1 over the tile's own pixels, x_s
    // [17][18][18] = the input over the tile and a one-pixel halo.
    float *x_s = buf + kC * kDzStride;
    stage<kC * P>(tid, make_rsrc(dz1 + (int64_t)f * kC * plane, fb),
                  [&](int e) { return own(e / P, e % P); },
                  [&](int e) { return dz_s + (e / P) * kDzStride + e % P; });
    // the 14 G-buffer channels, then the upsampled render
    stage<(kIn - 3) * kP1>(tid, make_rsrc(gbuf + (int64_t)f * (kIn - 3) * plane,
                                          4 * (kIn - 3) * plane),
                           [&](int e) { return halo(e / kP1, e % kP1); },
                           [&](int e) { return x_s + 3 * kP1 + e; });
    stage_up<kE1>(tid, make_rsrc(lowres + (int64_t)f * 3 * plane_lo, 4 * 3 * plane_lo), h, w,
                  oy0 - 1, ox0 - 1, x_s);
    __syncthreads();
    wgrad_gemm<kNJ1w>(dz_s, x_s, ones_s, kIn * 9, acc1, lane, wave);
    __syncthreads();
  }
  float *out = partial + (int64_t)blockIdx.x * kSrParams;
  wgrad_store<kNJ2>(acc2, kC * 9, out + kOffW2, out + kOffB2p, lane, wave);
  wgrad_store<kNJ1w>(acc1, kIn * 9, out, out + kC * kIn * 9, lane, wave);
  // head: lane (col, grp) holds rows 4 grp + i (outputs k) of column 16 wave + col
  if (wave < 3 && grp == 0) {
    const int nc = 16 * wave + col;
#pragma unroll
    for (int i = 0; i < kSrOut; ++i) {
      if (nc < kC) out[kOffW3p + i * kC + nc] = acc_h[i];
      else if (nc == kC) out[kOffB3p + i] = acc_h[i];
    }
  }
}

// grad_w[i] = sum over rows of partial[row][i] in fp32, in two fixed-order
// stages (deterministic): groups of kRedGroup consecutive rows, then the
// groups in order.
constexpr int kRedGroup = 64;

__global__ __launch_bounds__(kThreads) void sr_bwd_group_sum_kernel(
    const float *__restrict__ partial, int tiles, float *__restrict__ groups) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= kSrParams) return;
  const int t0 = blockIdx.y * kRedGroup, t1 = min(t0 + kRedGroup, tiles);
  float s = 0.0f;
  for (int t = t0; t < t1; ++t) s += partial[(int64_t)t * kSrParams + i];
  groups[(int64_t)blockIdx.y * kSrParams + i] = s;
}

__global__ __launch_bounds__(kThreads) void sr_bwd_reduce_kernel(const float *__restrict__ groups,
                                                                 int ngroups, float *__restrict__ gw) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= kSrParams) return;
  float s = 0.0f;
  for (int g = 0; g < ngroups; ++g) s += groups[(int64_t)g * kSrParams + i];
  gw[i] = s;
}

}  // namespace

hipError_t launch_sr_forward(const float *w, float *wt, const float *lowres, const float *gbuf,
                             float *out, int n, int h, int w_lo, hipStream_t stream) {
  hipLaunchKernelGGL(sr_relayout_kernel, dim3((kSrWtFloats + kThreads - 1) / kThreads),
                     dim3(kThreads), 0, stream, w, wt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)((2 * w_lo + kT - 1) / kT), (unsigned)((2 * h + kT - 1) / kT),
                  (unsigned)n);
  hipLaunchKernelGGL(sr_forward_kernel<false>, grid, dim3(kThreads), 0, stream, wt, lowres, gbuf,
                     out, h, w_lo, nullptr, nullptr);
  return hipGetLastError();
}

// Persistent workgroups of the weight-gradient kernel (two per CU).
constexpr int kWgBlocks = 512;

static int64_t wgrad_blocks(int n, int h, int w) {
  const int64_t tiles = (int64_t)n * ((2 * h + kT - 1) / kT) * ((2 * w + kT - 1) / kT);
  return std::min<int64_t>(tiles, kWgBlocks);
}

size_t sr_backward_workspace_bytes(int n, int h, int w) {
  const int64_t px = (int64_t)n * 4 * h * w;
  const int64_t rows = wgrad_blocks(n, h, w);
  const int64_t groups = (rows + kRedGroup - 1) / kRedGroup;
  return sizeof(float) * (size_t)(4 * kC * px + (rows + groups) * kSrParams);
}

hipError_t launch_sr_backward(const float *w, float *wt, const float *lowres, const float *gbuf,
                              const float *dy, float *gw, int n, int h, int w_lo, float *ws,
                              hipStream_t stream) {
  const int H = 2 * h, W = 2 * w_lo;
  const int64_t plane = (int64_t)H * W, px = (int64_t)n * plane;
  float *a1 = ws, *a2 = a1 + kC * px, *dz2 = a2 + kC * px, *dz1 = dz2 + kC * px;
  float *partial = dz1 + kC * px;
  hipLaunchKernelGGL(sr_relayout_kernel, dim3((kSrWtFloats + kThreads - 1) / kThreads),
                     dim3(kThreads), 0, stream, w, wt);
  const dim3 tiles((unsigned)((W + kT - 1) / kT), (unsigned)((H + kT - 1) / kT), (unsigned)n);
  hipLaunchKernelGGL(sr_forward_kernel<true>, tiles, dim3(kThreads), 0, stream, wt, lowres, gbuf,
                     nullptr, h, w_lo, a1, a2);
  const int64_t pb = std::min<int64_t>((px + kThreads - 1) / kThreads, 4096);
  hipLaunchKernelGGL(sr_bwd_dz2_kernel, dim3((unsigned)pb), dim3(kThreads), 0, stream, w, dy, a2,
                     dz2, n, plane);
  hipLaunchKernelGGL(sr_bwd_dz1_kernel, tiles, dim3(kThreads), 0, stream, wt, dz2, a1, dz1, H, W);
  // persistent workgroups; each writes one row of partial sums
  const int nblocks = (int)wgrad_blocks(n, h, w_lo);
  hipLaunchKernelGGL(sr_bwd_wgrad_kernel, dim3((unsigned)nblocks), dim3(kThreads), 0, stream,
                     lowres, gbuf, dy, a1, a2, dz1, dz2, partial, n, h, w_lo);
  const int ngroups = (nblocks + kRedGroup - 1) / kRedGroup;
  // the group sums follow the partials
  float *groups = partial + (int64_t)nblocks * kSrParams;
  const unsigned pblocks = (kSrParams + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(sr_bwd_group_sum_kernel, dim3(pblocks, (unsigned)ngroups), dim3(kThreads), 0,
                     stream, partial, nblocks, groups);
  hipLaunchKernelGGL(sr_bwd_reduce_kernel, dim3(pblocks), dim3(kThreads), 0, stream, groups,
                     ngroups, gw);
  return hipGetLastError();
}

}  // namespace gn
