// Plain fp32 GlassNet forward on the vector ALUs (no matrix cores).
//
// One thread evaluates one pixel (Sec. 3.4: F, T, B and R are per-pixel
// networks here).  Weights are read with wave-uniform addresses, so they come
// through the scalar cache and feed the FMAs as scalar operands.  A layer's
// input vector is streamed 8 values at a time from a per-thread scratch area
// in HBM; outputs are produced 64 at a time in registers.  The pooled sum of
// Eq. (5) stays in registers across the slot loop.
//
// Two exact rewrites of the per-slot network h are used (real arithmetic is
// unchanged, only the rounding order):
//   * h's first layer on [b_i; sigma] splits into W1b*b_i + (W1s*sigma + c1),
//     and the sigma part is computed once per pixel instead of once per slot;
//   * h's last layer is affine, so the masked sum over slots moves in front of
//     it: sum_i m_i (A3 a_i + c3) = A3 (sum_i m_i a_i) + (sum_i m_i) c3.
#include "valu_mlp.h"

namespace gn {
namespace {

using namespace valu;

constexpr int kThreads = 256;
constexpr int kOB = 64;   // outputs per register block

struct Fp32Args {
  FwdBatch b;
  unsigned *amax;                // optional: max of h's first-layer activation (as bits)
  float *__restrict__ scr;       // [4][W][nthr]
  int nthr;
  int pool;
};

template <int W>
__global__ __launch_bounds__(kThreads) void fwd_fp32_kernel(
    // restrict-qualified kernel parameters: the weights are never written by
    // this kernel, which lets their wave-uniform loads use the scalar cache
    const float *__restrict__ wm, const float *__restrict__ wt, Fp32Args a) {
  LayerOff lo[kNumLayers];
  // offsets are compile-time functions of W; recomputed here to stay uniform
  {
    int64_t off = 0;
    const int outs[kNumLayers] = {W, W, W, W, W, W, W, W, W, W, W, kNOUT};
    const int ins[kNumLayers] = {kNG + kNS, W, W, kNL + W, W, W, 2 * W, W, W, W + 3, W, W};
#pragma unroll
    for (int l = 0; l < kNumLayers; ++l) {
      lo[l].w = off;
      off += (int64_t)outs[l] * ins[l];
      lo[l].b = off;
      off += outs[l];
      lo[l].out = outs[l];
      lo[l].in = ins[l];
    }
  }
  // wm: master copy (biases are read from it); wt: matrices transposed per layer
#define LDO(l) lo[l].out
  const int tid = blockIdx.x * kThreads + threadIdx.x;
  const int stride = a.nthr;
  const int hw = a.b.hw, K = a.b.k;
  const int64_t npx = (int64_t)a.b.n * hw;
  float zmax = 0.0f;

  for (int64_t base = (int64_t)blockIdx.x * kThreads; base < npx;
       base += (int64_t)gridDim.x * kThreads) {
    // wave-uniform loop: weight addresses stay scalar; the tail lanes of the
    // last block recompute the last pixel and do not store
    // Opaque copies of the bases, re-made every iteration, keep the compiler
    // from hoisting hundreds of derived addresses out of this loop: weight
    // offsets then fold into scalar-load immediates and scratch rows into one
    // scalar add per access.
    const float *wmp = wm, *wtp = wt;
    float *scr = a.scr;
    asm volatile("" : "+s"(wmp), "+s"(wtp), "+s"(scr));
    cfloat *wm_ = (cfloat *)wmp;
    cfloat *wt_ = (cfloat *)wtp;
    float *sS = scr + (size_t)0 * W * stride;   // sigma          [W][stride]
    float *sU = scr + (size_t)1 * W * stride;   // hoisted sigma part of h's layer 1
    float *sA = scr + (size_t)2 * W * stride;   // ping
    float *sB = scr + (size_t)3 * W * stride;   // pong
    const bool valid = base + threadIdx.x < npx;
    const int64_t pix = valid ? base + threadIdx.x : npx - 1;
    const int f = (int)(pix / hw);
    const int q = (int)(pix - (int64_t)f * hw);
    const float *G = a.b.gbuf + (size_t)f * kNG * hw + q;
    const float *Ls = a.b.layers + (size_t)f * K * kNL * hw + q;
    const float *S = a.b.scene + (size_t)f * kNS;

    // ---- F: [G; s] -> sigma
    {
      float x[kNG + kNS];
#pragma unroll
      for (int c = 0; c < kNG; ++c) x[c] = G[(size_t)c * hw];
#pragma unroll
      for (int c = 0; c < kNS; ++c) x[kNG + c] = S[c];
      for (int ob = 0; ob < W; ob += kOB) {
        float acc[kOB];
#pragma unroll
        for (int o = 0; o < kOB; ++o) acc[o] = wm_[lo[L_F1].b + ob + o];
        acc_from_regs<kOB, kNG + kNS>(acc, wt_ + lo[L_F1].w, W, ob, 0, x);
#pragma unroll
        for (int o = 0; o < kOB; ++o) sA[(size_t)(ob + o) * stride + tid] = relu(acc[o]);
      }
    }
    for (int ob = 0; ob < W; ob += kOB) {
      float acc[kOB];
#pragma unroll
      for (int o = 0; o < kOB; ++o) acc[o] = wm_[lo[L_F2].b + ob + o];
      acc_from_scratch<kOB, W>(acc, wt_ + lo[L_F2].w, LDO(L_F2), ob, 0, sA, stride, tid);
#pragma unroll
      for (int o = 0; o < kOB; ++o) sB[(size_t)(ob + o) * stride + tid] = relu(acc[o]);
    }
    for (int ob = 0; ob < W; ob += kOB) {
      float acc[kOB];
#pragma unroll
      for (int o = 0; o < kOB; ++o) acc[o] = wm_[lo[L_F3].b + ob + o];
      acc_from_scratch<kOB, W>(acc, wt_ + lo[L_F3].w, LDO(L_F3), ob, 0, sB, stride, tid);
#pragma unroll
      for (int o = 0; o < kOB; ++o) sS[(size_t)(ob + o) * stride + tid] = acc[o];
    }
    // ---- h's layer 1, sigma part, once per pixel: u = W1s sigma + c1
    for (int ob = 0; ob < W; ob += kOB) {
      float acc[kOB];
#pragma unroll
      for (int o = 0; o < kOB; ++o) acc[o] = wm_[lo[L_T1].b + ob + o];
      acc_from_scratch<kOB, W>(acc, wt_ + lo[L_T1].w, LDO(L_T1), ob, kNL, sS, stride, tid);
#pragma unroll
      for (int o = 0; o < kOB; ++o) sU[(size_t)(ob + o) * stride + tid] = acc[o];
    }
    // ---- slot loop, Eq. (5): Z = sum_i m_i relu(A2 relu(W1b b_i + u) + c2)
    float Z[W];
#pragma unroll
    for (int o = 0; o < W; ++o) Z[o] = 0.0f;
    float cnt = 0.0f;
    for (int i = 0; i < K; ++i) {
      float bi[kNL];
#pragma unroll
      for (int c = 0; c < kNL; ++c) bi[c] = Ls[((size_t)i * kNL + c) * hw];
      const float m = bi[kAlpha] > 0.0f ? 1.0f : 0.0f;
      for (int ob = 0; ob < W; ob += kOB) {
        float acc[kOB];
#pragma unroll
        for (int o = 0; o < kOB; ++o) acc[o] = sU[(size_t)(ob + o) * stride + tid];
        acc_from_regs<kOB, kNL>(acc, wt_ + lo[L_T1].w, LDO(L_T1), ob, 0, bi);
#pragma unroll
        for (int o = 0; o < kOB; ++o) sA[(size_t)(ob + o) * stride + tid] = relu(acc[o]);
        if (a.amax) {
#pragma unroll
          for (int o = 0; o < kOB; ++o) zmax = fmaxf(zmax, relu(acc[o]));
        }
      }
#pragma unroll
      for (int ob = 0; ob < W; ob += kOB) {
        float acc[kOB];
#pragma unroll
        for (int o = 0; o < kOB; ++o) acc[o] = wm_[lo[L_T2].b + ob + o];
        acc_from_scratch<kOB, W>(acc, wt_ + lo[L_T2].w, LDO(L_T2), ob, 0, sA, stride, tid);
#pragma unroll
        for (int o = 0; o < kOB; ++o) Z[ob + o] = fmaf(m, relu(acc[o]), Z[ob + o]);
      }
      cnt += m;
    }
    // ---- pool and h's last layer: tau = A3 (Z * inv) + bscale * c3
    const float inv = a.pool == GN_POOL_MEAN ? 1.0f / fmaxf(cnt, 1.0f) : 1.0f;
    const float bscale = a.pool == GN_POOL_MEAN ? (cnt > 0.0f ? 1.0f : 0.0f) : cnt;
#pragma unroll
    for (int o = 0; o < W; ++o) sB[(size_t)o * stride + tid] = Z[o] * inv;
    for (int ob = 0; ob < W; ob += kOB) {
      float acc[kOB];
#pragma unroll
      for (int o = 0; o < kOB; ++o) acc[o] = bscale * wm_[lo[L_T3].b + ob + o];
      acc_from_scratch<kOB, W>(acc, wt_ + lo[L_T3].w, LDO(L_T3), ob, 0, sB, stride, tid);
#pragma unroll
      for (int o = 0; o < kOB; ++o) sA[(size_t)(ob + o) * stride + tid] = acc[o];
    }
    // ---- B: [sigma; tau] -> phi
    for (int ob = 0; ob < W; ob += kOB) {
      float acc[kOB];
#pragma unroll
      for (int o = 0; o < kOB; ++o) acc[o] = wm_[lo[L_B1].b + ob + o];
      acc_from_scratch<kOB, W>(acc, wt_ + lo[L_B1].w, LDO(L_B1), ob, 0, sS, stride, tid);
      acc_from_scratch<kOB, W>(acc, wt_ + lo[L_B1].w, LDO(L_B1), ob, W, sA, stride, tid);
#pragma unroll
      for (int o = 0; o < kOB; ++o) sB[(size_t)(ob + o) * stride + tid] = relu(acc[o]);
    }
    for (int ob = 0; ob < W; ob += kOB) {
      float acc[kOB];
#pragma unroll
      for (int o = 0; o < kOB; ++o) acc[o] = wm_[lo[L_B2].b + ob + o];
      acc_from_scratch<kOB, W>(acc, wt_ + lo[L_B2].w, LDO(L_B2), ob, 0, sB, stride, tid);
#pragma unroll
      for (int o = 0; o < kOB; ++o) sA[(size_t)(ob + o) * stride + tid] = relu(acc[o]);
    }
    for (int ob = 0; ob < W; ob += kOB) {
      float acc[kOB];
#pragma unroll
      for (int o = 0; o < kOB; ++o) acc[o] = wm_[lo[L_B3].b + ob + o];
      acc_from_scratch<kOB, W>(acc, wt_ + lo[L_B3].w, LDO(L_B3), ob, 0, sA, stride, tid);
#pragma unroll
      for (int o = 0; o < kOB; ++o) sB[(size_t)(ob + o) * stride + tid] = acc[o];
    }
    // ---- R: [phi; L_d] -> radiance
    {
      float ld[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) ld[c] = G[(size_t)(11 + c) * hw];
      for (int ob = 0; ob < W; ob += kOB) {
        float acc[kOB];
#pragma unroll
        for (int o = 0; o < kOB; ++o) acc[o] = wm_[lo[L_R1].b + ob + o];
        acc_from_scratch<kOB, W>(acc, wt_ + lo[L_R1].w, LDO(L_R1), ob, 0, sB, stride, tid);
        acc_from_regs<kOB, 3>(acc, wt_ + lo[L_R1].w, LDO(L_R1), ob, W, ld);
#pragma unroll
        for (int o = 0; o < kOB; ++o) sA[(size_t)(ob + o) * stride + tid] = relu(acc[o]);
      }
    }
    for (int ob = 0; ob < W; ob += kOB) {
      float acc[kOB];
#pragma unroll
      for (int o = 0; o < kOB; ++o) acc[o] = wm_[lo[L_R2].b + ob + o];
      acc_from_scratch<kOB, W>(acc, wt_ + lo[L_R2].w, LDO(L_R2), ob, 0, sA, stride, tid);
#pragma unroll
      for (int o = 0; o < kOB; ++o) sB[(size_t)(ob + o) * stride + tid] = relu(acc[o]);
    }
    {
      float acc[kNOUT];
#pragma unroll
      for (int o = 0; o < kNOUT; ++o) acc[o] = wm_[lo[L_R3].b + o];
      acc_from_scratch<kNOUT, W>(acc, wt_ + lo[L_R3].w, LDO(L_R3), 0, 0, sB, stride, tid);
      float *O = a.b.out + (size_t)f * kNOUT * hw + q;
      if (valid) {
#pragma unroll
        for (int o = 0; o < kNOUT; ++o) O[(size_t)o * hw] = acc[o];
      }
    }
  }
  if (a.amax) atomicMax(a.amax, __float_as_uint(zmax));   // zmax >= 0: bit order = value order
}

}  // namespace

int fp32_scratch_threads(int num_cus) { return num_cus * kThreads; }

hipError_t launch_fwd_fp32(int W, int pool, const float *master, const float *master_t,
                           const FwdBatch &b,
                           float *scratch, int scratch_threads, hipStream_t stream,
                           unsigned *amax) {
  Fp32Args a;
  a.amax = amax;
  a.b = b;
  a.scr = scratch;
  a.nthr = scratch_threads;
  a.pool = pool;
  const int grid = scratch_threads / kThreads;
  if (W == 64)
    hipLaunchKernelGGL(fwd_fp32_kernel<64>, dim3(grid), dim3(kThreads), 0, stream, master, master_t, a);
  else if (W == 128)
    hipLaunchKernelGGL(fwd_fp32_kernel<128>, dim3(grid), dim3(kThreads), 0, stream, master, master_t, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace gn
#undef LDO
