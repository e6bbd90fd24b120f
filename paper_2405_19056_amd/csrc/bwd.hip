// Hand-written backward of GlassNet's per-pixel evaluation (Sec. 3.5 trains
// F, T, B and R jointly end to end; this is dL/dw for a given dL/dy).
//
// Data flow (all fp32):
//   1. fwd_save:  recompute the forward per pixel and keep every per-pixel
//                 activation the gradient needs as a plane [row][pixel]
//                 (G/scene inputs, F's hidden layers, sigma, u, the pooled
//                 Z/max(c,1), tau, B's and R's hidden layers).  The per-slot
//                 activations of h are NOT kept.
//   2. head:      dy -> R -> B -> (dsigma from B, dtau) -> dZ through h's
//                 last layer and the pool.
//   3. slot i:    one transparency layer at a time, recompute z1_i, z2_i from
//                 (b_i, u), backprop through h's layers 2 and 1, add into du,
//                 and accumulate dW of those two layers over pixels.  Only one
//                 slot's activations exist at any time, so memory does not
//                 grow with the slot count (the streaming sum of Eq. (5)).
//   4. tail:      dsigma += A1s^T du, then F's layers.
//   5. dW:        each layer's weight gradient sum_p delta_p a_p^T is a GEMM
//                 with K = pixels on the fp32 matrix cores (16x16x4), split
//                 over pixel chunks; partials are reduced in a fixed order
//                 (deterministic, no atomics).  Bias gradients come from a row
//                 of ones appended to each activation block.
#include "gn_api_state.h"
#include "valu_mlp.h"

namespace gn {

struct BwdWorkspace {
  int W = 0;
  int64_t cap_px = 0;        // plane row length (padded pixel count)
  int64_t stride = -1;       // row length the constant rows were written for
  float *planes = nullptr;
  size_t plane_bytes = 0;
  float *part = nullptr;     // generic GEMM partials
  float *part_t2 = nullptr;  // h layer 2 partials (accumulated over slots)
  float *part_t1 = nullptr;  // h layer 1, slot part (accumulated over slots)
  size_t part_bytes = 0, part_t2_bytes = 0, part_t1_bytes = 0;
  int max_chunks = 0;
};

namespace {

using namespace valu;

constexpr int kThreads = 256;
constexpr int kOB = 64;
constexpr int kChunkPx = 4096;      // pixels per split-K chunk of the dW GEMMs

inline int rup(int x, int m) { return (x + m - 1) / m * m; }

// Row offsets of every plane block.  Activation blocks end with a row of
// ones (bias gradients) and are padded with zero rows to a multiple of 32.
struct Blocks {
  int xb, a1, a2, st, zs, d1, d2, pl, g1, g2, z1, bi, u, cnt;
  int dy, dg2, dg1, dphi, dd2, dd1, dtau, dzin, du, dsig, da2, da1, dz2, dz1;
  int rows;
};

Blocks make_blocks(int W) {
  Blocks b;
  int r = 0;
  auto take = [&](int n) { int o = r; r += n; return o; };
  const int RW = rup(W + 1, 32);
  b.xb = take(32);               // G 0..13, scene 14..29, ones 30
  b.a1 = take(RW);
  b.a2 = take(RW);
  b.st = take(rup(2 * W + 1, 32));   // sigma, tau, ones
  b.zs = take(RW);               // Z / max(c,1), then the bias scale of h's last layer
  b.d1 = take(RW);
  b.d2 = take(RW);
  b.pl = take(rup(W + 4, 32));   // phi, L_d (3), ones
  b.g1 = take(RW);
  b.g2 = take(RW);
  b.z1 = take(RW);               // slot i: z1, ones
  b.bi = take(32);               // slot i: b_i (12), ones at 12
  b.u = take(W);
  b.cnt = take(1);
  b.dy = take(32);
  b.dg2 = take(W); b.dg1 = take(W); b.dphi = take(W); b.dd2 = take(W); b.dd1 = take(W);
  b.dtau = take(W); b.dzin = take(W); b.du = take(W); b.dsig = take(W); b.da2 = take(W);
  b.da1 = take(W); b.dz2 = take(W); b.dz1 = take(W);
  b.rows = r;
  return b;
}

struct BwdArgs {
  const float *gbuf, *layers, *scene, *grad_out;
  int hw, k, pool;
  int64_t npx;
  float *planes;
  int stride;
  Blocks bl;
};

__device__ __forceinline__ void layer_offsets_dev(int W, LayerOff (&lo)[kNumLayers]) {
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

#define ROW(r) (a.planes + (size_t)(r) * a.stride)

// out rows = act(bias + W[:, col0:col0+NIN] . in rows), NOUT outputs.
template <int NOUT, int NIN, bool RELU>
__device__ __forceinline__ void fwd_layer(cfloat *wm, cfloat *wt, const LayerOff &lo, int col0,
                                          const float *in, float *out, int stride, int p) {
  for (int ob = 0; ob < NOUT; ob += kOB) {
    float acc[kOB];
#pragma unroll
    for (int o = 0; o < kOB; ++o) acc[o] = wm[lo.b + ob + o];
    acc_from_scratch<kOB, NIN>(acc, wt + lo.w, lo.out, ob, col0, in, stride, p);
#pragma unroll
    for (int o = 0; o < kOB; ++o) out[(size_t)(ob + o) * stride + p] = RELU ? relu(acc[o]) : acc[o];
  }
}

// out rows i in [0, NI) = mask_i * scale * sum_o W[o][col0 + i] d[o]  (o < NO),
// mask_i = [act_i > 0] when act != nullptr.  `init` rows are added if given.
template <int NI, int NO>
__device__ __forceinline__ void bwd_layer(cfloat *wm, const LayerOff &lo, int col0,
                                          const float *d, float *out, const float *act,
                                          const float *init, float scale, int stride, int p) {
  for (int ib = 0; ib < NI; ib += kOB) {
    float acc[kOB];
#pragma unroll
    for (int o = 0; o < kOB; ++o) acc[o] = 0.0f;
    acc_from_scratch<kOB, NO>(acc, wm + lo.w, lo.in, col0 + ib, 0, d, stride, p);
#pragma unroll
    for (int o = 0; o < kOB; ++o) {
      const size_t ix = (size_t)(ib + o) * stride + p;
      float v = acc[o] * scale;
      if (init) v += init[ix];
      if (act) v = act[ix] > 0.0f ? v : 0.0f;
      out[ix] = v;
    }
  }
}

// ---- 1. forward recompute, saving the planes -------------------------------
template <int W>
__global__ __launch_bounds__(kThreads) void fwd_save_kernel(const float *__restrict__ wm_,
                                                            const float *__restrict__ wt_,
                                                            BwdArgs a) {
  cfloat *wm = (cfloat *)wm_;
  cfloat *wt = (cfloat *)wt_;
  LayerOff lo[kNumLayers];
  layer_offsets_dev(W, lo);
  const int p = blockIdx.x * kThreads + threadIdx.x;
  const int64_t pc = p < a.npx ? p : a.npx - 1;
  const int f = (int)(pc / a.hw), q = (int)(pc - (int64_t)f * a.hw), hw = a.hw, K = a.k;
  const float *G = a.gbuf + (size_t)f * kNG * hw + q;
  const float *S = a.scene + (size_t)f * kNS;
  const float *Ls = a.layers + (size_t)f * K * kNL * hw + q;
  const Blocks &B = a.bl;
  const int st = a.stride;
  {
    float x[kNG + kNS];
#pragma unroll
    for (int c = 0; c < kNG; ++c) x[c] = G[(size_t)c * hw];
#pragma unroll
    for (int c = 0; c < kNS; ++c) x[kNG + c] = S[c];
#pragma unroll
    for (int c = 0; c < kNG + kNS; ++c) ROW(B.xb + c)[p] = x[c];
    for (int ob = 0; ob < W; ob += kOB) {
      float acc[kOB];
#pragma unroll
      for (int o = 0; o < kOB; ++o) acc[o] = wm[lo[L_F1].b + ob + o];
      acc_from_regs<kOB, kNG + kNS>(acc, wt + lo[L_F1].w, W, ob, 0, x);
#pragma unroll
      for (int o = 0; o < kOB; ++o) ROW(B.a1 + ob + o)[p] = relu(acc[o]);
    }
  }
  fwd_layer<W, W, true>(wm, wt, lo[L_F2], 0, ROW(B.a1), ROW(B.a2), st, p);
  fwd_layer<W, W, false>(wm, wt, lo[L_F3], 0, ROW(B.a2), ROW(B.st), st, p);       // sigma
  fwd_layer<W, W, false>(wm, wt, lo[L_T1], kNL, ROW(B.st), ROW(B.u), st, p);      // u
  // slot loop: Z = sum_i m_i relu(A2 relu(W1b b_i + u) + c2); z1 goes through the z1 rows
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
      for (int o = 0; o < kOB; ++o) acc[o] = ROW(B.u + ob + o)[p];
      acc_from_regs<kOB, kNL>(acc, wt + lo[L_T1].w, lo[L_T1].out, ob, 0, bi);
#pragma unroll
      for (int o = 0; o < kOB; ++o) ROW(B.z1 + ob + o)[p] = relu(acc[o]);
    }
#pragma unroll
    for (int ob = 0; ob < W; ob += kOB) {
      float acc[kOB];
#pragma unroll
      for (int o = 0; o < kOB; ++o) acc[o] = wm[lo[L_T2].b + ob + o];
      acc_from_scratch<kOB, W>(acc, wt + lo[L_T2].w, W, ob, 0, ROW(B.z1), st, p);
#pragma unroll
      for (int o = 0; o < kOB; ++o) Z[ob + o] = fmaf(m, relu(acc[o]), Z[ob + o]);
    }
    cnt += m;
  }
  const bool mean = a.pool == GN_POOL_MEAN;
  const float inv = mean ? 1.0f / fmaxf(cnt, 1.0f) : 1.0f;
  const float bs = mean ? (cnt > 0.0f ? 1.0f : 0.0f) : cnt;
#pragma unroll
  for (int o = 0; o < W; ++o) ROW(B.zs + o)[p] = Z[o] * inv;
  ROW(B.zs + W)[p] = bs;
  ROW(B.cnt)[p] = cnt;
  for (int ob = 0; ob < W; ob += kOB) {                                            // tau
    float acc[kOB];
#pragma unroll
    for (int o = 0; o < kOB; ++o) acc[o] = bs * wm[lo[L_T3].b + ob + o];
    acc_from_scratch<kOB, W>(acc, wt + lo[L_T3].w, W, ob, 0, ROW(B.zs), st, p);
#pragma unroll
    for (int o = 0; o < kOB; ++o) ROW(B.st + W + ob + o)[p] = acc[o];
  }
  fwd_layer<W, 2 * W, true>(wm, wt, lo[L_B1], 0, ROW(B.st), ROW(B.d1), st, p);
  fwd_layer<W, W, true>(wm, wt, lo[L_B2], 0, ROW(B.d1), ROW(B.d2), st, p);
  fwd_layer<W, W, false>(wm, wt, lo[L_B3], 0, ROW(B.d2), ROW(B.pl), st, p);       // phi
#pragma unroll
  for (int c = 0; c < 3; ++c) ROW(B.pl + W + c)[p] = G[(size_t)(11 + c) * hw];   // L_d
  for (int ob = 0; ob < W; ob += kOB) {
    float acc[kOB];
    float ld[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) ld[c] = ROW(B.pl + W + c)[p];
#pragma unroll
    for (int o = 0; o < kOB; ++o) acc[o] = wm[lo[L_R1].b + ob + o];
    acc_from_scratch<kOB, W>(acc, wt + lo[L_R1].w, W, ob, 0, ROW(B.pl), st, p);
    acc_from_regs<kOB, 3>(acc, wt + lo[L_R1].w, W, ob, W, ld);
#pragma unroll
    for (int o = 0; o < kOB; ++o) ROW(B.g1 + ob + o)[p] = relu(acc[o]);
  }
  fwd_layer<W, W, true>(wm, wt, lo[L_R2], 0, ROW(B.g1), ROW(B.g2), st, p);
}

// ---- 2. head: dy -> R -> B -> dsigma_B, dtau -> dZ ---------------------------
template <int W>
__global__ __launch_bounds__(kThreads) void head_kernel(const float *__restrict__ wm_, BwdArgs a) {
  cfloat *wm = (cfloat *)wm_;
  LayerOff lo[kNumLayers];
  layer_offsets_dev(W, lo);
  const int p = blockIdx.x * kThreads + threadIdx.x;
  const bool valid = p < a.npx;
  const int64_t pc = valid ? p : a.npx - 1;
  const int f = (int)(pc / a.hw), q = (int)(pc - (int64_t)f * a.hw);
  const Blocks &B = a.bl;
  const int st = a.stride;
  float dy[kNOUT];
#pragma unroll
  for (int c = 0; c < kNOUT; ++c) {
    dy[c] = valid ? a.grad_out[((size_t)f * kNOUT + c) * a.hw + q] : 0.0f;  // pad pixels: 0
    ROW(B.dy + c)[p] = dy[c];
  }
  for (int ib = 0; ib < W; ib += kOB) {                                          // R3^T
    float acc[kOB];
#pragma unroll
    for (int o = 0; o < kOB; ++o) acc[o] = 0.0f;
    acc_from_regs<kOB, kNOUT>(acc, wm + lo[L_R3].w, W, ib, 0, dy);
#pragma unroll
    for (int o = 0; o < kOB; ++o)
      ROW(B.dg2 + ib + o)[p] = ROW(B.g2 + ib + o)[p] > 0.0f ? acc[o] : 0.0f;
  }
  bwd_layer<W, W>(wm, lo[L_R2], 0, ROW(B.dg2), ROW(B.dg1), ROW(B.g1), nullptr, 1.0f, st, p);
  bwd_layer<W, W>(wm, lo[L_R1], 0, ROW(B.dg1), ROW(B.dphi), nullptr, nullptr, 1.0f, st, p);
  bwd_layer<W, W>(wm, lo[L_B3], 0, ROW(B.dphi), ROW(B.dd2), ROW(B.d2), nullptr, 1.0f, st, p);
  bwd_layer<W, W>(wm, lo[L_B2], 0, ROW(B.dd2), ROW(B.dd1), ROW(B.d1), nullptr, 1.0f, st, p);
  bwd_layer<W, W>(wm, lo[L_B1], 0, ROW(B.dd1), ROW(B.dsig), nullptr, nullptr, 1.0f, st, p);
  bwd_layer<W, W>(wm, lo[L_B1], W, ROW(B.dd1), ROW(B.dtau), nullptr, nullptr, 1.0f, st, p);
  const float c = ROW(B.cnt)[p];
  const float inv = a.pool == GN_POOL_MEAN ? 1.0f / fmaxf(c, 1.0f) : 1.0f;
  bwd_layer<W, W>(wm, lo[L_T3], 0, ROW(B.dtau), ROW(B.dzin), nullptr, nullptr, inv, st, p);
}

// ---- 3. one slot: recompute h's layers 1-2, backprop, accumulate du --------
template <int W>
__global__ __launch_bounds__(kThreads) void slot_kernel(const float *__restrict__ wm_,
                                                        const float *__restrict__ wt_, BwdArgs a,
                                                        int slot, int first) {
  cfloat *wm = (cfloat *)wm_;
  cfloat *wt = (cfloat *)wt_;
  LayerOff lo[kNumLayers];
  layer_offsets_dev(W, lo);
  const int p = blockIdx.x * kThreads + threadIdx.x;
  const int64_t pc = p < a.npx ? p : a.npx - 1;
  const int f = (int)(pc / a.hw), q = (int)(pc - (int64_t)f * a.hw), hw = a.hw;
  const Blocks &B = a.bl;
  const int st = a.stride;
  const float *Li = a.layers + ((size_t)f * a.k + slot) * kNL * hw + q;
  float bi[kNL];
#pragma unroll
  for (int c = 0; c < kNL; ++c) {
    bi[c] = Li[(size_t)c * hw];
    ROW(B.bi + c)[p] = bi[c];
  }
  const float m = bi[kAlpha] > 0.0f ? 1.0f : 0.0f;
  for (int ob = 0; ob < W; ob += kOB) {                                          // z1
    float acc[kOB];
#pragma unroll
    for (int o = 0; o < kOB; ++o) acc[o] = ROW(B.u + ob + o)[p];
    acc_from_regs<kOB, kNL>(acc, wt + lo[L_T1].w, lo[L_T1].out, ob, 0, bi);
#pragma unroll
    for (int o = 0; o < kOB; ++o) ROW(B.z1 + ob + o)[p] = relu(acc[o]);
  }
  for (int ob = 0; ob < W; ob += kOB) {                                          // dz2
    float acc[kOB];
#pragma unroll
    for (int o = 0; o < kOB; ++o) acc[o] = wm[lo[L_T2].b + ob + o];
    acc_from_scratch<kOB, W>(acc, wt + lo[L_T2].w, W, ob, 0, ROW(B.z1), st, p);
#pragma unroll
    for (int o = 0; o < kOB; ++o)
      ROW(B.dz2 + ob + o)[p] = acc[o] > 0.0f ? m * ROW(B.dzin + ob + o)[p] : 0.0f;
  }
  for (int ib = 0; ib < W; ib += kOB) {                                          // dz1, du
    float acc[kOB];
#pragma unroll
    for (int o = 0; o < kOB; ++o) acc[o] = 0.0f;
    acc_from_scratch<kOB, W>(acc, wm + lo[L_T2].w, W, ib, 0, ROW(B.dz2), st, p);
#pragma unroll
    for (int o = 0; o < kOB; ++o) {
      const float v = ROW(B.z1 + ib + o)[p] > 0.0f ? acc[o] : 0.0f;
      ROW(B.dz1 + ib + o)[p] = v;
      float *du = ROW(B.du + ib + o) + p;
      *du = first ? v : *du + v;
    }
  }
}

// ---- 4. tail: dsigma += A1s^T du, then F ------------------------------------
template <int W>
__global__ __launch_bounds__(kThreads) void tail_kernel(const float *__restrict__ wm_, BwdArgs a,
                                                        int have_slots) {
  cfloat *wm = (cfloat *)wm_;
  LayerOff lo[kNumLayers];
  layer_offsets_dev(W, lo);
  const int p = blockIdx.x * kThreads + threadIdx.x;
  const Blocks &B = a.bl;
  const int st = a.stride;
  if (have_slots)
    bwd_layer<W, W>(wm, lo[L_T1], kNL, ROW(B.du), ROW(B.dsig), nullptr, ROW(B.dsig), 1.0f, st, p);
  bwd_layer<W, W>(wm, lo[L_F3], 0, ROW(B.dsig), ROW(B.da2), ROW(B.a2), nullptr, 1.0f, st, p);
  bwd_layer<W, W>(wm, lo[L_F2], 0, ROW(B.da2), ROW(B.da1), ROW(B.a1), nullptr, 1.0f, st, p);
}

// ---- 5. weight gradients: sum over pixels on the fp32 matrix cores ---------
typedef float f32x4 __attribute__((ext_vector_type(4)));

// part[chunk][o][i] (+)= sum_{p in chunk} D[o][p] * A[i][p] for a 32 x 32 tile
// per wave.  Lane l feeds row (l & 15) and pixels 4 (l >> 4) + j of each
// 16-pixel step to both operands, so every pixel meets itself exactly once.
__global__ __launch_bounds__(64) void dw_gemm_kernel(const float *__restrict__ D,
                                                     const float *__restrict__ A, int stride,
                                                     int64_t npx_pad, float *__restrict__ part,
                                                     int o_pad, int i_pad, int accumulate) {
  const int lane = threadIdx.x;
  const int i0 = blockIdx.x * 32, o0 = blockIdx.y * 32, chunk = blockIdx.z;
  const int r = lane & 15, kq = lane >> 4;
  const int64_t p_begin = (int64_t)chunk * kChunkPx;
  const int64_t p_end = std::min<int64_t>(p_begin + kChunkPx, npx_pad);
  f32x4 acc[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = f32x4{0.f, 0.f, 0.f, 0.f};
  const float *d0 = D + (size_t)(o0 + r) * stride + 4 * kq;
  const float *d1 = d0 + (size_t)16 * stride;
  const float *a0 = A + (size_t)(i0 + r) * stride + 4 * kq;
  const float *a1 = a0 + (size_t)16 * stride;
  for (int64_t p = p_begin; p < p_end; p += 16) {
    const f32x4 da = *(const f32x4 *)(d0 + p), db = *(const f32x4 *)(d1 + p);
    const f32x4 aa = *(const f32x4 *)(a0 + p), ab = *(const f32x4 *)(a1 + p);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(da[j], aa[j], acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(da[j], ab[j], acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(db[j], aa[j], acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(db[j], ab[j], acc[1][1], 0, 0, 0);
    }
  }
  float *P = part + (size_t)chunk * o_pad * i_pad;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int o = o0 + 16 * mi + 4 * kq + rr, i = i0 + 16 * ni + r;
        float *dst = P + (size_t)o * i_pad + i;
        *dst = accumulate ? *dst + acc[mi][ni][rr] : acc[mi][ni][rr];
      }
}

// grad_w[layer][o][col0 + i] = sum_chunks part[c][o][i] (i < n_in);
// grad_w bias[o] = sum part[c][o][n_in] when has_bias.
__global__ void dw_reduce_kernel(const float *__restrict__ part, int nchunks, int o_pad, int i_pad,
                                 int n_out, int n_in, int has_bias, float *__restrict__ gw,
                                 LayerOff lo, int col0) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int ncol = n_in + (has_bias ? 1 : 0);
  if (e >= n_out * ncol) return;
  const int o = e / ncol, i = e - o * ncol;
  float s = 0.0f;
  for (int c = 0; c < nchunks; ++c) s += part[((size_t)c * o_pad + o) * i_pad + i];
  if (i < n_in)
    gw[lo.w + (int64_t)o * lo.in + col0 + i] = s;
  else
    gw[lo.b + o] = s;
}

__global__ void fill_rows_kernel(float *rows, int stride, int64_t n, float v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) rows[e] = v;
  (void)stride;
}

}  // namespace

}  // namespace gn

using namespace gn;

void gn_bwd_free(gn_handle *h) {
  if (!h->bwd) return;
  (void)hipFree(h->bwd->planes);
  (void)hipFree(h->bwd->part);
  (void)hipFree(h->bwd->part_t2);
  (void)hipFree(h->bwd->part_t1);
  delete h->bwd;
  h->bwd = nullptr;
}

size_t gn_bwd_bytes(gn_handle *h) {
  if (!h->bwd) return 0;
  return h->bwd->plane_bytes + h->bwd->part_bytes + h->bwd->part_t2_bytes + h->bwd->part_t1_bytes;
}

static hipError_t ensure_workspace(gn_handle *h, int64_t npx_pad) {
  BwdWorkspace *ws = h->bwd;
  if (ws && ws->cap_px >= npx_pad) return hipSuccess;
  gn_bwd_free(h);
  ws = new BwdWorkspace();
  h->bwd = ws;
  const Blocks bl = make_blocks(h->W);
  ws->W = h->W;
  ws->cap_px = npx_pad;
  ws->plane_bytes = sizeof(float) * (size_t)bl.rows * npx_pad;
  ws->max_chunks = (int)((npx_pad + kChunkPx - 1) / kChunkPx);
  const int W = h->W;
  ws->part_bytes = sizeof(float) * (size_t)ws->max_chunks * W * rup(2 * W + 1, 32);
  ws->part_t2_bytes = sizeof(float) * (size_t)ws->max_chunks * W * rup(W + 1, 32);
  ws->part_t1_bytes = sizeof(float) * (size_t)ws->max_chunks * W * 32;
  hipError_t e = hipMalloc((void **)&ws->planes, ws->plane_bytes);
  if (e == hipSuccess) e = hipMalloc((void **)&ws->part, ws->part_bytes);
  if (e == hipSuccess) e = hipMalloc((void **)&ws->part_t2, ws->part_t2_bytes);
  if (e == hipSuccess) e = hipMalloc((void **)&ws->part_t1, ws->part_t1_bytes);
  if (e == hipSuccess) e = hipMemset(ws->planes, 0, ws->plane_bytes);
  if (e != hipSuccess) gn_bwd_free(h);
  return e;
}

// Rows of ones (bias gradients) for a given plane row length.
static hipError_t init_constant_rows(gn_handle *h, int64_t stride, hipStream_t s) {
  BwdWorkspace *ws = h->bwd;
  if (ws->stride == stride) return hipSuccess;
  const Blocks bl = make_blocks(h->W);
  const int W = h->W;
  hipError_t e = hipMemsetAsync(ws->planes, 0, ws->plane_bytes, s);
  const int ones[] = {bl.xb + kNG + kNS, bl.a1 + W, bl.a2 + W, bl.st + 2 * W, bl.d1 + W,
                      bl.d2 + W, bl.pl + W + 3, bl.g1 + W, bl.g2 + W, bl.z1 + W, bl.bi + kNL};
  for (int r : ones) {
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(fill_rows_kernel, dim3((unsigned)((stride + 255) / 256)), dim3(256), 0, s,
                       ws->planes + (size_t)r * stride, (int)stride, stride, 1.0f);
    e = hipGetLastError();
  }
  if (e == hipSuccess) ws->stride = stride;
  return e;
}

struct GemmJob {
  int dblock, o_pad, ablock, i_pad;   // plane rows
  Layer layer;
  int n_out, n_in, has_bias, col0;
};

extern "C" gn_status glassnet_backward(gn_handle *h, const gn_frame *frame,
                                       const float *grad_out, float *grad_w, void *hip_stream) {
  if (!h) return gn_set_error(GN_E_INVAL, "handle is NULL");
  if (h->poisoned) return gn_set_error(GN_E_DEVICE, "handle poisoned by an earlier device error");
  if (!grad_out || !grad_w || ((uintptr_t)grad_out & 3) || ((uintptr_t)grad_w & 3))
    return gn_set_error(GN_E_INVAL, "grad_out and grad_w must be non-NULL, 4-byte aligned");
  gn_status st = gn_validate_frame(h, frame, nullptr);
  if (st != GN_OK) return st;
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (hipSetDevice(h->device) != hipSuccess) return gn_set_error(GN_E_DEVICE, "hipSetDevice failed");
  hipStream_t s = (hipStream_t)hip_stream;
  const int W = h->W;
  const int64_t hw = (int64_t)frame->h * frame->w;
  const int64_t npx = (int64_t)frame->n * hw;
  const int64_t npx_pad = (npx + kChunkPx - 1) / kChunkPx * kChunkPx;
  hipError_t e = ensure_workspace(h, npx_pad);
  if (e == hipSuccess) e = init_constant_rows(h, npx_pad, s);
  if (e != hipSuccess) {
    if (prev >= 0) (void)hipSetDevice(prev);
    return gn_check_device(h, e, "backward workspace");
  }
  BwdWorkspace *ws = h->bwd;
  const Blocks bl = make_blocks(W);
  BwdArgs a;
  a.gbuf = frame->gbuf;
  a.layers = frame->layers;
  a.scene = frame->scene;
  a.grad_out = grad_out;
  a.hw = (int)hw;
  a.k = frame->k;
  a.pool = h->cfg.pool;
  a.npx = npx;
  a.planes = ws->planes;
  a.stride = (int)npx_pad;
  a.bl = bl;
  const dim3 grid((unsigned)(npx_pad / kThreads)), block(kThreads);
  const float *wm = h->d_master, *wt = h->d_master_t;
  LayerOff lo[kNumLayers];
  layer_offsets(W, lo);
  const int nchunks = (int)(npx_pad / kChunkPx);
  auto plane = [&](int r) { return ws->planes + (size_t)r * npx_pad; };
  auto gemm = [&](const GemmJob &j, float *part, int accumulate) {
    hipLaunchKernelGGL(dw_gemm_kernel, dim3(j.i_pad / 32, j.o_pad / 32, nchunks), dim3(64), 0, s,
                       plane(j.dblock), plane(j.ablock), (int)npx_pad, npx_pad, part, j.o_pad,
                       j.i_pad, accumulate);
  };
  auto reduce = [&](const GemmJob &j, const float *part) {
    const int n = j.n_out * (j.n_in + (j.has_bias ? 1 : 0));
    hipLaunchKernelGGL(dw_reduce_kernel, dim3((n + 255) / 256), dim3(256), 0, s, part, nchunks,
                       j.o_pad, j.i_pad, j.n_out, j.n_in, j.has_bias, grad_w, lo[j.layer], j.col0);
  };
  const int RW = rup(W + 1, 32);

  if (W == 64) {
    hipLaunchKernelGGL(fwd_save_kernel<64>, grid, block, 0, s, wm, wt, a);
    hipLaunchKernelGGL(head_kernel<64>, grid, block, 0, s, wm, a);
  } else {
    hipLaunchKernelGGL(fwd_save_kernel<128>, grid, block, 0, s, wm, wt, a);
    hipLaunchKernelGGL(head_kernel<128>, grid, block, 0, s, wm, a);
  }
  // slot loop: recompute, backprop, accumulate dW of h's layers 1 (slot part) and 2
  const GemmJob jT2{bl.dz2, W, bl.z1, RW, L_T2, W, W, 1, 0};
  const GemmJob jT1a{bl.dz1, W, bl.bi, 32, L_T1, W, kNL, 1, 0};
  for (int i = 0; i < frame->k; ++i) {
    if (W == 64)
      hipLaunchKernelGGL(slot_kernel<64>, grid, block, 0, s, wm, wt, a, i, i == 0);
    else
      hipLaunchKernelGGL(slot_kernel<128>, grid, block, 0, s, wm, wt, a, i, i == 0);
    gemm(jT2, ws->part_t2, i > 0);
    gemm(jT1a, ws->part_t1, i > 0);
  }
  if (frame->k > 0) {
    reduce(jT2, ws->part_t2);
    reduce(jT1a, ws->part_t1);
  } else {
    // no slot: h's layers 1 (slot part and bias) and 2 get zero gradient
    e = hipMemsetAsync(grad_w + lo[L_T2].w, 0, sizeof(float) * (size_t)(W * W + W), s);
    for (int o = 0; o < W && e == hipSuccess; ++o)
      e = hipMemsetAsync(grad_w + lo[L_T1].w + (int64_t)o * lo[L_T1].in, 0, sizeof(float) * kNL, s);
    if (e == hipSuccess) e = hipMemsetAsync(grad_w + lo[L_T1].b, 0, sizeof(float) * W, s);
    if (e == hipSuccess) e = hipMemsetAsync(plane(bl.du), 0, sizeof(float) * W * npx_pad, s);
  }
  if (W == 64)
    hipLaunchKernelGGL(tail_kernel<64>, grid, block, 0, s, wm, a, frame->k > 0);
  else
    hipLaunchKernelGGL(tail_kernel<128>, grid, block, 0, s, wm, a, frame->k > 0);

  const GemmJob jobs[] = {
      {bl.dy, 32, bl.g2, RW, L_R3, kNOUT, W, 1, 0},
      {bl.dg2, W, bl.g1, RW, L_R2, W, W, 1, 0},
      {bl.dg1, W, bl.pl, rup(W + 4, 32), L_R1, W, W + 3, 1, 0},
      {bl.dphi, W, bl.d2, RW, L_B3, W, W, 1, 0},
      {bl.dd2, W, bl.d1, RW, L_B2, W, W, 1, 0},
      {bl.dd1, W, bl.st, rup(2 * W + 1, 32), L_B1, W, 2 * W, 1, 0},
      {bl.dtau, W, bl.zs, RW, L_T3, W, W, 1, 0},
      {bl.du, W, bl.st, rup(W, 32), L_T1, W, W, 0, kNL},
      {bl.dsig, W, bl.a2, RW, L_F3, W, W, 1, 0},
      {bl.da2, W, bl.a1, RW, L_F2, W, W, 1, 0},
      {bl.da1, W, bl.xb, 32, L_F1, W, kNG + kNS, 1, 0},
  };
  for (const GemmJob &j : jobs) {
    gemm(j, ws->part, 0);
    reduce(j, ws->part);
  }
  if (e == hipSuccess) e = hipGetLastError();
  if (prev >= 0) (void)hipSetDevice(prev);
  return gn_check_device(h, e, "backward launch");
}
