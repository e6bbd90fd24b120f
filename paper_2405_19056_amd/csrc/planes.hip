// The fp32 plane pipeline: GlassNet's FP32 forward (Sec. 3.3-3.4), the FP8
// calibration pass, and the hand-written backward (Sec. 3.5 trains F, T, B
// and R jointly end to end; dL/dw for a given dL/dy).
//
// Every per-pixel quantity lives in a plane [row][pixel] of fp32 in HBM, and
// every linear map of the forward and of the backward is one plane GEMM on
// the fp32 matrix cores,
//     out[m][p] = epilogue( sum_k A[m][k] X[k][p] ),
// with A a weight matrix (or its transpose) and X a block of planes.  The
// epilogues fuse what sits between two linear maps: bias, ReLU, the ReLU
// derivative mask, the alpha mask and pool of Eq. (5) and per-pixel scales.
//
//   1. prep:      gather G, the scene vector, L_d, the active-slot count and
//                 dL/dy into planes.
//   2. forward:   F; u = W_T1,sigma sigma + b_T1 (the sigma-hoist); per slot
//                 z1_i and z2_i with the masked pool accumulated in the
//                 epilogue; T3; B; R's hidden layers.  The slot activations
//                 are overwritten slot by slot, never kept for all slots.
//                 The FP32 forward ends with R's last layer into the output;
//                 the calibration stops after h's first layer of every slot.
//   3. head:      R^T, B^T -> (dsigma_B, dtau) -> dZ through T3 and the pool.
//   4. slot i:    recompute z1_i, then dz2_i (z2_i's ReLU mask in the
//                 epilogue), dz1_i, du += dz1_i, and accumulate dW of T2 and
//                 of T1's slot columns.
//   5. tail:      dsigma += W_T1,sigma^T du, then F^T.
//   6. dW:        each layer's sum_p delta_p a_p^T on the matrix cores, split
//                 over pixel chunks, partials reduced in a fixed order
//                 (deterministic, no atomics).  Bias gradients come from a row
//                 of ones appended to each activation block.
//
// With the canonical slot order (slot_order.h) prep also ranks every
// pixel's slots, and slot step i gathers each pixel's slot of rank i: the
// pool is an fp32 running sum whose order depends only on the slot records.
#include <string.h>

#include "gn_api_state.h"
#include "slot_order.h"

namespace gn {

typedef float f32x4 __attribute__((ext_vector_type(4)));

struct BwdWorkspace {
  int W = 0;
  int64_t cap_px = 0;        // plane row length (padded pixel count)
  int64_t stride = -1;       // row length the constant rows were written for
  float *planes = nullptr;
  size_t plane_bytes = 0;
  f32x4 *frag = nullptr;     // weight fragments of every plane GEMM
  size_t frag_bytes = 0;
  float *part = nullptr;     // generic dW partials
  float *part_t2 = nullptr;  // T2 partials (accumulated over slots)
  float *part_t1 = nullptr;  // T1 slot-column partials (accumulated over slots)
  size_t part_bytes = 0, part_t2_bytes = 0, part_t1_bytes = 0;
  uint8_t *perm = nullptr;   // canonical slot order: [rank][padded pixel] slot indices
  size_t perm_bytes = 0;
  int max_chunks = 0;
};

namespace {

constexpr int kThreads = 256;
constexpr int kChunkPx = 4096;      // plane rows hold the pixels rounded up to this
// Plane rows are npx_pad + kRowSkew floats apart: a power-of-two pitch puts
// the same pixel of every row on the same HBM channel.
constexpr int kRowSkew = 1056;
// Operand loads use 32-bit byte offsets within a plane block (up to 288 rows
// plus a 16-row tile): this bounds the pixels of one backward call.
constexpr int64_t kMaxPx = (int64_t)3 << 20;

inline int rup(int x, int m) { return (x + m - 1) / m * m; }

// Row offsets of every plane block.  Activation blocks end with a row of
// ones (bias gradients) and are padded with zero rows to a multiple of 32.
struct Blocks {
  int xb, a1, a2, st, u, zs, d1, d2, pl, g1, g2, z1, bi, px, y;
  int dy, dg2, dg1, dphi, dd2, dd1, dsig, dtau, dzin, du, da2, da1, dz2, dz1;
  int rows;
};
enum { PX_INV = 0, PX_M = 1 };     // rows of the per-pixel scalar block

// Width of F's input and of h's slot input after positional encoding.
inline int enc_x(int pe) { return (kNG + kNS) * pe_blocks(pe); }
inline int enc_b(int pe) { return kNL * pe_blocks(pe); }

Blocks make_blocks(int W, int pe) {
  Blocks b;
  int r = 0;
  auto take = [&](int n) { int o = r; r += n; return o; };
  const int RW = rup(W + 1, 32);
  b.xb = take(rup(enc_x(pe) + 1, 32));   // encoding blocks of [G 0..13; scene 0..15], ones
  b.a1 = take(RW);
  b.a2 = take(RW);
  b.st = take(rup(2 * W + 1, 32));   // sigma, tau, ones
  b.u = take(W);
  b.zs = take(RW);                   // pooled Z / max(c,1); row W: bias scale of T3
  b.d1 = take(RW);
  b.d2 = take(RW);
  b.pl = take(rup(W + 4, 32));       // phi, L_d (3), ones
  b.g1 = take(RW);
  b.g2 = take(RW);
  b.z1 = take(RW);                   // slot i: z1, ones
  b.bi = take(rup(enc_b(pe) + 1, 32));   // slot i: encoding blocks of b_i (12), ones
  b.px = take(32);                   // 1/max(c,1) (mean) or 1; slot mask m_i
  b.y = take(32);                    // R's 3 outputs (16-row GEMM tile), forward only
  b.dy = take(32);
  b.dg2 = take(W); b.dg1 = take(W); b.dphi = take(W); b.dd2 = take(W); b.dd1 = take(W);
  b.dsig = take(W); b.dtau = take(W);    // adjacent: B1^T writes both at once
  b.dzin = take(W); b.du = take(W); b.da2 = take(W); b.da1 = take(W);
  b.dz2 = take(W); b.dz1 = take(W);
  b.rows = r;
  return b;
}

// ---- weight fragments of the plane GEMMs ------------------------------------
// Op o multiplies A (M x K) into planes.  A[m][k] = W[m][col0 + k] of a layer
// (trans = 0) or W[k][col0 + m] (trans = 1, the backward maps).  Fragments are
// stored [mt][q][lane] as f32x4: element j of lane l holds
// A[16 mt + (l & 15)][16 q + 4 j + (l >> 4)], the operand lane l presents to
// v_mfma_f32_16x16x4f32 in K-step 4q + j; zero outside M x K.  The group
// count is even, so every input block has at least 32 * ceil(K / 32) rows
// (zero rows beyond the data, or the ones row, meet zero weights).
enum Op {
  O_F1, O_F2, O_F3, O_T1S, O_T1A, O_T2, O_T3, O_B1, O_B2, O_B3, O_R1, O_R2, O_R3,
  O_R3T, O_R2T, O_R1T, O_B3T, O_B2T, O_B1T, O_T3T, O_T2T, O_T1ST, O_F3T, O_F2T, kNumOps
};

struct OpDesc {
  int64_t woff;      // float offset of the layer's matrix in the master vector
  int64_t off;       // f32x4 offset of the fragments
  int32_t ld;        // the layer's input count (master row length)
  int32_t trans, col0, M, K, mt, kq, pad;
};

struct OpTable {
  OpDesc op[kNumOps];
  int64_t total;     // f32x4 count
};

OpTable make_ops(int W, int pe) {
  LayerOff lo[kNumLayers];
  layer_offsets(W, pe, lo);
  const int nb = enc_b(pe);
  struct S { Op o; Layer l; int trans, col0, M, K; };
  const S s[kNumOps] = {
      {O_F1, L_F1, 0, 0, W, enc_x(pe)}, {O_F2, L_F2, 0, 0, W, W},  {O_F3, L_F3, 0, 0, W, W},
      {O_T1S, L_T1, 0, nb, W, W},       {O_T1A, L_T1, 0, 0, W, nb}, {O_T2, L_T2, 0, 0, W, W},
      {O_T3, L_T3, 0, 0, W, W},         {O_B1, L_B1, 0, 0, W, 2 * W}, {O_B2, L_B2, 0, 0, W, W},
      {O_B3, L_B3, 0, 0, W, W},         {O_R1, L_R1, 0, 0, W, W + 3}, {O_R2, L_R2, 0, 0, W, W},
      {O_R3, L_R3, 0, 0, kNOUT, W},
      {O_R3T, L_R3, 1, 0, W, kNOUT},    {O_R2T, L_R2, 1, 0, W, W},  {O_R1T, L_R1, 1, 0, W, W},
      {O_B3T, L_B3, 1, 0, W, W},        {O_B2T, L_B2, 1, 0, W, W},  {O_B1T, L_B1, 1, 0, 2 * W, W},
      {O_T3T, L_T3, 1, 0, W, W},        {O_T2T, L_T2, 1, 0, W, W},  {O_T1ST, L_T1, 1, nb, W, W},
      {O_F3T, L_F3, 1, 0, W, W},        {O_F2T, L_F2, 1, 0, W, W}};
  OpTable t;
  int64_t off = 0;
  for (int i = 0; i < kNumOps; ++i) {
    OpDesc &d = t.op[s[i].o];
    d.woff = lo[s[i].l].w;
    d.ld = lo[s[i].l].in;
    d.trans = s[i].trans;
    d.col0 = s[i].col0;
    d.M = s[i].M;
    d.K = s[i].K;
    d.mt = (d.M + 15) / 16;
    d.kq = (d.K + 31) / 32 * 2;     // even: the GEMM consumes groups in pairs
    d.pad = 0;
    d.off = off;
    off += (int64_t)d.mt * d.kq * 64;
  }
  t.total = off;
  return t;
}

__global__ __launch_bounds__(kThreads) void pack_ops_kernel(const float *__restrict__ master,
                                                            OpTable t, f32x4 *__restrict__ frag) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= t.total) return;
  int o = 0;
  while (o + 1 < kNumOps && e >= t.op[o + 1].off) ++o;
  const OpDesc d = t.op[o];
  const int64_t r = e - d.off;
  const int lane = (int)(r & 63);
  const int64_t fq = r >> 6;
  const int mt = (int)(fq / d.kq), q = (int)(fq % d.kq);
  const int m = 16 * mt + (lane & 15);
  f32x4 v;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int k = 16 * q + 4 * j + (lane >> 4);
    float x = 0.0f;
    if (m < d.M && k < d.K)
      x = d.trans ? master[d.woff + (int64_t)k * d.ld + d.col0 + m]
                  : master[d.woff + (int64_t)m * d.ld + d.col0 + k];
    v[j] = x;
  }
  frag[e] = v;
}

// ---- the plane GEMM ----------------------------------------------------------
// A wave owns 64 pixels and 16*MT rows.  Pixel tile t (0..3) of the wave
// presents pixel p0 + 4n + t as MFMA column n, so lane l reads and writes four
// consecutive pixels of a row (16-byte accesses, 256 contiguous bytes per 16
// lanes) and holds, after the K loop, rows 16 mt + 4 (l >> 4) + r of them.
enum { EP_FWD = 0, EP_DZ2 = 1, EP_BWD = 2 };

struct PgArgs {
  const f32x4 *frag;     // the op's fragments
  int kq;                // 16-deep K groups
  int64_t stride;        // plane row length
  const float *x;        // first row of the input block
  float *out;            // first output row
  const float *bias;     // [M], or null
  const float *bscale;   // per-pixel row multiplying the bias, or null
  const float *add;      // block added to the result (EP_DZ2: the gradient selected)
  const float *mask;     // block: result kept where mask > 0, or null
  const float *pscale;   // per-pixel row multiplying the result, or null
  const float *post;     // per-pixel row multiplying after accumulation, or null
  float *out2;           // EP_BWD: second block that receives (or accumulates) the result
  int relu, accumulate, accumulate2;
};

__device__ __forceinline__ f32x4 ld4(const float *p) { return *(const f32x4 *)p; }

// Operand loads go through buffer resources: one 32-bit per-lane byte offset
// plus a wave-uniform offset per row, instead of a 64-bit address per row.
// Raw addressing over 4 GiB from the base; word 3 selects 32-bit data.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
__device__ __forceinline__ rsrc_t make_rsrc(const void *base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, -1, 0x00020000);
}
__device__ __forceinline__ f32x4 bld4(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
__device__ __forceinline__ void st4(float *p, f32x4 v) { *(f32x4 *)p = v; }

template <int MT, int EP, int RS>
__global__ __launch_bounds__(kThreads) void plane_gemm_kernel(PgArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = lane & 15, g = lane >> 4;
  // RS waves share 64 pixels and split the workgroup's 16 MT RS rows
  const int pgrp = wave / RS, rs = wave - pgrp * RS;
  const int64_t pq = ((int64_t)blockIdx.x * (4 / RS) + pgrp) * 64 + 4 * n;
  const int mt0 = (blockIdx.y * RS + rs) * MT;
  const int64_t st = a.stride;
  f32x4 acc[MT][4];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[mt][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const uint32_t fstride = (uint32_t)a.kq * 64 * 16;        // bytes per fragment row
  const uint32_t row = (uint32_t)st * 4;                      // bytes per plane row
  const rsrc_t xr = make_rsrc(a.x), frr = make_rsrc(a.frag + (size_t)mt0 * a.kq * 64);
  const uint32_t xoff = (uint32_t)(((size_t)g * st + pq) * 4), foff = (uint32_t)lane * 16;
  // Two operand sets in flight: the loads of group q + 1 are issued before
  // the MFMAs of group q (loads of a clamped group past the end are harmless
  // re-reads).
  f32x4 xa[4], wa[MT], xb[4], wb[MT];
  auto load = [&](int q, f32x4 (&x)[4], f32x4 (&w)[MT]) {
    q = q < a.kq ? q : a.kq - 1;
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = bld4(xr, xoff, (uint32_t)(16 * q + 4 * j) * row);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) w[mt] = bld4(frr, foff, mt * fstride + (uint32_t)q * 1024);
  };
  auto mfma = [&](const f32x4 (&x)[4], const f32x4 (&w)[MT]) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[mt][j], x[j][t], acc[mt][t], 0, 0, 0);
  };
  load(0, xa, wa);
  // The scheduling barriers keep each group's loads ahead of the previous
  // group's MFMAs (left alone, the scheduler sinks them next to their use).
  for (int q = 0; q < a.kq; q += 2) {      // kq is even
    load(q + 1, xb, wb);
    __builtin_amdgcn_sched_barrier(0);
    mfma(xa, wa);
    __builtin_amdgcn_sched_barrier(0);
    load(q + 2, xa, wa);
    __builtin_amdgcn_sched_barrier(0);
    mfma(xb, wb);
    __builtin_amdgcn_sched_barrier(0);
  }
  const f32x4 one = {1.f, 1.f, 1.f, 1.f};
  const f32x4 bsc = a.bscale ? ld4(a.bscale + pq) : one;
  const f32x4 psc = a.pscale ? ld4(a.pscale + pq) : one;
  const f32x4 pst = a.post ? ld4(a.post + pq) : one;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = 16 * (mt0 + mt) + 4 * g + r;
      const size_t ix = (size_t)m * st + pq;
      f32x4 v = {acc[mt][0][r], acc[mt][1][r], acc[mt][2][r], acc[mt][3][r]};
      if (EP == EP_FWD) {
        if (a.bias) v += a.bias[m] * bsc;
        if (a.add) v += ld4(a.add + ix);
        if (a.relu) {
#pragma unroll
          for (int t = 0; t < 4; ++t) v[t] = fmaxf(v[t], 0.0f);
        }
        v *= psc;
        if (a.accumulate) v += ld4(a.out + ix);
        v *= pst;
      } else if (EP == EP_DZ2) {
        const f32x4 z = v + a.bias[m];
        const f32x4 d = ld4(a.add + ix);
#pragma unroll
        for (int t = 0; t < 4; ++t) v[t] = z[t] > 0.0f ? psc[t] * d[t] : 0.0f;
      } else {
        v *= psc;
        if (a.add) v += ld4(a.add + ix);
        if (a.mask) {
          const f32x4 mk = ld4(a.mask + ix);
#pragma unroll
          for (int t = 0; t < 4; ++t) v[t] = mk[t] > 0.0f ? v[t] : 0.0f;
        }
      }
      st4(a.out + ix, v);
      if (EP == EP_BWD && a.out2) {
        if (a.accumulate2) v += ld4(a.out2 + ix);
        st4(a.out2 + ix, v);
      }
    }
}

// ---- gathers into planes -------------------------------------------------------
struct PrepArgs {
  const float *gbuf, *layers, *scene, *grad_out;
  int hw, k, pool, W, pe;
  int64_t npx, stride;
  float *planes;
  uint8_t *perm;     // canonical order: [rank][npx_pad] slot indices; null: input order
  int64_t npx_pad;
  Blocks bl;
};

#define ROW(r) (a.planes + (size_t)(r) * a.stride)

// Positional-encoding block b of x (Sec. 3.4): x for b = 0, then
// sin(2^k pi x) for b = 2k + 1 and cos(2^k pi x) for b = 2k + 2 (sinpi and
// cospi reduce the argument exactly; the scaling by 2^k is exact).
__device__ __forceinline__ float pe_value(float x, int b) {
  if (b == 0) return x;
  const float t = x * (float)(1 << ((b - 1) >> 1));
  return (b & 1) ? sinpif(t) : cospif(t);
}

// G and the scene vector (F's input), L_d (R's), the mean's 1/max(c,1), T3's
// bias scale and dL/dy.  Padding pixels repeat the last pixel with dL/dy = 0,
// so every gradient they could carry is zero.  A null gbuf or scene (object
// streaming calls that do not run F or R) leaves those planes untouched.
__global__ __launch_bounds__(kThreads) void prep_kernel(PrepArgs a) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const bool valid = p < a.npx;
  const int64_t pc = valid ? p : a.npx - 1;
  const int f = (int)(pc / a.hw), q = (int)(pc - (int64_t)f * a.hw), hw = a.hw, W = a.W;
  const Blocks &B = a.bl;
  const int nblk = pe_blocks(a.pe);
  if (a.gbuf) {
    const float *G = a.gbuf + (size_t)f * kNG * hw + q;
    for (int c = 0; c < kNG; ++c) {
      const float x = G[(size_t)c * hw];
      for (int b = 0; b < nblk; ++b) ROW(B.xb + b * (kNG + kNS) + c)[p] = pe_value(x, b);
    }
    for (int c = 0; c < 3; ++c) ROW(B.pl + W + c)[p] = G[(size_t)(11 + c) * hw];
  }
  if (a.scene)
    for (int c = 0; c < kNS; ++c) {
      const float x = a.scene[(size_t)f * kNS + c];
      for (int b = 0; b < nblk; ++b) ROW(B.xb + b * (kNG + kNS) + kNG + c)[p] = pe_value(x, b);
    }
  float cnt = 0.0f;
  const float *Lf = a.layers + (size_t)f * a.k * kNL * hw + q;
  for (int i = 0; i < a.k; ++i) cnt += Lf[((size_t)i * kNL + kAlpha) * hw] > 0.0f ? 1.0f : 0.0f;
  if (a.perm && a.k > 1)      // slot i goes to its rank's row of the order table
    for (int i = 0; i < a.k; ++i)
      a.perm[(size_t)slot_rank(Lf, (size_t)hw, a.k, i) * a.npx_pad + p] = (uint8_t)i;
  const bool mean = a.pool == GN_POOL_MEAN;
  ROW(B.px + PX_INV)[p] = mean ? 1.0f / fmaxf(cnt, 1.0f) : 1.0f;
  ROW(B.zs + W)[p] = mean ? (cnt > 0.0f ? 1.0f : 0.0f) : cnt;
  for (int c = 0; c < kNOUT; ++c)
    ROW(B.dy + c)[p] = valid && a.grad_out ? a.grad_out[((size_t)f * kNOUT + c) * hw + q] : 0.0f;
}

// Step i's slot (the pixel's slot of rank i in canonical order, or slot i):
// its 12 channels (and their encodings) and its mask m_i = [alpha > 0].
__global__ __launch_bounds__(kThreads) void slot_gather_kernel(PrepArgs a, int step) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t pc = p < a.npx ? p : a.npx - 1;
  const int f = (int)(pc / a.hw), q = (int)(pc - (int64_t)f * a.hw), hw = a.hw;
  const int slot = a.perm && a.k > 1 ? (int)a.perm[(size_t)step * a.npx_pad + p] : step;
  const float *Li = a.layers + ((size_t)f * a.k + slot) * kNL * hw + q;
  const Blocks &B = a.bl;
  const int nblk = pe_blocks(a.pe);
  for (int c = 0; c < kNL; ++c) {
    const float x = Li[(size_t)c * hw];
    for (int b = 0; b < nblk; ++b) ROW(B.bi + b * kNL + c)[p] = pe_value(x, b);
  }
  ROW(B.px + PX_M)[p] = Li[(size_t)kAlpha * hw] > 0.0f ? 1.0f : 0.0f;
}

#undef ROW

// Object streaming: add the call's active-slot count of every pixel to the
// state's count row (or set it, on the first call).
__global__ __launch_bounds__(kThreads) void stream_count_kernel(const float *__restrict__ layers,
                                                                int k, int hw, int64_t npx,
                                                                float *__restrict__ cnt, int fresh) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= npx) return;
  const int f = (int)(p / hw), q = (int)(p - (int64_t)f * hw);
  const float *Lf = layers + (size_t)f * k * kNL * hw + q;
  float c = fresh ? 0.0f : cnt[p];
  for (int i = 0; i < k; ++i) c += Lf[((size_t)i * kNL + kAlpha) * hw] > 0.0f ? 1.0f : 0.0f;
  cnt[p] = c;
}

// Object streaming: the pool of Eq. (5) from the state, T3's input block:
// zs[r] = Z[r] / max(c, 1) (mean) or Z[r] (sum), and T3's bias scale row, as
// the forward's last slot epilogue and prep compute them.
__global__ __launch_bounds__(kThreads) void stream_pool_kernel(const float *__restrict__ Z,
                                                               const float *__restrict__ cnt,
                                                               int64_t npx, int W, int mean,
                                                               float *__restrict__ zs,
                                                               int64_t stride) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= npx) return;
  const float c = cnt[p];
  const float inv = mean ? 1.0f / fmaxf(c, 1.0f) : 1.0f;
  for (int r = 0; r < W; ++r) zs[(size_t)r * stride + p] = Z[(size_t)r * npx + p] * inv;
  zs[(size_t)W * stride + p] = mean ? (c > 0.0f ? 1.0f : 0.0f) : c;
}

// ---- weight gradients: sums over pixels on the fp32 matrix cores -----------
constexpr int kDwPx = 1024;     // pixels per chunk: one workgroup, one partial tile
constexpr size_t kDwLds = 160 * 1024;   // LDS bytes per workgroup
constexpr int kDwStep = 32;     // pixels per LDS stage: 8 chunks of 16 bytes per row
// LDS stages of dw_lds_kernel<MO, MI>, each (MO + MI) x 32 rows of kDwStep
// fp32: at most 4, and at least 2 for every shape with MO + MI <= 20.
constexpr int dw_lds_stages(int MO, int MI) {
  return (int)(kDwLds / ((size_t)(MO + MI) * 32 * kDwStep * 4)) < 4
             ? (int)(kDwLds / ((size_t)(MO + MI) * 32 * kDwStep * 4))
             : 4;
}

// part[chunk][o][i] (+)= sum over the chunk's pixels of D[o][p] A[i][p] for
// the whole (32 MO) x (32 MI) tile of one weight gradient; the four waves
// split it into 2 x 2 quadrants of (16 MO) x (16 MI) and each writes its own.
// Every 32-pixel step of D's and A's rows is copied into LDS once, with direct
// global->LDS loads, up to nst - 1 steps ahead of the matrix cores; row r keeps
// its 16-byte chunk c at slot c ^ (r & 7), so the rows that 8 lanes read
// together fall into distinct banks.  Lane l feeds row (l & 15) and the four
// pixels of chunk 4 h + (l >> 4) of step half h to both operands, so every
// pixel meets itself exactly once; the sums run in a fixed order.
template <int MO, int MI>
__global__ __launch_bounds__(kThreads) void dw_lds_kernel(const float *__restrict__ D,
                                                         const float *__restrict__ A,
                                                         int64_t stride, float *__restrict__ part,
                                                         int accumulate) {
  constexpr int nst = dw_lds_stages(MO, MI);
  constexpr int kRows = 32 * (MO + MI);          // D's rows, then A's
  constexpr int kStage = kRows * 8;              // 16-byte slots per stage
  constexpr int kFills = kStage / 256;           // fill instructions per wave per stage
  constexpr int kSteps = kDwPx / kDwStep;
  extern __shared__ __attribute__((aligned(16))) f32x4 slab[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, kq = lane >> 4;
  const int wo = wave >> 1, wi = wave & 1;
  const int chunk = blockIdx.x;
  const int64_t p0 = (int64_t)chunk * kDwPx;
  auto fill = [&](int st) {
    f32x4 *dst = slab + (size_t)(st % nst) * kStage;
    const int64_t px = p0 + (int64_t)st * kDwStep;
#pragma unroll
    for (int f = 0; f < kFills; ++f) {
      const int base = (f * 4 + wave) * 64;
      const int idx = base + lane, row = idx >> 3, c = (idx & 7) ^ (row & 7);
      const float *src = row < 32 * MO ? D + (size_t)row * stride
                                       : A + (size_t)(row - 32 * MO) * stride;
      __builtin_amdgcn_global_load_lds((const void *)(src + px + 4 * c),
                                       (__attribute__((address_space(3))) void *)(dst + base),
                                       16, 0, 0);
    }
  };
  f32x4 acc[MO][MI];
#pragma unroll
  for (int mo = 0; mo < MO; ++mo)
#pragma unroll
    for (int mi = 0; mi < MI; ++mi) acc[mo][mi] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int drow = 16 * MO * wo + r, arow = 32 * MO + 16 * MI * wi + r;
  for (int st = 0; st < nst - 1 && st < kSteps; ++st) fill(st);
  for (int st = 0; st < kSteps; ++st) {
    // stage st has landed once only the fills of later stages may be pending
    const int pend = min(nst - 2, kSteps - 1 - st);
    if (pend >= 2)
      asm volatile("s_waitcnt vmcnt(%0)" ::"n"(2 * kFills) : "memory");
    else if (pend == 1)
      asm volatile("s_waitcnt vmcnt(%0)" ::"n"(kFills) : "memory");
    else
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();     // stage st visible; every wave is done with stage st - 1
    if (st + nst - 1 < kSteps) fill(st + nst - 1);     // into stage st - 1's buffer
    const f32x4 *S = slab + (size_t)(st % nst) * kStage;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = 4 * h + kq;
      f32x4 d[MO], x[MI];
#pragma unroll
      for (int mo = 0; mo < MO; ++mo) {
        const int row = drow + 16 * mo;
        d[mo] = S[row * 8 + (c ^ (row & 7))];
      }
#pragma unroll
      for (int mi = 0; mi < MI; ++mi) {
        const int row = arow + 16 * mi;
        x[mi] = S[row * 8 + (c ^ (row & 7))];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int mo = 0; mo < MO; ++mo)
#pragma unroll
          for (int mi = 0; mi < MI; ++mi)
            acc[mo][mi] = __builtin_amdgcn_mfma_f32_16x16x4f32(d[mo][j], x[mi][j], acc[mo][mi],
                                                                0, 0, 0);
    }
  }
  constexpr int kIPad = 32 * MI;
  float *P = part + (size_t)chunk * (32 * MO) * kIPad;
#pragma unroll
  for (int mo = 0; mo < MO; ++mo)
#pragma unroll
    for (int mi = 0; mi < MI; ++mi)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int o = 16 * MO * wo + 16 * mo + 4 * kq + rr, i = 16 * MI * wi + 16 * mi + r;
        float *dst = P + (size_t)o * kIPad + i;
        *dst = accumulate ? *dst + acc[mo][mi][rr] : acc[mo][mi][rr];
      }
}

template <int MO, int MI>
static hipError_t launch_dw_lds(const float *D, const float *A, int64_t stride, float *part,
                                int accumulate, int nchunks, hipStream_t s) {
  constexpr int nst = dw_lds_stages(MO, MI);
  static_assert(nst >= 2, "dw_lds_kernel needs two LDS stages");
  constexpr size_t lds = (size_t)nst * (MO + MI) * 32 * kDwStep * 4;
  static bool attr_set = false;     // per process; the attribute is per function
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)dw_lds_kernel<MO, MI>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((dw_lds_kernel<MO, MI>), dim3((unsigned)nchunks), dim3(kThreads), lds, s, D,
                     A, stride, part, accumulate);
  return hipGetLastError();
}

// grad_w[layer][o][col0 + i] = sum_chunks part[c][o][i] (i < n_in);
// grad_w bias[o] = sum part[c][o][n_in] when has_bias.  A workgroup owns 16
// float4 columns of the padded (o_pad x i_pad) tile; its thread group g sums
// chunks g, g + 16, g + 32, ... in order and group 0 adds the 16 sums in group
// order, so the result does not depend on the launch.
__global__ __launch_bounds__(kThreads) void dw_reduce_kernel(const float *__restrict__ part,
                                                             int nchunks, int o_pad, int i_pad,
                                                             int n_out, int n_in, int has_bias,
                                                             float *__restrict__ gw, LayerOff lo,
                                                             int col0) {
  __shared__ f32x4 red[16][16];
  const int v = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int n4 = o_pad * i_pad / 4, e4 = blockIdx.x * 16 + v;
  f32x4 s = f32x4{0.f, 0.f, 0.f, 0.f};
  if (e4 < n4) {
    const f32x4 *src = (const f32x4 *)part + e4;
    int c = g;
    for (; c + 48 < nchunks; c += 64) {
      const f32x4 a0 = src[(size_t)c * n4], a1 = src[(size_t)(c + 16) * n4];
      const f32x4 a2 = src[(size_t)(c + 32) * n4], a3 = src[(size_t)(c + 48) * n4];
      s += a0;
      s += a1;
      s += a2;
      s += a3;
    }
    for (; c < nchunks; c += 16) s += src[(size_t)c * n4];
  }
  red[g][v] = s;
  __syncthreads();
  if (g != 0 || e4 >= n4) return;
  for (int k = 1; k < 16; ++k) s += red[k][v];
  const int o = 4 * e4 / i_pad, i0 = 4 * e4 - o * i_pad;
  if (o >= n_out) return;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int i = i0 + t;
    if (i < n_in)
      gw[lo.w + (int64_t)o * lo.in + col0 + i] = s[t];
    else if (has_bias && i == n_in)
      gw[lo.b + o] = s[t];
  }
}

__global__ void fill_kernel(float *dst, int64_t n, float v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) dst[e] = v;
}

// R's 3 output rows (plus their biases) into the caller's [n][3][hw] layout.
__global__ __launch_bounds__(kThreads) void scatter_out_kernel(const float *__restrict__ y,
                                                               int64_t stride, int64_t npx, int hw,
                                                               const float *__restrict__ b3,
                                                               float *__restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= npx) return;
  const int f = (int)(p / hw), q = (int)(p - (int64_t)f * hw);
  for (int c = 0; c < kNOUT; ++c)
    out[((size_t)f * kNOUT + c) * hw + q] = y[(size_t)c * stride + p] + b3[c];
}

// max over rows [0, n) and pixels [0, npx) of a non-negative plane block, as
// float bits (for non-negative floats the bit order is the value order).
__global__ __launch_bounds__(kThreads) void amax_kernel(const float *__restrict__ rows, int n,
                                                        int64_t stride, int64_t npx,
                                                        unsigned *amax) {
  __shared__ float red[kThreads];
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  float m = 0.0f;
  if (p < npx)
    for (int r = 0; r < n; ++r) m = fmaxf(m, rows[(size_t)r * stride + p]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(amax, __float_as_uint(red[0]));
}

}  // namespace

}  // namespace gn

using namespace gn;

void gn_bwd_free(gn_handle *h) {
  if (!h->bwd) return;
  (void)hipFree(h->bwd->planes);
  (void)hipFree(h->bwd->frag);
  (void)hipFree(h->bwd->part);
  (void)hipFree(h->bwd->part_t2);
  (void)hipFree(h->bwd->part_t1);
  (void)hipFree(h->bwd->perm);
  delete h->bwd;
  h->bwd = nullptr;
}

size_t gn_bwd_bytes(gn_handle *h) {
  if (!h->bwd) return 0;
  return h->bwd->plane_bytes + h->bwd->frag_bytes + h->bwd->part_bytes + h->bwd->part_t2_bytes +
         h->bwd->part_t1_bytes + h->bwd->perm_bytes;
}

static hipError_t ensure_workspace(gn_handle *h, int64_t npx_pad) {
  BwdWorkspace *ws = h->bwd;
  if (ws && ws->cap_px >= npx_pad) return hipSuccess;
  gn_bwd_free(h);
  ws = new BwdWorkspace();
  h->bwd = ws;
  const Blocks bl = make_blocks(h->W, h->pl.pe);
  const OpTable ops = make_ops(h->W, h->pl.pe);
  ws->W = h->W;
  ws->cap_px = npx_pad;
  ws->plane_bytes = sizeof(float) * (size_t)bl.rows * (npx_pad + kRowSkew);
  ws->frag_bytes = sizeof(f32x4) * (size_t)ops.total;
  ws->max_chunks = (int)((npx_pad + kDwPx - 1) / kDwPx);
  const int W = h->W, pe = h->pl.pe;
  // partial tiles: o_pad <= W rows; the widest input blocks are B1's
  // [sigma; tau; 1] and F1's encoded input (part), T2's (part_t2) and h's
  // encoded slot input (part_t1)
  const int wide = std::max(rup(2 * W + 1, 32), rup(enc_x(pe) + 1, 32));
  ws->part_bytes = sizeof(float) * (size_t)ws->max_chunks * W * wide;
  ws->part_t2_bytes = sizeof(float) * (size_t)ws->max_chunks * W * rup(W + 1, 32);
  ws->part_t1_bytes = sizeof(float) * (size_t)ws->max_chunks * W * rup(enc_b(pe) + 1, 32);
  hipError_t e = hipMalloc((void **)&ws->planes, ws->plane_bytes);
  if (e == hipSuccess) e = hipMalloc((void **)&ws->frag, ws->frag_bytes);
  if (e == hipSuccess) e = hipMalloc((void **)&ws->part, ws->part_bytes);
  if (e == hipSuccess) e = hipMalloc((void **)&ws->part_t2, ws->part_t2_bytes);
  if (e == hipSuccess) e = hipMalloc((void **)&ws->part_t1, ws->part_t1_bytes);
  // the slot-order table: one byte per slot of the handle's largest count
  ws->perm_bytes = (size_t)std::max(h->cfg.k_max, 1) * npx_pad;
  if (e == hipSuccess) e = hipMalloc((void **)&ws->perm, ws->perm_bytes);
  if (e != hipSuccess) gn_bwd_free(h);
  return e;
}

static hipError_t fill(float *dst, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, n, v);
  return hipGetLastError();
}

// Zero every plane (padding rows are read as zero K rows by the GEMMs) and
// write the rows of ones, for a given plane row length.
static hipError_t init_constant_rows(gn_handle *h, int64_t stride, hipStream_t s) {
  BwdWorkspace *ws = h->bwd;
  if (ws->stride == stride) return hipSuccess;
  const Blocks bl = make_blocks(h->W, h->pl.pe);
  const int W = h->W;
  hipError_t e = fill(ws->planes, (int64_t)bl.rows * stride, 0.0f, s);
  const int pe = h->pl.pe;
  const int ones[] = {bl.xb + enc_x(pe), bl.a1 + W, bl.a2 + W, bl.st + 2 * W, bl.d1 + W,
                      bl.d2 + W, bl.pl + W + 3, bl.g1 + W, bl.g2 + W, bl.z1 + W,
                      bl.bi + enc_b(pe)};
  for (int r : ones)
    if (e == hipSuccess) e = fill(ws->planes + (size_t)r * stride, stride, 1.0f, s);
  if (e == hipSuccess) ws->stride = stride;
  return e;
}

struct GemmJob {
  int dblock, o_pad, ablock, i_pad;   // plane rows
  Layer layer;
  int n_out, n_in, has_bias, col0;
};

// One call of the plane pipeline over a frame batch.  begin() validates the
// size, prepares the workspace and operand fragments and gathers the inputs;
// the phases enqueue their launches on the call's stream in order.
class Pipeline {
 public:
  Pipeline(gn_handle *h, hipStream_t s)
      : h_(h), s_(s), W_(h->W), pe_(h->pl.pe), bl_(make_blocks(h->W, h->pl.pe)),
        ops_(make_ops(h->W, h->pl.pe)) {
    layer_offsets(W_, pe_, lo_);
  }

  // canonical: pool each pixel's slots in canonical order (object streaming
  // passes false: it adds objects in call order).
  gn_status begin(const gn_frame *f, const float *grad_out, const char *what,
                  bool canonical = true) {
    const int64_t hw = (int64_t)f->h * f->w;
    npx_ = (int64_t)f->n * hw;
    npx_pad_ = (npx_ + kChunkPx - 1) / kChunkPx * kChunkPx;
    ld_ = npx_pad_ + kRowSkew;
    if (npx_pad_ > kMaxPx) return gn_set_error(GN_E_INVAL, "more than 3 * 2^20 pixels in one call");
    hw_ = (int)hw;
    K_ = f->k;
    e_ = ensure_workspace(h_, npx_pad_);
    if (e_ == hipSuccess) e_ = init_constant_rows(h_, ld_, s_);
    if (e_ != hipSuccess) return gn_check_device(h_, e_, what);
    ws_ = h_->bwd;
    wm_ = h_->d_master;
    pa_.gbuf = f->gbuf;
    pa_.layers = f->layers;
    pa_.scene = f->scene;
    pa_.grad_out = grad_out;
    pa_.hw = hw_;
    pa_.k = K_;
    pa_.pool = h_->cfg.pool;
    pa_.W = W_;
    pa_.pe = pe_;
    pa_.npx = npx_;
    pa_.stride = ld_;
    pa_.planes = ws_->planes;
    pa_.perm = canonical && gn_slot_kmax(h_) > 1 ? ws_->perm : nullptr;
    pa_.npx_pad = npx_pad_;
    pa_.bl = bl_;
    hipLaunchKernelGGL(pack_ops_kernel, dim3((unsigned)((ops_.total + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s_, wm_, ops_, ws_->frag);
    hipLaunchKernelGGL(prep_kernel, pgrid(), dim3(kThreads), 0, s_, pa_);
    return GN_OK;
  }

  // F, then u = W_T1,sigma sigma + b_T1 (the sigma-hoist).
  void trunk() {
    fwd(O_F1, bl_.xb, bl_.a1, L_F1, true);
    fwd(O_F2, bl_.a1, bl_.a2, L_F2, true);
    fwd(O_F3, bl_.a2, bl_.st, L_F3, false);                  // sigma
    fwd(O_T1S, bl_.st, bl_.u, L_T1, false);                  // u
  }

  // Z = sum_i m_i relu(W_T2 z1_i + b_T2), an fp32 running sum over the
  // slots in gather order, then / max(c, 1) for the mean.
  void slots() {
    const bool mean = h_->cfg.pool == GN_POOL_MEAN;
    for (int i = 0; i < K_; ++i) {
      gather(i);
      z1();
      PgArgs a = args();
      a.bias = wm_ + lo_[L_T2].b;
      a.relu = 1;
      a.pscale = plane(bl_.px + PX_M);
      a.accumulate = i > 0;
      if (i == K_ - 1 && mean) a.post = plane(bl_.px + PX_INV);
      gemm(O_T2, EP_FWD, bl_.z1, bl_.zs, a);
    }
    if (K_ == 0) fill_rows(bl_.zs, W_);
  }

  // T3 (tau), B (phi) and R's hidden layers.
  void head() {
    PgArgs a = args();                                       // tau = W_T3 zs + bs b_T3
    a.bias = wm_ + lo_[L_T3].b;
    a.bscale = plane(bl_.zs + W_);
    gemm(O_T3, EP_FWD, bl_.zs, bl_.st + W_, a);
    fwd(O_B1, bl_.st, bl_.d1, L_B1, true);
    fwd(O_B2, bl_.d1, bl_.d2, L_B2, true);
    fwd(O_B3, bl_.d2, bl_.pl, L_B3, false);                  // phi
    fwd(O_R1, bl_.pl, bl_.g1, L_R1, true);
    fwd(O_R2, bl_.g1, bl_.g2, L_R2, true);
  }

  // R's last layer (no bias in the GEMM: its 3 biases are added while the
  // rows are scattered into the caller's [n][3][h][w] output).
  void output(float *out) {
    gemm(O_R3, EP_FWD, bl_.g2, bl_.y, args());
    hipLaunchKernelGGL(scatter_out_kernel, pgrid(), dim3(kThreads), 0, s_, plane(bl_.y),
                       ld_, npx_, hw_, wm_ + lo_[L_R3].b, out);
  }

  // FP8 calibration: the largest first-layer activation of h over every slot
  // of every pixel, as float bits (non-negative, so bit order = value order).
  void calibrate(unsigned *amax) {
    for (int i = 0; i < K_; ++i) {
      gather(i);
      z1();
      hipLaunchKernelGGL(amax_kernel, pgrid(), dim3(kThreads), 0, s_, plane(bl_.z1), W_,
                         ld_, npx_, amax);
    }
  }

  // dL/dw given the forward planes (trunk, slots, head) and dL/dy (begin).
  void backward(float *grad_w) {
    const bool mean = h_->cfg.pool == GN_POOL_MEAN;
    const int W = W_;
    // ---- head: R^T, B^T -> (dsigma_B, dtau) -> dZ
    bwd(O_R3T, bl_.dy, bl_.dg2, bl_.g2);
    bwd(O_R2T, bl_.dg2, bl_.dg1, bl_.g1);
    bwd(O_R1T, bl_.dg1, bl_.dphi, -1);
    bwd(O_B3T, bl_.dphi, bl_.dd2, bl_.d2);
    bwd(O_B2T, bl_.dd2, bl_.dd1, bl_.d1);
    bwd(O_B1T, bl_.dd1, bl_.dsig, -1);                        // dsigma_B and dtau
    {
      PgArgs a = args();                                      // dZ = W_T3^T dtau / max(c,1)
      if (mean) a.pscale = plane(bl_.px + PX_INV);
      gemm(O_T3T, EP_BWD, bl_.dtau, bl_.dzin, a);
    }
    // ---- slot loop
    const int RW = rup(W + 1, 32);
    const GemmJob jT2{bl_.dz2, W, bl_.z1, RW, L_T2, W, W, 1, 0};
    const int nb = enc_b(pe_), nx = enc_x(pe_);
    const GemmJob jT1a{bl_.dz1, W, bl_.bi, rup(nb + 1, 32), L_T1, W, nb, 1, 0};
    for (int i = 0; i < K_; ++i) {
      gather(i);
      z1();
      {
        PgArgs a = args();                                    // dz2 = [z2 > 0] m_i dZ
        a.bias = wm_ + lo_[L_T2].b;
        a.add = plane(bl_.dzin);
        a.pscale = plane(bl_.px + PX_M);
        gemm(O_T2, EP_DZ2, bl_.z1, bl_.dz2, a);
      }
      {
        PgArgs a = args();                                    // dz1 = [z1 > 0] W_T2^T dz2; du += dz1
        a.mask = plane(bl_.z1);
        a.out2 = plane(bl_.du);
        a.accumulate2 = i > 0;
        gemm(O_T2T, EP_BWD, bl_.dz2, bl_.dz1, a);
      }
      dw_gemm(jT2, ws_->part_t2, ws_->part_t2_bytes, i > 0);
      dw_gemm(jT1a, ws_->part_t1, ws_->part_t1_bytes, i > 0);
    }
    // with no slot, T2 and T1's slot columns and bias get zero gradient (no chunks)
    reduce(jT2, ws_->part_t2, K_ > 0 ? nchunks() : 0, grad_w);
    reduce(jT1a, ws_->part_t1, K_ > 0 ? nchunks() : 0, grad_w);
    // ---- tail
    if (K_ > 0) {
      PgArgs a = args();                                      // dsigma += W_T1,sigma^T du
      a.add = plane(bl_.dsig);
      gemm(O_T1ST, EP_BWD, bl_.du, bl_.dsig, a);
    } else {
      fill_rows(bl_.du, W);
    }
    bwd(O_F3T, bl_.dsig, bl_.da2, bl_.a2);
    bwd(O_F2T, bl_.da2, bl_.da1, bl_.a1);
    // ---- weight gradients
    const GemmJob jobs[] = {
        {bl_.dy, 32, bl_.g2, RW, L_R3, kNOUT, W, 1, 0},
        {bl_.dg2, W, bl_.g1, RW, L_R2, W, W, 1, 0},
        {bl_.dg1, W, bl_.pl, rup(W + 4, 32), L_R1, W, W + 3, 1, 0},
        {bl_.dphi, W, bl_.d2, RW, L_B3, W, W, 1, 0},
        {bl_.dd2, W, bl_.d1, RW, L_B2, W, W, 1, 0},
        {bl_.dd1, W, bl_.st, rup(2 * W + 1, 32), L_B1, W, 2 * W, 1, 0},
        {bl_.dtau, W, bl_.zs, RW, L_T3, W, W, 1, 0},
        {bl_.du, W, bl_.st, W, L_T1, W, W, 0, nb},
        {bl_.dsig, W, bl_.a2, RW, L_F3, W, W, 1, 0},
        {bl_.da2, W, bl_.a1, RW, L_F2, W, W, 1, 0},
        {bl_.da1, W, bl_.xb, rup(nx + 1, 32), L_F1, W, nx, 1, 0},
    };
    for (const GemmJob &j : jobs) {
      dw_gemm(j, ws_->part, ws_->part_bytes, 0);
      reduce(j, ws_->part, nchunks(), grad_w);
    }
  }

  // ---- object streaming: the state is [sigma (W rows); Z (W rows); count]
  // of npx fp32 elements per row.  begin: F, sigma out.  accumulate: sigma
  // in, u, the call's slots added to Z (continued from the state unless
  // fresh), the count.  finish: sigma and the pool in, T3, B, R.  The
  // arithmetic and its order are the input-order forward's.
  void stream_begin(float *state) {
    trunk();
    copy_rows(state, npx_, plane(bl_.st), ld_, W_);
  }
  void stream_accumulate(float *state, bool fresh) {
    copy_rows(plane(bl_.st), ld_, state, npx_, W_);
    fwd(O_T1S, bl_.st, bl_.u, L_T1, false);                  // u, as in trunk()
    float *z = state + (size_t)W_ * npx_;
    if (!fresh) copy_rows(plane(bl_.zs), ld_, z, npx_, W_);
    for (int i = 0; i < K_; ++i) {
      gather(i);
      z1();
      PgArgs a = args();
      a.bias = wm_ + lo_[L_T2].b;
      a.relu = 1;
      a.pscale = plane(bl_.px + PX_M);
      a.accumulate = i > 0 || !fresh;
      gemm(O_T2, EP_FWD, bl_.z1, bl_.zs, a);
    }
    if (K_ > 0 || fresh) {
      if (K_ == 0) fill_rows(bl_.zs, W_);
      copy_rows(z, npx_, plane(bl_.zs), ld_, W_);
    }
    hipLaunchKernelGGL(stream_count_kernel, pgrid(), dim3(kThreads), 0, s_, pa_.layers, K_, hw_,
                       npx_, state + (size_t)2 * W_ * npx_, fresh ? 1 : 0);
  }
  void stream_finish(const float *state, bool fresh, float *out) {
    copy_rows(plane(bl_.st), ld_, state, npx_, W_);
    if (fresh) {
      fill_rows(bl_.zs, W_ + 1);           // no object: empty pool, zero bias scale
    } else {
      hipLaunchKernelGGL(stream_pool_kernel, pgrid(), dim3(kThreads), 0, s_,
                         (const float *)(state + (size_t)W_ * npx_),
                         state + (size_t)2 * W_ * npx_, npx_, W_,
                         h_->cfg.pool == GN_POOL_MEAN ? 1 : 0, plane(bl_.zs), ld_);
    }
    head();
    output(out);
  }

  gn_status finish(const char *what) {
    if (e_ == hipSuccess) e_ = hipGetLastError();
    return gn_check_device(h_, e_, what);
  }

 private:
  dim3 pgrid() const { return dim3((unsigned)(npx_pad_ / kThreads)); }
  int nchunks() const { return (int)(npx_pad_ / kDwPx); }
  float *plane(int r) const { return ws_->planes + (size_t)r * ld_; }
  static PgArgs args() {
    PgArgs a;
    memset(&a, 0, sizeof a);
    return a;
  }
  void fill_rows(int row, int n) {
    if (e_ == hipSuccess) e_ = fill(plane(row), (int64_t)n * ld_, 0.0f, s_);
  }
  void gather(int i) {
    hipLaunchKernelGGL(slot_gather_kernel, pgrid(), dim3(kThreads), 0, s_, pa_, i);
  }
  // n rows of npx elements between row-major blocks of different row lengths
  template <class T>
  void copy_rows(T *dst, int64_t dst_len, const T *src, int64_t src_len, int n) {
    if (e_ == hipSuccess)
      e_ = hipMemcpy2DAsync(dst, sizeof(T) * dst_len, src, sizeof(T) * src_len, sizeof(T) * npx_,
                            n, hipMemcpyDeviceToDevice, s_);
  }

  // One plane GEMM: op `o` from block `xrow` into block `orow`.
  void gemm(Op o, int ep, int xrow, int orow, PgArgs a) {
    const OpDesc &d = ops_.op[o];
    a.frag = ws_->frag + d.off;
    a.kq = d.kq;
    a.stride = ld_;
    a.x = plane(xrow);
    a.out = plane(orow);
    const dim3 block(kThreads);
    if (d.mt < 4) {             // R3: one 16-row tile, 64-pixel waves
      const dim3 grid((unsigned)(npx_pad_ / kThreads), 1);
      hipLaunchKernelGGL((plane_gemm_kernel<1, EP_FWD, 1>), grid, block, 0, s_, a);
      return;
    }
    // 64-row waves; two waves share a pixel group when the op has 128+ rows
    const int rsplit = d.mt >= 8 ? 2 : 1;
    const dim3 grid((unsigned)(npx_pad_ / (kThreads / rsplit)), (unsigned)(d.mt / (4 * rsplit)));
#define PG(EP, RS) hipLaunchKernelGGL((plane_gemm_kernel<4, EP, RS>), grid, block, 0, s_, a)
    if (rsplit == 2) {
      if (ep == EP_FWD) PG(EP_FWD, 2); else if (ep == EP_DZ2) PG(EP_DZ2, 2); else PG(EP_BWD, 2);
    } else {
      if (ep == EP_FWD) PG(EP_FWD, 1); else if (ep == EP_DZ2) PG(EP_DZ2, 1); else PG(EP_BWD, 1);
    }
#undef PG
  }
  void fwd(Op o, int xrow, int orow, Layer l, bool relu) {
    PgArgs a = args();
    a.bias = wm_ + lo_[l].b;
    a.relu = relu;
    gemm(o, EP_FWD, xrow, orow, a);
  }
  void bwd(Op o, int xrow, int orow, int maskrow) {
    PgArgs a = args();
    if (maskrow >= 0) a.mask = plane(maskrow);
    gemm(o, EP_BWD, xrow, orow, a);
  }
  void z1() {                                                // z1_i = relu(W_T1,b b_i + u)
    PgArgs a = args();
    a.add = plane(bl_.u);
    a.relu = 1;
    gemm(O_T1A, EP_FWD, bl_.bi, bl_.z1, a);
  }
  void dw_gemm(const GemmJob &j, float *part, size_t part_bytes, int accumulate) {
    // the whole (o_pad x i_pad) gradient per workgroup, operands staged in LDS
    const int MO = j.o_pad / 32, MI = j.i_pad / 32;
    if (sizeof(float) * (size_t)nchunks() * j.o_pad * j.i_pad > part_bytes) {
      if (e_ == hipSuccess) e_ = hipErrorInvalidValue;     // partials would not fit
      return;
    }
    const float *D = plane(j.dblock), *Ap = plane(j.ablock);
#define DL(A, B)                                                                       \
  if (MO == A && MI == B) {                                                            \
    const hipError_t e = launch_dw_lds<A, B>(D, Ap, ld_, part, accumulate, nchunks(), s_); \
    if (e_ == hipSuccess) e_ = e;                                                      \
    return;                                                                            \
  }
    DL(1, 5) DL(4, 5) DL(4, 9) DL(4, 4) DL(4, 1)     // W = 128
    DL(4, 3) DL(4, 7) DL(4, 2)                       //   with encoded inputs
    DL(1, 3) DL(2, 3) DL(2, 5) DL(2, 2) DL(2, 1)     // W = 64
    DL(2, 7) DL(2, 9) DL(2, 4)                       //   with encoded inputs
#undef DL
    e_ = hipErrorInvalidValue;     // no other gradient shape exists for the widths and levels
  }
  void reduce(const GemmJob &j, const float *part, int nch, float *grad_w) {
    const int n4 = j.o_pad * j.i_pad / 4;
    hipLaunchKernelGGL(dw_reduce_kernel, dim3((n4 + 15) / 16), dim3(kThreads), 0, s_, part, nch,
                       j.o_pad, j.i_pad, j.n_out, j.n_in, j.has_bias, grad_w, lo_[j.layer], j.col0);
  }

  gn_handle *h_;
  hipStream_t s_;
  int W_, pe_;
  Blocks bl_;
  OpTable ops_;
  LayerOff lo_[kNumLayers];
  BwdWorkspace *ws_ = nullptr;
  const float *wm_ = nullptr;
  PrepArgs pa_{};
  int64_t npx_ = 0, npx_pad_ = 0, ld_ = 0;   // pixels, padded pixels, plane row pitch
  int hw_ = 0, K_ = 0;
  hipError_t e_ = hipSuccess;
};

// Runs fn(pipeline) on the handle's device; restores the caller's device.
template <class Fn>
static gn_status with_device(gn_handle *h, Fn fn) {
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (hipSetDevice(h->device) != hipSuccess) return gn_set_error(GN_E_DEVICE, "hipSetDevice failed");
  const gn_status st = fn();
  if (prev >= 0) (void)hipSetDevice(prev);
  return st;
}

gn_status gn_planes_forward(gn_handle *h, const gn_frame *frame, float *out, hipStream_t s) {
  return with_device(h, [&]() {
    Pipeline p(h, s);
    gn_status st = p.begin(frame, nullptr, "fp32 forward");
    if (st != GN_OK) return st;
    p.trunk();
    p.slots();
    p.head();
    p.output(out);
    return p.finish("fp32 forward");
  });
}

gn_status gn_planes_calibrate(gn_handle *h, const gn_frame *frame, unsigned *amax, hipStream_t s) {
  return with_device(h, [&]() {
    Pipeline p(h, s);
    gn_status st = p.begin(frame, nullptr, "calibration");
    if (st != GN_OK) return st;
    p.trunk();
    p.calibrate(amax);
    return p.finish("calibration");
  });
}

// Object streaming on the plane pipeline (GN_FP32 handles); state holds
// gn_planes_stream_bytes floats.
size_t gn_planes_stream_bytes(int W, int64_t npx) {
  return sizeof(float) * (size_t)(2 * W + 1) * (size_t)npx;   // sigma, Z, count
}

gn_status gn_planes_stream(gn_handle *h, const gn_frame *frame, int mode, float *state, int fresh,
                           float *out, hipStream_t s) {
  return with_device(h, [&]() {
    Pipeline p(h, s);
    gn_status st = p.begin(frame, nullptr, "fp32 stream", false);
    if (st != GN_OK) return st;
    if (mode == FWD_BEGIN)
      p.stream_begin(state);
    else if (mode == FWD_ACC)
      p.stream_accumulate(state, fresh != 0);
    else
      p.stream_finish(state, fresh != 0, out);
    return p.finish("fp32 stream");
  });
}

extern "C" gn_status glassnet_backward(gn_handle *h, const gn_frame *frame,
                                       const float *grad_out, float *grad_w, void *hip_stream) {
  if (!h) return gn_set_error(GN_E_INVAL, "handle is NULL");
  if (h->poisoned) return gn_set_error(GN_E_DEVICE, "handle poisoned by an earlier device error");
  if (!grad_out || !grad_w || ((uintptr_t)grad_out & 3) || ((uintptr_t)grad_w & 3))
    return gn_set_error(GN_E_INVAL, "grad_out and grad_w must be non-NULL, 4-byte aligned");
  gn_status st = gn_validate_frame(h, frame, nullptr);
  if (st != GN_OK) return st;
  return with_device(h, [&]() {
    Pipeline p(h, (hipStream_t)hip_stream);
    gn_status st2 = p.begin(frame, grad_out, "backward workspace");
    if (st2 != GN_OK) return st2;
    p.trunk();
    p.slots();
    p.head();
    p.backward(grad_w);
    return p.finish("backward launch");
  });
}
