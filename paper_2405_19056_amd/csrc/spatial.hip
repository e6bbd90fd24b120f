// The spatial GlassNet networks (Sec. 3.4): F and B as U-Nets, h and R as
// CNNs whose first layers are 3 x 3 convolutions, on the gfx950 matrix cores
// (bf16 operands, fp32 accumulation).
//
// Reading of the architecture (the paper gives no widths, depths or levels):
//   U-Net (F on [G; s], B on [sigma; tau]): e1 = relu(conv3 x); d = 2 x 2
//     average of e1; m = relu(conv3 d) at half resolution; u = m repeated
//     2 x 2; e2 = relu(conv3 [e1; u]); out = conv1 e2.
//   h(b_i, sigma) = conv1 relu(conv1 relu(conv3 [b_i; sigma])); the pool of
//     Eq. (5) per pixel over the buffers with alpha > 0 there.
//   R = conv1 relu(conv3 relu(conv3 [phi; L_d])) with 3 outputs.
// conv3: 3 x 3, zero padding of one pixel; conv1: 1 x 1; every conv has a
// bias.  Width W (64 or 128) throughout.
//
// Layout.  Activations live in HBM as bf16 [n][H][W][C] (channels innermost,
// C a multiple of 32), so the 8 channels one lane presents to the matrix
// core for one pixel are one 16-byte load.  Every conv is an implicit GEMM,
// Y^T = A X^T: the weights are the A operand (16 output channels per M-tile),
// 16 pixels of one row the B operand, K = (tap, input channel) in 32-deep
// steps; the zero padding is a zero B fragment.  Two inputs can be
// concatenated along the channels, the second optionally at half resolution
// and read through a 2 x 2 nearest upsample (the U-Net's skip join), so the
// concatenation and the upsample are never materialised.
//
// Work split.  A workgroup of 8 waves owns 512 output pixels, each wave 64
// consecutive pixels of one row (4 N-tiles) and every output channel (up to
// 8 M-tiles: 32 accumulators of 4 floats).  The weights stream through LDS
// in chunks of kChunk K-steps (direct global->LDS copies, two buffers, one
// chunk ahead), every fragment read once per wave and used for its 4 N-tiles.
// The input fragments of the next K-step are loaded while the current one's
// MFMAs run.
//
// Epilogues: bias, ReLU, then one of: bf16 activation store, fp32 store, or
// R's 3 outputs to the caller's [n][3][H][W] fp32 image.
//
// h over the buffers, the pool and T's last layer run in one kernel of their
// own (sp_slots_kernel below): the per-buffer activations and the running
// sum stay on the chip.  (The generic table also packs T's layers as
// ordinary convs; only their biases are read from it.)
#include <algorithm>

#include "gn_internal.h"

namespace gn {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 8, kThreads = kWaves * 64;
// N-tiles (16 pixels) per wave of the generic conv: 4 for the narrow convs,
// 2 for the W = 128 ones (half the registers: two workgroups per CU, four
// waves per SIMD to hide the input loads' latency)
constexpr int kChunk = 4;                    // K-steps per LDS weight chunk (even)
static_assert(kChunk % 2 == 0, "the conv loop takes the steps of a chunk in pairs");

// K-steps of a conv's packed weights: taps x 32-channel blocks, rounded up to
// whole chunks with zero fragments (the conv loop then runs whole chunks,
// straight-line code the compiler keeps its loads ahead in).
__host__ __device__ inline int padded_steps(int taps, int cbt) {
  return (taps * cbt + kChunk - 1) / kChunk * kChunk;
}
constexpr int kFrag = 1024;                  // one A fragment: 64 lanes x 16 bytes

__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, bf16x2));
}

__device__ __forceinline__ f32x4 mma(u32x4 a, u32x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t v) {
  return __uint_as_float((uint32_t)v << 16);
}

// Input loads go through buffer resources bounded by the input's size: a
// load at an offset past the bound returns zeros (the conv's zero padding),
// so no select on the loaded value holds up the next K-step's loads.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr uint32_t kOutside = 0x80000000u;     // past every bound (inputs stay under 2 GiB)
__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                           0x00020000);
}
__device__ __forceinline__ u32x4 bld(rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

}  // namespace

// One convolution launch (host fills it; see SpConv in the launcher).
struct SpConvArgs {
  const uint8_t *in0;       // bf16 [n][H][W][c0]
  const uint8_t *in1;       // bf16 [n][H1][W1][c1] or null; up1: H1 = H / 2, W1 = W / 2
  int c0, c1, up1;
  const uint8_t *wfrag;     // A fragments [step][mt][lane] (16 B each)
  const float *bias;        // [MT * 16] (zero past the real outputs)
  int steps;                // K-steps = taps x (c0 + c1) / 32
  int steps_pad;            // the packed steps: steps rounded up to whole chunks
  int ksize;                // 1 or 3
  int n, H, Wd;             // output (= in0) size
  int cout_pad;             // output channel count of the bf16 / fp32 layouts (MT * 16)
  // epilogue
  int relu;
  uint8_t *out_bf;          // bf16 [n][H][W][cout_pad], or null
  float *out_f32;           // fp32 [n][H][W][cout_pad], or null
  float *out_rgb;           // fp32 [n][3][H][W] (3 real outputs), or null
};

namespace {

template <int MT, int kNT>
__global__ __launch_bounds__(kThreads, kNT == 2 ? 4 : 1) void sp_conv_kernel(SpConvArgs a) {
  constexpr int kWavePx = kNT * 16;            // pixels per wave (one row segment)
  extern __shared__ __attribute__((aligned(1024))) uint8_t lds[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, col = lane & 15;
  const int H = a.H, Wd = a.Wd;
  const int segs = (Wd + kWavePx - 1) / kWavePx;          // row segments per row
  // Workgroups reach the 8 XCDs round-robin: give each XCD a contiguous run
  // of tiles, so that the rows a 3 x 3 conv reads twice more (for the rows
  // above and below) are mostly in its own L2.
  const int full = gridDim.x & ~7;
  const int tile = (int)blockIdx.x < full ? (blockIdx.x & 7) * (full >> 3) + (blockIdx.x >> 3)
                                          : (int)blockIdx.x;
  const int64_t seg = (int64_t)tile * kWaves + wave;
  const int64_t nseg = (int64_t)a.n * H * segs;
  const bool live = seg < nseg;
  const int64_t sg = live ? seg : nseg - 1;
  // the wave's row segment (wave-uniform)
  const int f = __builtin_amdgcn_readfirstlane((int)(sg / ((int64_t)H * segs)));
  const int rem = (int)(sg - (int64_t)f * H * segs);
  const int y = __builtin_amdgcn_readfirstlane(rem / segs);
  const int x0 = __builtin_amdgcn_readfirstlane((rem - (rem / segs) * segs) * kWavePx);
  const int r = a.ksize >> 1;
  const int cb0 = a.c0 >> 5;                              // 32-channel blocks of in0
  const int cbt = (a.c0 + a.c1) >> 5;

  constexpr int kChunkBytes = kChunk * MT * kFrag;
  const int nchunks = a.steps_pad / kChunk;
  auto fill = [&](int c) {
    const uint8_t *src = a.wfrag + (int64_t)c * kChunkBytes;
    // a compile-time count of copies per wave (the compiler then knows how
    // many vector-memory operations are in flight behind them)
    constexpr int kCopies = (kChunk * MT + kWaves - 1) / kWaves;
#pragma unroll
    for (int i = 0; i < kCopies; ++i) {
      const int off = (i * kWaves + wave) * kFrag;
      if (off >= kChunkBytes) break;
      __builtin_amdgcn_global_load_lds((const void *)(src + off + lane * 16),
                                       (__attribute__((address_space(3))) void *)(lds + (c & 1) * kChunkBytes + off),
                                       16, 0, 0);
    }
  };

  // B fragment of K-step s for N-tile t: pixel (y + dy - r, x0 + 16 t + col + dx - r),
  // channels 32 cb + 8 g .. + 7 of the concatenated input; outside the frame
  // the offset is past the buffer's bound and the load returns zeros.  Every
  // lane loads, so each step issues exactly kNT loads: the chunk waits below
  // count on that.
  const int H1 = a.up1 ? H >> 1 : H, W1 = a.up1 ? Wd >> 1 : Wd;
  const uint8_t *in0 = a.in0, *in1 = a.in1 ? a.in1 : a.in0;
  const uint32_t bytes0 = (uint32_t)((int64_t)a.n * H * Wd * a.c0 * 2);
  const uint32_t bytes1 = (uint32_t)((int64_t)a.n * H1 * W1 * a.c1 * 2);
  auto load_b = [&](int s, u32x4 (&b)[kNT]) {
    const int tap = s / cbt, cb = s - tap * cbt;
    const int dy = tap / a.ksize - r, dx = tap % a.ksize - r;
    const int yy = y + dy;
    const bool yok = yy >= 0 && yy < H;
    const int yc = min(max(yy, 0), H - 1);
    const bool first = cb < cb0;
    const int shift = first ? 0 : a.up1;
    const int cs = first ? a.c0 : a.c1;
    // byte offset of the row's first pixel and the channel block
    const uint32_t rowoff =
        first ? (uint32_t)((((int64_t)f * H + yc) * Wd * a.c0 + 32 * cb) * 2)
              : (uint32_t)((((int64_t)f * H1 + (yc >> shift)) * W1 * a.c1 + 32 * (cb - cb0)) * 2);
    uint32_t off[kNT];
#pragma unroll
    for (int t = 0; t < kNT; ++t) {
      const int xx = x0 + 16 * t + col + dx;
      const bool ok = yok && xx >= 0 && xx < Wd;
      off[t] = ok ? rowoff + (uint32_t)((((xx >> shift) * cs) + 8 * g) * 2) : kOutside;
    }
    // the source is wave-uniform: its resource is built in scalar registers
    const rsrc_t rs = make_rsrc(first ? in0 : in1, first ? bytes0 : bytes1);
#pragma unroll
    for (int t = 0; t < kNT; ++t) b[t] = bld(rs, off[t]);
  };

  f32x4 acc[kNT][MT];
#pragma unroll
  for (int t = 0; t < kNT; ++t)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[t][mt] = f32x4{0.f, 0.f, 0.f, 0.f};

  // one K-step: all MT weight fragments requested from LDS first (held there
  // by a scheduling barrier, else each read sinks next to its MFMAs and is
  // waited for alone), then the MFMAs
  // (With two N-tiles per wave the fragments come in two groups of MT / 2,
  // the second group's reads issued behind the first group's MFMAs: fewer
  // registers, for four waves per SIMD.)
  auto step = [&](const uint8_t *Ws, const u32x4 (&b)[kNT]) {
    constexpr int kG = kNT >= 4 || MT < 8 ? MT : MT / 2;
#pragma unroll
    for (int m0 = 0; m0 < MT; m0 += kG) {
      u32x4 w[kG];
#pragma unroll
      for (int i = 0; i < kG; ++i) w[i] = *(const u32x4 *)(Ws + (m0 + i) * kFrag + lane * 16);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < kG; ++i)
#pragma unroll
        for (int t = 0; t < kNT; ++t) acc[t][m0 + i] = mma(w[i], b[t], acc[t][m0 + i]);
      __builtin_amdgcn_sched_barrier(0);
    }
  };

  fill(0);
  // Two input sets: b0 holds the current step's fragments (chunks have an
  // even step count, so each chunk starts with its first step in b0); the
  // next step's loads (clamped to the last step: a harmless re-read) are in
  // flight while the current step's MFMAs run.
  u32x4 b0[kNT], b1[kNT];
  load_b(0, b0);
  for (int c = 0; c < nchunks; ++c) {
    // The chunk's weights have landed: each wave waits for its own copies,
    // then for everyone's.  Issued after the copies of chunk c (at the start
    // of chunk c - 1) are only the input loads of chunk c - 1's steps, kNT per
    // step, the last kChunk kNT of them still allowed in flight.
    // (A plain __syncthreads would also drain those input loads.)  The
    // LDS reads of the buffer the next fill overwrites are drained too.
    if (c == 0)
      asm volatile("s_waitcnt vmcnt(0)\n\ts_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    else
      asm volatile("s_waitcnt vmcnt(%0)\n\ts_waitcnt lgkmcnt(0)\n\ts_barrier" ::"n"(kChunk * kNT)
                   : "memory");
    if (c + 1 < nchunks) fill(c + 1);
    const uint8_t *Wc = lds + (c & 1) * kChunkBytes;
    const int s0 = c * kChunk;
    // steps past the real ones multiply zero weights (their inputs re-read
    // the last real step's)
#pragma unroll
    for (int j = 0; j < kChunk; j += 2) {
      load_b(min(s0 + j + 1, a.steps - 1), b1);
      __builtin_amdgcn_sched_barrier(0);
      step(Wc + j * MT * kFrag, b0);
      load_b(min(s0 + j + 2, a.steps - 1), b0);
      __builtin_amdgcn_sched_barrier(0);
      step(Wc + (j + 1) * MT * kFrag, b1);
    }
  }

  if (!live) return;
  // ---- epilogue: lane (g, col) holds output channels 16 mt + 4 g + j of pixel col
#pragma unroll
  for (int t = 0; t < kNT; ++t) {
    const int xx = x0 + 16 * t + col;
    if (xx >= Wd) continue;
    const int64_t px = ((int64_t)f * H + y) * Wd + xx;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int c0 = 16 * mt + 4 * g;
      f32x4 v = acc[t][mt] + *(const f32x4 *)(a.bias + c0);
      if (a.relu) {
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = fmaxf(v[j], 0.0f);
      }
      if (a.out_bf) {
        uint2 pk = {pk_bf16(v[0], v[1]), pk_bf16(v[2], v[3])};
        *(uint2 *)(a.out_bf + (px * a.cout_pad + c0) * 2) = pk;
      }
      if (a.out_f32) *(f32x4 *)(a.out_f32 + px * a.cout_pad + c0) = v;
      if (a.out_rgb && mt == 0 && g == 0) {
        const int64_t hw = (int64_t)H * Wd, q = (int64_t)y * Wd + xx;
        a.out_rgb[((int64_t)f * 3 + 0) * hw + q] = v[0];
        a.out_rgb[((int64_t)f * 3 + 1) * hw + q] = v[1];
        a.out_rgb[((int64_t)f * 3 + 2) * hw + q] = v[2];
      }
    }
  }
}

// ---- h over every buffer, the pool and T's last layer, in one kernel ----------
// With sigma's part u = conv3 sigma + c1 computed once, each buffer i needs
//   z1 = relu(conv3_b b_i + u), z2 = relu(A2 z1 + c2), Z += [alpha_i > 0] z2,
// and after the last buffer tau = A3 (Z / max(c, 1)) + [c > 0] c3 (mean; the
// sum: A3 Z + c c3).  A wave owns 16 pixels of one row and every channel; u
// and Z stay in registers across the buffers and z1 feeds h's second layer
// from registers, so the per-buffer activations never leave the chip.
//
// Weights stay in LDS for the whole kernel (persistent workgroups):
//   conv3_b: 5 K-steps; lane group g of step s presents tap 2 s + (g >> 1)
//     (the tenth tap is zero), channels 8 (g & 1) .. + 7 of the buffer
//     (12 real, 16 packed);
//   A2, A3: W / 32 K-steps in register order: element e of lane group g in
//     step s multiplies channel 32 s + 4 g + e (e < 4) or 32 s + 16 + 4 g +
//     e - 4, which is where M-tiles 2 s and 2 s + 1 of the previous layer's
//     accumulators hold them.
struct SpSlotsArgs {
  const uint8_t *frag;      // conv3_b, A2, A3 fragments, contiguous
  const float *bias;        // c2 then c3, 16 MT floats each
  const uint8_t *bpk;       // bf16 [n][k][H][W][16]: each buffer's 12 channels, zero padded
  const float *layers;      // the caller's buffers (alpha)
  const float *u;           // fp32 [n][H][W][16 MT]
  uint8_t *tau;             // bf16 [n][H][W][16 MT]
  int n, H, Wd, k, mean;
};

constexpr int kSlotSteps1 = 5;               // conv3_b K-steps (9 taps x 16 channels)

template <int MT>
__global__ __launch_bounds__(kThreads) void sp_slots_kernel(SpSlotsArgs a) {
  extern __shared__ __attribute__((aligned(1024))) uint8_t lds[];
  constexpr int W = 16 * MT, KS = MT / 2;
  constexpr int kBytes = (kSlotSteps1 + 2 * KS) * MT * kFrag;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, col = lane & 15;
  // every fragment, then the biases, into LDS once
  for (int off = wave * kFrag; off < kBytes; off += kWaves * kFrag)
    __builtin_amdgcn_global_load_lds((const void *)(a.frag + off + lane * 16),
                                     (__attribute__((address_space(3))) void *)(lds + off), 16, 0, 0);
  float *lbias = (float *)(lds + kBytes);
  if (threadIdx.x < 2 * W) lbias[threadIdx.x] = a.bias[threadIdx.x];
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  const uint8_t *F1 = lds, *F2 = lds + kSlotSteps1 * MT * kFrag, *F3 = F2 + KS * MT * kFrag;

  const int H = a.H, Wd = a.Wd, k = a.k;
  const int64_t hw = (int64_t)H * Wd;
  const int segs = (Wd + 15) >> 4;
  const int64_t nseg = (int64_t)a.n * H * segs;
  const int64_t ntiles = (nseg + kWaves - 1) / kWaves;
  // workgroups reach the 8 XCDs round-robin: each XCD takes a contiguous run
  // of tiles (neighbouring rows share its L2)
  const int per = gridDim.x >> 3, xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  for (int64_t base = 0; base < ntiles; base += gridDim.x) {
    const int64_t seg = (base + (int64_t)xcd * per + slot) * kWaves + wave;
    if (seg >= nseg) continue;
    const int f = __builtin_amdgcn_readfirstlane((int)(seg / ((int64_t)H * segs)));
    const int rem = (int)(seg - (int64_t)f * H * segs);
    const int y = __builtin_amdgcn_readfirstlane(rem / segs);
    const int x0 = __builtin_amdgcn_readfirstlane((rem - y * segs) * 16);
    const int x = x0 + col;
    const bool xin = x < Wd;
    const int xc = min(x, Wd - 1);
    const int64_t px = ((int64_t)f * H + y) * Wd + xc;

    f32x4 u[MT], Z[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      u[mt] = *(const f32x4 *)(a.u + px * W + 16 * mt + 4 * g);
      Z[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    float cnt = 0.0f;
    // buffer i's conv3 inputs (tap 2 s + (g >> 1); outside the frame the
    // offset is past the plane's bound and the load returns zeros) and its
    // alpha; the next buffer's are loaded while this one's MFMAs run
    auto load_slot = [&](int i, u32x4 (&b)[kSlotSteps1], float &al) {
      const int64_t fb = (int64_t)f * k + i;
      al = a.layers[(fb * kNL + kAlpha) * hw + (int64_t)y * Wd + xc];
      const rsrc_t rb = make_rsrc(a.bpk + fb * hw * 32, (uint32_t)(hw * 32));
#pragma unroll
      for (int s = 0; s < kSlotSteps1; ++s) {
        const int tap = 2 * s + (g >> 1);
        const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
        const bool ok = tap < 9 && yy >= 0 && yy < H && xx >= 0 && xx < Wd;
        b[s] = bld(rb, ok ? (uint32_t)(yy * Wd + xx) * 32 + 16 * (g & 1) : kOutside);
      }
    };
    u32x4 b[kSlotSteps1], bn[kSlotSteps1];
    float al = 0.0f, aln = 0.0f;
    if (k > 0) load_slot(0, b, al);
    for (int i = 0; i < k; ++i) {
      if (i + 1 < k) load_slot(i + 1, bn, aln);
      __builtin_amdgcn_sched_barrier(0);
      const bool act = xin && al > 0.0f;
      if (!__builtin_amdgcn_ballot_w64(act)) {          // adds exactly nothing
#pragma unroll
        for (int s = 0; s < kSlotSteps1; ++s) b[s] = bn[s];
        al = aln;
        continue;
      }
      f32x4 acc[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt] = u[mt];
#pragma unroll
      for (int s = 0; s < kSlotSteps1; ++s)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          acc[mt] = mma(*(const u32x4 *)(F1 + (s * MT + mt) * kFrag + lane * 16), b[s], acc[mt]);
      // z1 in register order, then h's second layer
      u32x4 zb[KS];
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const f32x4 p = acc[2 * s], q = acc[2 * s + 1];
        zb[s] = u32x4{pk_bf16(fmaxf(p[0], 0.f), fmaxf(p[1], 0.f)),
                      pk_bf16(fmaxf(p[2], 0.f), fmaxf(p[3], 0.f)),
                      pk_bf16(fmaxf(q[0], 0.f), fmaxf(q[1], 0.f)),
                      pk_bf16(fmaxf(q[2], 0.f), fmaxf(q[3], 0.f))};
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt] = *(const f32x4 *)(lbias + 16 * mt + 4 * g);
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          acc[mt] = mma(*(const u32x4 *)(F2 + (s * MT + mt) * kFrag + lane * 16), zb[s], acc[mt]);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) Z[mt][j] += act ? fmaxf(acc[mt][j], 0.0f) : 0.0f;
      cnt += act ? 1.0f : 0.0f;
#pragma unroll
      for (int s = 0; s < kSlotSteps1; ++s) b[s] = bn[s];
      al = aln;
    }
    // the pool's finish and T's last layer
    const float inv = a.mean ? 1.0f / fmaxf(cnt, 1.0f) : 1.0f;
    const float bs = a.mean ? (cnt > 0.0f ? 1.0f : 0.0f) : cnt;
    u32x4 zb[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const f32x4 p = Z[2 * s] * inv, q = Z[2 * s + 1] * inv;
      zb[s] = u32x4{pk_bf16(p[0], p[1]), pk_bf16(p[2], p[3]), pk_bf16(q[0], q[1]),
                    pk_bf16(q[2], q[3])};
    }
    f32x4 acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[mt] = *(const f32x4 *)(lbias + W + 16 * mt + 4 * g) * bs;
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
        acc[mt] = mma(*(const u32x4 *)(F3 + (s * MT + mt) * kFrag + lane * 16), zb[s], acc[mt]);
    if (xin) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const uint2 pk = {pk_bf16(acc[mt][0], acc[mt][1]), pk_bf16(acc[mt][2], acc[mt][3])};
        *(uint2 *)(a.tau + (px * W + 16 * mt + 4 * g) * 2) = pk;
      }
    }
  }
}

// ---- input packing and the pooling steps ------------------------------------
// x = [G 0..13; scene 0..15; 0, 0] as bf16 [n][H][W][32].
__global__ void sp_pack_x_kernel(const float *__restrict__ gbuf, const float *__restrict__ scene,
                                 int64_t npx, int hw, uint8_t *__restrict__ x) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npx) return;
  const int f = (int)(p / hw), q = (int)(p - (int64_t)f * hw);
  uint32_t w[16];
  for (int j = 0; j < 16; ++j) {
    float v[2];
    for (int e = 0; e < 2; ++e) {
      const int c = 2 * j + e;
      v[e] = c < kNG ? gbuf[((int64_t)f * kNG + c) * hw + q]
                     : (c < kNG + kNS ? scene[(int64_t)f * kNS + c - kNG] : 0.0f);
    }
    w[j] = pk_bf16(v[0], v[1]);
  }
  u32x4 *dst = (u32x4 *)(x + p * 64);
  for (int j = 0; j < 4; ++j) dst[j] = u32x4{w[4 * j], w[4 * j + 1], w[4 * j + 2], w[4 * j + 3]};
}

// `nch` planes (plane stride hw, frame stride fstride floats) from `src` as
// bf16 [n][H][W][32], zero past nch.
__global__ void sp_pack_planes_kernel(const float *__restrict__ src, int nch, int64_t fstride,
                                      int64_t npx, int hw, uint8_t *__restrict__ x) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npx) return;
  const int f = (int)(p / hw), q = (int)(p - (int64_t)f * hw);
  uint32_t w[16];
  for (int j = 0; j < 16; ++j) {
    float v[2];
    for (int e = 0; e < 2; ++e) {
      const int c = 2 * j + e;
      v[e] = c < nch ? src[(int64_t)f * fstride + (int64_t)c * hw + q] : 0.0f;
    }
    w[j] = pk_bf16(v[0], v[1]);
  }
  u32x4 *dst = (u32x4 *)(x + p * 64);
  for (int j = 0; j < 4; ++j) dst[j] = u32x4{w[4 * j], w[4 * j + 1], w[4 * j + 2], w[4 * j + 3]};
}

// Every buffer's 12 planes as bf16 [n][k][H][W][16] (zero channels 12..15):
// one thread per (frame, buffer, pixel).
__global__ void sp_pack_slots_kernel(const float *__restrict__ layers, int64_t total, int hw,
                                     uint8_t *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int64_t fb = i / hw;                 // frame * k + buffer
  const int q = (int)(i - fb * hw);
  const float *src = layers + fb * kNL * hw + q;
  uint32_t w[8];
  for (int j = 0; j < 8; ++j) {
    const int c = 2 * j;
    w[j] = pk_bf16(c < kNL ? src[(int64_t)c * hw] : 0.0f, c + 1 < kNL ? src[(int64_t)(c + 1) * hw] : 0.0f);
  }
  u32x4 *dst = (u32x4 *)(out + i * 32);
  dst[0] = u32x4{w[0], w[1], w[2], w[3]};
  dst[1] = u32x4{w[4], w[5], w[6], w[7]};
}

// The fragments of sp_slots_kernel: blockIdx.y 0 packs conv3_b (T1's buffer
// columns, master [W][12 + W][3][3]), 1 and 2 pack A2 and A3 ([W][W]) in
// register order.  Fragment (s, mt), lane l = 16 g + m, element j.
__global__ void sp_pack_slots_frag_kernel(const float *__restrict__ master, int W, int64_t t1,
                                          int64_t t2, int64_t t3, uint8_t *__restrict__ out) {
  const int MT = W / 16, KS = MT / 2, which = blockIdx.y;
  const int steps = which == 0 ? kSlotSteps1 : KS;
  const int64_t base = which == 0 ? 0 : (int64_t)(kSlotSteps1 + (which - 1) * KS) * MT * 512;
  const int64_t n = (int64_t)steps * MT * 512;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(e & 7), l = (int)((e >> 3) & 63);
    const int64_t frag = e >> 9;
    const int mt = (int)(frag % MT), s = (int)(frag / MT);
    const int g = l >> 4, row = 16 * mt + (l & 15);
    float v = 0.0f;
    if (which == 0) {
      const int tap = 2 * s + (g >> 1), ch = 8 * (g & 1) + j;
      if (tap < 9 && ch < kNL) v = master[t1 + ((int64_t)row * (kNL + W) + ch) * 9 + tap];
    } else {
      const int ch = 32 * s + (j < 4 ? 4 * g + j : 16 + 4 * g + j - 4);
      v = master[(which == 1 ? t2 : t3) + (int64_t)row * W + ch];
    }
    ((__bf16 *)(out + base * 2))[e] = (__bf16)v;
  }
}

// 2 x 2 average of a bf16 [n][H][W][C] block (H, W even) into [n][H/2][W/2][C]:
// one thread per output pixel and 8 channels, the sum in fp32.
__global__ void sp_avgpool_kernel(const uint8_t *__restrict__ in, int n, int H, int Wd, int C,
                                  uint8_t *__restrict__ out) {
  const int H2 = H >> 1, W2 = Wd >> 1, cg = C >> 3;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)n * H2 * W2 * cg;
  if (i >= total) return;
  const int c8 = (int)(i % cg);
  const int64_t p = i / cg;
  const int x = (int)(p % W2);
  const int64_t fy = p / W2;
  const int yy = (int)(fy % H2), f = (int)(fy / H2);
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int dy = 0; dy < 2; ++dy)
    for (int dx = 0; dx < 2; ++dx) {
      const uint16_t *src =
          (const uint16_t *)(in + ((((int64_t)f * H + 2 * yy + dy) * Wd + 2 * x + dx) * C + 8 * c8) * 2);
      for (int j = 0; j < 8; ++j) s[j] += bf16_to_f32(src[j]);
    }
  uint32_t w[4];
  for (int j = 0; j < 4; ++j) w[j] = pk_bf16(0.25f * s[2 * j], 0.25f * s[2 * j + 1]);
  *(u32x4 *)(out + (p * C + 8 * c8) * 2) = u32x4{w[0], w[1], w[2], w[3]};
}

// Weight fragments of one conv: element e of fragment (step, mt), lane l,
// position j holds W[16 mt + (l & 15)][ci][tap] for step = tap * cbt + cb and
// concatenated input channel 32 cb + 8 (l >> 4) + j, mapped to the master
// input column (zero for padding channels and rows past cout).
struct SpPackDesc {
  int64_t woff;             // float offset of the weight tensor [cout][cin][k][k]
  int64_t out_off;          // byte offset of the fragments in the packed buffer
  int cout, cin, k;         // master tensor shape
  int col0;                 // first master input column this conv multiplies
  int c0real, c0pad, c1real, c1pad;   // its two sources (channels, padded to 32)
  int mt;                   // M-tiles
};

// All convolutions in one launch: blockIdx.y selects the conv; the biases
// (padded to whole M-tiles, zero past cout and for T1's buffer part, whose
// bias T1's sigma part carries) go after the fragments.
struct SpPackAll {
  SpPackDesc d[15];
  int64_t bias_src[15];     // master float offset of each conv's bias (-1: none)
  int64_t bias_dst[15];     // float offset in the packed bias block
  int64_t bias_block;       // byte offset of the bias block
};

__global__ void sp_pack_all_kernel(const float *__restrict__ master, SpPackAll all,
                                   uint8_t *__restrict__ packed) {
  const SpPackDesc &d = all.d[blockIdx.y];
  const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x < 16 * d.mt) {
    const int o = threadIdx.x;
    const int64_t src = all.bias_src[blockIdx.y];
    ((float *)(packed + all.bias_block))[all.bias_dst[blockIdx.y] + o] =
        src >= 0 && o < d.cout ? master[src + o] : 0.0f;
  }
  const int cbt = (d.c0pad + d.c1pad) >> 5;
  const int steps = d.k * d.k * cbt;
  const int64_t n = (int64_t)padded_steps(d.k * d.k, cbt) * d.mt * 64 * 8;
  for (int64_t e = e0; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(e & 7), l = (int)((e >> 3) & 63);
    const int64_t frag = e >> 9;
    const int mt = (int)(frag % d.mt), step = (int)(frag / d.mt);
    const int tap = step / cbt, cb = step - tap * cbt;
    const int row = 16 * mt + (l & 15);
    const int cc = 32 * cb + 8 * (l >> 4) + j;           // concatenated padded channel
    int ci = -1;
    if (cc < d.c0pad) {
      if (cc < d.c0real) ci = cc;
    } else if (cc - d.c0pad < d.c1real) {
      ci = d.c0real + (cc - d.c0pad);
    }
    float v = 0.0f;
    if (step < steps && row < d.cout && ci >= 0)      // padding steps stay zero
      v = master[d.woff + (((int64_t)row * d.cin + d.col0 + ci) * d.k * d.k) + tap];
    ((__bf16 *)(packed + d.out_off))[e] = (__bf16)v;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side: the layer sequence.

// The 14 convolutions (and T1's split into its buffer and sigma parts).
enum SpConvId {
  SP_F1, SP_F2, SP_F3, SP_F4, SP_T1B, SP_T1S, SP_T2, SP_T3, SP_B1, SP_B2, SP_B3, SP_B4,
  SP_R1, SP_R2, SP_R3, kSpConvs
};

struct SpLayout {
  int W;
  SpPackDesc d[kSpConvs];
  int64_t bias_off[kSpConvs];      // float offset of each conv's padded bias in the bias block
  int64_t frag_bytes, bias_floats;
  int64_t slots_off, slots_bytes;  // sp_slots_kernel's fragments (after the bias block)
  int64_t t1, t2, t3;              // master offsets of T's three weight tensors
};

static int64_t sp_master_offsets(int W, int64_t woff[14], int64_t boff[14], int cout[14],
                                 int cin[14], int ks[14]) {
  const int spec[14][3] = {{W, kNG + kNS, 3}, {W, W, 3}, {W, 2 * W, 3}, {W, W, 1},
                           {W, kNL + W, 3}, {W, W, 1}, {W, W, 1},
                           {W, 2 * W, 3}, {W, W, 3}, {W, 2 * W, 3}, {W, W, 1},
                           {W, W + 3, 3}, {W, W, 3}, {kNOUT, W, 1}};
  int64_t off = 0;
  for (int i = 0; i < 14; ++i) {
    cout[i] = spec[i][0];
    cin[i] = spec[i][1];
    ks[i] = spec[i][2];
    woff[i] = off;
    off += (int64_t)cout[i] * cin[i] * ks[i] * ks[i];
    boff[i] = off;
    off += cout[i];
  }
  return off;
}

size_t spatial_num_params(int W) {
  if (W != 64 && W != 128) return 0;
  int64_t wo[14], bo[14];
  int co[14], ci[14], k[14];
  return (size_t)sp_master_offsets(W, wo, bo, co, ci, k);
}

static SpLayout sp_layout(int W) {
  int64_t wo[14], bo[14];
  int co[14], ci[14], k[14];
  sp_master_offsets(W, wo, bo, co, ci, k);
  // master tensor index of every conv; (col0, sources) of each
  struct M { int m, col0, c0real, c0pad, c1real, c1pad; };
  const M map[kSpConvs] = {
      {0, 0, kNG + kNS, 32, 0, 0},   {1, 0, W, W, 0, 0},  {2, 0, W, W, W, W}, {3, 0, W, W, 0, 0},
      {4, 0, kNL, 32, 0, 0},         {4, kNL, W, W, 0, 0},                     // T1: b part, sigma part
      {5, 0, W, W, 0, 0},            {6, 0, W, W, 0, 0},
      {7, 0, W, W, W, W},            {8, 0, W, W, 0, 0},  {9, 0, W, W, W, W}, {10, 0, W, W, 0, 0},
      {11, 0, W, W, 3, 32},          {12, 0, W, W, 0, 0}, {13, 0, W, W, 0, 0}};
  SpLayout L;
  L.W = W;
  int64_t fb = 0, bf = 0;
  for (int c = 0; c < kSpConvs; ++c) {
    const M &m = map[c];
    SpPackDesc &d = L.d[c];
    d.woff = wo[m.m];
    d.cout = co[m.m];
    d.cin = ci[m.m];
    d.k = k[m.m];
    d.col0 = m.col0;
    d.c0real = m.c0real;
    d.c0pad = m.c0pad;
    d.c1real = m.c1real;
    d.c1pad = m.c1pad;
    d.mt = (d.cout + 15) / 16;
    d.out_off = fb;
    fb += (int64_t)padded_steps(d.k * d.k, (d.c0pad + d.c1pad) / 32) * d.mt * kFrag;
    L.bias_off[c] = bf;
    bf += d.mt * 16;
  }
  L.frag_bytes = fb;
  L.bias_floats = bf;
  const int MT = W / 16;
  L.slots_off = (fb + 4 * bf + 1023) / 1024 * 1024;
  L.slots_bytes = (int64_t)(kSlotSteps1 + MT) * MT * kFrag;
  L.t1 = wo[4];
  L.t2 = wo[5];
  L.t3 = wo[6];
  return L;
}

// Master bias offset of conv c (T1's two parts share T1's bias; the sigma
// part carries it, the buffer part adds none).
static int64_t sp_bias_master(int W, int c, bool *zero) {
  int64_t wo[14], bo[14];
  int co[14], ci[14], k[14];
  sp_master_offsets(W, wo, bo, co, ci, k);
  const int m[kSpConvs] = {0, 1, 2, 3, 4, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13};
  *zero = c == SP_T1B;
  return bo[m[c]];
}

size_t spatial_weight_bytes(int W) {
  const SpLayout L = sp_layout(W);
  return (size_t)(L.slots_off + L.slots_bytes);
}

// Device bytes of the activations a call of n frames of H x W with k buffers
// needs.
size_t spatial_workspace_bytes(int W, int n, int H, int Wd, int k) {
  const int64_t px = (int64_t)n * H * Wd, half = px / 4;
  // bf16: x/L_d (32 ch), e1, e2, sigma, tau, phi, r1, r2 (W ch each), half-res
  // d and m (W ch), the k buffers (16 ch each); fp32: u (W ch); rounding slack
  return (size_t)(2 * (px * 32 + 7 * px * W + 2 * half * W + px * 16 * (int64_t)k) +
                  4 * px * W + 16 * 256);
}

hipError_t spatial_pack(const float *master, int W, uint8_t *packed, hipStream_t s) {
  const SpLayout L = sp_layout(W);
  static_assert(kSpConvs == 15, "SpPackAll holds 15 convolutions");
  SpPackAll all;
  int64_t most = 0;
  for (int c = 0; c < kSpConvs; ++c) {
    all.d[c] = L.d[c];
    bool zero = false;
    const int64_t bo = sp_bias_master(W, c, &zero);
    all.bias_src[c] = zero ? -1 : bo;
    all.bias_dst[c] = L.bias_off[c];
    const SpPackDesc &d = L.d[c];
    most = std::max<int64_t>(most, (int64_t)padded_steps(d.k * d.k, (d.c0pad + d.c1pad) / 32) *
                                       d.mt * 512);
  }
  all.bias_block = L.frag_bytes;
  const unsigned bx = (unsigned)std::min<int64_t>((most + 255) / 256, 1024);
  hipLaunchKernelGGL(sp_pack_all_kernel, dim3(bx, kSpConvs), dim3(256), 0, s, master, all,
                     packed);
  hipLaunchKernelGGL(sp_pack_slots_frag_kernel, dim3(64, 3), dim3(256), 0, s, master, W, L.t1,
                     L.t2, L.t3, packed + L.slots_off);
  return hipGetLastError();
}

template <int MT>
static hipError_t sp_slots_launch(const SpSlotsArgs &a, hipStream_t s) {
  static bool attr = false;
  const size_t lds = (size_t)(kSlotSteps1 + MT) * MT * kFrag + 2 * 16 * MT * sizeof(float);
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void *)sp_slots_kernel<MT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int64_t nseg = (int64_t)a.n * a.H * ((a.Wd + 15) / 16);
  const int64_t ntiles = (nseg + kWaves - 1) / kWaves;
  // persistent: one workgroup per CU (the weights fill most of its LDS), a
  // multiple of the 8 XCDs
  const unsigned grid = (unsigned)std::min<int64_t>(256, (ntiles + 7) / 8 * 8);
  hipLaunchKernelGGL(sp_slots_kernel<MT>, dim3(grid), dim3(kThreads), lds, s, a);
  return hipGetLastError();
}

template <int MT, int NT>
static hipError_t sp_launch(const SpConvArgs &a, hipStream_t s) {
  static bool attr = false;
  const size_t lds = 2 * (size_t)kChunk * MT * kFrag;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void *)sp_conv_kernel<MT, NT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int64_t segs = (int64_t)a.n * a.H * ((a.Wd + 16 * NT - 1) / (16 * NT));
  const unsigned grid = (unsigned)((segs + kWaves - 1) / kWaves);
  hipLaunchKernelGGL((sp_conv_kernel<MT, NT>), dim3(grid), dim3(kThreads), lds, s, a);
  return hipGetLastError();
}

static hipError_t sp_conv(const SpConvArgs &a0, int mt, hipStream_t s) {
  switch (mt) {
    case 1: return sp_launch<1, 4>(a0, s);
    case 4: return sp_launch<4, 4>(a0, s);
    case 8: return sp_launch<8, 2>(a0, s);
  }
  return hipErrorInvalidValue;
}

hipError_t spatial_forward(const uint8_t *packed, int W, int pool, const float *gbuf,
                           const float *layers, const float *scene, int n, int H, int Wd, int k,
                           float *out, uint8_t *ws, hipStream_t s) {
  const SpLayout L = sp_layout(W);
  const float *bias = (const float *)(packed + L.frag_bytes);
  const int64_t px = (int64_t)n * H * Wd, half = px / 4;
  const int hw = H * Wd;
  // workspace carve-up (see spatial_workspace_bytes)
  uint8_t *p = ws;
  auto take = [&](int64_t bytes) { uint8_t *q = p; p += (bytes + 255) & ~(int64_t)255; return q; };
  uint8_t *x32 = take(px * 32 * 2);                   // x, then each b_i, then L_d
  uint8_t *e1 = take(px * W * 2), *e2 = take(px * W * 2), *sig = take(px * W * 2);
  uint8_t *tau = take(px * W * 2);
  uint8_t *phi = take(px * W * 2), *r1 = take(px * W * 2), *r2 = take(px * W * 2);
  uint8_t *dh = take(half * W * 2), *mh = take(half * W * 2);
  uint8_t *bpk = take(px * 16 * 2 * (int64_t)k);
  float *u = (float *)take(px * W * 4);
  const int MT = W / 16;
  const unsigned pg = (unsigned)((px + 255) / 256);
  hipError_t e = hipSuccess;

  auto conv = [&](int c, const uint8_t *in0, int c0, const uint8_t *in1, int c1, int up1,
                  int Hc, int Wc) {
    SpConvArgs a = {};
    const SpPackDesc &d = L.d[c];
    a.in0 = in0;
    a.in1 = in1;
    a.c0 = c0;
    a.c1 = c1;
    a.up1 = up1;
    a.wfrag = packed + d.out_off;
    a.bias = bias + L.bias_off[c];
    a.ksize = d.k;
    a.steps = d.k * d.k * ((c0 + c1) / 32);
    a.steps_pad = padded_steps(d.k * d.k, (c0 + c1) / 32);
    a.n = n;
    a.H = Hc;
    a.Wd = Wc;
    a.cout_pad = d.mt * 16;
    return a;
  };
  auto run = [&](const SpConvArgs &a, int mt) {
    if (e == hipSuccess) e = sp_conv(a, mt, s);
  };
  auto unet = [&](int c1st, const uint8_t *in0, int c0, const uint8_t *in1, int c1, uint8_t *outp) {
    SpConvArgs a = conv(c1st, in0, c0, in1, c1, 0, H, Wd);        // e1
    a.relu = 1;
    a.out_bf = e1;
    run(a, MT);
    const int64_t tot = half * (W / 8);
    hipLaunchKernelGGL(sp_avgpool_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, e1,
                       n, H, Wd, W, dh);
    a = conv(c1st + 1, dh, W, nullptr, 0, 0, H / 2, Wd / 2);      // m (half resolution)
    a.relu = 1;
    a.out_bf = mh;
    run(a, MT);
    a = conv(c1st + 2, e1, W, mh, W, 1, H, Wd);                   // e2 = relu(conv3 [e1; up m])
    a.relu = 1;
    a.out_bf = e2;
    run(a, MT);
    a = conv(c1st + 3, e2, W, nullptr, 0, 0, H, Wd);              // out = conv1 e2
    a.out_bf = outp;
    run(a, MT);
  };

  // F: sigma = U-Net([G; s])
  hipLaunchKernelGGL(sp_pack_x_kernel, dim3(pg), dim3(256), 0, s, gbuf, scene, px, hw, x32);
  unet(SP_F1, x32, 32, nullptr, 0, sig);
  // T: u = conv3 sigma (T1's sigma columns) + c1; then, in one kernel, per
  // buffer z1 = relu(conv3 b_i + u), Z += [alpha_i > 0] relu(A2 z1 + c2), and
  // tau = A3 (Z / max(c, 1)) + [c > 0] c3 (mean) or A3 Z + c c3 (sum)
  {
    SpConvArgs a = conv(SP_T1S, sig, W, nullptr, 0, 0, H, Wd);
    a.out_f32 = u;
    run(a, MT);
  }
  if (k > 0) {
    const int64_t tot = px * k;
    hipLaunchKernelGGL(sp_pack_slots_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                       layers, tot, hw, bpk);
  }
  {
    SpSlotsArgs a;
    a.frag = packed + L.slots_off;
    a.bias = bias + L.bias_off[SP_T2];       // c2, then c3 (T3's bias block follows T2's)
    a.bpk = bpk;
    a.layers = layers;
    a.u = u;
    a.tau = tau;
    a.n = n;
    a.H = H;
    a.Wd = Wd;
    a.k = k;
    a.mean = pool == GN_POOL_MEAN ? 1 : 0;
    if (e == hipSuccess) e = MT == 8 ? sp_slots_launch<8>(a, s) : sp_slots_launch<4>(a, s);
  }
  // B: phi = U-Net([sigma; tau])
  unet(SP_B1, sig, W, tau, W, phi);
  // R: y = conv1 relu(conv3 relu(conv3 [phi; L_d]))
  hipLaunchKernelGGL(sp_pack_planes_kernel, dim3(pg), dim3(256), 0, s, gbuf + 11 * hw, 3,
                     (int64_t)kNG * hw, px, hw, x32);
  {
    SpConvArgs a = conv(SP_R1, phi, W, x32, 32, 0, H, Wd);
    a.relu = 1;
    a.out_bf = r1;
    run(a, MT);
    a = conv(SP_R2, r1, W, nullptr, 0, 0, H, Wd);
    a.relu = 1;
    a.out_bf = r2;
    run(a, MT);
    a = conv(SP_R3, r2, W, nullptr, 0, 0, H, Wd);
    a.out_rgb = out;
    run(a, 1);
  }
  if (e == hipSuccess) e = hipGetLastError();
  return e;
}

}  // namespace gn
