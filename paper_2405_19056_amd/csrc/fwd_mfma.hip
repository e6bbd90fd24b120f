// Fused GlassNet forward on the gfx950 matrix cores (bf16 / fp8 in, fp32 acc).
//
// Formulation.  Every layer is Y^T = A X^T with the weights A as the MFMA
// "A" operand (16 output neurons per M-tile) and 16 pixels per N-tile as the
// "B" operand.  The fp32 accumulator of v_mfma_f32_16x16x32_bf16 leaves lane
// l holding 4 consecutive output rows (4*(l>>4) + r) of pixel l & 15; two
// M-tiles give exactly the 8 values that lane must present as the B operand
// of the next layer's 32-deep K-step.  The next layer's weights are stored
// with their input columns permuted the same way, so activations go from one
// layer to the next by a ReLU and a bf16 convert, without leaving registers.
//
// Work split.  A workgroup of 8 waves owns a tile of 256 pixels (32 per wave,
// two N-tiles).  Weights are staged into LDS chunk by chunk with direct
// global->LDS loads, double-buffered: while a stage computes, the next
// stage's chunk streams in.  The weights of the per-slot network h that run
// inside the slot loop stay resident.  Grid = number of CUs; each workgroup
// walks tiles with a stride of the grid (tiles may come from a table that
// mixes frames of different sizes and slot counts).
//
// The method (Sec. 3.3-3.4): sigma = F([G; s]); tau = pool_i h(b_i, sigma)
// over slots with alpha_i > 0 (Eq. (5)); phi = B([sigma; tau]);
// y = R([phi; L_d]).  Two exact rewrites of h are used: its first layer's
// sigma part is computed once per pixel (u = W1s sigma + c1), and because its
// last layer is affine the masked pool moves in front of it:
// sum_i m_i (A3 a_i + c3) = A3 (sum_i m_i a_i) + (sum_i m_i) c3.  The running
// sum is fp32 in registers, so memory does not grow with the slot count.
#include "gn_internal.h"
#include "slot_order.h"

namespace gn {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef const float __attribute__((address_space(1))) gcfloat;
typedef float __attribute__((address_space(1))) gfloat;
typedef u32x4 __attribute__((address_space(1))) gu32x4;
typedef f32x4 __attribute__((address_space(1))) gf32x4;

constexpr int kWaves = 8;
constexpr int kNT = 2;                // N-tiles of 16 pixels per wave
constexpr int kThreads = kWaves * 64;
static_assert(kWaves * kNT * 16 == kTilePx, "tile = waves x N-tiles x 16 pixels");
constexpr int kFrag = 1024;            // one bf16 A fragment: 64 lanes x 16 B

struct MfmaArgs {
  const uint8_t *packed;
  int64_t stage_off[kMaxStages + 1];
  int64_t res_off, res_bytes, bias_off, t2q_off, t2s_off;
  FwdBatch b;
  const FrameDesc *frames;
  const TileRef *tiles;
  int ntiles;
  int tiles_per_frame;
  int pool;
  float sa, inv_sa;                    // fp8 activation scale and its inverse
  uint8_t *sig_scratch;                // per (workgroup, wave): sigma fragments, stage 1 -> 3
  int sig_lds_waves;                   // waves 0 .. n-1 park sigma in LDS instead:
  int sig_tail_waves;                  // the first n - t after the stage buffers, the
                                       // last t in the stage buffers' idle tails
  uint8_t *state;                      // object streaming: per-tile state (modes other than FULL)
  int state_load;                      // 1: the state holds a running sum to continue from
  int canon;                           // FULL: pool each pixel's slots in canonical order
  int kpad;                            // bytes per pixel of the LDS slot-order table
  int aslots;                          // slots whose alphas the LDS alpha table holds
  int alpha_alias;                     // 1: the alpha table sits in sigma's parking area
};

// Two floats -> packed bf16 pair (round to nearest even), one v_cvt_pk_bf16_f32.
__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, bf16x2));
}

// max(x, 0) in one v_med3_f32 (fmaxf on a matrix-core result would first
// canonicalise its operand, costing a second instruction).
__device__ __forceinline__ float relu1(float x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 3.402823466e+38f); }

__device__ __forceinline__ f32x4 mma(u32x4 a, u32x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// 16x16x16 bf16 MFMA: lane group g supplies inputs 4g..4g+3.
__device__ __forceinline__ f32x4 mma16(uint2 a, uint2 b, f32x4 c) {
  typedef short s16x4 __attribute__((ext_vector_type(4)));
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s16x4, a),
                                                   __builtin_bit_cast(s16x4, b), c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 relu4(f32x4 v) {
  return f32x4{relu1(v.x), relu1(v.y), relu1(v.z), relu1(v.w)};
}

// ReLU of two packed bf16: sign-magnitude values order like signed 16-bit
// integers, so max(x, 0) as int16 zeroes exactly the negative numbers.
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t x) {
  typedef short s16x2 __attribute__((ext_vector_type(2)));
  s16x2 v = __builtin_bit_cast(s16x2, x);
  s16x2 z = {0, 0};
  v = __builtin_elementwise_max(v, z);
  return __builtin_bit_cast(uint32_t, v);
}

// Four floats -> four OCP E4M3 bytes (round to nearest even) of
// min(max(v, 0), 448): ReLU and the clamp to the format's largest finite
// magnitude in one v_med3 each.
__device__ __forceinline__ int relu_pack_fp8x4(f32x4 v) {
  const float M = 448.0f;
  const float x = __builtin_amdgcn_fmed3f(v.x, 0.0f, M), y = __builtin_amdgcn_fmed3f(v.y, 0.0f, M);
  const float z = __builtin_amdgcn_fmed3f(v.z, 0.0f, M), w = __builtin_amdgcn_fmed3f(v.w, 0.0f, M);
  int r = __builtin_amdgcn_cvt_pk_fp8_f32(x, y, 0, false);
  return __builtin_amdgcn_cvt_pk_fp8_f32(z, w, r, true);
}

// 16x16x128 E4M3 x E4M3 -> fp32 on the gfx950 matrix cores, unit block scales.
__device__ __forceinline__ f32x4 mma_fp8(i32x8 a, i32x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
}

__device__ __forceinline__ void wait_vm() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// The positional-encoding blocks of x (Sec. 3.4) up to block NB - 1: x, then
// sin(2^k pi x) (block 2k + 1) and cos(2^k pi x) (block 2k + 2).  Level 0
// comes from the hardware sine and cosine, which take revolutions: x / 2 is
// reduced exactly to [0, 1) first.  Each further level follows from the one
// before by the double-angle identities (sin 2a = 2 sin a cos a,
// cos 2a = 1 - 2 sin^2 a): a few fp32 roundings per level, far below the
// bf16 rounding the values then get.
template <int NB>
__device__ __forceinline__ void pe_blocks_of(float x, float (&e)[NB]) {
  e[0] = x;
  if constexpr (NB > 1) {
    const float r = __builtin_amdgcn_fractf(x * 0.5f);
    float sn = __builtin_amdgcn_sinf(r), cs = __builtin_amdgcn_cosf(r);
#pragma unroll
    for (int b = 1; b < NB; b += 2) {
      if (b > 1) {
        const float s2 = 2.0f * sn * cs;
        cs = __builtin_fmaf(-2.0f * sn, sn, 1.0f);
        sn = s2;
      }
      e[b] = sn;
      if (b + 1 < NB) e[b + 1] = cs;
    }
  }
}

// Stage boundary that leaves the newest N vector-memory operations in flight:
// N global stores issued after the next stage's LDS fill, whose completion
// nothing in the workgroup waits for.  The fill itself (older) has landed in
// LDS once vmcnt <= N; LDS traffic is drained and every wave has arrived.
template <int N>
__device__ __forceinline__ void stage_sync_after_stores() {
  asm volatile("s_waitcnt vmcnt(%0)\n\ts_waitcnt lgkmcnt(0)\n\ts_barrier" ::"n"(N) : "memory");
}

// Copy `bytes` (a multiple of 1 KiB) from global to LDS: each wave moves whole
// 1 KiB blocks, lane i writing bytes [16 i, 16 i + 16) of its block.
__device__ __forceinline__ void lds_fill(uint8_t *dst, const uint8_t *src, int64_t bytes,
                                         int wave, int lane) {
  for (int64_t off = (int64_t)wave * kFrag; off < bytes; off += kWaves * kFrag) {
    __builtin_amdgcn_global_load_lds(
        (const void *)(src + off + lane * 16),
        (__attribute__((address_space(3))) void *)(dst + off), 16, 0, 0);
  }
}

__device__ __forceinline__ u32x4 ld_frag(const uint8_t *chunk, int idx, int lane) {
  return *(const u32x4 *)(chunk + (size_t)idx * kFrag + lane * 16);
}

// One A fragment of the 16x16x16 bf16 instruction: 64 lanes x 8 bytes.
__device__ __forceinline__ uint2 ld_frag16(const uint8_t *chunk, int idx, int lane) {
  return *(const uint2 *)(chunk + (size_t)idx * 512 + lane * 8);
}

// One fp8 A fragment of the 16x16x128 instruction: 64 lanes x 32 bytes,
// stored as two 1 KiB halves (bytes 0-15 of every lane, then bytes 16-31),
// so each 16-byte LDS read has consecutive lanes 16 bytes apart (a 32-byte
// lane stride would put two lanes on every bank).
__device__ __forceinline__ i32x8 ld_frag8(const uint8_t *chunk, int idx, int lane) {
  const uint8_t *f = chunk + (size_t)idx * 2 * kFrag + lane * 16;
  const i32x4 lo = *(const i32x4 *)f, hi = *(const i32x4 *)(f + kFrag);
  return i32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}

template <int MT_>
__device__ __forceinline__ void bias_init(f32x4 (&acc)[kNT][MT_], const float *bias, int g) {
#pragma unroll
  for (int mt = 0; mt < MT_; ++mt) {
    const f32x4 b = *(const f32x4 *)(bias + 16 * mt + 4 * g);
#pragma unroll
    for (int t = 0; t < kNT; ++t) acc[t][mt] = b;
  }
}

// Accumulator rows -> next layer's B fragments (M-tiles 2j and 2j+1 make K-step j).
template <int MT_, bool RELU>
__device__ __forceinline__ void to_frags(const f32x4 (&acc)[kNT][MT_], u32x4 (&out)[kNT][MT_ / 2]) {
#pragma unroll
  for (int t = 0; t < kNT; ++t) {
#pragma unroll
    for (int mt = 0; mt < MT_; ++mt) {
      const f32x4 v = acc[t][mt];
      uint32_t lo = pk_bf16(v.x, v.y), hi = pk_bf16(v.z, v.w);
      if (RELU) {
        lo = relu_bf16x2(lo);
        hi = relu_bf16x2(hi);
      }
      out[t][mt >> 1][2 * (mt & 1)] = lo;
      out[t][mt >> 1][2 * (mt & 1) + 1] = hi;
    }
  }
}

// One chained layer, an M-tile pair at a time: out[t][p] = pack(act(A in + bias))
// for M-tiles 2p and 2p+1.  The pair's weight fragments are read up front and
// the next pair's are requested before this pair's MFMAs issue, so LDS
// latency overlaps matrix-core work instead of stalling every K-step.
// EARLY: a scheduling barrier keeps the next M-tiles' fragment reads ahead of
// the current M-tiles' MFMAs (left alone, the scheduler sinks each read next
// to its MFMAs and waits for it alone): 3.5-5% of the bf16 frame, 2% of the
// fp8 one, whose kernel spills with it in T3 and B's first layer and there
// leaves the placement to the scheduler.
template <int MT_, int KS_, bool RELU, bool EARLY>
__device__ __forceinline__ void layer(u32x4 (&out)[kNT][MT_ / 2], const uint8_t *chunk,
                                      const u32x4 (&in)[kNT][KS_], const float *bias, int g,
                                      int lane) {
  u32x4 wb[2][2][KS_];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int ks = 0; ks < KS_; ++ks) wb[0][h][ks] = ld_frag(chunk, h * KS_ + ks, lane);
#pragma unroll
  for (int p = 0; p < MT_ / 2; ++p) {
    const int cur = p & 1;
    if (p + 1 < MT_ / 2) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int ks = 0; ks < KS_; ++ks)
          wb[cur ^ 1][h][ks] = ld_frag(chunk, (2 * (p + 1) + h) * KS_ + ks, lane);
    }
    if constexpr (EARLY) __builtin_amdgcn_sched_barrier(0);
    f32x4 acc[kNT][2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const f32x4 b = *(const f32x4 *)(bias + 16 * (2 * p + h) + 4 * g);
#pragma unroll
      for (int t = 0; t < kNT; ++t) acc[t][h] = b;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int ks = 0; ks < KS_; ++ks) {
#pragma unroll
        for (int t = 0; t < kNT; ++t) acc[t][h] = mma(wb[cur][h][ks], in[t][ks], acc[t][h]);
      }
    }
#pragma unroll
    for (int t = 0; t < kNT; ++t) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const f32x4 v = acc[t][h];
        uint32_t lo = pk_bf16(v.x, v.y), hi = pk_bf16(v.z, v.w);
        if (RELU) {
          lo = relu_bf16x2(lo);
          hi = relu_bf16x2(hi);
        }
        out[t][p][2 * h] = lo;
        out[t][p][2 * h + 1] = hi;
      }
    }
  }
}

// acc[t][mt] += A(chunk) . in[t] over the chunk's KS_ K-steps, one M-tile's
// fragments read ahead of its MFMAs and the next M-tile's requested early
// (EARLY as for layer).
template <int MT_, int KS_, bool EARLY>
__device__ __forceinline__ void mm(f32x4 (&acc)[kNT][MT_], const uint8_t *chunk,
                                   const u32x4 (&in)[kNT][KS_], int lane) {
  u32x4 wb[2][KS_];
#pragma unroll
  for (int ks = 0; ks < KS_; ++ks) wb[0][ks] = ld_frag(chunk, ks, lane);
#pragma unroll
  for (int mt = 0; mt < MT_; ++mt) {
    const int cur = mt & 1;
    if (mt + 1 < MT_) {
#pragma unroll
      for (int ks = 0; ks < KS_; ++ks) wb[cur ^ 1][ks] = ld_frag(chunk, (mt + 1) * KS_ + ks, lane);
    }
    if constexpr (EARLY) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int ks = 0; ks < KS_; ++ks)
#pragma unroll
      for (int t = 0; t < kNT; ++t) acc[t][mt] = mma(wb[cur][ks], in[t][ks], acc[t][mt]);
  }
}

// F's encoded input as B fragments: K-step b (of N) is encoding block B0 + b
// of the 8 raw channels the lane holds.
template <int B0, int N>
__device__ __forceinline__ void enc_frags(const float (&xr)[kNT][8], u32x4 (&x)[kNT][N]) {
#pragma unroll
  for (int t = 0; t < kNT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float e0[B0 + N], e1[B0 + N];
      pe_blocks_of<B0 + N>(xr[t][2 * q], e0);
      pe_blocks_of<B0 + N>(xr[t][2 * q + 1], e1);
#pragma unroll
      for (int b = 0; b < N; ++b) x[t][b][q] = pk_bf16(e0[B0 + b], e1[B0 + b]);
    }
}

template <int W>
struct Shape {
  static constexpr int MT = W / 16, KS = W / 32;
  static constexpr int kBiasBytes = kNumLayers * W * 4;
};

// Object-streaming state of one tile (modes other than FWD_FULL): sigma as
// bf16 B fragments [wave][t][ks][lane], the running masked sum Z of h's hidden
// layer as fp32 accumulator rows [wave][t][mt][lane], the active-slot count
// [wave][t][pixel column].  Every access is a whole 16-byte lane vector.
template <int W>
struct StreamTile {
  static constexpr int64_t kSig = (int64_t)kWaves * kNT * (W / 32) * kFrag;
  static constexpr int64_t kZ = (int64_t)kWaves * kNT * (W / 16) * kFrag;
  static constexpr int64_t kCnt = (int64_t)kWaves * kNT * 16 * 4;
  static constexpr int64_t kBytes = kSig + kZ + kCnt;
};

// MODE selects the part of the path one launch runs: FWD_FULL the whole
// forward; FWD_BEGIN stages 0-1 (sigma into the state); FWD_ACC stage 2 (the
// slot loop, continuing the state's running sum); FWD_FINISH stages 3-9 from
// the state.  FWD_FULL compiles to the code it had before the modes existed.
//
// PE > 0: F's and h's inputs are positionally encoded with PE levels; F1 then
// runs over two stages of its own (stage indices below), and h's first layer
// takes pe_k16_steps(PE) 16-deep K-steps per slot.
template <int W, int PREC, int MODE, int PE>
__global__ __launch_bounds__(kThreads) void fwd_mfma_kernel(MfmaArgs a) {
  constexpr int MT = Shape<W>::MT, KS = Shape<W>::KS;
  constexpr int kShift = stage_shift(PE), kStages = kNumStages + kShift;
  // stage of each weight group (F1 and F2 share stage 0 without encoding)
  constexpr int sF1 = 0, sF1B = 1, sF2 = kShift, sF3 = 1 + kShift, sT1S = 2 + kShift,
                sT3 = 3 + kShift, sB1S = 4 + kShift, sB1T = 5 + kShift, sB2 = 6 + kShift,
                sB3 = 7 + kShift, sR1 = 8 + kShift, sR2 = 9 + kShift;
  constexpr int kE = pe_blocks(PE);                   // encoding blocks
  constexpr int kF1A = PE > 0 ? (kE + 1) / 2 : 1;     // F1's blocks in stage sF1
  constexpr int kF1B = kE - kF1A;                     // and in stage sF1B
  constexpr int kNK16 = PE > 0 ? pe_k16_steps(PE) : 1;   // h layer 1's K=16 steps
  constexpr bool kSlots = MODE == FWD_FULL || MODE == FWD_ACC;     // runs the slot loop
  constexpr bool kTrunk = MODE == FWD_FULL || MODE == FWD_BEGIN;   // runs F
  constexpr bool kHead = MODE == FWD_FULL || MODE == FWD_FINISH;   // runs T3, B, R
  extern __shared__ __attribute__((aligned(1024))) uint8_t lds[];
  const int wave = threadIdx.x >> 6;

  // LDS map: [resident | biases | slot order | stage buffer 0 | stage buffer 1]
  const int64_t res_bytes = a.res_bytes;
  uint8_t *L_res = lds;
  float *L_bias = (float *)(lds + res_bytes);
  int64_t stage_max = 0;
#pragma unroll
  for (int s = 0; s < kStages; ++s)
    stage_max = max(stage_max, a.stage_off[s + 1] - a.stage_off[s]);
  // slot-order table: for each pixel of the tile, its slots' indices in
  // canonical order (kpad bytes per pixel, a multiple of 4), and the tile's
  // alphas [slot][pixel] that the order is computed from (aslots slots)
  // (in sigma's LDS parking area, free until F's last layer ends, when that
  // area holds at least the table)
  uint8_t *L_perm = lds + res_bytes + Shape<W>::kBiasBytes;
  uint8_t *L_stage0 =
      L_perm + (size_t)kTilePx * a.kpad + (a.alpha_alias ? 0 : (size_t)kTilePx * 4 * a.aslots);
  uint8_t *L_stage1 = L_stage0 + stage_max;
  float *L_alpha = a.alpha_alias ? (float *)(L_stage1 + stage_max)
                                 : (float *)(L_perm + (size_t)kTilePx * a.kpad);
  // FWD_FINISH runs an odd number of stages per tile, so its buffer parity
  // flips from one tile to the next (par); every other mode keeps par = 0.
  int par = 0;
  auto stage_buf = [&](int s) { return ((s + par) & 1) ? L_stage1 : L_stage0; };
  // resident weights of the slot loop and all biases, once per workgroup
  const int lane0 = threadIdx.x & 63;
  auto fill_stage0 = [&](int s) {
    lds_fill(stage_buf(s), a.packed + a.stage_off[s], a.stage_off[s + 1] - a.stage_off[s], wave,
             lane0);
  };
  // bf16: [T1A | T2 (bf16)]; fp8: [T1A | T2 (fp8, 2 KiB fragments) | T2 row scales]
  constexpr bool kFp8 = PREC == GN_FP8_T;
  // fragment reads held ahead of their MFMAs (layer, mm): everywhere in bf16;
  // in fp8 everywhere but T3 and B's first layer (it spills there)
  constexpr bool kEarly = true, kEarlyT3B1 = !kFp8;
  constexpr int kT1ABytes = (MT * kNK16 * 512 + 1023) & ~1023;   // K=16 fragments of 512 B
  if constexpr (kSlots) {
    if (kFp8) {
      constexpr int64_t t1a = kT1ABytes;
      lds_fill(L_res, a.packed + a.res_off, t1a, wave, lane0);
      lds_fill(L_res + t1a, a.packed + a.t2q_off, res_bytes - t1a, wave, lane0);
    } else {
      lds_fill(L_res, a.packed + a.res_off, res_bytes, wave, lane0);
    }
  }
  lds_fill((uint8_t *)L_bias, a.packed + a.bias_off, Shape<W>::kBiasBytes, wave, lane0);
  if ((int)blockIdx.x < a.ntiles) {
    // FULL streams every stage; BEGIN (without encoding) and ACC keep their
    // few stages resident for the whole launch; BEGIN with encoding streams
    // its four stages per tile; FINISH starts its pipeline at T3's stage.
    if constexpr (MODE == FWD_FULL) fill_stage0(sF1);
    if constexpr (MODE == FWD_BEGIN) {
      fill_stage0(sF1);
      if constexpr (PE == 0) fill_stage0(sF3);
    }
    if constexpr (MODE == FWD_ACC) fill_stage0(sT1S);
    if constexpr (MODE == FWD_FINISH) fill_stage0(sT3);
  }
  wait_vm();
  __syncthreads();

  const uint8_t *T1A = L_res;
  const uint8_t *T2 = L_res + kT1ABytes;                           // bf16 form
  float *T2scale = (float *)(L_res + kT1ABytes + MT * 2 * kFrag);  // fp8 form
  if (kFp8 && kSlots) {
    // dequantisation factor s of the fp8 layer (weight row scale x activation
    // scale), and that layer's bias divided by it: the slot loop sums
    // relu(acc + c2 / s) = relu(s acc + c2) / s (s > 0) and the pool
    // multiplies by s once
    if ((int)threadIdx.x < W) {
      const float sc = T2scale[threadIdx.x] * a.sa;
      T2scale[threadIdx.x] = sc;
      L_bias[L_T2 * W + threadIdx.x] /= sc;
    }
    __syncthreads();
  }
  const float *bF1 = L_bias + L_F1 * W, *bF2 = L_bias + L_F2 * W, *bF3 = L_bias + L_F3 * W;
  const float *bT1 = L_bias + L_T1 * W, *bT2 = L_bias + L_T2 * W, *bT3 = L_bias + L_T3 * W;
  const float *bB1 = L_bias + L_B1 * W, *bB2 = L_bias + L_B2 * W, *bB3 = L_bias + L_B3 * W;
  const float *bR1 = L_bias + L_R1 * W, *bR2 = L_bias + L_R2 * W, *bR3 = L_bias + L_R3 * W;
  const int64_t f1_bytes = (int64_t)MT * kFrag;          // F1 precedes F2 in stage 0
  const int64_t r1p_bytes = (int64_t)MT * KS * kFrag;    // R1P precedes R1L in stage 8
  const int64_t r2_bytes = (int64_t)MT * KS * kFrag;     // R2 precedes R3 in stage 9

  // ---- tile -> frame pointers, first pixel
  // Frame pointers in the global address space: loads and stores through
  // them are global (vector-memory counter only).  Through generic pointers
  // they would be flat operations, which also count against the LDS counter,
  // so every wait for an LDS fragment would also wait for the HBM loads in
  // flight (the prefetched slot inputs among them).
  struct TileInfo {
    gcfloat *G, *L, *S;
    gfloat *O;
    int hw, K, q0;
  };
  auto resolve = [&](int tile) {
    TileInfo ti;
    if (a.tiles) {
      const TileRef tr = a.tiles[tile];
      const FrameDesc fd = a.frames[tr.frame];
      ti.G = (gcfloat *)fd.g; ti.L = (gcfloat *)fd.L; ti.S = (gcfloat *)fd.s;
      ti.O = (gfloat *)fd.out; ti.hw = fd.hw; ti.K = fd.k;
      ti.q0 = tr.q0;
    } else {
      const int f = tile / a.tiles_per_frame;
      ti.hw = a.b.hw;
      ti.K = a.b.k;
      ti.q0 = (tile - f * a.tiles_per_frame) * kTilePx;
      ti.G = (gcfloat *)(a.b.gbuf + (size_t)f * kNG * ti.hw);
      ti.L = (gcfloat *)(a.b.layers + (size_t)f * ti.K * kNL * ti.hw);
      ti.S = (gcfloat *)(a.b.scene + (size_t)f * kNS);
      ti.O = (gfloat *)(a.b.out + (size_t)f * kNOUT * ti.hw);
    }
    return ti;
  };
  // F's input (G-buffer planes 0..13, scene 0..15, zero pad) of a tile: lane
  // group g holds columns 8g..8g+7 of its pixel.  Loaded one tile ahead.
  auto load_x = [&](const TileInfo &ti, int ln, float (&xr)[kNT][8]) {
    const int gg = ln >> 4, cc = ln & 15;
#pragma unroll
    for (int t = 0; t < kNT; ++t) {
      const int q = ti.q0 + wave * (kNT * 16) + t * 16 + cc;
      const int qq = q < ti.hw ? q : ti.hw - 1;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int c = 8 * gg + j;
        xr[t][j] = c < kNG ? ti.G[(size_t)c * ti.hw + qq] : (c < kNG + kNS ? ti.S[c - kNG] : 0.0f);
      }
    }
  };
  // Canonical slot order (FULL mode, if the handle asks for it): each
  // pixel's slots are pooled in an order that depends only on their records,
  // so the rounding of the running sum cannot depend on the order the caller
  // passed them in.  With up to kFastK slots the tile's alphas are copied to
  // LDS during F's last layer and ranked at the start of the slot stage.
  constexpr int kFastK = 8;
  float xr[kNT][8];
  TileInfo nti;
  if ((int)blockIdx.x < a.ntiles) {
    nti = resolve(blockIdx.x);
    if constexpr (kTrunk) load_x(nti, lane0, xr);
  }

  for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    const bool has_next = tile + (int)gridDim.x < a.ntiles;
    // Opaque per-tile copies of the lane id and the packed-weight base keep
    // the compiler from hoisting every derived address (staging sources of
    // all stages, channel masks) out of the tile loop and holding them in
    // registers for its whole length.
    int lane = threadIdx.x & 63;
    const uint8_t *packed = a.packed;
    asm volatile("" : "+v"(lane), "+s"(packed));
    const int g = lane >> 4, col = lane & 15;
    auto fill_stage = [&](int s) {
      lds_fill(stage_buf(s), packed + a.stage_off[s], a.stage_off[s + 1] - a.stage_off[s], wave,
               lane);
    };
    // ---- the tile's frame (resolved one tile ahead)
    const TileInfo ti = nti;
    gcfloat *Gp = ti.G, *Lp = ti.L;
    gfloat *Op = ti.O;
    const int hw = ti.hw, K = ti.K, q0 = ti.q0;
    int qc[kNT];
    bool valid[kNT];
#pragma unroll
    for (int t = 0; t < kNT; ++t) {
      const int q = q0 + wave * (kNT * 16) + t * 16 + col;
      valid[t] = q < hw;
      qc[t] = valid[t] ? q : hw - 1;          // tail lanes recompute a real pixel
    }
    // this wave's part of the tile's streaming state
    uint8_t *st = a.state + (size_t)tile * StreamTile<W>::kBytes;
    gu32x4 *st_sig = (gu32x4 *)(st + (size_t)wave * (kNT * KS * kFrag)) + lane;
    gf32x4 *st_z = (gf32x4 *)(st + StreamTile<W>::kSig + (size_t)wave * (kNT * MT * kFrag)) + lane;
    gfloat *st_cnt = (gfloat *)(st + StreamTile<W>::kSig + StreamTile<W>::kZ) + wave * (kNT * 16) + col;
    u32x4 sig[kNT][KS];   // sigma: from F (FULL, BEGIN) or from the state (ACC)
    f32x4 Z[kNT][MT];     // running masked sum of h's hidden layer, and
    float cnt[kNT];       // the number of active slots it holds

    // FULL: sigma is needed again only by B's first layer: park it in this wave's
    // scratch instead of holding 32 registers through the slot loop
    // (LDS left free by the weights holds it for the first sig_lds_waves
    // waves; the others use a per-wave slot in HBM)
    constexpr int kSigBytes = kNT * KS * kFrag;
    // Both stage buffers hold only stages 1-4's fragments (stage_max bytes or
    // fewer) while sigma is parked, so their tails serve the last waves.
    const bool sig_in_lds = wave < a.sig_lds_waves;
    const int nfree = a.sig_lds_waves - a.sig_tail_waves;
    uint8_t *sig_lds = wave < nfree ? L_stage1 + stage_max + (size_t)wave * kSigBytes
                                    : ((wave - nfree) & 1 ? L_stage1 : L_stage0) + stage_max -
                                          (size_t)(1 + (wave - nfree) / 2) * kSigBytes;
    uint8_t *sig_slot = a.sig_scratch + ((size_t)blockIdx.x * kWaves + wave) * kSigBytes;

    // The tile's alphas, slot by slot, into the LDS alpha table (canonical
    // order with up to kFastK slots): 64-pixel blocks, lane i copying pixel i
    // of its block (clamped to the frame).  Issued with F's second layer and
    // ranked before its last.
    const bool canon_fast = MODE == FWD_FULL && a.canon && K > 1 && K <= kFastK;
    auto copy_alphas = [&]() {
      for (int b = wave; b < 4 * K; b += kWaves) {
        const int j = b >> 2, p0 = (b & 3) * 64;
        const int q = min(q0 + p0 + lane, hw - 1);
        __builtin_amdgcn_global_load_lds(
            (const void *)(Lp + ((size_t)j * kNL + kAlpha) * hw + q),
            (__attribute__((address_space(3))) void *)(L_alpha + j * kTilePx + p0), 4, 0, 0);
      }
    };

    if constexpr (kTrunk) {
      u32x4 h2[kNT][KS];
      if constexpr (PE == 0) {
        // ================= stage 0: F layers 1-2 =================
        if constexpr (MODE == FWD_FULL) fill_stage(sF3);
        if (canon_fast) copy_alphas();
        {
          u32x4 x[kNT][1];
#pragma unroll
          for (int t = 0; t < kNT; ++t)
            x[t][0] = u32x4{pk_bf16(xr[t][0], xr[t][1]), pk_bf16(xr[t][2], xr[t][3]),
                            pk_bf16(xr[t][4], xr[t][5]), pk_bf16(xr[t][6], xr[t][7])};
          const uint8_t *S = stage_buf(sF1);
          u32x4 h1[kNT][KS];
          layer<MT, 1, true, kEarly>(h1, S, x, bF1, g, lane);
          layer<MT, KS, true, kEarly>(h2, S + f1_bytes, h1, bF2, g, lane);
        }
        if constexpr (MODE == FWD_FULL) {
          wait_vm();
          __syncthreads();
        }
      } else {
        // ====== stages 0-1: F layer 1 on the encoded input; stage 2: F layer 2 ======
        fill_stage(sF1B);
        f32x4 acc[kNT][MT];
        bias_init(acc, bF1, g);
        {
          u32x4 x[kNT][kF1A];
          enc_frags<0, kF1A>(xr, x);
          mm<MT, kF1A, kEarly>(acc, stage_buf(sF1), x, lane);
        }
        wait_vm();
        __syncthreads();
        fill_stage(sF2);
        u32x4 h1[kNT][KS];
        {
          u32x4 x[kNT][kF1B];
          enc_frags<kF1A, kF1B>(xr, x);
          mm<MT, kF1B, kEarly>(acc, stage_buf(sF1B), x, lane);
          to_frags<MT, true>(acc, h1);
        }
        wait_vm();
        __syncthreads();
        fill_stage(sF3);
        if (canon_fast) copy_alphas();
        layer<MT, KS, true, kEarly>(h2, stage_buf(sF2), h1, bF2, g, lane);
        wait_vm();
        __syncthreads();
      }

      // ================= F layer 3 -> sigma =================
      if constexpr (MODE == FWD_FULL) fill_stage(sT1S);
      // Canonical order of each pixel's slots, into this wave's part of the
      // LDS table (byte r of a pixel's entry: its slot of rank r).  Keys: the
      // bits of alpha for active slots, 0xFFFFFF00 + j for an inactive slot j
      // (above every active key, distinct), 0xFFFFFFFF past K.  With up to
      // kFastK slots each lane ranks its lane group's slots g and g + 4 from the
      // alphas in LDS (they landed by the last barrier); two active slots of
      // equal alpha (and more than kFastK slots) take the full comparison of
      // slot_order.h.
      if (MODE == FWD_FULL && a.canon && K > 1) {
        uint8_t *perm_px[kNT];
#pragma unroll
        for (int t = 0; t < kNT; ++t)
          perm_px[t] = L_perm + (size_t)(wave * (kNT * 16) + t * 16 + col) * a.kpad;
        if (K <= kFastK) {
          float alk[kNT][kFastK];
#pragma unroll
          for (int t = 0; t < kNT; ++t)
#pragma unroll
            for (int j = 0; j < kFastK; ++j)
              alk[t][j] = j < K ? L_alpha[j * kTilePx + wave * (kNT * 16) + t * 16 + col] : 0.0f;
          unsigned slow = 0;
#pragma unroll
          for (int t = 0; t < kNT; ++t) {
            uint32_t key[kFastK];
#pragma unroll
            for (int j = 0; j < kFastK; ++j)
              key[j] = j >= K ? 0xFFFFFFFFu
                              : (alk[t][j] > 0.0f ? __float_as_uint(alk[t][j]) : 0xFFFFFF00u + j);
#pragma unroll
            for (int sl = 0; sl < 2; ++sl) {
              const int i = g + 4 * sl;
              uint32_t ki = key[4 * sl];
#pragma unroll
              for (int jj = 1; jj < 4; ++jj) ki = g == jj ? key[4 * sl + jj] : ki;
              int lt = 0, le = 0;
#pragma unroll
              for (int j = 0; j < kFastK; ++j) {
                lt += key[j] < ki ? 1 : 0;
                le += key[j] <= ki ? 1 : 0;
              }
              if (i < K) {
                if (le == lt + 1)
                  perm_px[t][lt] = ki >= 0xFFFFFF00u ? (uint8_t)0xFF : (uint8_t)i;
                else
                  slow |= 1u << (2 * t + sl);
              }
            }
          }
          if (__builtin_amdgcn_ballot_w64(slow != 0)) {
#pragma unroll
            for (int t = 0; t < kNT; ++t)
#pragma unroll
              for (int sl = 0; sl < 2; ++sl)
                if (slow & (1u << (2 * t + sl)))
                  perm_px[t][slot_rank(Lp + qc[t], (size_t)hw, K, g + 4 * sl)] =
                      slot_active(Lp + qc[t], hw, g + 4 * sl) ? (uint8_t)(g + 4 * sl) : (uint8_t)0xFF;
          }
        } else {
#pragma unroll
          for (int t = 0; t < kNT; ++t)
            for (int i = g; i < K; i += 4)
              perm_px[t][slot_rank(Lp + qc[t], (size_t)hw, K, i)] =
                  slot_active(Lp + qc[t], hw, i) ? (uint8_t)i : (uint8_t)0xFF;
        }
        // the wave reads the table back in its own slot loop (LDS operations of
        // one wave complete in order)
      }
      // the alpha table shares sigma's parking area: every wave has read it
      // before any wave parks sigma there
      if (canon_fast && a.alpha_alias) __syncthreads();
      if constexpr (MODE == FWD_BEGIN && PE > 0) {
        if (has_next) fill_stage(sF1);      // the next tile's first stage
      }
      layer<MT, KS, false, kEarly>(sig, stage_buf(sF3), h2, bF3, g, lane);
      if constexpr (MODE == FWD_BEGIN) {
        // sigma goes to the streaming state; the next tile's F input is requested
#pragma unroll
        for (int t = 0; t < kNT; ++t)
#pragma unroll
          for (int k = 0; k < KS; ++k) st_sig[(t * KS + k) * 64] = sig[t][k];
        if (has_next) {
          nti = resolve(tile + gridDim.x);
          load_x(nti, lane, xr);
        }
        if constexpr (PE > 0) {
          // the next tile's first stage has landed; this stage's buffer is free
          wait_vm();
          __syncthreads();
        }
      } else {
        if (sig_in_lds) {
#pragma unroll
          for (int t = 0; t < kNT; ++t)
#pragma unroll
            for (int k = 0; k < KS; ++k) *(u32x4 *)(sig_lds + (t * KS + k) * kFrag + lane * 16) = sig[t][k];
        } else {
#pragma unroll
          for (int t = 0; t < kNT; ++t)
#pragma unroll
            for (int k = 0; k < KS; ++k) *(u32x4 *)(sig_slot + (t * KS + k) * kFrag + lane * 16) = sig[t][k];
        }
        // the kNT x KS stores above stay in flight; the same wave reads them back
        // in stage 3, after stage 2's full wait
        if (sig_in_lds)
          stage_sync_after_stores<0>();
        else
          stage_sync_after_stores<kNT * KS>();
      }
    }

    if constexpr (kSlots) {
      // ================= stage 2: u = W1s sigma + c1, then the slot loop =======
      if constexpr (MODE == FWD_FULL) fill_stage(sT3);
      if constexpr (MODE == FWD_ACC) {
#pragma unroll
        for (int t = 0; t < kNT; ++t)
#pragma unroll
          for (int k = 0; k < KS; ++k) sig[t][k] = st_sig[(t * KS + k) * 64];
      }
      {
        // the slot-order table of this tile (written above): the lane's pixel
        // of N-tile t has its entry at byte pofs + 16 t kpad
        const bool canon = MODE == FWD_FULL && a.canon && K > 1;
        const uint32_t pofs = (uint32_t)(wave * (kNT * 16) + col) * a.kpad;
        // u = W1s sigma + c1 in fp32 accumulator layout: the C operand of h's
        // first layer for every slot
        f32x4 u[kNT][MT];
        bias_init(u, bT1, g);
        mm<MT, KS, kEarly>(u, stage_buf(sT1S), sig, lane);

        if constexpr (kFp8) {
          // fp8: h's first layer runs in units of the activation scale (its
          // inputs b_i and u are divided by it), so its output quantises directly
#pragma unroll
          for (int t = 0; t < kNT; ++t)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) u[t][mt] *= a.inv_sa;
        }
#pragma unroll
        for (int t = 0; t < kNT; ++t) {
          cnt[t] = 0.0f;
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) Z[t][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        if constexpr (MODE == FWD_ACC) {
          if (a.state_load) {     // continue the running sum of earlier calls
#pragma unroll
            for (int t = 0; t < kNT; ++t) {
              cnt[t] = st_cnt[t * 16];
#pragma unroll
              for (int mt = 0; mt < MT; ++mt) Z[t][mt] = st_z[(t * MT + mt) * 64];
            }
          }
        }
        // Slot inputs: lane group g < 3 carries planes 4g..4g+3 of its pixel (the
        // K=16 operand of h's first layer; with encoding, lane group g carries
        // planes 3g..3g+2 and their encodings); the next slot's planes are
        // loaded one slot ahead so their latency overlaps the current slot's work.
        constexpr int kRaw = PE > 0 ? 3 : 4;
        float nxt[kNT][kRaw];
        // Iteration i takes each pixel's slot of rank i (canonical order) or
        // slot i (input order).  In canonical order the inactive slots come
        // last and their table bytes are 0xFF: such a pixel loads nothing and
        // presents zeros (alpha 0: its term is masked out exactly), so half the
        // loads of the workloads' slot stage never reach the memory system.
        auto load_slot = [&](int i) {
          uint32_t qs[kNT];      // element offsets (frames of the MFMA path stay below 2^32)
          bool act[kNT];
#pragma unroll
          for (int t = 0; t < kNT; ++t) {
            const int si = canon ? (int)L_perm[pofs + t * 16 * a.kpad + i] : i;
            act[t] = si != 0xFF;
            qs[t] = (uint32_t)si * (uint32_t)(kNL * hw) + (uint32_t)qc[t];
            asm volatile("" : "+v"(qs[t]));   // per-slot addresses stay in the loop body
          }
#pragma unroll
          for (int t = 0; t < kNT; ++t)
#pragma unroll
            for (int j = 0; j < kRaw; ++j) {
              if constexpr (PE > 0)
                nxt[t][j] = act[t] ? Lp[(size_t)(3 * g + j) * hw + qs[t]] : 0.0f;
              else
                nxt[t][j] = g < 3 && act[t] ? Lp[(size_t)(4 * g + j) * hw + qs[t]] : 0.0f;
            }
        };
        if (K > 0) load_slot(0);
        for (int i = 0; i < K; ++i) {
          float cur[kNT][kRaw];
#pragma unroll
          for (int t = 0; t < kNT; ++t)
#pragma unroll
            for (int j = 0; j < kRaw; ++j) cur[t][j] = nxt[t][j];
          if (i + 1 < K) load_slot(i + 1);
          // A slot in which no pixel of this wave takes part adds exactly zero
          // to the running sum and the count: skip its two layers.  The lanes
          // that loaded alpha decide (lane group 2 position 1, or with
          // encoding lane group 3 position 0).
          bool any = false;
#pragma unroll
          for (int t = 0; t < kNT; ++t)
            any = any || (PE > 0 ? (g == 3 && cur[t][0] > 0.0f) : (g == 2 && cur[t][1] > 0.0f));
          if (__builtin_amdgcn_ballot_w64(any) == 0) continue;
          uint2 bi[kNT][kNK16];
          float m[kNT];
#pragma unroll
          for (int t = 0; t < kNT; ++t) {
            if constexpr (PE > 0) {
              // value v = 4 s + j of the lane group's list: block v / 3 of raw
              // plane 3 g + v % 3 (zero past the last block)
              float enc[3][kE];
#pragma unroll
              for (int c = 0; c < 3; ++c) pe_blocks_of<kE>(cur[t][c], enc[c]);
              float e[4 * kNK16];
#pragma unroll
              for (int v = 0; v < 4 * kNK16; ++v) {
                const float x = v / 3 < kE ? enc[v % 3][v / 3] : 0.0f;
                e[v] = kFp8 ? x * a.inv_sa : x;
              }
#pragma unroll
              for (int st = 0; st < kNK16; ++st)
                bi[t][st] = uint2{pk_bf16(e[4 * st], e[4 * st + 1]),
                                  pk_bf16(e[4 * st + 2], e[4 * st + 3])};
              // alpha (plane 9) sits in lane group 3 at position 0: broadcast it
              const float al = __int_as_float(
                  __builtin_amdgcn_ds_bpermute((col + 48) * 4, __float_as_int(cur[t][0])));
              m[t] = al > 0.0f ? 1.0f : 0.0f;
            } else {
              if constexpr (kFp8)
                bi[t][0] = uint2{pk_bf16(cur[t][0] * a.inv_sa, cur[t][1] * a.inv_sa),
                                 pk_bf16(cur[t][2] * a.inv_sa, cur[t][3] * a.inv_sa)};
              else
                bi[t][0] = uint2{pk_bf16(cur[t][0], cur[t][1]), pk_bf16(cur[t][2], cur[t][3])};
              // alpha (plane 9) sits in lane group 2 at position 1: broadcast it
              const float al = __int_as_float(
                  __builtin_amdgcn_ds_bpermute((col + 32) * 4, __float_as_int(cur[t][1])));
              m[t] = al > 0.0f ? 1.0f : 0.0f;
            }
          }
          if constexpr (kFp8) {
          // h layer 1 (bf16 MFMA, in activation-scale units), quantised to
          // E4M3: lane byte 4*mt + r holds row 16*mt + 4*g + r, the order the
          // fp8 weights of layer 2 were packed in.
          i32x8 zq[kNT];
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            if constexpr (PE > 0) {
              f32x4 acc1[kNT];
#pragma unroll
              for (int t = 0; t < kNT; ++t) acc1[t] = u[t][mt];
#pragma unroll
              for (int st = 0; st < kNK16; ++st) {
                const uint2 w = ld_frag16(T1A, mt * kNK16 + st, lane);
#pragma unroll
                for (int t = 0; t < kNT; ++t) acc1[t] = mma16(w, bi[t][st], acc1[t]);
              }
#pragma unroll
              for (int t = 0; t < kNT; ++t) zq[t][mt] = relu_pack_fp8x4(acc1[t]);
            } else {
              const uint2 w = ld_frag16(T1A, mt, lane);
#pragma unroll
              for (int t = 0; t < kNT; ++t)
                zq[t][mt] = relu_pack_fp8x4(mma16(w, bi[t][0], u[t][mt]));
            }
          }
          __builtin_amdgcn_s_setprio(1);   // as for the bf16 layer 2 below
          // h layer 2 on the fp8 matrix cores (K = 128 in one instruction),
          // the running sum kept in units of the dequantisation factor s
          // (applied at the pool); each M-tile's fragment is requested one
          // M-tile ahead of its MFMAs.
          i32x8 wn = ld_frag8(T2, 0, lane);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            const i32x8 w = wn;
            if (mt + 1 < MT) wn = ld_frag8(T2, mt + 1, lane);
            const f32x4 b = *(const f32x4 *)(bT2 + 16 * mt + 4 * g);     // c2 / s
#pragma unroll
            for (int t = 0; t < kNT; ++t) {
              const f32x4 r = relu4(mma_fp8(w, zq[t], b));
              Z[t][mt].x = fmaf(m[t], r.x, Z[t][mt].x);
              Z[t][mt].y = fmaf(m[t], r.y, Z[t][mt].y);
              Z[t][mt].z = fmaf(m[t], r.z, Z[t][mt].z);
              Z[t][mt].w = fmaf(m[t], r.w, Z[t][mt].w);
            }
          }
          } else {
          // h layer 1: z1 = relu(W1b b_i + u)
          u32x4 z1[kNT][KS];
#pragma unroll
          for (int p = 0; p < KS; ++p) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              f32x4 acc1[kNT];
              if constexpr (PE > 0) {
#pragma unroll
                for (int t = 0; t < kNT; ++t) acc1[t] = u[t][2 * p + h];
#pragma unroll
                for (int st = 0; st < kNK16; ++st) {
                  const uint2 w = ld_frag16(T1A, (2 * p + h) * kNK16 + st, lane);
#pragma unroll
                  for (int t = 0; t < kNT; ++t) acc1[t] = mma16(w, bi[t][st], acc1[t]);
                }
              } else {
                const uint2 w = ld_frag16(T1A, 2 * p + h, lane);
#pragma unroll
                for (int t = 0; t < kNT; ++t) acc1[t] = mma16(w, bi[t][0], u[t][2 * p + h]);
              }
#pragma unroll
              for (int t = 0; t < kNT; ++t) {
                const f32x4 v = acc1[t];
                z1[t][p][2 * h] = relu_bf16x2(pk_bf16(v.x, v.y));
                z1[t][p][2 * h + 1] = relu_bf16x2(pk_bf16(v.z, v.w));
              }
            }
          }
          // h layer 2 at raised wave priority: of the two waves that share a
          // SIMD, the one in this layer issues first, which offsets the pair
          // so that one's matrix-core work overlaps the other's layer 1 and
          // LDS reads (1-1.5% of the 512^2 K = 8 frame in bf16, ~1% in fp8;
          // issuing the next M-tile's MFMAs before each M-tile's relu and
          // running sum was slower in both forms).
          __builtin_amdgcn_s_setprio(1);
          // h layer 2 and the masked running sum: Z += m * relu(A2 z1 + c2).
          // The fragments stream one K-step ahead of the MFMAs that use them.
          u32x4 wnext = ld_frag(T2, 0, lane);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            const f32x4 b = *(const f32x4 *)(bT2 + 16 * mt + 4 * g);
            f32x4 acc[kNT];
#pragma unroll
            for (int t = 0; t < kNT; ++t) acc[t] = b;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
              const u32x4 w = wnext;
              if (mt * KS + ks + 1 < MT * KS) wnext = ld_frag(T2, mt * KS + ks + 1, lane);
#pragma unroll
              for (int t = 0; t < kNT; ++t) acc[t] = mma(w, z1[t][ks], acc[t]);
            }
#pragma unroll
            for (int t = 0; t < kNT; ++t) {
              const f32x4 r = relu4(acc[t]);    // one v_med3 each
              Z[t][mt].x = fmaf(m[t], r.x, Z[t][mt].x);
              Z[t][mt].y = fmaf(m[t], r.y, Z[t][mt].y);
              Z[t][mt].z = fmaf(m[t], r.z, Z[t][mt].z);
              Z[t][mt].w = fmaf(m[t], r.w, Z[t][mt].w);
            }
          }
          }
#pragma unroll
          for (int t = 0; t < kNT; ++t) cnt[t] += m[t];
          __builtin_amdgcn_s_setprio(0);
        }
      }
      if constexpr (MODE == FWD_ACC) {
#pragma unroll
        for (int t = 0; t < kNT; ++t) {
          if (g == 0) st_cnt[t * 16] = cnt[t];
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) st_z[(t * MT + mt) * 64] = Z[t][mt];
        }
        if (has_next) nti = resolve(tile + gridDim.x);
      } else {
        wait_vm();
        __syncthreads();
      }
    }

    if constexpr (kHead) {
      // ================= stage 3: pool and h layer 3 -> tau =================
      fill_stage(sB1S);
      u32x4 sig2[kNT][KS];
      if constexpr (MODE == FWD_FINISH) {
        // the pool state and sigma come from the streaming state
#pragma unroll
        for (int t = 0; t < kNT; ++t) {
          cnt[t] = a.state_load ? st_cnt[t * 16] : 0.0f;
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
            Z[t][mt] = a.state_load ? st_z[(t * MT + mt) * 64] : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int k = 0; k < KS; ++k) sig2[t][k] = st_sig[(t * KS + k) * 64];
        }
      } else {
#pragma unroll
        for (int t = 0; t < kNT; ++t)
#pragma unroll
          for (int k = 0; k < KS; ++k)
            sig2[t][k] = sig_in_lds ? *(const u32x4 *)(sig_lds + (t * KS + k) * kFrag + lane * 16)
                                    : *(const u32x4 *)(sig_slot + (t * KS + k) * kFrag + lane * 16);
      }
      u32x4 tau[kNT][KS];
      {
        // fp8: the running sum is in units of the dequantisation factor s
        // (weight row scale x activation scale) of the slot loop's fp8 layer
        f32x4 s8[MT];
        if constexpr (kFp8) {
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            if constexpr (MODE == FWD_FULL)
              s8[mt] = *(const f32x4 *)(T2scale + 16 * mt + 4 * g);
            else
              s8[mt] = *(const f32x4 *)((const float *)(a.packed + a.t2s_off) + 16 * mt + 4 * g) *
                       a.sa;
          }
        }
        u32x4 zs[kNT][KS];
        f32x4 acc[kNT][MT];
#pragma unroll
        for (int t = 0; t < kNT; ++t) {
          const bool mean = a.pool == GN_POOL_MEAN;
          const float inv = mean ? 1.0f / fmaxf(cnt[t], 1.0f) : 1.0f;
          const float bs = mean ? (cnt[t] > 0.0f ? 1.0f : 0.0f) : cnt[t];
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            const f32x4 v = kFp8 ? (Z[t][mt] * s8[mt]) * inv : Z[t][mt] * inv;
            zs[t][mt >> 1][2 * (mt & 1)] = pk_bf16(v.x, v.y);
            zs[t][mt >> 1][2 * (mt & 1) + 1] = pk_bf16(v.z, v.w);
            acc[t][mt] = *(const f32x4 *)(bT3 + 16 * mt + 4 * g) * bs;
          }
        }
        mm<MT, KS, kEarlyT3B1>(acc, stage_buf(sT3), zs, lane);
        to_frags<MT, false>(acc, tau);
      }
      wait_vm();
      __syncthreads();

      // ================= stages 4-5: B layer 1 on [sigma; tau] =================
      fill_stage(sB1T);
      f32x4 accB[kNT][MT];
      bias_init(accB, bB1, g);
      mm<MT, KS, kEarlyT3B1>(accB, stage_buf(sB1S), sig2, lane);
      wait_vm();
      __syncthreads();

      fill_stage(sB2);
      u32x4 hb[kNT][KS];
      mm<MT, KS, kEarlyT3B1>(accB, stage_buf(sB1T), tau, lane);
      to_frags<MT, true>(accB, hb);
      wait_vm();
      __syncthreads();

      // ================= stage 6: B layer 2 =================
      fill_stage(sB3);
      // L_d for R's first layer (stage 8), requested two stages early
      float ldr[kNT][3];
#pragma unroll
      for (int t = 0; t < kNT; ++t)
#pragma unroll
        for (int c = 0; c < 3; ++c) ldr[t][c] = g == 0 ? Gp[(size_t)(11 + c) * hw + qc[t]] : 0.0f;
      {
        u32x4 hb2[kNT][KS];
        layer<MT, KS, true, kEarly>(hb2, stage_buf(sB2), hb, bB2, g, lane);
#pragma unroll
        for (int t = 0; t < kNT; ++t)
#pragma unroll
          for (int k = 0; k < KS; ++k) hb[t][k] = hb2[t][k];
      }
      wait_vm();
      __syncthreads();

      // ================= stage 7: B layer 3 -> phi =================
      fill_stage(sR1);
      u32x4 phi[kNT][KS];
      layer<MT, KS, false, kEarly>(phi, stage_buf(sB3), hb, bB3, g, lane);
      wait_vm();
      __syncthreads();

      // ================= stage 8: R layer 1 on [phi; L_d] =================
      fill_stage(sR2);
      u32x4 hr[kNT][KS];
      {
        u32x4 ld[kNT][1];
#pragma unroll
        for (int t = 0; t < kNT; ++t)
          ld[t][0] = u32x4{pk_bf16(ldr[t][0], ldr[t][1]), pk_bf16(ldr[t][2], 0.0f), 0u, 0u};
        f32x4 acc[kNT][MT];
        bias_init(acc, bR1, g);
        mm<MT, KS, kEarly>(acc, stage_buf(sR1), phi, lane);
        mm<MT, 1, kEarly>(acc, stage_buf(sR1) + r1p_bytes, ld, lane);
        to_frags<MT, true>(acc, hr);
      }
      wait_vm();
      __syncthreads();

      // ================= stage 9: R layers 2-3 -> radiance =================
      if (has_next) {
        if constexpr (MODE == FWD_FULL) {
          fill_stage(sF1);
          nti = resolve(tile + gridDim.x);
          load_x(nti, lane, xr);
        } else {
          // the next tile's T3 stage goes to the buffer this tile's R1 stage used
          lds_fill(((sT3 + (par ^ 1)) & 1) ? L_stage1 : L_stage0, packed + a.stage_off[sT3],
                   a.stage_off[sT3 + 1] - a.stage_off[sT3], wave, lane);
          nti = resolve(tile + gridDim.x);
        }
      }
      {
        u32x4 hr2[kNT][KS];
        layer<MT, KS, true, kEarly>(hr2, stage_buf(sR2), hr, bR2, g, lane);
        f32x4 y[kNT][1];
        bias_init(y, bR3, g);
        mm<1, KS, kEarly>(y, stage_buf(sR2) + r2_bytes, hr2, lane);
        // Lane group 0 holds rows 0..2.  Tail lanes store the value of pixel
        // hw - 1 they recomputed (bitwise the same as that pixel's own lane),
        // so exactly 3 kNT store instructions issue, with a non-empty mask.
#pragma unroll
        for (int t = 0; t < kNT; ++t) {
          if (g == 0) {
            Op[qc[t]] = y[t][0].x;
            Op[(size_t)hw + qc[t]] = y[t][0].y;
            Op[(size_t)2 * hw + qc[t]] = y[t][0].z;
          }
        }
      }
      stage_sync_after_stores<3 * kNT>();
      if constexpr (MODE == FWD_FINISH) par ^= 1;
    }
  }
}

// ---- weight packing ---------------------------------------------------------
struct PackArgs {
  const float *master;
  uint8_t *packed;
  ChunkDesc chunk[kNumChunks];
  LayerOff lo[kNumLayers];
  int W;
  int64_t bias_off;
};

__device__ __forceinline__ int chain_col(int ks, int g, int j) {
  return 32 * ks + (j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4));
}

// One thread per bf16 element of one chunk (blockIdx.y = chunk).
__global__ void pack_bf16_kernel(PackArgs p) {
  const ChunkDesc d = p.chunk[blockIdx.y];
  const int lg = d.kmap == KMAP_MEM16 || d.kmap == KMAP_PE16 ? 2 : 3;   // log2 elements per lane
  const int64_t n = (int64_t)d.mt * d.ks * 64 << lg;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int j = (int)(e & ((1 << lg) - 1));
  const int lane = (int)((e >> lg) & 63);
  const int fragi = (int)(e >> (lg + 6));
  const int mt = fragi / d.ks, ks = fragi - mt * d.ks;
  const int row = 16 * mt + (lane & 15);
  const int g = lane >> 4;
  int k;
  if (d.kmap == KMAP_ENC) {
    const int c = 8 * g + j;
    k = c < d.raw ? (d.ks0 + ks) * d.raw + c : d.ncols;
  } else if (d.kmap == KMAP_PE16) {
    const int v = 4 * ks + j, blk = v / 3;
    k = blk < d.nblocks ? blk * d.raw + 3 * g + v % 3 : d.ncols;
  } else {
    k = d.kmap == KMAP_MEM     ? 32 * ks + 8 * g + j
        : d.kmap == KMAP_MEM16 ? 16 * ks + 4 * g + j
                               : chain_col(ks, g, j);
  }
  const LayerOff lo = p.lo[d.layer];
  float v = 0.0f;
  if (row < d.nrows && k < d.ncols) v = p.master[lo.w + (int64_t)row * lo.in + d.col0 + k];
  __bf16 h = (__bf16)v;
  ((__bf16 *)(p.packed + d.offset))[e] = h;
}

// fp8 copy of h's second layer (the layer that runs once per slot): per output
// row n a scale s_n = max_k |A2[n][k]| / 448 and bytes E4M3(A2[n][k] / s_n),
// stored as MT fragments of 64 lanes x 32 bytes.  Lane 16 g + (n & 15) of
// fragment n >> 4 holds, at byte 4 q + r, input k = 16 q + 4 g + r; a
// fragment keeps bytes 0-15 of every lane in its first KiB and bytes 16-31
// in its second (ld_frag8).
// One block per output row, one thread per input.
__global__ void pack_fp8_t2_kernel(PackArgs p, uint8_t *q8, float *scale) {
  __shared__ float red[256];
  const int n = blockIdx.x, k = threadIdx.x, W = p.W;
  const LayerOff lo = p.lo[L_T2];
  const float v = k < W ? p.master[lo.w + (int64_t)n * W + k] : 0.0f;
  red[k] = fabsf(v);
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (k < w) red[k] = fmaxf(red[k], red[k + w]);
    __syncthreads();
  }
  const float s = red[0] > 0.0f ? red[0] / 448.0f : 1.0f;
  if (k == 0) scale[n] = s;
  if (k >= W) return;
  const float x = fminf(fmaxf(v / s, -448.0f), 448.0f);
  const uint8_t b = (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.0f, 0, false) & 0xff);
  const int g = (k & 15) >> 2, j = 4 * (k >> 4) + (k & 3);
  const int lane = 16 * g + (n & 15);
  q8[(size_t)(n >> 4) * 2048 + (j >> 4) * 1024 + lane * 16 + (j & 15)] = b;
}

__global__ void pack_bias_kernel(PackArgs p) {
  const int l = blockIdx.x, o = threadIdx.x;
  if (o >= p.W) return;
  const LayerOff lo = p.lo[l];
  float v = o < lo.out ? p.master[lo.b + o] : 0.0f;
  ((float *)(p.packed + p.bias_off))[(int64_t)l * p.W + o] = v;
}

}  // namespace

size_t mfma_sig_scratch_bytes(int W, int grid) {
  return (size_t)grid * kWaves * kNT * (W / 32) * kFrag;
}

hipError_t launch_pack_weights(const float *master, uint8_t *packed, const PackedLayout &pl,
                               float fp8_act_scale, hipStream_t stream) {
  (void)fp8_act_scale;
  PackArgs p;
  p.master = master;
  p.packed = packed;
  for (int c = 0; c < kNumChunks; ++c) p.chunk[c] = pl.chunk[c];
  layer_offsets(pl.W, pl.pe, p.lo);
  p.W = pl.W;
  p.bias_off = pl.bias_off;
  int64_t maxn = 0;
  for (int c = 0; c < kNumChunks; ++c)
    maxn = std::max<int64_t>(maxn, (int64_t)pl.chunk[c].mt * pl.chunk[c].ks * 512);
  hipLaunchKernelGGL(pack_bf16_kernel, dim3((unsigned)((maxn + 255) / 256), kNumChunks), dim3(256),
                     0, stream, p);
  hipLaunchKernelGGL(pack_bias_kernel, dim3(kNumLayers), dim3(pl.W), 0, stream, p);
  hipLaunchKernelGGL(pack_fp8_t2_kernel, dim3(pl.W), dim3(pl.W), 0, stream, p,
                     packed + pl.t2q_off, (float *)(packed + pl.t2scale_off));
  return hipGetLastError();
}

// Resident LDS bytes of the slot loop's weights for a precision.
static int64_t resident_bytes(const PackedLayout &pl, int precision) {
  const int MT = pl.W / 16;
  if (precision == GN_FP8_T)
    return (((int64_t)MT * pl.chunk[C_T1A].ks * 512 + 1023) & ~(int64_t)1023) +
           (pl.t2scale_off - pl.t2q_off) + (pl.total_bytes - pl.t2scale_off);
  return pl.resident_bytes;
}

// order_bytes: the canonical order's LDS tables (order and alphas) per tile.
static size_t mfma_base_lds_bytes(const PackedLayout &pl, int precision, int order_bytes) {
  int64_t stage_max = 0;
  for (int s = 0; s < pl.nstages; ++s)
    stage_max = std::max<int64_t>(stage_max, pl.stage_off[s + 1] - pl.stage_off[s]);
  return (size_t)(resident_bytes(pl, precision) + (int64_t)kNumLayers * pl.W * 4 +
                  (int64_t)order_bytes + 2 * stage_max);
}

// Waves whose sigma fits in the LDS the weights leave free (160 KiB per CU),
// and how many of them sit in the stage buffers' tails: from F3's stage to
// B1S's (stages 1-4, shifted by two with encoded inputs) buffer 1 holds the
// first and third of them, buffer 0 the second and fourth.
static void mfma_sig_lds(const PackedLayout &pl, int precision, int order_bytes, int *nlds,
                         int *ntail) {
  constexpr size_t kLdsMax = 160 * 1024;
  const size_t per_wave = (size_t)kNT * (pl.W / 32) * kFrag;
  const size_t base = mfma_base_lds_bytes(pl, precision, order_bytes);
  int64_t stage_max = 0;
  for (int s = 0; s < pl.nstages; ++s)
    stage_max = std::max<int64_t>(stage_max, pl.stage_off[s + 1] - pl.stage_off[s]);
  const int sh = stage_shift(pl.pe);
  auto size = [&](int s) { return pl.stage_off[sh + s + 1] - pl.stage_off[sh + s]; };
  const int64_t tail1 = stage_max - std::max(size(1), size(3));
  const int64_t tail0 = stage_max - std::max(size(2), size(4));
  const int free_waves = base >= kLdsMax ? 0 : (int)((kLdsMax - base) / per_wave);
  int t = 0;
  // tails are used alternately (buffer 0, buffer 1, buffer 0, ...)
  for (int64_t used0 = 0, used1 = 0;; ++t) {
    int64_t &u = (t & 1) ? used1 : used0;
    const int64_t cap = (t & 1) ? tail1 : tail0;
    if (u + (int64_t)per_wave > cap) break;
    u += per_wave;
  }
  const int n = std::min(kWaves, free_waves + t);
  *ntail = std::max(0, n - free_waves);
  *nlds = n;
}

static int mfma_sig_free_waves(const PackedLayout &pl, int precision, int order_bytes) {
  int n, t;
  mfma_sig_lds(pl, precision, order_bytes, &n, &t);
  return n - t;
}

static size_t mfma_lds_bytes(const PackedLayout &pl, int precision, int order_bytes) {
  return mfma_base_lds_bytes(pl, precision, order_bytes) +
         (size_t)mfma_sig_free_waves(pl, precision, order_bytes) * kNT * (pl.W / 32) * kFrag;
}

template <int W, int PREC, int MODE, int PE>
static hipError_t launch_one(const MfmaArgs &a, int grid, size_t lds, hipStream_t stream) {
  // The attribute is per function; a layout of a different size (another
  // handle's) raises it again.
  static size_t attr_lds = 0;
  if (lds > attr_lds) {
    hipError_t e = hipFuncSetAttribute((const void *)fwd_mfma_kernel<W, PREC, MODE, PE>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_lds = lds;
  }
  hipLaunchKernelGGL((fwd_mfma_kernel<W, PREC, MODE, PE>), dim3(grid), dim3(kThreads), lds, stream,
                     a);
  return hipGetLastError();
}

template <int W, int PREC, int PE>
static hipError_t launch_mode(int mode, const MfmaArgs &a, int grid, size_t lds,
                              hipStream_t stream) {
  switch (mode) {
    case FWD_FULL: return launch_one<W, PREC, FWD_FULL, PE>(a, grid, lds, stream);
    case FWD_BEGIN: return launch_one<W, PREC, FWD_BEGIN, PE>(a, grid, lds, stream);
    case FWD_ACC: return launch_one<W, PREC, FWD_ACC, PE>(a, grid, lds, stream);
    case FWD_FINISH: return launch_one<W, PREC, FWD_FINISH, PE>(a, grid, lds, stream);
  }
  return hipErrorInvalidValue;
}

template <int W, int PREC>
static hipError_t launch_pe(int pe, int mode, const MfmaArgs &a, int grid, size_t lds,
                            hipStream_t stream) {
  switch (pe) {
    case 0: return launch_mode<W, PREC, 0>(mode, a, grid, lds, stream);
    case 1: return launch_mode<W, PREC, 1>(mode, a, grid, lds, stream);
    case 2: return launch_mode<W, PREC, 2>(mode, a, grid, lds, stream);
    case 3: return launch_mode<W, PREC, 3>(mode, a, grid, lds, stream);
    case 4: return launch_mode<W, PREC, 4>(mode, a, grid, lds, stream);
  }
  return hipErrorInvalidValue;
}
static_assert(kMaxPe == 4, "launch_pe covers encoding levels 0..4");

size_t stream_state_tile_bytes(int W) {
  return W == 64 ? (size_t)StreamTile<64>::kBytes : (size_t)StreamTile<128>::kBytes;
}

static hipError_t launch_impl(int W, int precision, int pool, const uint8_t *packed,
                              const PackedLayout &pl, const FwdBatch *batch,
                              const FrameDesc *frames, const TileRef *tiles, int ntiles,
                              float fp8_act_scale, int grid, uint8_t *sig_scratch, int mode,
                              uint8_t *state, int state_load, int slot_kmax,
                              hipStream_t stream) {
  MfmaArgs a;
  a.sig_scratch = sig_scratch;
  a.state = state;
  a.state_load = state_load;
  // canonical order: a table of slot_kmax bytes per pixel, rounded up to 4
  a.canon = slot_kmax > 1 ? 1 : 0;
  a.kpad = a.canon ? (slot_kmax + 3) / 4 * 4 : 0;
  a.aslots = a.canon ? std::min(slot_kmax, 8) : 0;
  // the alpha table goes into sigma's parking area when that area holds it,
  // else into LDS of its own
  int order_bytes = kTilePx * a.kpad;
  mfma_sig_lds(pl, precision, order_bytes, &a.sig_lds_waves, &a.sig_tail_waves);
  const int alpha_bytes = kTilePx * 4 * a.aslots;
  a.alpha_alias = (a.sig_lds_waves - a.sig_tail_waves) * kNT * (W / 32) * kFrag >= alpha_bytes;
  if (!a.alpha_alias) {
    order_bytes += alpha_bytes;
    mfma_sig_lds(pl, precision, order_bytes, &a.sig_lds_waves, &a.sig_tail_waves);
  }
  a.packed = packed;
  for (int s = 0; s <= kMaxStages; ++s) a.stage_off[s] = s <= pl.nstages ? pl.stage_off[s] : 0;
  a.res_off = pl.resident_off;
  a.res_bytes = resident_bytes(pl, precision);
  a.bias_off = pl.bias_off;
  a.t2q_off = pl.t2q_off;
  a.t2s_off = pl.t2scale_off;
  if (batch) {
    a.b = *batch;
    a.tiles_per_frame = (batch->hw + kTilePx - 1) / kTilePx;
  } else {
    a.b = FwdBatch{};
    a.tiles_per_frame = 1;
  }
  a.frames = frames;
  a.tiles = tiles;
  a.ntiles = ntiles;
  a.pool = pool;
  a.sa = fp8_act_scale;
  a.inv_sa = 1.0f / fp8_act_scale;
  if (ntiles <= 0) return hipSuccess;
  grid = std::max(1, std::min(grid, ntiles));   // the scratch holds `grid` workgroups
  const size_t lds = mfma_lds_bytes(pl, precision, order_bytes);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (precision == GN_BF16) {
    if (W == 64) return launch_pe<64, GN_BF16>(pl.pe, mode, a, grid, lds, stream);
    if (W == 128) return launch_pe<128, GN_BF16>(pl.pe, mode, a, grid, lds, stream);
  }
  if (precision == GN_FP8_T && W == 128)
    return launch_pe<128, GN_FP8_T>(pl.pe, mode, a, grid, lds, stream);
  return hipErrorInvalidValue;
}

hipError_t launch_fwd_mfma(int W, int precision, int pool, const uint8_t *packed,
                           const PackedLayout &pl, const FwdBatch *batch,
                           const FrameDesc *frames, const TileRef *tiles, int ntiles,
                           float fp8_act_scale, int grid, uint8_t *sig_scratch,
                           int slot_kmax, hipStream_t stream) {
  return launch_impl(W, precision, pool, packed, pl, batch, frames, tiles, ntiles, fp8_act_scale,
                     grid, sig_scratch, FWD_FULL, nullptr, 0, slot_kmax, stream);
}

hipError_t launch_fwd_stream(int W, int precision, int pool, const uint8_t *packed,
                             const PackedLayout &pl, const FwdBatch &batch, float fp8_act_scale,
                             int grid, int mode, uint8_t *state, int state_load,
                             hipStream_t stream) {
  if (mode == FWD_FULL || !state) return hipErrorInvalidValue;
  const int tpf = (batch.hw + kTilePx - 1) / kTilePx;
  return launch_impl(W, precision, pool, packed, pl, &batch, nullptr, nullptr, batch.n * tpf,
                     fp8_act_scale, grid, nullptr, mode, state, state_load, 0, stream);
}

}  // namespace gn
