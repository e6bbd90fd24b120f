// Host-side layout tables: master weight offsets and the packed MFMA layout;
// the seeded weight initialisation; Adam's bias corrections.
#include <math.h>
#include <string.h>

#include "gn_internal.h"

namespace gn {

void layer_offsets(int W, int pe, LayerOff lo[kNumLayers]) {
  const int e = pe_blocks(pe);
  const int outs[kNumLayers] = {W, W, W, W, W, W, W, W, W, W, W, kNOUT};
  const int ins[kNumLayers] = {(kNG + kNS) * e, W, W, kNL * e + W, W, W, 2 * W, W, W, W + 3, W, W};
  int64_t off = 0;
  for (int l = 0; l < kNumLayers; ++l) {
    lo[l].w = off;
    off += (int64_t)outs[l] * ins[l];
    lo[l].b = off;
    off += outs[l];
    lo[l].out = outs[l];
    lo[l].in = ins[l];
  }
}

size_t num_params(int W, int pe) {
  if (W != 64 && W != 128) return 0;
  if (pe < 0 || pe > kMaxPe) return 0;
  return (size_t)11 * W * W + (size_t)59 * W + 3 + (size_t)84 * pe * W;
}

// SplitMix64's output function (Steele, Lea and Flood, OOPSLA 2014): a
// bijective mix of a 64-bit counter, arithmetic modulo 2^64.
static inline uint64_t splitmix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void seeded_weights(int W, int pe, uint64_t seed, float *w) {
  LayerOff lo[kNumLayers];
  layer_offsets(W, pe, lo);
  for (int l = 0; l < kNumLayers; ++l) {
    // He et al.'s uniform bound for ReLU layers on the matrix, 1/sqrt(fan_in)
    // on the bias
    const double wb = sqrt(6.0 / lo[l].in), bb = 1.0 / sqrt((double)lo[l].in);
    const int64_t nw = (int64_t)lo[l].out * lo[l].in;
    for (int64_t e = lo[l].w; e < lo[l].b + lo[l].out; ++e) {
      const uint64_t x = splitmix64(seed + (uint64_t)(e + 1) * 0x9E3779B97F4A7C15ull);
      const double u = (double)(x >> 11) * 0x1.0p-53;
      w[e] = (float)((2.0 * u - 1.0) * (e < lo[l].w + nw ? wb : bb));
    }
  }
}

void adam_bias_corrections(float b1, float b2, int step, float *c1, float *c2) {
  *c1 = (float)(1.0 / (1.0 - pow((double)b1, (double)step)));
  *c2 = (float)(1.0 / (1.0 - pow((double)b2, (double)step)));
}

void make_packed_layout(int W, int pe, PackedLayout *pl) {
  memset(pl, 0, sizeof(*pl));
  pl->W = W;
  pl->pe = pe;
  const int MT = W / 16, KS = W / 32, E = pe_blocks(pe), NK16 = pe_k16_steps(pe);
  auto set = [&](Chunk c, int layer, int col0, int ncols, int nrows, int mt, int ks, int kmap) {
    ChunkDesc &d = pl->chunk[c];
    d.layer = layer;
    d.col0 = col0;
    d.ncols = ncols;
    d.nrows = nrows;
    d.mt = mt;
    d.ks = ks;
    d.kmap = kmap;
    d.elem_bytes = 2;
    d.nblocks = E;
  };
  // F1: one 32-deep K-step per encoding block; with encoded inputs its blocks
  // are split over two stages (the first ceil(E / 2) blocks, then the rest)
  const int f1a = pe > 0 ? (E + 1) / 2 : 1;
  set(C_F1, L_F1, 0, (kNG + kNS) * E, W, MT, f1a, KMAP_ENC);
  pl->chunk[C_F1].raw = kNG + kNS;
  set(C_F1B, L_F1, 0, (kNG + kNS) * E, W, pe > 0 ? MT : 0, E - f1a, KMAP_ENC);
  pl->chunk[C_F1B].raw = kNG + kNS;
  pl->chunk[C_F1B].ks0 = f1a;
  set(C_F2, L_F2, 0, W, W, MT, KS, KMAP_CHAIN);
  set(C_F3, L_F3, 0, W, W, MT, KS, KMAP_CHAIN);
  set(C_T1S, L_T1, kNL * E, W, W, MT, KS, KMAP_CHAIN);
  set(C_T3, L_T3, 0, W, W, MT, KS, KMAP_CHAIN);
  set(C_B1S, L_B1, 0, W, W, MT, KS, KMAP_CHAIN);
  set(C_B1T, L_B1, W, W, W, MT, KS, KMAP_CHAIN);
  set(C_B2, L_B2, 0, W, W, MT, KS, KMAP_CHAIN);
  set(C_B3, L_B3, 0, W, W, MT, KS, KMAP_CHAIN);
  set(C_R1P, L_R1, 0, W, W, MT, KS, KMAP_CHAIN);
  set(C_R1L, L_R1, W, 3, W, MT, 1, KMAP_MEM);
  set(C_R2, L_R2, 0, W, W, MT, KS, KMAP_CHAIN);
  set(C_R3, L_R3, 0, W, kNOUT, 1, KS, KMAP_CHAIN);
  if (pe > 0) {
    set(C_T1A, L_T1, 0, kNL * E, W, MT, NK16, KMAP_PE16);
    pl->chunk[C_T1A].raw = kNL;
  } else {
    set(C_T1A, L_T1, 0, kNL, W, MT, 1, KMAP_MEM16);
  }
  set(C_T2, L_T2, 0, W, W, MT, KS, KMAP_CHAIN);

  // Stage groups in kernel order; every fragment is 1 KiB so stages stay
  // multiples of 1 KiB.
  const Chunk none = kNumChunks;
  const Chunk plain[kNumStages][2] = {
      {C_F1, C_F2}, {C_F3, none}, {C_T1S, none}, {C_T3, none},
      {C_B1S, none}, {C_B1T, none}, {C_B2, none}, {C_B3, none},
      {C_R1P, C_R1L}, {C_R2, C_R3}};
  const Chunk encoded[kMaxStages][2] = {
      {C_F1, none}, {C_F1B, none}, {C_F2, none}, {C_F3, none}, {C_T1S, none}, {C_T3, none},
      {C_B1S, none}, {C_B1T, none}, {C_B2, none}, {C_B3, none},
      {C_R1P, C_R1L}, {C_R2, C_R3}};
  pl->nstages = kNumStages + stage_shift(pe);
  int64_t off = 0;
  for (int s = 0; s < pl->nstages; ++s) {
    pl->stage_off[s] = off;
    for (int j = 0; j < 2; ++j) {
      Chunk c = pe > 0 ? encoded[s][j] : plain[s][j];
      if (c == none) continue;
      pl->chunk[c].offset = off;
      off += (int64_t)pl->chunk[c].mt * pl->chunk[c].ks * 1024;
    }
  }
  pl->stage_off[pl->nstages] = off;
  pl->resident_off = off;
  pl->chunk[C_T1A].offset = off;
  off += ((int64_t)MT * pl->chunk[C_T1A].ks * 512 + 1023) & ~(int64_t)1023;   // K=16: 512 B each
  pl->chunk[C_T2].offset = off;
  off += (int64_t)MT * KS * 1024;
  pl->resident_bytes = off - pl->resident_off;
  pl->bias_off = off;
  off += (int64_t)kNumLayers * W * 4;
  off = (off + 1023) & ~(int64_t)1023;
  pl->t2q_off = off;                       // fp8 T2: MT fragments of 64 lanes x 32 B
  off += (int64_t)MT * 2048;
  pl->t2scale_off = off;                   // fp32 per-row scales, padded to 1 KiB
  off += ((int64_t)W * 4 + 1023) & ~(int64_t)1023;
  pl->total_bytes = off;
}

}  // namespace gn
