// Internal declarations shared by the GlassNet library sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "glassnet.h"

namespace gn {

constexpr int kNG = GN_NUM_G, kNL = GN_NUM_L, kNS = GN_NUM_S, kNOUT = GN_NUM_OUT;
constexpr int kAlpha = GN_ALPHA_PLANE;
constexpr int kMaxPe = GN_MAX_PE_LEVELS;

// Positional encoding (Sec. 3.4): an input vector x of C channels becomes
// (1 + 2 L) blocks of C: x, then sin(2^k pi x) and cos(2^k pi x) for
// k = 0 .. L-1.  It widens F's input (30 channels) and h's slot input (12).
constexpr int pe_blocks(int pe) { return 1 + 2 * pe; }
// h's slot input in 16-deep K-steps of the fused kernel: lane group g owns
// raw channels 3g .. 3g+2 and presents their encodings in block order.
constexpr int pe_k16_steps(int pe) { return (3 * pe_blocks(pe) + 3) / 4; }

// One frame as the kernels see it: pointers already offset to the frame.
struct FrameDesc {
  const float *g;    // [14][hw]
  const float *L;    // [k][12][hw]
  const float *s;    // [16]
  float *out;        // [3][hw]
  int32_t hw;
  int32_t k;
  int32_t pad0, pad1;
};

// A tile of the fused MFMA kernel: kTilePx pixels of one frame from q0.
struct TileRef {
  int32_t frame;     // index into a FrameDesc table
  int32_t q0;
};

// The 12 linear layers in the flat master vector.
enum Layer { L_F1, L_F2, L_F3, L_T1, L_T2, L_T3, L_B1, L_B2, L_B3, L_R1, L_R2, L_R3, kNumLayers };

struct LayerOff {
  int64_t w, b;      // float offsets of matrix and bias
  int32_t out, in;
};

void layer_offsets(int W, int pe, LayerOff lo[kNumLayers]);
size_t num_params(int W, int pe);
// The seeded initialisation of glassnet_create (host): num_params(W, pe)
// floats.
void seeded_weights(int W, int pe, uint64_t seed, float *w);

// ---- packed (fragment-ordered) weights of the MFMA forward -----------------
// A chunk is the part of one layer's matrix that multiplies one input source.
// It is stored as MT x KS fragments of 64 lanes x 16 bytes: lane l of fragment
// (mt, ks) holds row 16*mt + (l & 15) and the 8 inputs of K-step ks that lane
// group l >> 4 presents to the matrix core.  Inputs that come straight from
// memory use the natural order (8 consecutive channels per lane group);
// inputs produced by a previous layer use the order in which that layer's
// accumulator rows sit in the lanes, so activations chain from one layer to
// the next without leaving registers.
enum Chunk {
  C_F1, C_F2, C_F3, C_T1S, C_T3, C_B1S, C_B1T, C_B2, C_B3, C_R1P, C_R1L, C_R2, C_R3,
  C_T1A, C_T2,            // resident in LDS through the slot loop
  C_F1B,                  // encoded inputs: F1's second half of K-steps (empty otherwise)
  kNumChunks
};
// KMAP_MEM16: a 16-deep K-step of v_mfma_f32_16x16x16bf16_1k, lane group g
// holding inputs 4g..4g+3 (fragments of 64 lanes x 8 bytes).
// KMAP_ENC: 32-deep K-step ks0 + ks is encoding block ks0 + ks of the raw
// inputs, lane group g holding raw channels 8g..8g+7 of that block.
// KMAP_PE16: 16-deep K-steps of the encoded slot input (pe_k16_steps):
// element j of lane group g in K-step s is value v = 4s + j of the group's
// list (block v / 3, raw channel 3g + v % 3).
enum KMap { KMAP_CHAIN = 0, KMAP_MEM = 1, KMAP_MEM16 = 2, KMAP_ENC = 3, KMAP_PE16 = 4 };

struct ChunkDesc {
  int32_t layer;     // Layer
  int32_t col0;      // first input column of the master layer this chunk covers
  int32_t ncols;     // real input columns (K padded to 32*ks)
  int32_t nrows;     // real output rows (M padded to 16*mt)
  int32_t mt, ks;
  int32_t kmap;
  int32_t elem_bytes;  // 2 (bf16) or 1 (fp8)
  int32_t raw;         // KMAP_ENC / KMAP_PE16: raw channels per encoding block
  int32_t ks0;         // KMAP_ENC: encoding block of the chunk's first K-step
  int32_t nblocks;     // KMAP_ENC / KMAP_PE16: encoding blocks (1 + 2 L)
  int32_t pad;
  int64_t offset;      // byte offset in the packed buffer
};

// Ten stages; with encoded inputs F1 takes two stages of its own before F2's
// (an even number, so every later stage keeps its buffer parity).
constexpr int kNumStages = 10;
constexpr int kMaxStages = 12;
constexpr int stage_shift(int pe) { return pe > 0 ? 2 : 0; }

struct PackedLayout {
  int W, pe;
  int nstages;
  ChunkDesc chunk[kNumChunks];
  int64_t stage_off[kMaxStages + 1];   // byte ranges of the staged chunks
  int64_t resident_off, resident_bytes;  // T1A + T2 (bf16)
  int64_t bias_off;                    // fp32 biases: 12 x W floats
  int64_t t2q_off;                     // fp8 copy of T2 (FP8_T), MT x 1 fragments of 64 x 32 B
  int64_t t2scale_off;                 // fp32 per-row dequant scales of the fp8 T2 (W floats)
  int64_t total_bytes;
};

void make_packed_layout(int W, int pe, PackedLayout *pl);

// ---- launches (all asynchronous on `stream`) --------------------------------
struct BwdWorkspace;
struct FwdBatch {
  // Arithmetic mode: n frames of equal hw/k laid out as in gn_frame.
  const float *gbuf, *layers, *scene;
  float *out;
  int32_t n, hw, k;
};

hipError_t launch_pack_weights(const float *master, uint8_t *packed, const PackedLayout &pl,
                               float fp8_act_scale, hipStream_t stream);


// sig_scratch: mfma_sig_scratch_bytes(W, grid) bytes private to this launch
// (launches that may overlap need different scratch buffers).  slot_kmax > 1:
// every pixel's slots are pooled in canonical order (slot_order.h), for
// frames of up to slot_kmax slots; 0: in input order.
hipError_t launch_fwd_mfma(int W, int precision, int pool, const uint8_t *packed,
                           const PackedLayout &pl, const FwdBatch *batch,
                           const FrameDesc *frames, const TileRef *tiles, int ntiles,
                           float fp8_act_scale, int grid, uint8_t *sig_scratch,
                           int slot_kmax, hipStream_t stream);
size_t mfma_sig_scratch_bytes(int W, int grid);
constexpr int kTilePx = 256;

// Object streaming: the parts of the fused forward one launch runs.  BEGIN
// evaluates F and stores sigma in the state; ACC runs the slot loop over the
// batch's k slots, continuing the state's running sum when state_load is 1
// (starting from zero otherwise); FINISH pools and runs T3, B and R from the
// state (an empty pool when state_load is 0) and writes batch.out.  The state
// holds stream_state_tile_bytes(W) bytes per tile of kTilePx pixels of each
// frame (n x ceil(hw / kTilePx) tiles).
enum FwdMode { FWD_FULL = 0, FWD_BEGIN = 1, FWD_ACC = 2, FWD_FINISH = 3 };
size_t stream_state_tile_bytes(int W);
hipError_t launch_fwd_stream(int W, int precision, int pool, const uint8_t *packed,
                             const PackedLayout &pl, const FwdBatch &batch, float fp8_act_scale,
                             int grid, int mode, uint8_t *state, int state_load,
                             hipStream_t stream);

// L1 term; grad (optional) = sign(out - target) / count x *grad_scale (a
// device scalar; null: 1).
hipError_t launch_l1(const float *out, const float *target, uint64_t count, float *loss,
                     float *grad, const float *grad_scale, float *partials, int npart,
                     hipStream_t stream);
// DSSIM term: planes = n x 3 images of h x w (h, w >= 11); ws holds
// dssim_workspace_bytes(planes, h, w) bytes; grad may be null.
size_t dssim_workspace_bytes(int planes, int h, int w);
// The allocation-free DSSIM form's fixed per-device workspace: its size, the
// set-up of its device address (once per device, that device current) and
// the address (null before set-up).
constexpr size_t kDssimScratchBytes = (size_t)16 << 20;
constexpr int kMaxDevices = 64;
hipError_t dssim_scratch_init(int device);
float *dssim_scratch(int device);
hipError_t launch_dssim(const float *out, const float *target, int planes, int h, int w,
                        float *loss, float *grad, int accumulate, float *ws, hipStream_t stream);
// x2 super-sampling network: widths and the packed parameter count.
constexpr int kSrWidth = 32, kSrIn = 3 + 14, kSrOut = 3;
constexpr int kSrParams = kSrWidth * kSrIn * 9 + kSrWidth + kSrWidth * kSrWidth * 9 + kSrWidth +
                          kSrOut * kSrWidth + kSrOut;
// Floats of the kernel's re-laid weight copy (conv1's K padded to 20 input
// channels per tap).
constexpr int kSrWtFloats = (9 * 20 / 4) * 2 * 64 + kSrWidth + (9 * kSrWidth / 4) * 2 * 64 +
                            kSrWidth + kSrOut * kSrWidth + kSrOut +
                            (9 * kSrWidth / 4) * 2 * 64;  // + conv2's transpose (backward)
// w: packed weights (device, kSrParams floats); wt: kSrWtFloats floats of
// device scratch for their re-laid copy; lowres [n][3][h][w], gbuf
// [n][14][2h][2w], out [n][3][2h][2w].
hipError_t launch_sr_forward(const float *w, float *wt, const float *lowres, const float *gbuf,
                             float *out, int n, int h, int w_lo, hipStream_t stream);
// Its weight gradient for dy = dL/d(out): grad_w (kSrParams floats)
// overwritten; ws holds sr_backward_workspace_bytes(n, h, w) bytes.
size_t sr_backward_workspace_bytes(int n, int h, int w);
hipError_t launch_sr_backward(const float *w, float *wt, const float *lowres, const float *gbuf,
                              const float *dy, float *gw, int n, int h, int w_lo, float *ws,
                              hipStream_t stream);
// Spatial networks (spatial.hip): parameter count, bytes of the packed
// weights and of one call's activations, the packing (from a device fp32
// master vector) and the forward (bf16 matrix cores, fp32 accumulation).
size_t spatial_num_params(int W);
size_t spatial_weight_bytes(int W);
size_t spatial_workspace_bytes(int W, int n, int H, int Wd, int k);
hipError_t spatial_pack(const float *master, int W, uint8_t *packed, hipStream_t s);
hipError_t spatial_forward(const uint8_t *packed, int W, int pool, const float *gbuf,
                           const float *layers, const float *scene, int n, int H, int Wd, int k,
                           float *out, uint8_t *ws, hipStream_t s);
// One Adam step on w (n floats) from gradient g, moments m and v, with the
// bias corrections c1 = 1 / (1 - b1^t) and c2 = 1 / (1 - b2^t) of step t.
hipError_t launch_adam(float *w, const float *g, float *m, float *v, int64_t n, float c1, float c2,
                       float lr, float b1, float b2, float eps, float wd, hipStream_t stream);
// Adam's bias corrections for step t >= 1 (host).
void adam_bias_corrections(float b1, float b2, int step, float *c1, float *c2);


}  // namespace gn
