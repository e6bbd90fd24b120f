/*
 * glassnet.h -- C ABI of the GlassNet per-pixel evaluator for MI355X (gfx950).
 *
 * The method (Zhang & Simo-Serra, "Neural Scene Baking for Permutation
 * Invariant Transparency Rendering with Real-time Global Illumination"):
 *   Sec. 3.2   a separated opaque G-buffer plus one transparency buffer per
 *              transparent object, w x h x c*(t+1) planes in total;
 *   Sec. 3.3   Eq. (5): tau = sum_i h(b_i, sigma), one network h shared by all
 *              transparency buffers followed by a symmetric pool;
 *   Sec. 3.4   scene encoder F -> sigma, blend network B([sigma; tau]) -> phi,
 *              rendering network R([phi; L_d]) -> output radiance;
 *   Sec. 3.5   end-to-end training with an L1 term.
 * Every network is a per-pixel 3-layer MLP (Linear-ReLU-Linear-ReLU-Linear) of
 * hidden width W; a transparency slot takes part iff its alpha > 0.
 *
 * Conventions shared by every call
 *   - Plain C types only.  Pointers documented "device" are HIP device
 *     allocations owned by the caller; "host" pointers are ordinary memory.
 *   - Every call returns a gn_status; nothing throws across the ABI.  On
 *     failure glassnet_last_error() gives a message for the calling thread.
 *   - Compute calls are asynchronous and stream-ordered on the hip_stream the
 *     caller passes (a hipStream_t; NULL = the null stream).  Device buffers
 *     must stay valid until that stream work has completed.
 *   - A handle's forward/backward/l1/set_weights calls are used by one host
 *     thread at a time; serve_submit/serve_poll may be called concurrently.
 *   - An asynchronous device fault observed by the library poisons the handle:
 *     every later call returns GN_E_DEVICE.
 */
#ifndef GLASSNET_H
#define GLASSNET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Planes per pixel (fp32).  G-buffer: position(3), unit normal(3), albedo(3),
 * roughness, metallic, direct light L_d(3) -- L_d are planes 11..13.
 * Transparency layer: position(3), unit normal(3), tint(3), alpha (plane 9),
 * IOR, depth.  Scene vector: 16 variable scene parameters per frame. */
#define GN_NUM_G 14
#define GN_NUM_L 12
#define GN_NUM_S 16
#define GN_NUM_OUT 3
#define GN_ALPHA_PLANE 9
#define GN_MAX_K 64
#define GN_MAX_PE_LEVELS 4

typedef int32_t gn_status;
#define GN_OK 0
#define GN_E_INVAL (-1)        /* bad argument: shape, pointer, alignment, size */
#define GN_E_NOMEM (-2)        /* device or host allocation failed */
#define GN_E_DEVICE (-3)       /* HIP runtime or kernel error; handle poisoned */
#define GN_E_UNSUPPORTED (-4)  /* valid request the library does not implement */
#define GN_E_AGAIN (-5)        /* serving: result not ready yet */
#define GN_E_BUSY (-6)         /* serving: pending queue full */

/* Arithmetic of the forward pass.
 *   GN_FP32    fp32 weights and activations on the fp32 matrix cores, layer by
 *              layer through a workspace of fp32 planes (about 14.5 KB per
 *              pixel at W = 128, kept by the handle and shared with the
 *              backward: FP32 forward and backward calls on different
 *              streams must be ordered by the caller).
 *   GN_BF16    bf16 weights/activations on MFMA, fp32 accumulation, fp32 pool.
 *   GN_FP8_T   the per-slot hidden layer of h in FP8-E4M3 (per-output-channel
 *              fp32 weight scales, static activation scale), the rest as GN_BF16.
 *   GN_FP8_ALL every layer in FP8-E4M3.  Not built: glassnet_create returns
 *              GN_E_UNSUPPORTED.  Emulated with the same scales on the 512^2,
 *              K = 8 input distribution its error against the exact forward
 *              is about 8e-2 (relative Frobenius), above the 6e-2 an FP8 form
 *              is held to; GN_FP8_T's is about 1.5e-2 to 3.5e-2.
 * Backward and loss always accumulate in fp32. */
typedef int32_t gn_precision;
#define GN_FP32 0
#define GN_BF16 1
#define GN_FP8_T 2
#define GN_FP8_ALL 3

/* The symmetric function g of Eq. (5).
 *   GN_POOL_SUM   tau = sum over active slots of h(b_i, sigma)   (Eq. (5))
 *   GN_POOL_MEAN  tau = that sum / max(#active, 1); no active slot gives 0. */
typedef int32_t gn_pool;
#define GN_POOL_MEAN 0
#define GN_POOL_SUM 1

/* The order in which a pixel's slots are added into the pool of Eq. (5).
 * The pool is a symmetric function, so the method's result does not depend
 * on the order of the transparency buffers (Sec. 3.3; Sec. 4.3's order-
 * inversion table); a floating-point sum does, by its rounding.
 *   GN_ORDER_CANONICAL  every forward path (GN_FP32, GN_BF16, GN_FP8_T, the
 *                       backward's recompute and serving) adds each pixel's
 *                       slots in one order fixed by their records: active
 *                       slots (alpha > 0) by the bits of alpha as an unsigned
 *                       integer, equal alphas by the bit patterns of planes
 *                       0..11 in turn, equal records by index; then inactive
 *                       slots by index.  The output is then bitwise the same
 *                       under any permutation of a pixel's slots.
 *   GN_ORDER_INPUT      slot 0, 1, ..., k - 1 (object streaming always adds
 *                       objects in call order). */
typedef int32_t gn_slot_order;
#define GN_ORDER_CANONICAL 0
#define GN_ORDER_INPUT 1

typedef struct gn_config {
  int32_t width;              /* W: 64 or 128 */
  int32_t k_max;              /* largest slot count a call may pass, 0..GN_MAX_K */
  gn_pool pool;
  gn_precision precision;
  uint64_t hbm_budget_bytes;  /* serving admission budget; 0 = 64 GiB */
  int32_t device;             /* HIP device ordinal */
  int32_t max_pending;        /* serving: pending-queue bound; 0 = 65536 */
  int32_t pe_levels;          /* positional encoding levels L, 0..GN_MAX_PE_LEVELS
                                 (Sec. 3.4 encodes every network input).  With
                                 L > 0, F's input [G; s] (30 channels) and h's
                                 slot input b_i (12) each become 1 + 2 L blocks
                                 of their channels: x, then sin(2^k pi x) and
                                 cos(2^k pi x) for k = 0 .. L-1.  sigma, R's
                                 L_d and the alpha mask stay raw.  0 = none. */
  gn_slot_order slot_order;   /* GN_ORDER_CANONICAL (0, the default) or GN_ORDER_INPUT */
  uint64_t seed;              /* glassnet_create with host_weights == NULL: the
                                 weights are drawn from this seed (see there) */
} gn_config;

typedef struct gn_handle gn_handle;

/* A batch of n frames of h x w pixels with k transparency slots each.  All
 * three arrays are device memory, fp32, C-contiguous, 4-byte aligned:
 *   gbuf   [n][GN_NUM_G][h][w]
 *   layers [n][k][GN_NUM_L][h][w]   (may be NULL when k == 0)
 *   scene  [n][GN_NUM_S]                                                  */
typedef struct gn_frame {
  int32_t n, h, w, k;
  const float *gbuf;
  const float *layers;
  const float *scene;
} gn_frame;

/* Serving timestamps, seconds on the host's steady clock. */
typedef struct gn_timing {
  double t_submit, t_admit, t_start, t_done;
} gn_timing;

/* Number of fp32 parameters for width W and L positional-encoding levels:
 * 11 W^2 + 59 W + 3 + 84 L W.
 * Flat layout: nets F, T, B, R; layers 1, 2, 3; per layer the matrix row-major
 * [out][in] then the bias.  Input order: F [G-buffer 0..13; scene 0..15],
 * T [slot planes 0..11; sigma], B [sigma; tau], R [phi; L_d]; with L > 0 F's
 * columns are the 1 + 2 L encoding blocks of [G; scene] in block order (raw,
 * sin level 0, cos level 0, sin level 1, ...) and T's the blocks of the slot
 * planes, then sigma.  Returns 0 for an unsupported width or level count. */
size_t glassnet_num_params(int32_t width, int32_t pe_levels);

/* Create a handle on cfg->device and upload host_weights (host, n floats,
 * n == glassnet_num_params(width, pe_levels)).  The library owns the fp32
 * master copy, its bf16/fp8 packed forms and every workspace.  *out is set on
 * GN_OK.  GN_E_UNSUPPORTED for a width other than 64 or 128, GN_FP8_ALL,
 * GN_FP8_T at width 64, or pe_levels outside 0..GN_MAX_PE_LEVELS; GN_E_INVAL for other bad
 * fields or a wrong n; GN_E_DEVICE / GN_E_NOMEM from the device.
 *
 * Seeded initialisation: with host_weights == NULL (and n == 0 or the
 * parameter count) the weights are drawn from cfg->seed, He et al.'s uniform
 * initialisation for ReLU networks: every matrix entry of a layer with
 * fan_in inputs uniform in +-sqrt(6 / fan_in), every bias uniform in
 * +-1 / sqrt(fan_in).  Element e of the flat layout (0-based) uses
 * u_e = (SplitMix64(seed + (e + 1) * 0x9E3779B97F4A7C15) >> 11) * 2^-53 in
 * [0, 1) (Steele, Lea and Flood's SplitMix64 finaliser, computed modulo
 * 2^64) and the value (2 u_e - 1) * bound, rounded to fp32.
 * glassnet_get_weights reads the result back. */
gn_status glassnet_create(const gn_config *cfg, const float *host_weights, size_t n,
                          gn_handle **out);

/* Drain outstanding serving work, free every library allocation.  NULL is a no-op. */
gn_status glassnet_destroy(gn_handle *h);

/* Copy the fp32 master weights to host memory (n floats).  Synchronous. */
gn_status glassnet_get_weights(gn_handle *h, float *host_weights, size_t n);

/* Replace the master weights from DEVICE memory (n floats) and re-derive the
 * packed forms, stream-ordered on hip_stream (used by training loops). */
gn_status glassnet_set_weights(gn_handle *h, const float *dev_weights, size_t n,
                               void *hip_stream);

/* GN_FP8_T: static activation scale of the FP8 layer's input (the per-slot
 * hidden activation of h).  scales[0] > 0 maps the activation range onto
 * E4M3; n must be 1.  The default is derived at create time. */
gn_status glassnet_set_act_scales(gn_handle *h, const float *scales, size_t n);

/* GN_FP8_T calibration: evaluates h's first layer in fp32 over every slot of
 * every pixel of frame and sets the activation scale to (largest value)/448,
 * so the representative frame's range maps onto E4M3 without clipping.
 * Runs the fp32 plane pipeline of GN_FP32 (same workspace, same pixel limit).
 * Synchronous (waits for hip_stream). */
gn_status glassnet_calibrate(gn_handle *h, const gn_frame *frame, void *hip_stream);

/* Forward (Sec. 3.3-3.4): out [n][GN_NUM_OUT][h][w] fp32 device.
 * Requires 0 <= k <= k_max, n, h, w >= 1 and fewer than 2^32 floats of slot
 * planes per frame (k * GN_NUM_L * h * w); every call that takes a gn_frame
 * checks these.  Out must not alias inputs.  Each pixel's slots are pooled in
 * the handle's slot order (gn_config.slot_order).
 * GN_FP32: at most 3 * 2^20 pixels (n * h * w) per call (GN_E_INVAL beyond).
 * Forward calls of one handle share a small device scratch (GN_BF16 /
 * GN_FP8_T) or the plane workspace (GN_FP32): calls on different streams must
 * be ordered by the caller.  Serving has its own. */
gn_status glassnet_forward(gn_handle *h, const gn_frame *frame, float *out, void *hip_stream);

/* Backward of the forward above with respect to the weights (Sec. 3.5), fp32.
 * grad_out is dL/d(out), device, shaped like out.  grad_w (device, n_params
 * floats) is overwritten with dL/dw in the flat layout.  Per-slot activations
 * of h are recomputed, never stored for all k.  The transparency mask is a
 * hard selection: no gradient flows through alpha's threshold.  At most
 * 3 * 2^20 pixels (n * h * w) per call (GN_E_INVAL beyond).  The library keeps
 * a workspace of about 14.5 KB per pixel (W = 128) between calls. */
gn_status glassnet_backward(gn_handle *h, const gn_frame *frame, const float *grad_out,
                            float *grad_w, void *hip_stream);

/* Structural-dissimilarity term of the loss (Sec. 3.5 trains with SSIM and L1;
 * DSSIM = (1 - SSIM) / 2).  SSIM as Wang et al. define it: an 11 x 11
 * Gaussian window of sigma 1.5 over every fully contained window of each of
 * the 3 channels of each image, K1 = 0.01, K2 = 0.03, dynamic range 1.
 *   out, target  device [n][3][height][width] fp32 (height, width >= 11)
 *   loss         device scalar: (1 - mean SSIM over windows, channels and
 *                images) / 2
 *   grad_out     device, shaped like out, or NULL: d loss / d out, written
 *                (accumulate == 0) or added to its contents (accumulate != 0,
 *                e.g. after glassnet_l1_loss for the L1 + DSSIM loss).
 * The library keeps a workspace of about 12 bytes per pixel (grown on a
 * larger call, after the stream's earlier work).  GN_E_INVAL for smaller
 * images or aliasing buffers. */
gn_status glassnet_dssim_loss(gn_handle *h, const float *out, const float *target, int32_t n,
                              int32_t height, int32_t width, float *loss, float *grad_out,
                              int32_t accumulate, void *hip_stream);

/* glassnet_dssim_loss for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving or training loops, harnesses that
 * forbid hipMalloc.  Same arguments, kernels and result (bitwise); the
 * workspace is a fixed 16 MiB array of device memory that the library
 * holds on every GPU it runs on until the process ends, instead of the
 * handle's grown workspace.  The call allocates and frees nothing (no HIP or
 * other allocating routine) and synchronises nothing.  Every call on one GPU
 * shares that GPU's array: calls that may overlap on one GPU (different
 * streams, or handles on the same device used concurrently) race and must be
 * ordered by the caller.  Sizes whose workspace exceeds the array (more than
 * about 1.39 million SSIM windows: n x 3 x (height - 10) x (width - 10)) get
 * GN_E_INVAL; other errors as glassnet_dssim_loss. */
gn_status glassnet_dssim_loss_noalloc(gn_handle *h, const float *out, const float *target,
                                      int32_t n, int32_t height, int32_t width, float *loss,
                                      float *grad_out, int32_t accumulate, void *hip_stream);

/* One optimiser step on the handle's fp32 master weights (Sec. 4 trains with
 * Adam, Kingma & Ba, and weight decay), then the packed forms re-derived;
 * stream-ordered on hip_stream.  Weight decay is an L2 term added to the
 * gradient: g' = grad_w + weight_decay w, m = beta1 m + (1 - beta1) g',
 * v = beta2 v + (1 - beta2) g'^2, w -= lr m_hat / (sqrt(v_hat) + eps) with
 * m_hat = m / (1 - beta1^step), v_hat = v / (1 - beta2^step).
 *   grad_w  device, n = glassnet_num_params(...) floats (e.g. from
 *           glassnet_backward); read only.
 *   state   device, 2 n floats owned by the caller: m then v, zero before
 *           step 1, updated in place; one state per training run.
 *   step    1, 2, 3, ... (the bias corrections' t).
 * GN_E_INVAL for n other than the handle's parameter count, step < 1, lr or
 * weight_decay negative, beta outside [0, 1), eps <= 0, or overlapping
 * buffers.  An FP8_T handle keeps its activation scale. */
gn_status glassnet_adam_step(gn_handle *h, const float *grad_w, float *state, size_t n,
                             int32_t step, float lr, float beta1, float beta2, float eps,
                             float weight_decay, void *hip_stream);

/* x2 super-sampling network (Sec. 3.4 closes with a small multi-layer CNN
 * that doubles the resolution of GlassNet's render, helped by textures and
 * G-buffers the rasterizer produces cheaply at the higher resolution; Sec. 4.1
 * renders 256^2 and super-samples to 512^2).  The layers are a reading (the
 * paper gives none): input = the render upsampled x2 bilinearly (sample
 * centres at half-pixel offsets, sources clamped at the edges) followed by
 * the 14 full-resolution G-buffer planes; conv 3x3 17 -> 32 + ReLU, conv 3x3
 * 32 -> 32 + ReLU (both zero-padded, size kept), conv 1x1 32 -> 3; output =
 * upsampled render + that.  fp32 throughout.
 *   sr_w     device, glassnet_sr_num_params() floats: conv1 W [32][17][3][3]
 *            then b [32], conv2 W [32][32][3][3] then b [32], conv3 W [3][32]
 *            then b [3]; read only.
 *   height, width   the render's size; the output is 2 height x 2 width.
 *   lowres   device [n][3][height][width] (e.g. glassnet_forward's out).
 *   gbuf_hi  device [n][14][2 height][2 width], channels as in gn_frame.
 *   out      device [n][3][2 height][2 width]; must not overlap the inputs.
 * Independent of the handle's width and precision: the handle supplies the
 * device and a 97 KB copy of sr_w re-laid for the kernels (allocated on the
 * first call), which calls on different streams share: order them.
 * GN_E_INVAL for n outside 1..65535, height or width outside 1..2^18, NULL or
 * misaligned pointers, or out overlapping an input. */
size_t glassnet_sr_num_params(void);
gn_status glassnet_sr_forward(gn_handle *h, const float *sr_w, int32_t n, int32_t height,
                              int32_t width, const float *lowres, const float *gbuf_hi, float *out,
                              void *hip_stream);

/* The spatial networks (Sec. 3.4 names F and B U-Nets and h, R multi-layer
 * CNNs with 3 x 3 kernels before R's final 1 x 1 ones).  Architecture read
 * from that description (widths and depths are not given; W = the handle's
 * width):
 *   U-Net (F on [G; s], B on [sigma; tau]): e1 = relu(conv3 x);
 *     d = 2 x 2 average of e1; m = relu(conv3 d) at half resolution;
 *     e2 = relu(conv3 [e1; m repeated 2 x 2]); output = conv1 e2;
 *   h(b_i, sigma) = conv1 relu(conv1 relu(conv3 [b_i; sigma])), pooled per
 *     pixel over the buffers with alpha > 0 there (the handle's pool);
 *   R = conv1 relu(conv3 relu(conv3 [phi; L_d])), 3 outputs;
 * conv3: 3 x 3 correlation with zero padding of one pixel; conv1: 1 x 1;
 * every conv has a bias.  F's scene input is 16 constant planes.
 * glassnet_spatial_num_params(W): the flat fp32 parameter count (0 for a
 * width other than 64 or 128); layout: nets F (4 convs), T (3), B (4), R (3),
 * per conv W [out][in][kh][kw] row-major then b; input channel orders as the
 * concatenations above. */
size_t glassnet_spatial_num_params(int32_t width);

/* Spatial forward of a frame batch: sp_w (device, glassnet_spatial_num_params
 * floats, caller-owned) is re-laid into the handle's bf16 copy, then every
 * conv runs on the bf16 matrix cores with fp32 accumulation (whatever the
 * handle's precision), activations stored as bf16, the pool of Eq. (5) in
 * fp32 in buffer order.  frame as for glassnet_forward with even h and w and
 * at most 2^22 pixels per call; out [n][3][h][w] fp32 device.  A permutation
 * of the transparency buffers is a permutation of whole images (h sees a
 * buffer's neighbourhood).  The handle keeps the weight copy and a workspace
 * of about 3.5 KB per pixel at W = 128 (grown on a larger call, after the
 * stream's earlier work).  GN_E_INVAL for odd sizes, bad frames or aliasing
 * buffers. */
gn_status glassnet_spatial_forward(gn_handle *h, const float *sp_w, const gn_frame *frame,
                                   float *out, void *hip_stream);

/* Weight gradient of glassnet_sr_forward (Sec. 4.1 trains the super-sampling
 * network on its own), fp32: grad_out = dL/d(out) [n][3][2 height][2 width],
 * device; grad_w (device, glassnet_sr_num_params() floats, packed like sr_w)
 * is overwritten with dL/d(sr_w).  The forward is recomputed with the same
 * arithmetic as glassnet_sr_forward (so the ReLU masks are the ones behind
 * its output; the derivative of ReLU is 0 at 0), per-tile partial sums are
 * added in fp32 in a fixed order: the result is deterministic.  At most 2^22
 * output pixels per call (n 4 height width) and height, width <= 2^16
 * (GN_E_INVAL beyond, or for NULL, misaligned or aliasing pointers).  The
 * handle keeps a workspace of 512 bytes per output pixel plus at most 35 MB
 * (grown on a larger call, after the stream's earlier work). */
gn_status glassnet_sr_backward(gn_handle *h, const float *sr_w, int32_t n, int32_t height,
                               int32_t width, const float *lowres, const float *gbuf_hi,
                               const float *grad_out, float *grad_w, void *hip_stream);

/* The same Adam step on a caller-owned fp32 device vector w of n floats
 * (e.g. the super-sampling network's weights, trained apart from GlassNet in
 * Sec. 4.1), with the update rule of glassnet_adam_step; state is 2 n floats
 * (m then v, zero before step 1).  The handle supplies the device.  GN_E_INVAL
 * for n outside 1..2^31, step < 1, hyperparameters as in glassnet_adam_step,
 * or overlapping buffers. */
gn_status glassnet_adam_update(gn_handle *h, float *w, const float *grad_w, float *state,
                               size_t n, int32_t step, float lr, float beta1, float beta2,
                               float eps, float weight_decay, void *hip_stream);

/* L1 term of Sec. 3.5 over count elements: *loss = mean |out - target| and
 * grad_out = sign(out - target) / count (0 where equal), times *grad_scale
 * when grad_scale is not NULL (a device scalar, e.g. the upstream gradient of
 * an autograd graph; read on the device, no host synchronisation).  All
 * device.  grad_out may be NULL.  GN_E_INVAL for NULL out, target or loss,
 * misaligned pointers, or grad_out overlapping out, target or grad_scale. */
gn_status glassnet_l1_loss(gn_handle *h, const float *out, const float *target,
                           uint64_t count, float *loss, float *grad_out, const float *grad_scale,
                           void *hip_stream);

/* Device bytes the handle holds for forward work: weights, packed forms and
 * workspaces.  Independent of the slot count k (the pool is a running sum). */
gn_status glassnet_workspace_bytes(gn_handle *h, uint64_t *bytes);

/* Object streaming (Sec. 3.3, Eq. (5); Sec. 4.4.2 and Fig. "MemUsage"): tau
 * is a sum over transparency buffers, so each object's buffer can be
 * evaluated on its own and added to a running sum, and device memory stays
 * constant in the number of transparent objects.  A frame batch is evaluated
 * as begin (F -> sigma), then any number of accumulate calls (k >= 0 objects
 * each), then finish (pool, T3, B, R -> out).  Objects are pooled in call
 * order: the result is bitwise the glassnet_forward result, on a handle of
 * the same configuration with slot_order GN_ORDER_INPUT, over all accumulated
 * slots in call order (same arithmetic, same order).  finish may follow any accumulate
 * call (a progressive result) and accumulation may continue after it.
 *
 * The state is caller-owned device memory of glassnet_stream_state_bytes
 * bytes, whatever the number of objects: sigma, the fp32 running sum of h's
 * hidden layer and the active-slot count, in a layout private to the library
 * (GN_BF16 / GN_FP8_T: sigma in bf16, 772 bytes per pixel at W = 128, 388 at
 * W = 64; GN_FP32: sigma, the running sum and the count in fp32, (2 W + 1) x
 * 4 bytes per pixel, through the plane workspace of the FP32 forward with
 * its pixel limit).  Calls on one state
 * are ordered on the hip_stream each passes; calls on different streams must
 * be ordered by the caller. */
gn_status glassnet_stream_state_bytes(gn_handle *h, int32_t n, int32_t hgt, int32_t wid,
                                      uint64_t *bytes);

/* Start a frame batch: evaluate F on frame->gbuf and frame->scene into state
 * (frame->k and frame->layers are ignored).  state: 16-byte aligned device
 * memory of state_bytes >= glassnet_stream_state_bytes(n, h, w) bytes; a
 * state begun earlier that overlaps this memory is forgotten. */
gn_status glassnet_stream_begin(gn_handle *h, const gn_frame *frame, void *state,
                                uint64_t state_bytes, void *hip_stream);

/* Add frame->k objects, frame->layers [n][k][GN_NUM_L][h][w], to the state's
 * running sum (gbuf and scene are ignored).  n, h, w must be those of the
 * begin call; 0 <= k <= k_max, and k = 0 is a no-op.  GN_E_INVAL for a state
 * not begun on this handle. */
gn_status glassnet_stream_accumulate(gn_handle *h, const gn_frame *frame, void *state,
                                     void *hip_stream);

/* Pool the objects accumulated so far (none: an empty pool) and evaluate T3,
 * B and R: out [n][GN_NUM_OUT][h][w] fp32 device, L_d read from frame->gbuf
 * (layers, scene and k are ignored).  The state is left unchanged. */
gn_status glassnet_stream_finish(gn_handle *h, const gn_frame *frame, void *state, float *out,
                                 void *hip_stream);

/* Forget a begun state (its memory stays the caller's).  GN_E_INVAL if unknown. */
gn_status glassnet_stream_release(gn_handle *h, void *state);

/* Serving (continuous batching).  serve_submit enqueues a frame batch whose
 * device buffers the library may read until serve_poll reports done; out is
 * written then.  Frames are admitted while the bytes of admitted-but-unfinished
 * frames (inputs + output) fit hbm_budget_bytes; tiles of admitted frames of
 * any size and k share kernel launches.  Returns GN_E_INVAL for a frame larger
 * than the whole budget, GN_E_BUSY when the pending queue is full.  Never
 * blocks on the GPU. */
gn_status serve_submit(gn_handle *h, const gn_frame *frame, float *out, uint64_t *ticket);

/* *done = 1 once the ticket's output is complete (timing filled, may be NULL),
 * 0 otherwise.  A ticket whose work failed returns GN_E_DEVICE; an unknown
 * ticket GN_E_INVAL.  A completed ticket may be polled again until the next
 * serve_forget or destroy. */
gn_status serve_poll(gn_handle *h, uint64_t ticket, int32_t *done, gn_timing *timing);

/* Block until every submitted frame is done (or failed). */
gn_status serve_drain(gn_handle *h);

/* Drop the bookkeeping of a completed ticket. */
gn_status serve_forget(gn_handle *h, uint64_t ticket);

/* Message of the last failed call on this thread ("" if none). */
const char *glassnet_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GLASSNET_H */
