// Handle state shared by the C-ABI sources (api.cpp, backward, serving).
#pragma once

#include <atomic>
#include <map>
#include <mutex>

#include "gn_internal.h"

struct GnServer;

// A caller-owned object-streaming state the handle knows about (begun by
// glassnet_stream_begin): the frame geometry it was sized for, its bytes, and
// whether any slot has been accumulated into it yet.
struct GnStreamRec {
  int32_t n, hgt, wid;
  uint64_t bytes;
  bool fresh;
};

struct gn_handle {
  gn_config cfg{};
  int W = 0;
  int device = 0;
  int num_cus = 0;
  size_t nparams = 0;
  float *d_master = nullptr;      // fp32 master weights (flat layout)
  uint8_t *d_packed = nullptr;    // fragment-ordered bf16/fp8 weights + biases
  gn::PackedLayout pl{};
  uint8_t *d_sig_scratch[2] = {nullptr, nullptr};  // MFMA forward: caller streams, serving
  float *d_l1_partials = nullptr;
  float *d_loss_ws = nullptr;     // DSSIM term: coefficient maps and partial sums
  float *d_sr_wt = nullptr;       // super-sampling network: re-laid weight copy
  float *d_sr_ws = nullptr;       // super-sampling backward: activations and partials
  size_t sr_ws_bytes = 0;
  uint8_t *d_sp_packed = nullptr; // spatial networks: weight fragments and biases
  uint8_t *d_sp_ws = nullptr;     // spatial networks: activations of one call
  size_t sp_ws_bytes = 0;
  size_t loss_ws_bytes = 0;
  int l1_npart = 0;
  float act_scale = 0.0f;         // fp8 activation scale
  std::atomic<bool> poisoned{false};
  size_t bytes_held = 0;          // device bytes of the forward state
  gn::BwdWorkspace *bwd = nullptr;
  GnServer *server = nullptr;
  std::mutex stream_mu;                          // guards streams
  std::map<uintptr_t, GnStreamRec> streams;      // keyed by state address
};

// Largest slot count whose pixels the fused forward orders canonically (0:
// the handle pools in input order).
inline int gn_slot_kmax(const gn_handle *h) {
  return h->cfg.slot_order == GN_ORDER_CANONICAL ? h->cfg.k_max : 0;
}

gn_status gn_set_error(gn_status code, const char *msg);
gn_status gn_check_device(gn_handle *h, hipError_t e, const char *what);
gn_status gn_validate_frame(gn_handle *h, const gn_frame *f, const float *out);
gn_status gn_prepare_weights(gn_handle *h, hipStream_t stream);

gn_status gn_serve_init(gn_handle *h);
void gn_serve_shutdown(gn_handle *h);
void gn_bwd_free(gn_handle *h);
// The fp32 plane pipeline (planes.hip): the FP32 forward and the FP8
// calibration (amax: device float bits of the largest h-layer-1 activation).
gn_status gn_planes_forward(gn_handle *h, const gn_frame *frame, float *out, hipStream_t s);
gn_status gn_planes_calibrate(gn_handle *h, const gn_frame *frame, unsigned *amax, hipStream_t s);
// Object streaming on the plane pipeline (GN_FP32): mode FWD_BEGIN, FWD_ACC or
// FWD_FINISH; the state holds gn_planes_stream_bytes(W, n h w) bytes.
size_t gn_planes_stream_bytes(int W, int64_t npx);
gn_status gn_planes_stream(gn_handle *h, const gn_frame *frame, int mode, float *state, int fresh,
                           float *out, hipStream_t s);
size_t gn_bwd_bytes(gn_handle *h);
