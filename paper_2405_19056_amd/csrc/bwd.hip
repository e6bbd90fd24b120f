// Backward pass (placeholder until the hand-written kernels land).
#include "gn_api_state.h"

void gn_bwd_free(gn_handle *h) { (void)h; }
size_t gn_bwd_bytes(gn_handle *h) { (void)h; return 0; }

extern "C" gn_status glassnet_backward(gn_handle *h, const gn_frame *frame,
                                       const float *grad_out, float *grad_w, void *hip_stream) {
  (void)h; (void)frame; (void)grad_out; (void)grad_w; (void)hip_stream;
  return gn_set_error(GN_E_UNSUPPORTED, "backward not built yet");
}
