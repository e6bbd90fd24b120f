// Serving (placeholder until the scheduler lands).
#include "gn_api_state.h"

gn_status gn_serve_init(gn_handle *h) { (void)h; return GN_OK; }
void gn_serve_shutdown(gn_handle *h) { (void)h; }

extern "C" {
gn_status serve_submit(gn_handle *h, const gn_frame *f, float *out, uint64_t *ticket) {
  (void)h; (void)f; (void)out; (void)ticket;
  return gn_set_error(GN_E_UNSUPPORTED, "serving not built yet");
}
gn_status serve_poll(gn_handle *h, uint64_t t, int32_t *done, gn_timing *tm) {
  (void)h; (void)t; (void)done; (void)tm;
  return gn_set_error(GN_E_UNSUPPORTED, "serving not built yet");
}
gn_status serve_drain(gn_handle *h) { (void)h; return gn_set_error(GN_E_UNSUPPORTED, "serving not built yet"); }
gn_status serve_forget(gn_handle *h, uint64_t t) { (void)h; (void)t; return gn_set_error(GN_E_UNSUPPORTED, "serving not built yet"); }
}
