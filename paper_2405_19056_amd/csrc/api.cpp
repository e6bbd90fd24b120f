// The C ABI of libglassnet: argument validation, handle state, launches.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "gn_api_state.h"

namespace {

thread_local std::string g_err;

gn_status fail(gn_status code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

// Sets the handle's device for the duration of a call, restores the caller's.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

bool aligned4(const void *p) { return ((uintptr_t)p & 3u) == 0; }

bool overlaps(const void *a, size_t an, const void *b, size_t bn) {
  if (!a || !b || !an || !bn) return false;
  const char *x = (const char *)a, *y = (const char *)b;
  return x < y + bn && y < x + an;
}

}  // namespace

gn_status gn_set_error(gn_status code, const char *msg) { return fail(code, "%s", msg); }

gn_status gn_check_device(gn_handle *h, hipError_t e, const char *what) {
  if (e == hipSuccess) return GN_OK;
  h->poisoned = true;
  return fail(GN_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

gn_status gn_validate_frame(gn_handle *h, const gn_frame *f, const float *out) {
  if (!f) return fail(GN_E_INVAL, "frame is NULL");
  if (f->n < 1 || f->h < 1 || f->w < 1)
    return fail(GN_E_INVAL, "frame shape n=%d h=%d w=%d must be >= 1", f->n, f->h, f->w);
  if (f->k < 0 || f->k > h->cfg.k_max)
    return fail(GN_E_INVAL, "k=%d outside [0, k_max=%d]", f->k, h->cfg.k_max);
  const int64_t hw = (int64_t)f->h * f->w;
  // the fused kernel addresses a frame's slot planes with 32-bit offsets
  if (hw * gn::kNG > INT32_MAX || (int64_t)f->n * hw > INT32_MAX ||
      hw * (int64_t)std::max(f->k, 1) * gn::kNL >= ((int64_t)1 << 32))
    return fail(GN_E_INVAL, "frame too large (%d x %d x %d, k=%d)", f->n, f->h, f->w, f->k);
  if (!f->gbuf || !f->scene) return fail(GN_E_INVAL, "gbuf and scene must be non-NULL");
  if (f->k > 0 && !f->layers) return fail(GN_E_INVAL, "layers is NULL with k=%d", f->k);
  if (!aligned4(f->gbuf) || !aligned4(f->scene) || !aligned4(f->layers) || !aligned4(out))
    return fail(GN_E_INVAL, "device pointers must be 4-byte aligned");
  if (out) {
    const size_t ob = sizeof(float) * (size_t)f->n * gn::kNOUT * hw;
    if (overlaps(out, ob, f->gbuf, sizeof(float) * (size_t)f->n * gn::kNG * hw) ||
        overlaps(out, ob, f->layers, sizeof(float) * (size_t)f->n * f->k * gn::kNL * hw) ||
        overlaps(out, ob, f->scene, sizeof(float) * (size_t)f->n * gn::kNS))
      return fail(GN_E_INVAL, "out aliases an input buffer");
  }
  return GN_OK;
}

static gn_status precheck(gn_handle *h) {
  if (!h) return fail(GN_E_INVAL, "handle is NULL");
  if (h->poisoned) return fail(GN_E_DEVICE, "handle poisoned by an earlier device error");
  // surface asynchronous faults from earlier work on this device
  hipError_t e = hipPeekAtLastError();
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return gn_check_device(h, e, "earlier asynchronous device error");
  }
  return GN_OK;
}

gn_status gn_prepare_weights(gn_handle *h, hipStream_t stream) {
  hipError_t e = gn::launch_pack_weights(h->d_master, h->d_packed, h->pl, h->act_scale, stream);
  return gn_check_device(h, e, "weight packing");
}

extern "C" {

size_t glassnet_num_params(int32_t width, int32_t pe_levels) {
  return gn::num_params(width, pe_levels);
}

const char *glassnet_last_error(void) { return g_err.c_str(); }

gn_status glassnet_create(const gn_config *cfg, const float *host_weights, size_t n,
                          gn_handle **out) {
  if (!cfg || !out) return fail(GN_E_INVAL, "cfg and out must be non-NULL");
  *out = nullptr;
  if (cfg->width != 64 && cfg->width != 128)
    return fail(GN_E_UNSUPPORTED, "width %d not supported (64 or 128)", cfg->width);
  if (cfg->k_max < 0 || cfg->k_max > GN_MAX_K)
    return fail(GN_E_INVAL, "k_max %d outside [0, %d]", cfg->k_max, GN_MAX_K);
  if (cfg->pool != GN_POOL_MEAN && cfg->pool != GN_POOL_SUM)
    return fail(GN_E_INVAL, "unknown pool %d", cfg->pool);
  if (cfg->precision == GN_FP8_ALL)
    return fail(GN_E_UNSUPPORTED, "GN_FP8_ALL is not built: FP8 in every layer misses the "
                                  "6e-2 error bar (about 8e-2); use GN_FP8_T");
  if (cfg->precision != GN_FP32 && cfg->precision != GN_BF16 && cfg->precision != GN_FP8_T)
    return fail(GN_E_INVAL, "unknown precision %d", cfg->precision);
  if (cfg->precision == GN_FP8_T && cfg->width != 128)
    return fail(GN_E_UNSUPPORTED, "GN_FP8_T needs width 128");
  if (cfg->slot_order != GN_ORDER_CANONICAL && cfg->slot_order != GN_ORDER_INPUT)
    return fail(GN_E_INVAL, "unknown slot order %d", cfg->slot_order);
  if (cfg->pe_levels < 0 || cfg->pe_levels > GN_MAX_PE_LEVELS)
    return fail(GN_E_UNSUPPORTED, "pe_levels %d outside [0, %d]", cfg->pe_levels,
                GN_MAX_PE_LEVELS);
  const size_t np = gn::num_params(cfg->width, cfg->pe_levels);
  if (n != np && !(host_weights == nullptr && n == 0))
    return fail(GN_E_INVAL, "expected %zu weights for width %d and %d encoding levels, got %zu",
                np, cfg->width, cfg->pe_levels, n);
  std::vector<float> seeded;
  if (!host_weights) {
    seeded.resize(np);
    gn::seeded_weights(cfg->width, cfg->pe_levels, cfg->seed, seeded.data());
    host_weights = seeded.data();
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return fail(GN_E_DEVICE, "no HIP device available");
  if (cfg->device < 0 || cfg->device >= ndev)
    return fail(GN_E_INVAL, "device %d outside [0, %d)", cfg->device, ndev);
  DeviceGuard dg(cfg->device);
  if (!dg.ok) return fail(GN_E_DEVICE, "hipSetDevice(%d) failed", cfg->device);

  gn_handle *h = new (std::nothrow) gn_handle();
  if (!h) return fail(GN_E_NOMEM, "host allocation failed");
  h->cfg = *cfg;
  if (!h->cfg.hbm_budget_bytes) h->cfg.hbm_budget_bytes = (uint64_t)64 << 30;
  if (!h->cfg.max_pending) h->cfg.max_pending = 65536;
  h->W = cfg->width;
  h->device = cfg->device;
  h->nparams = np;
  h->act_scale = 8.0f / 448.0f;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, cfg->device) != hipSuccess) {
    delete h;
    return fail(GN_E_DEVICE, "hipGetDeviceProperties failed");
  }
  h->num_cus = prop.multiProcessorCount;
  gn::make_packed_layout(h->W, cfg->pe_levels, &h->pl);
  h->l1_npart = 4 * h->num_cus;

  const size_t wbytes = sizeof(float) * np;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMalloc((void **)&h->d_master, wbytes);
  if (e == hipSuccess) e = hipMalloc((void **)&h->d_packed, (size_t)h->pl.total_bytes);
  if (e == hipSuccess) e = hipMalloc((void **)&h->d_l1_partials, sizeof(float) * h->l1_npart);
  const size_t sig_bytes = gn::mfma_sig_scratch_bytes(h->W, h->num_cus);
  if (cfg->precision != GN_FP32)
    for (int i = 0; i < 2 && e == hipSuccess; ++i)
      e = hipMalloc((void **)&h->d_sig_scratch[i], sig_bytes);
  if (e == hipSuccess) e = hipMemcpy(h->d_master, host_weights, wbytes, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(h->d_packed, 0, (size_t)h->pl.total_bytes);
  if (e != hipSuccess) {
    gn_status st = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
                       ? fail(GN_E_NOMEM, "device allocation failed: %s", hipGetErrorString(e))
                       : fail(GN_E_DEVICE, "device setup failed: %s", hipGetErrorString(e));
    glassnet_destroy(h);
    return st;
  }
  // the allocation-free DSSIM form's workspace address on this device (once)
  if (e == hipSuccess) {
    e = gn::dssim_scratch_init(cfg->device);
    if (e != hipSuccess) {
      glassnet_destroy(h);
      return fail(GN_E_DEVICE, "DSSIM scratch address: %s", hipGetErrorString(e));
    }
  }
  h->bytes_held = wbytes + (size_t)h->pl.total_bytes + sizeof(float) * h->l1_npart +
                  (cfg->precision == GN_FP32 ? 0 : 2 * sig_bytes);
  gn_status st = gn_prepare_weights(h, nullptr);
  if (st == GN_OK) {
    e = hipDeviceSynchronize();
    st = gn_check_device(h, e, "weight packing");
  }
  if (st != GN_OK) {
    std::string msg = g_err;
    glassnet_destroy(h);
    return fail(st, "%s", msg.c_str());
  }
  st = gn_serve_init(h);
  if (st != GN_OK) {
    std::string msg = g_err;
    glassnet_destroy(h);
    return fail(st, "%s", msg.c_str());
  }
  *out = h;
  return GN_OK;
}

gn_status glassnet_destroy(gn_handle *h) {
  if (!h) return GN_OK;
  DeviceGuard dg(h->device);
  gn_serve_shutdown(h);
  gn_bwd_free(h);
  if (!h->poisoned) (void)hipDeviceSynchronize();
  (void)hipFree(h->d_master);
  (void)hipFree(h->d_packed);
  (void)hipFree(h->d_l1_partials);
  (void)hipFree(h->d_loss_ws);
  (void)hipFree(h->d_sr_wt);
  (void)hipFree(h->d_sr_ws);
  (void)hipFree(h->d_sp_packed);
  (void)hipFree(h->d_sp_ws);
  (void)hipFree(h->d_sig_scratch[0]);
  (void)hipFree(h->d_sig_scratch[1]);
  delete h;
  return GN_OK;
}

gn_status glassnet_get_weights(gn_handle *h, float *host_weights, size_t n) {
  gn_status st = precheck(h);
  if (st != GN_OK) return st;
  if (!host_weights || n != h->nparams)
    return fail(GN_E_INVAL, "need a host buffer of %zu floats", h->nparams);
  DeviceGuard dg(h->device);
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess)
    e = hipMemcpy(host_weights, h->d_master, sizeof(float) * n, hipMemcpyDeviceToHost);
  return gn_check_device(h, e, "get_weights");
}

gn_status glassnet_set_weights(gn_handle *h, const float *dev_weights, size_t n,
                               void *hip_stream) {
  gn_status st = precheck(h);
  if (st != GN_OK) return st;
  if (!dev_weights || n != h->nparams || !aligned4(dev_weights))
    return fail(GN_E_INVAL, "need %zu aligned device floats", h->nparams);
  DeviceGuard dg(h->device);
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t e = hipSuccess;
  if (dev_weights != h->d_master)
    e = hipMemcpyAsync(h->d_master, dev_weights, sizeof(float) * n, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return gn_check_device(h, e, "set_weights copy");
  return gn_prepare_weights(h, s);
}

gn_status glassnet_set_act_scales(gn_handle *h, const float *scales, size_t n) {
  gn_status st = precheck(h);
  if (st != GN_OK) return st;
  if (!scales || n != 1 || !(scales[0] > 0.0f) || !(scales[0] < 1e30f))
    return fail(GN_E_INVAL, "need exactly one finite positive activation scale");
  h->act_scale = scales[0];
  return GN_OK;
}

gn_status glassnet_calibrate(gn_handle *h, const gn_frame *frame, void *hip_stream) {
  gn_status st = precheck(h);
  if (st != GN_OK) return st;
  st = gn_validate_frame(h, frame, nullptr);
  if (st != GN_OK) return st;
  DeviceGuard dg(h->device);
  hipStream_t s = (hipStream_t)hip_stream;
  unsigned *amax = nullptr;
  hipError_t e = hipMalloc((void **)&amax, sizeof(unsigned));
  if (e == hipSuccess) e = hipMemsetAsync(amax, 0, sizeof(unsigned), s);
  if (e != hipSuccess) {
    (void)hipFree(amax);
    return gn_check_device(h, e, "calibration");
  }
  st = gn_planes_calibrate(h, frame, amax, s);
  unsigned bits = 0;
  if (st == GN_OK) {
    e = hipMemcpyAsync(&bits, amax, sizeof bits, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    st = gn_check_device(h, e, "calibration");
  }
  (void)hipFree(amax);
  if (st != GN_OK) return st;
  float m;
  memcpy(&m, &bits, sizeof m);
  if (m > 0.0f && m < 1e30f) h->act_scale = m / 448.0f;
  return GN_OK;
}

gn_status glassnet_workspace_bytes(gn_handle *h, uint64_t *bytes) {
  if (!h || !bytes) return fail(GN_E_INVAL, "NULL argument");
  *bytes = h->bytes_held + gn_bwd_bytes(h);
  return GN_OK;
}

gn_status glassnet_forward(gn_handle *h, const gn_frame *frame, float *out, void *hip_stream) {
  gn_status st = precheck(h);
  if (st != GN_OK) return st;
  if (!out) return fail(GN_E_INVAL, "out is NULL");
  st = gn_validate_frame(h, frame, out);
  if (st != GN_OK) return st;
  DeviceGuard dg(h->device);
  hipStream_t s = (hipStream_t)hip_stream;
  gn::FwdBatch b;
  b.gbuf = frame->gbuf;
  b.layers = frame->layers;
  b.scene = frame->scene;
  b.out = out;
  b.n = frame->n;
  b.hw = frame->h * frame->w;
  b.k = frame->k;
  if (h->cfg.precision == GN_FP32) return gn_planes_forward(h, frame, out, s);
  const int tpf = (b.hw + gn::kTilePx - 1) / gn::kTilePx;
  const hipError_t e = gn::launch_fwd_mfma(h->W, h->cfg.precision, h->cfg.pool, h->d_packed, h->pl,
                                           &b, nullptr, nullptr, b.n * tpf, h->act_scale,
                                           h->num_cus, h->d_sig_scratch[0], gn_slot_kmax(h), s);
  return gn_check_device(h, e, "forward launch");
}

// ---- object streaming ---------------------------------------------------------

static gn_status stream_geometry(gn_handle *h, int32_t n, int32_t hgt, int32_t wid,
                                 uint64_t *bytes) {
  if (n < 1 || hgt < 1 || wid < 1)
    return fail(GN_E_INVAL, "frame shape n=%d h=%d w=%d must be >= 1", n, hgt, wid);
  const int64_t hw = (int64_t)hgt * wid;
  if (hw * gn::kNG > INT32_MAX || (int64_t)n * hw > INT32_MAX)
    return fail(GN_E_INVAL, "frame too large (%d x %d x %d)", n, hgt, wid);
  if (h->cfg.precision == GN_FP32) {          // plane pipeline: [sigma; Z; count] rows
    *bytes = gn_planes_stream_bytes(h->W, (int64_t)n * hw);
    return GN_OK;
  }
  const uint64_t tiles = (uint64_t)n * (uint64_t)((hw + gn::kTilePx - 1) / gn::kTilePx);
  *bytes = tiles * gn::stream_state_tile_bytes(h->W);
  return GN_OK;
}

// One streaming launch: the fused kernel's mode, or the plane pipeline (GN_FP32).
static gn_status stream_launch(gn_handle *h, const gn::FwdBatch &b, const gn_frame *f, int mode,
                               void *state, int state_load, float *out, hipStream_t s,
                               const char *what) {
  if (h->cfg.precision == GN_FP32) {
    gn_frame pf = *f;
    pf.gbuf = b.gbuf;
    pf.layers = b.layers;
    pf.scene = b.scene;
    pf.k = b.k;
    return gn_planes_stream(h, &pf, mode, (float *)state, state_load ? 0 : 1, out, s);
  }
  const hipError_t e = gn::launch_fwd_stream(h->W, h->cfg.precision, h->cfg.pool, h->d_packed,
                                             h->pl, b, h->act_scale, h->num_cus, mode,
                                             (uint8_t *)state, state_load, s);
  return gn_check_device(h, e, what);
}

// The record of a begun state whose geometry matches the frame (caller holds stream_mu).
static gn_status stream_lookup(gn_handle *h, const gn_frame *f, const void *state,
                               GnStreamRec **rec) {
  auto it = h->streams.find((uintptr_t)state);
  if (it == h->streams.end())
    return fail(GN_E_INVAL, "state %p was not begun with glassnet_stream_begin", state);
  const GnStreamRec &r = it->second;
  if (f->n != r.n || f->h != r.hgt || f->w != r.wid)
    return fail(GN_E_INVAL, "frame %d x %d x %d does not match the state's %d x %d x %d", f->n,
                f->h, f->w, r.n, r.hgt, r.wid);
  *rec = &it->second;
  return GN_OK;
}

static gn::FwdBatch stream_batch(const gn_frame *f) {
  gn::FwdBatch b;
  b.gbuf = f->gbuf;
  b.layers = f->layers;
  b.scene = f->scene;
  b.out = nullptr;
  b.n = f->n;
  b.hw = f->h * f->w;
  b.k = f->k;
  return b;
}

gn_status glassnet_stream_state_bytes(gn_handle *h, int32_t n, int32_t hgt, int32_t wid,
                                      uint64_t *bytes) {
  if (!h || !bytes) return fail(GN_E_INVAL, "NULL argument");
  return stream_geometry(h, n, hgt, wid, bytes);
}

gn_status glassnet_stream_begin(gn_handle *h, const gn_frame *frame, void *state,
                                uint64_t state_bytes, void *hip_stream) {
  gn_status st = precheck(h);
  if (st != GN_OK) return st;
  if (!frame || !state) return fail(GN_E_INVAL, "frame and state must be non-NULL");
  uint64_t need = 0;
  st = stream_geometry(h, frame->n, frame->h, frame->w, &need);
  if (st != GN_OK) return st;
  if (state_bytes < need)
    return fail(GN_E_INVAL, "state holds %llu bytes, the frame needs %llu",
                (unsigned long long)state_bytes, (unsigned long long)need);
  if (((uintptr_t)state & 15u) != 0) return fail(GN_E_INVAL, "state must be 16-byte aligned");
  if (!frame->gbuf || !frame->scene) return fail(GN_E_INVAL, "gbuf and scene must be non-NULL");
  if (!aligned4(frame->gbuf) || !aligned4(frame->scene))
    return fail(GN_E_INVAL, "device pointers must be 4-byte aligned");
  const size_t hw = (size_t)frame->h * frame->w;
  if (overlaps(state, need, frame->gbuf, sizeof(float) * frame->n * gn::kNG * hw) ||
      overlaps(state, need, frame->scene, sizeof(float) * frame->n * gn::kNS))
    return fail(GN_E_INVAL, "state aliases an input buffer");
  DeviceGuard dg(h->device);
  {
    std::lock_guard<std::mutex> lk(h->stream_mu);
    // a state that reuses (part of) the memory of earlier ones replaces them
    for (auto it = h->streams.begin(); it != h->streams.end();) {
      if (overlaps((const void *)it->first, it->second.bytes, state, need))
        it = h->streams.erase(it);
      else
        ++it;
    }
    h->streams[(uintptr_t)state] = GnStreamRec{frame->n, frame->h, frame->w, need, true};
  }
  gn::FwdBatch b = stream_batch(frame);
  b.layers = nullptr;     // BEGIN reads the G-buffer and the scene vector only
  b.k = 0;
  return stream_launch(h, b, frame, gn::FWD_BEGIN, state, 0, nullptr, (hipStream_t)hip_stream,
                       "stream begin launch");
}

gn_status glassnet_stream_accumulate(gn_handle *h, const gn_frame *frame, void *state,
                                     void *hip_stream) {
  gn_status st = precheck(h);
  if (st != GN_OK) return st;
  if (!frame || !state) return fail(GN_E_INVAL, "frame and state must be non-NULL");
  if (frame->k < 0 || frame->k > h->cfg.k_max)
    return fail(GN_E_INVAL, "k=%d outside [0, k_max=%d]", frame->k, h->cfg.k_max);
  if (frame->k > 0 && !frame->layers) return fail(GN_E_INVAL, "layers is NULL with k=%d", frame->k);
  if (!aligned4(frame->layers)) return fail(GN_E_INVAL, "device pointers must be 4-byte aligned");
  std::lock_guard<std::mutex> lk(h->stream_mu);
  GnStreamRec *rec = nullptr;
  st = stream_lookup(h, frame, state, &rec);
  if (st != GN_OK) return st;
  if (frame->k == 0) return GN_OK;
  const size_t hw = (size_t)frame->h * frame->w;
  if (overlaps(state, rec->bytes, frame->layers, sizeof(float) * frame->n * frame->k * gn::kNL * hw))
    return fail(GN_E_INVAL, "state aliases the layers buffer");
  DeviceGuard dg(h->device);
  gn::FwdBatch b = stream_batch(frame);
  b.gbuf = nullptr;       // ACC reads the objects' layers only
  b.scene = nullptr;
  st = stream_launch(h, b, frame, gn::FWD_ACC, state, rec->fresh ? 0 : 1, nullptr,
                     (hipStream_t)hip_stream, "stream accumulate launch");
  if (st == GN_OK) rec->fresh = false;
  return st;
}

gn_status glassnet_stream_finish(gn_handle *h, const gn_frame *frame, void *state, float *out,
                                 void *hip_stream) {
  gn_status st = precheck(h);
  if (st != GN_OK) return st;
  if (!frame || !state || !out) return fail(GN_E_INVAL, "frame, state and out must be non-NULL");
  if (!frame->gbuf) return fail(GN_E_INVAL, "gbuf must be non-NULL");
  if (!aligned4(frame->gbuf) || !aligned4(out))
    return fail(GN_E_INVAL, "device pointers must be 4-byte aligned");
  std::lock_guard<std::mutex> lk(h->stream_mu);
  GnStreamRec *rec = nullptr;
  st = stream_lookup(h, frame, state, &rec);
  if (st != GN_OK) return st;
  const size_t hw = (size_t)frame->h * frame->w;
  const size_t ob = sizeof(float) * frame->n * gn::kNOUT * hw;
  if (overlaps(out, ob, frame->gbuf, sizeof(float) * frame->n * gn::kNG * hw) ||
      overlaps(out, ob, state, rec->bytes))
    return fail(GN_E_INVAL, "out aliases gbuf or the state");
  DeviceGuard dg(h->device);
  gn::FwdBatch b = stream_batch(frame);
  b.layers = nullptr;     // FINISH reads L_d from the G-buffer and the state only
  b.scene = nullptr;
  b.k = 0;
  b.out = out;
  return stream_launch(h, b, frame, gn::FWD_FINISH, state, rec->fresh ? 0 : 1, out,
                       (hipStream_t)hip_stream, "stream finish launch");
}

gn_status glassnet_stream_release(gn_handle *h, void *state) {
  if (!h || !state) return fail(GN_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(h->stream_mu);
  if (!h->streams.erase((uintptr_t)state))
    return fail(GN_E_INVAL, "state %p was not begun with glassnet_stream_begin", state);
  return GN_OK;
}

gn_status glassnet_l1_loss(gn_handle *h, const float *out, const float *target, uint64_t count,
                           float *loss, float *grad_out, const float *grad_scale,
                           void *hip_stream) {
  gn_status st = precheck(h);
  if (st != GN_OK) return st;
  if (!out || !target || !loss) return fail(GN_E_INVAL, "out, target and loss must be non-NULL");
  if (!aligned4(out) || !aligned4(target) || !aligned4(loss) || !aligned4(grad_out) ||
      !aligned4(grad_scale))
    return fail(GN_E_INVAL, "device pointers must be 4-byte aligned");
  if (grad_out && (overlaps(grad_out, 4 * count, out, 4 * count) ||
                   overlaps(grad_out, 4 * count, target, 4 * count) ||
                   (grad_scale && overlaps(grad_out, 4 * count, grad_scale, 4))))
    return fail(GN_E_INVAL, "grad_out aliases out, target or grad_scale");
  DeviceGuard dg(h->device);
  hipError_t e = gn::launch_l1(out, target, count, loss, grad_out, grad_scale, h->d_l1_partials,
                               h->l1_npart, (hipStream_t)hip_stream);
  return gn_check_device(h, e, "l1 launch");
}

// Arguments of the DSSIM term (both forms).
static gn_status dssim_check(gn_handle *h, const float *out, const float *target, int32_t n,
                             int32_t height, int32_t width, const float *loss,
                             const float *grad_out) {
  gn_status st = precheck(h);
  if (st != GN_OK) return st;
  if (n < 1 || height < 11 || width < 11)
    return fail(GN_E_INVAL, "need n >= 1 and images of at least 11 x 11 (got %d x %d x %d)", n,
                height, width);
  if ((int64_t)n * gn::kNOUT * height * width > ((int64_t)1 << 31))
    return fail(GN_E_INVAL, "more than 2^31 elements");
  if (!out || !target || !loss) return fail(GN_E_INVAL, "out, target and loss must be non-NULL");
  if (!aligned4(out) || !aligned4(target) || !aligned4(loss) || !aligned4(grad_out))
    return fail(GN_E_INVAL, "device pointers must be 4-byte aligned");
  const size_t bytes = sizeof(float) * (size_t)n * gn::kNOUT * height * width;
  if (grad_out && (overlaps(grad_out, bytes, out, bytes) || overlaps(grad_out, bytes, target, bytes) ||
                   overlaps(grad_out, bytes, loss, 4)))
    return fail(GN_E_INVAL, "grad_out aliases out, target or loss");
  if (overlaps(loss, 4, out, bytes) || overlaps(loss, 4, target, bytes))
    return fail(GN_E_INVAL, "loss aliases out or target");
  return GN_OK;
}

gn_status glassnet_dssim_loss(gn_handle *h, const float *out, const float *target, int32_t n,
                              int32_t height, int32_t width, float *loss, float *grad_out,
                              int32_t accumulate, void *hip_stream) {
  gn_status st = dssim_check(h, out, target, n, height, width, loss, grad_out);
  if (st != GN_OK) return st;
  DeviceGuard dg(h->device);
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t need = gn::dssim_workspace_bytes(n * gn::kNOUT, height, width);
  if (need > h->loss_ws_bytes) {
    // grown workspaces replace the old one once the stream's earlier work is done
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipFree(h->d_loss_ws);
    h->d_loss_ws = nullptr;
    h->loss_ws_bytes = 0;
    if (e == hipSuccess) e = hipMalloc((void **)&h->d_loss_ws, need);
    if (e != hipSuccess) {
      h->d_loss_ws = nullptr;
      return e == hipErrorOutOfMemory ? fail(GN_E_NOMEM, "DSSIM workspace of %zu bytes", need)
                                      : gn_check_device(h, e, "DSSIM workspace");
    }
    h->loss_ws_bytes = need;
  }
  hipError_t e = gn::launch_dssim(out, target, n * gn::kNOUT, height, width, loss, grad_out,
                                  accumulate ? 1 : 0, h->d_loss_ws, s);
  return gn_check_device(h, e, "DSSIM launch");
}

gn_status glassnet_dssim_loss_noalloc(gn_handle *h, const float *out, const float *target,
                                      int32_t n, int32_t height, int32_t width, float *loss,
                                      float *grad_out, int32_t accumulate, void *hip_stream) {
  gn_status st = dssim_check(h, out, target, n, height, width, loss, grad_out);
  if (st != GN_OK) return st;
  const size_t need = gn::dssim_workspace_bytes(n * gn::kNOUT, height, width);
  if (need > gn::kDssimScratchBytes)
    return fail(GN_E_INVAL, "DSSIM of %d x 3 x %d x %d needs %zu workspace bytes, above the %zu "
                "of the allocation-free form", n, height, width, need, gn::kDssimScratchBytes);
  float *ws = gn::dssim_scratch(h->device);
  if (!ws) return fail(GN_E_DEVICE, "DSSIM scratch not set up on device %d", h->device);
  DeviceGuard dg(h->device);
  hipError_t e = gn::launch_dssim(out, target, n * gn::kNOUT, height, width, loss, grad_out,
                                  accumulate ? 1 : 0, ws, (hipStream_t)hip_stream);
  return gn_check_device(h, e, "DSSIM launch");
}

size_t glassnet_sr_num_params(void) { return (size_t)gn::kSrParams; }

}  // extern "C"

namespace {
// the handle's device copy of the super-sampling weights in kernel order
gn_status sr_weight_copy(gn_handle *h) {
  if (h->d_sr_wt) return GN_OK;
  hipError_t e = hipMalloc((void **)&h->d_sr_wt, sizeof(float) * (size_t)gn::kSrWtFloats);
  if (e == hipSuccess) return GN_OK;
  h->d_sr_wt = nullptr;
  return e == hipErrorOutOfMemory ? fail(GN_E_NOMEM, "super-sampling weight copy")
                                  : gn_check_device(h, e, "super-sampling weight copy");
}
}  // namespace

extern "C" {

size_t glassnet_spatial_num_params(int32_t width) { return gn::spatial_num_params(width); }

gn_status glassnet_spatial_forward(gn_handle *h, const float *sp_w, const gn_frame *frame,
                                   float *out, void *hip_stream) {
  gn_status st = precheck(h);
  if (st != GN_OK) return st;
  st = gn_validate_frame(h, frame, out);
  if (st != GN_OK) return st;
  if (!sp_w || !aligned4(sp_w) || !out)
    return fail(GN_E_INVAL, "sp_w and out must be non-NULL, 4-byte aligned");
  if ((frame->h & 1) || (frame->w & 1))
    return fail(GN_E_INVAL, "the U-Nets need even frame sizes (got %d x %d)", frame->h, frame->w);
  if ((int64_t)frame->n * frame->h * frame->w > ((int64_t)1 << 22))
    return fail(GN_E_INVAL, "more than 2^22 pixels in one call");
  const size_t w_b = sizeof(float) * gn::spatial_num_params(h->W);
  const size_t out_b = sizeof(float) * (size_t)frame->n * gn::kNOUT * frame->h * frame->w;
  if (overlaps(out, out_b, sp_w, w_b)) return fail(GN_E_INVAL, "out aliases sp_w");
  DeviceGuard dg(h->device);
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t e = hipSuccess;
  if (!h->d_sp_packed) {
    e = hipMalloc((void **)&h->d_sp_packed, gn::spatial_weight_bytes(h->W));
    if (e != hipSuccess) {
      h->d_sp_packed = nullptr;
      return e == hipErrorOutOfMemory ? fail(GN_E_NOMEM, "spatial weight copy")
                                      : gn_check_device(h, e, "spatial weight copy");
    }
  }
  const size_t need = gn::spatial_workspace_bytes(h->W, frame->n, frame->h, frame->w, frame->k) + 4096;
  if (need > h->sp_ws_bytes) {
    // grown workspaces replace the old one once the stream's earlier work is done
    e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipFree(h->d_sp_ws);
    h->d_sp_ws = nullptr;
    h->sp_ws_bytes = 0;
    if (e == hipSuccess) e = hipMalloc((void **)&h->d_sp_ws, need);
    if (e != hipSuccess) {
      h->d_sp_ws = nullptr;
      return e == hipErrorOutOfMemory ? fail(GN_E_NOMEM, "spatial workspace of %zu bytes", need)
                                      : gn_check_device(h, e, "spatial workspace");
    }
    h->sp_ws_bytes = need;
  }
  e = gn::spatial_pack(sp_w, h->W, h->d_sp_packed, s);
  if (e == hipSuccess)
    e = gn::spatial_forward(h->d_sp_packed, h->W, h->cfg.pool, frame->gbuf, frame->layers,
                            frame->scene, frame->n, frame->h, frame->w, frame->k, out, h->d_sp_ws,
                            s);
  return gn_check_device(h, e, "spatial forward launch");
}

gn_status glassnet_sr_forward(gn_handle *h, const float *sr_w, int32_t n, int32_t height,
                              int32_t width, const float *lowres, const float *gbuf_hi, float *out,
                              void *hip_stream) {
  gn_status st = precheck(h);
  if (st != GN_OK) return st;
  if (n < 1 || n > 65535 || height < 1 || width < 1 || height > (1 << 18) || width > (1 << 18))
    return fail(GN_E_INVAL, "need 1 <= n <= 65535 and 1 <= height, width <= 2^18 (got %d x %d x %d)",
                n, height, width);
  if (!sr_w || !lowres || !gbuf_hi || !out)
    return fail(GN_E_INVAL, "sr_w, lowres, gbuf_hi and out must be non-NULL");
  if (!aligned4(sr_w) || !aligned4(lowres) || !aligned4(gbuf_hi) || !aligned4(out))
    return fail(GN_E_INVAL, "device pointers must be 4-byte aligned");
  const size_t plane_hi = (size_t)4 * height * width;
  const size_t out_b = sizeof(float) * (size_t)n * gn::kNOUT * plane_hi;
  const size_t g_b = sizeof(float) * (size_t)n * GN_NUM_G * plane_hi;
  const size_t lo_b = sizeof(float) * (size_t)n * gn::kNOUT * height * width;
  const size_t w_b = sizeof(float) * (size_t)gn::kSrParams;
  if (overlaps(out, out_b, lowres, lo_b) || overlaps(out, out_b, gbuf_hi, g_b) ||
      overlaps(out, out_b, sr_w, w_b))
    return fail(GN_E_INVAL, "out aliases lowres, gbuf_hi or sr_w");
  DeviceGuard dg(h->device);
  st = sr_weight_copy(h);
  if (st != GN_OK) return st;
  hipError_t e = gn::launch_sr_forward(sr_w, h->d_sr_wt, lowres, gbuf_hi, out, n, height, width,
                                       (hipStream_t)hip_stream);
  return gn_check_device(h, e, "super-sampling launch");
}

gn_status glassnet_sr_backward(gn_handle *h, const float *sr_w, int32_t n, int32_t height,
                               int32_t width, const float *lowres, const float *gbuf_hi,
                               const float *grad_out, float *grad_w, void *hip_stream) {
  gn_status st = precheck(h);
  if (st != GN_OK) return st;
  if (n < 1 || height < 1 || width < 1 || height > (1 << 16) || width > (1 << 16) ||
      (int64_t)n * 4 * height * width > ((int64_t)1 << 22))
    return fail(GN_E_INVAL,
                "need n, height, width >= 1, height, width <= 2^16 and at most 2^22 output "
                "pixels (got %d x %d x %d)", n, height, width);
  if (!sr_w || !lowres || !gbuf_hi || !grad_out || !grad_w)
    return fail(GN_E_INVAL, "sr_w, lowres, gbuf_hi, grad_out and grad_w must be non-NULL");
  if (!aligned4(sr_w) || !aligned4(lowres) || !aligned4(gbuf_hi) || !aligned4(grad_out) ||
      !aligned4(grad_w))
    return fail(GN_E_INVAL, "device pointers must be 4-byte aligned");
  const size_t plane_hi = (size_t)4 * height * width;
  const size_t w_b = sizeof(float) * (size_t)gn::kSrParams;
  const size_t go_b = sizeof(float) * (size_t)n * gn::kNOUT * plane_hi;
  const size_t g_b = sizeof(float) * (size_t)n * GN_NUM_G * plane_hi;
  const size_t lo_b = sizeof(float) * (size_t)n * gn::kNOUT * height * width;
  if (overlaps(grad_w, w_b, sr_w, w_b) || overlaps(grad_w, w_b, lowres, lo_b) ||
      overlaps(grad_w, w_b, gbuf_hi, g_b) || overlaps(grad_w, w_b, grad_out, go_b))
    return fail(GN_E_INVAL, "grad_w aliases an input");
  DeviceGuard dg(h->device);
  hipStream_t s = (hipStream_t)hip_stream;
  st = sr_weight_copy(h);
  if (st != GN_OK) return st;
  const size_t need = gn::sr_backward_workspace_bytes(n, height, width);
  if (need > h->sr_ws_bytes) {
    // grown workspaces replace the old one once the stream's earlier work is done
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipFree(h->d_sr_ws);
    h->d_sr_ws = nullptr;
    h->sr_ws_bytes = 0;
    if (e == hipSuccess) e = hipMalloc((void **)&h->d_sr_ws, need);
    if (e != hipSuccess) {
      h->d_sr_ws = nullptr;
      return e == hipErrorOutOfMemory
                 ? fail(GN_E_NOMEM, "super-sampling backward workspace of %zu bytes", need)
                 : gn_check_device(h, e, "super-sampling backward workspace");
    }
    h->sr_ws_bytes = need;
  }
  hipError_t e = gn::launch_sr_backward(sr_w, h->d_sr_wt, lowres, gbuf_hi, grad_out, grad_w, n,
                                        height, width, h->d_sr_ws, s);
  return gn_check_device(h, e, "super-sampling backward launch");
}

gn_status glassnet_adam_step(gn_handle *h, const float *grad_w, float *state, size_t n,
                             int32_t step, float lr, float beta1, float beta2, float eps,
                             float weight_decay, void *hip_stream) {
  gn_status st = precheck(h);
  if (st != GN_OK) return st;
  if (n != h->nparams) return fail(GN_E_INVAL, "expected %zu parameters, got %zu", h->nparams, n);
  if (!grad_w || !state || !aligned4(grad_w) || !aligned4(state))
    return fail(GN_E_INVAL, "grad_w and state must be non-NULL 4-byte aligned device pointers");
  if (step < 1) return fail(GN_E_INVAL, "step %d must be >= 1", step);
  if (!(lr >= 0.0f && lr < 1e30f) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
      !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f && eps < 1e30f) ||
      !(weight_decay >= 0.0f && weight_decay < 1e30f))
    return fail(GN_E_INVAL, "need lr >= 0, 0 <= beta1, beta2 < 1, eps > 0, weight_decay >= 0");
  const size_t b = sizeof(float) * n;
  if (overlaps(state, 2 * b, grad_w, b) || overlaps(state, 2 * b, h->d_master, b) ||
      overlaps(grad_w, b, h->d_master, b))
    return fail(GN_E_INVAL, "grad_w, state and the handle's weights must not overlap");
  DeviceGuard dg(h->device);
  hipStream_t s = (hipStream_t)hip_stream;
  float c1, c2;
  gn::adam_bias_corrections(beta1, beta2, step, &c1, &c2);
  hipError_t e = gn::launch_adam(h->d_master, grad_w, state, state + n, (int64_t)n, c1, c2, lr,
                                 beta1, beta2, eps, weight_decay, s);
  if (e != hipSuccess) return gn_check_device(h, e, "adam launch");
  return gn_prepare_weights(h, s);
}

gn_status glassnet_adam_update(gn_handle *h, float *w, const float *grad_w, float *state,
                               size_t n, int32_t step, float lr, float beta1, float beta2,
                               float eps, float weight_decay, void *hip_stream) {
  gn_status st = precheck(h);
  if (st != GN_OK) return st;
  if (n < 1 || n > ((size_t)1 << 31)) return fail(GN_E_INVAL, "n must be in 1..2^31, got %zu", n);
  if (!w || !grad_w || !state || !aligned4(w) || !aligned4(grad_w) || !aligned4(state))
    return fail(GN_E_INVAL, "w, grad_w and state must be non-NULL 4-byte aligned device pointers");
  if (step < 1) return fail(GN_E_INVAL, "step %d must be >= 1", step);
  if (!(lr >= 0.0f && lr < 1e30f) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
      !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f && eps < 1e30f) ||
      !(weight_decay >= 0.0f && weight_decay < 1e30f))
    return fail(GN_E_INVAL, "need lr >= 0, 0 <= beta1, beta2 < 1, eps > 0, weight_decay >= 0");
  const size_t b = sizeof(float) * n;
  if (overlaps(state, 2 * b, grad_w, b) || overlaps(state, 2 * b, w, b) || overlaps(grad_w, b, w, b))
    return fail(GN_E_INVAL, "w, grad_w and state must not overlap");
  DeviceGuard dg(h->device);
  float c1, c2;
  gn::adam_bias_corrections(beta1, beta2, step, &c1, &c2);
  hipError_t e = gn::launch_adam(w, grad_w, state, state + n, (int64_t)n, c1, c2, lr, beta1, beta2,
                                 eps, weight_decay, (hipStream_t)hip_stream);
  return gn_check_device(h, e, "adam launch");
}

}  // extern "C"
