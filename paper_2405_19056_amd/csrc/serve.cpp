// Serving: the continuous-batching scheduler of serve_core.h driving the fused
// MFMA forward in tile-table mode on a library-owned HIP stream.
#include <string.h>

#include <memory>
#include <mutex>

#include "gn_api_state.h"
#include "serve_core.h"

namespace {

constexpr int kMaxInflight = 2;
constexpr int kChunkTiles = 1024;      // 262144 pixels per launch at most
constexpr int kMaxDescs = 8192;

static_assert(sizeof(gn::TileRef) == sizeof(gn::serve::Tile), "tile records must match");

class HipExecutor : public gn::serve::Executor {
 public:
  explicit HipExecutor(gn_handle *h) : h_(h) {}

  hipError_t init() {
    hipError_t e = hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipHostMalloc((void **)&h_descs_, sizeof(gn::FrameDesc) * kMaxDescs, 0);
    if (e == hipSuccess) e = hipMalloc((void **)&d_descs_, sizeof(gn::FrameDesc) * kMaxDescs);
    for (int s = 0; s < kMaxInflight && e == hipSuccess; ++s) {
      e = hipHostMalloc((void **)&h_tiles_[s], sizeof(gn::TileRef) * kChunkTiles, 0);
      if (e == hipSuccess) e = hipMalloc((void **)&d_tiles_[s], sizeof(gn::TileRef) * kChunkTiles);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_[s], hipEventDisableTiming);
    }
    return e;
  }

  ~HipExecutor() override {
    if (stream_) (void)hipStreamSynchronize(stream_);
    for (int s = 0; s < kMaxInflight; ++s) {
      if (ev_[s]) (void)hipEventDestroy(ev_[s]);
      (void)hipHostFree(h_tiles_[s]);
      (void)hipFree(d_tiles_[s]);
    }
    (void)hipHostFree(h_descs_);
    (void)hipFree(d_descs_);
    if (stream_) (void)hipStreamDestroy(stream_);
  }

  size_t device_bytes() const {
    return sizeof(gn::FrameDesc) * kMaxDescs + sizeof(gn::TileRef) * kChunkTiles * kMaxInflight;
  }

  int launch(int slot, const std::vector<std::pair<int32_t, gn::serve::FrameIn>> &new_descs,
             const gn::serve::Tile *tiles, int ntiles) override {
    (void)hipSetDevice(h_->device);
    hipError_t e = hipSuccess;
    for (const auto &nd : new_descs) {
      gn::FrameDesc &d = h_descs_[nd.first];
      d.g = nd.second.g;
      d.L = nd.second.L;
      d.s = nd.second.s;
      d.out = nd.second.out;
      d.hw = nd.second.hw;
      d.k = nd.second.k;
      d.pad0 = d.pad1 = 0;
      e = hipMemcpyAsync(d_descs_ + nd.first, &d, sizeof d, hipMemcpyHostToDevice, stream_);
      if (e != hipSuccess) return -1;
    }
    memcpy(h_tiles_[slot], tiles, sizeof(gn::TileRef) * ntiles);
    e = hipMemcpyAsync(d_tiles_[slot], h_tiles_[slot], sizeof(gn::TileRef) * ntiles,
                       hipMemcpyHostToDevice, stream_);
    if (e == hipSuccess)
      e = gn::launch_fwd_mfma(h_->W, h_->cfg.precision, h_->cfg.pool, h_->d_packed, h_->pl,
                              nullptr, d_descs_, d_tiles_[slot], ntiles, h_->act_scale,
                              h_->num_cus, h_->d_sig_scratch[1], gn_slot_kmax(h_), stream_);
    if (e == hipSuccess) e = hipEventRecord(ev_[slot], stream_);
    if (e != hipSuccess) {
      h_->poisoned = true;
      return -1;
    }
    return 0;
  }

  int query(int slot) override {
    const hipError_t e = hipEventQuery(ev_[slot]);
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) return 0;
    h_->poisoned = true;
    return -1;
  }

 private:
  gn_handle *h_;
  hipStream_t stream_ = nullptr;
  gn::FrameDesc *h_descs_ = nullptr, *d_descs_ = nullptr;
  gn::TileRef *h_tiles_[kMaxInflight] = {}, *d_tiles_[kMaxInflight] = {};
  hipEvent_t ev_[kMaxInflight] = {};
};

}  // namespace

struct GnServer {
  std::unique_ptr<HipExecutor> exec;
  std::unique_ptr<gn::serve::Scheduler> sched;
};

gn_status gn_serve_init(gn_handle *h) {
  (void)h;   // created on first submit
  return GN_OK;
}

void gn_serve_shutdown(gn_handle *h) {
  if (!h->server) return;
  h->server->sched->drain();
  h->server->sched->stop();
  h->server->sched.reset();
  h->server->exec.reset();
  delete h->server;
  h->server = nullptr;
}

static std::mutex g_init_mu;

static gn_status ensure_server(gn_handle *h) {
  std::lock_guard<std::mutex> lk(g_init_mu);
  if (h->server) return GN_OK;
  if (h->cfg.precision == GN_FP32)
    return gn_set_error(GN_E_UNSUPPORTED, "serving runs the fused MFMA forward (bf16 or fp8_t)");
  (void)hipSetDevice(h->device);
  auto *srv = new GnServer();
  srv->exec.reset(new HipExecutor(h));
  hipError_t e = srv->exec->init();
  if (e != hipSuccess) {
    delete srv;
    return gn_check_device(h, e, "serving setup");
  }
  gn::serve::Scheduler::Options o;
  o.budget_bytes = h->cfg.hbm_budget_bytes;
  o.max_pending = h->cfg.max_pending;
  o.chunk_tiles = kChunkTiles;
  o.max_inflight = kMaxInflight;
  o.max_descs = kMaxDescs;
  srv->sched.reset(new gn::serve::Scheduler(srv->exec.get(), o));
  h->bytes_held += srv->exec->device_bytes();
  h->server = srv;
  return GN_OK;
}

extern "C" {

gn_status serve_submit(gn_handle *h, const gn_frame *f, float *out, uint64_t *ticket) {
  if (!h || !ticket || !out) return gn_set_error(GN_E_INVAL, "handle, out and ticket must be non-NULL");
  if (h->poisoned) return gn_set_error(GN_E_DEVICE, "handle poisoned by an earlier device error");
  gn_status st = gn_validate_frame(h, f, out);
  if (st != GN_OK) return st;
  st = ensure_server(h);
  if (st != GN_OK) return st;
  const int64_t hw = (int64_t)f->h * f->w;
  std::vector<gn::serve::FrameIn> frames;
  frames.reserve(f->n);
  for (int i = 0; i < f->n; ++i) {
    gn::serve::FrameIn fi;
    fi.g = f->gbuf + (size_t)i * gn::kNG * hw;
    fi.L = f->layers ? f->layers + (size_t)i * f->k * gn::kNL * hw : nullptr;
    fi.s = f->scene + (size_t)i * gn::kNS;
    fi.out = out + (size_t)i * gn::kNOUT * hw;
    fi.hw = (int32_t)hw;
    fi.k = f->k;
    frames.push_back(fi);
  }
  const int rc = h->server->sched->submit(frames, ticket);
  if (rc == gn::serve::S_INVAL)
    return gn_set_error(GN_E_INVAL, "frame larger than the HBM budget (or too many frames)");
  if (rc == gn::serve::S_BUSY) return gn_set_error(GN_E_BUSY, "pending queue full");
  return rc;
}

gn_status serve_poll(gn_handle *h, uint64_t ticket, int32_t *done, gn_timing *timing) {
  if (!h || !done) return gn_set_error(GN_E_INVAL, "handle and done must be non-NULL");
  if (!h->server) return gn_set_error(GN_E_INVAL, "unknown ticket");
  gn::serve::Timing tm;
  int d = 0;
  const int rc = h->server->sched->poll(ticket, &d, &tm);
  if (rc == gn::serve::S_INVAL) return gn_set_error(GN_E_INVAL, "unknown ticket");
  *done = d;
  if (timing) {
    timing->t_submit = tm.t_submit;
    timing->t_admit = tm.t_admit;
    timing->t_start = tm.t_start;
    timing->t_done = tm.t_done;
  }
  if (rc == gn::serve::S_DEVICE) return gn_set_error(GN_E_DEVICE, "the ticket's work failed");
  return GN_OK;
}

gn_status serve_drain(gn_handle *h) {
  if (!h) return gn_set_error(GN_E_INVAL, "handle is NULL");
  if (!h->server) return GN_OK;
  const int rc = h->server->sched->drain();
  if (rc != 0) return gn_set_error(GN_E_DEVICE, "some served frames failed");
  return GN_OK;
}

gn_status serve_forget(gn_handle *h, uint64_t ticket) {
  if (!h) return gn_set_error(GN_E_INVAL, "handle is NULL");
  if (!h->server) return gn_set_error(GN_E_INVAL, "unknown ticket");
  const int rc = h->server->sched->forget(ticket);
  if (rc == gn::serve::S_INVAL) return gn_set_error(GN_E_INVAL, "unknown ticket");
  if (rc == gn::serve::S_AGAIN) return gn_set_error(GN_E_AGAIN, "ticket not finished");
  return GN_OK;
}

}  // extern "C"
