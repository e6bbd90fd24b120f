// Host-only harness: drives the serving scheduler with a fake executor so its
// admission, ordering, completion and failure logic can be tested on a CPU.
#include <atomic>
#include <mutex>
#include <vector>

#include "serve_core.h"

using namespace gn::serve;

namespace {

class FakeExecutor : public Executor {
 public:
  int launch(int slot, const std::vector<std::pair<int32_t, FrameIn>> &new_descs,
             const Tile *tiles, int ntiles) override {
    std::lock_guard<std::mutex> lk(mu);
    for (const auto &d : new_descs) desc_hw[d.first] = d.second.hw;
    for (int i = 0; i < ntiles; ++i) seen.push_back({desc_hw[tiles[i].desc], tiles[i].q0});
    if (fail_launch > 0) {
      --fail_launch;
      return -1;
    }
    state[slot] = 0;
    fail_this[slot] = fail_query > 0;
    if (fail_query > 0) --fail_query;
    return 0;
  }
  int query(int slot) override {
    std::lock_guard<std::mutex> lk(mu);
    if (hold) return 0;
    return fail_this[slot] ? -1 : 1;
  }
  std::mutex mu;
  std::vector<std::pair<int, int>> seen;   // (frame hw, q0) in launch order
  int desc_hw[1 << 16] = {};
  int state[16] = {};
  bool fail_this[16] = {};
  int fail_launch = 0, fail_query = 0;
  std::atomic<bool> hold{false};
};

struct Harness {
  FakeExecutor ex;
  Scheduler *s = nullptr;
  std::vector<float> dummy = std::vector<float>(16);
};

}  // namespace

extern "C" {

void *h_create(unsigned long long budget, int max_pending, int chunk, int inflight, int max_descs,
               int hold) {
  Harness *h = new Harness();
  h->ex.hold = hold != 0;
  Scheduler::Options o;
  o.budget_bytes = budget;
  o.max_pending = max_pending;
  o.chunk_tiles = chunk;
  o.max_inflight = inflight;
  o.max_descs = max_descs;
  o.idle_poll_s = 1e-5;
  h->s = new Scheduler(&h->ex, o);
  return h;
}

int h_submit(void *p, int hw, int k, int nframes, unsigned long long *ticket) {
  Harness *h = (Harness *)p;
  std::vector<FrameIn> fr(nframes, FrameIn{h->dummy.data(), h->dummy.data(), h->dummy.data(),
                                           h->dummy.data(), hw, k});
  uint64_t t = 0;
  int rc = h->s->submit(fr, &t);
  *ticket = t;
  return rc;
}

int h_poll(void *p, unsigned long long ticket, int *done, double *tm) {
  Timing t{};
  int rc = ((Harness *)p)->s->poll(ticket, done, &t);
  tm[0] = t.t_submit;
  tm[1] = t.t_admit;
  tm[2] = t.t_start;
  tm[3] = t.t_done;
  return rc;
}

int h_drain(void *p) { return ((Harness *)p)->s->drain(); }
int h_forget(void *p, unsigned long long t) { return ((Harness *)p)->s->forget(t); }
void h_hold(void *p, int hold) { ((Harness *)p)->ex.hold = hold != 0; }
void h_fail(void *p, int launches, int queries) {
  Harness *h = (Harness *)p;
  std::lock_guard<std::mutex> lk(h->ex.mu);
  h->ex.fail_launch = launches;
  h->ex.fail_query = queries;
}
unsigned long long h_max_inflight_bytes(void *p) { return ((Harness *)p)->s->max_in_flight_bytes(); }
long long h_launches(void *p) { return ((Harness *)p)->s->launches(); }
long long h_mixed(void *p) { return ((Harness *)p)->s->mixed_launches(); }
unsigned long long h_frame_bytes(int hw, int k) {
  return Scheduler::frame_bytes(FrameIn{nullptr, nullptr, nullptr, nullptr, hw, k});
}

// Tiles launched so far as (descriptor hw, q0) pairs.
int h_tiles(void *p, int *out, int max) {
  Harness *h = (Harness *)p;
  std::lock_guard<std::mutex> lk(h->ex.mu);
  int n = 0;
  for (const auto &t : h->ex.seen) {
    if (n >= max) break;
    out[2 * n] = t.first;
    out[2 * n + 1] = t.second;
    ++n;
  }
  return (int)h->ex.seen.size();
}

void h_destroy(void *p) {
  Harness *h = (Harness *)p;
  h->ex.hold = false;
  delete h->s;
  delete h;
}
}
