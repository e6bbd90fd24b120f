// Continuous-batching scheduler for frame requests (host logic only).
//
// Requests are frames (or small batches of frames) whose inputs are already
// resident in device memory.  A scheduler thread
//   1. admits pending requests in arrival order while the bytes of admitted,
//      unfinished requests stay within the HBM budget;
//   2. cuts the admitted requests into tiles of kTilePx pixels and appends
//      them to one work list, so tiles of frames of any size and slot count
//      share launches;
//   3. keeps up to `max_inflight` launches of at most `chunk_tiles` tiles in
//      flight, each completing asynchronously;
//   4. on completion credits every request with its tiles and finishes a
//      request when all of its tiles are done (or fails it if a launch that
//      held its tiles failed).
// The device side is an Executor, so the same logic runs against the HIP
// executor or a fake one in host-only tests.
#pragma once

#include <stdint.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace gn {
namespace serve {

constexpr int kServeTilePx = 256;

struct FrameIn {
  const float *g, *L, *s;
  float *out;
  int32_t hw, k;
};

struct Tile {
  int32_t desc;   // descriptor slot of the frame
  int32_t q0;     // first pixel of the tile
};

struct Timing {
  double t_submit, t_admit, t_start, t_done;
};

// Device side.  launch() receives the descriptors that must be visible to the
// device before the tiles run (newly admitted frames) and the tiles.
class Executor {
 public:
  virtual ~Executor() = default;
  // Returns 0 on success.  `slot` identifies the launch buffer (< max_inflight).
  virtual int launch(int slot, const std::vector<std::pair<int32_t, FrameIn>> &new_descs,
                     const Tile *tiles, int ntiles) = 0;
  // 1 = finished, 0 = still running, < 0 = failed.
  virtual int query(int slot) = 0;
};

enum { REQ_PENDING = 0, REQ_ADMITTED = 1, REQ_DONE = 2, REQ_FAILED = 3 };
enum { S_OK = 0, S_INVAL = -1, S_DEVICE = -3, S_AGAIN = -5, S_BUSY = -6 };

inline double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

class Scheduler {
 public:
  struct Options {
    uint64_t budget_bytes = (uint64_t)64 << 30;
    int max_pending = 65536;
    int chunk_tiles = 1024;
    int max_inflight = 2;
    int max_descs = 8192;
    double idle_poll_s = 20e-6;   // event polling period while launches are in flight
  };

  Scheduler(Executor *ex, const Options &o) : ex_(ex), opt_(o) {
    for (int i = o.max_descs - 1; i >= 0; --i) free_descs_.push_back(i);
    slots_.resize(o.max_inflight);
    thread_ = std::thread([this] { run(); });
  }

  ~Scheduler() { stop(); }

  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stopping_) return;
      stopping_ = true;
    }
    cv_.notify_all();
    if (thread_.joinable()) thread_.join();
  }

  static uint64_t frame_bytes(const FrameIn &f) {
    return (uint64_t)4 * ((uint64_t)f.hw * (14 + 12 * (uint64_t)f.k + 3) + 16);
  }

  int submit(const std::vector<FrameIn> &frames, uint64_t *ticket) {
    uint64_t bytes = 0;
    int64_t tiles = 0;
    for (const FrameIn &f : frames) {
      bytes += frame_bytes(f);
      tiles += (f.hw + kServeTilePx - 1) / kServeTilePx;
    }
    std::lock_guard<std::mutex> lk(mu_);
    if (stopping_) return S_INVAL;
    if (bytes > opt_.budget_bytes || (int)frames.size() > opt_.max_descs) return S_INVAL;
    if ((int)pending_.size() >= opt_.max_pending) return S_BUSY;
    const uint64_t t = ++next_ticket_;
    Req &r = reqs_[t];
    r.frames = frames;
    r.bytes = bytes;
    r.tiles_left = tiles;
    r.tm.t_submit = now_s();
    pending_.push_back(t);
    ++outstanding_;
    *ticket = t;
    cv_.notify_all();
    return S_OK;
  }

  int poll(uint64_t ticket, int *done, Timing *tm) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return S_INVAL;
    const Req &r = it->second;
    if (tm) *tm = r.tm;
    if (r.state == REQ_FAILED) {
      *done = 1;
      return S_DEVICE;
    }
    *done = r.state == REQ_DONE;
    return S_OK;
  }

  int forget(uint64_t ticket) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return S_INVAL;
    if (it->second.state != REQ_DONE && it->second.state != REQ_FAILED) return S_AGAIN;
    reqs_.erase(it);
    return S_OK;
  }

  // Waits until every submitted request finished; returns S_DEVICE if any failed.
  int drain() {
    std::unique_lock<std::mutex> lk(mu_);
    done_cv_.wait(lk, [this] { return outstanding_ == 0; });
    return failed_since_drain_ ? (failed_since_drain_ = false, S_DEVICE) : S_OK;
  }

  // Introspection for tests.
  uint64_t in_flight_bytes() {
    std::lock_guard<std::mutex> lk(mu_);
    return inflight_bytes_;
  }
  uint64_t max_in_flight_bytes() {
    std::lock_guard<std::mutex> lk(mu_);
    return max_inflight_bytes_;
  }
  int64_t launches() {
    std::lock_guard<std::mutex> lk(mu_);
    return n_launches_;
  }
  int64_t mixed_launches() {
    std::lock_guard<std::mutex> lk(mu_);
    return n_mixed_launches_;
  }

 private:
  struct Req {
    std::vector<FrameIn> frames;
    std::vector<int32_t> descs;
    uint64_t bytes = 0;
    int64_t tiles_left = 0;
    int state = REQ_PENDING;
    Timing tm{0, 0, 0, 0};
  };
  struct WorkTile {
    Tile tile;
    uint64_t ticket;
  };
  struct Slot {
    bool busy = false;
    std::vector<std::pair<uint64_t, int64_t>> credit;   // ticket -> tiles in this launch
  };

  void admit_locked() {
    while (!pending_.empty()) {
      const uint64_t t = pending_.front();
      Req &r = reqs_[t];
      if (inflight_bytes_ + r.bytes > opt_.budget_bytes) break;          // FIFO: wait
      if ((int)free_descs_.size() < (int)r.frames.size()) break;
      pending_.pop_front();
      r.state = REQ_ADMITTED;
      r.tm.t_admit = now_s();
      inflight_bytes_ += r.bytes;
      if (inflight_bytes_ > max_inflight_bytes_) max_inflight_bytes_ = inflight_bytes_;
      for (const FrameIn &f : r.frames) {
        const int32_t d = free_descs_.back();
        free_descs_.pop_back();
        r.descs.push_back(d);
        new_descs_.push_back({d, f});
        for (int32_t q0 = 0; q0 < f.hw; q0 += kServeTilePx) work_.push_back({{d, q0}, t});
      }
      if (r.frames.empty()) finish_locked(t, r, REQ_DONE);
    }
  }

  void launch_locked() {
    for (int s = 0; s < (int)slots_.size() && !work_.empty(); ++s) {
      Slot &sl = slots_[s];
      if (sl.busy) continue;
      const int n = (int)std::min<size_t>(work_.size(), (size_t)opt_.chunk_tiles);
      tiles_.resize(n);
      sl.credit.clear();
      const double t = now_s();
      for (int i = 0; i < n; ++i) {
        const WorkTile &wt = work_.front();
        tiles_[i] = wt.tile;
        if (sl.credit.empty() || sl.credit.back().first != wt.ticket) {
          sl.credit.push_back({wt.ticket, 0});
          Req &r = reqs_[wt.ticket];
          if (r.tm.t_start == 0) r.tm.t_start = t;
        }
        sl.credit.back().second += 1;
        work_.pop_front();
      }
      ++n_launches_;
      if (sl.credit.size() > 1) ++n_mixed_launches_;
      const int rc = ex_->launch(s, new_descs_, tiles_.data(), n);
      new_descs_.clear();
      if (rc != 0) {
        fail_slot_locked(sl);
      } else {
        sl.busy = true;
      }
    }
  }

  void poll_locked() {
    for (Slot &sl : slots_) {
      if (!sl.busy) continue;
    }
    for (int s = 0; s < (int)slots_.size(); ++s) {
      Slot &sl = slots_[s];
      if (!sl.busy) continue;
      const int q = ex_->query(s);
      if (q == 0) continue;
      sl.busy = false;
      if (q < 0) {
        fail_slot_locked(sl);
        continue;
      }
      for (auto &c : sl.credit) {
        Req &r = reqs_[c.first];
        if (r.state != REQ_ADMITTED) continue;
        r.tiles_left -= c.second;
        if (r.tiles_left == 0) finish_locked(c.first, r, REQ_DONE);
      }
      sl.credit.clear();
    }
  }

  void fail_slot_locked(Slot &sl) {
    for (auto &c : sl.credit) {
      Req &r = reqs_[c.first];
      if (r.state == REQ_ADMITTED) finish_locked(c.first, r, REQ_FAILED);
    }
    sl.credit.clear();
    sl.busy = false;
  }

  void finish_locked(uint64_t ticket, Req &r, int state) {
    r.state = state;
    r.tm.t_done = now_s();
    if (state == REQ_FAILED) {
      failed_since_drain_ = true;
      // drop this request's tiles that have not been launched yet
      std::deque<WorkTile> keep;
      for (const WorkTile &w : work_)
        if (w.ticket != ticket) keep.push_back(w);
      work_.swap(keep);
    }
    inflight_bytes_ -= r.bytes;
    for (int32_t d : r.descs) free_descs_.push_back(d);
    r.descs.clear();
    --outstanding_;
    done_cv_.notify_all();
  }

  bool any_busy_locked() const {
    for (const Slot &s : slots_)
      if (s.busy) return true;
    return false;
  }

  void run() {
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      admit_locked();
      poll_locked();
      admit_locked();       // completions may have freed budget
      launch_locked();
      const bool busy = any_busy_locked();
      if (stopping_ && !busy && pending_.empty() && work_.empty()) break;
      if (busy) {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::duration<double>(opt_.idle_poll_s));
        lk.lock();
      } else if (pending_.empty() && work_.empty()) {
        cv_.wait(lk, [this] { return stopping_ || !pending_.empty(); });
      } else if (!pending_.empty() && work_.empty()) {
        // head of the queue does not fit and nothing is running: it never will
        // fit unless budget frees, which cannot happen -- fail it
        const uint64_t t = pending_.front();
        pending_.pop_front();
        Req &r = reqs_[t];
        r.state = REQ_FAILED;
        r.tm.t_done = now_s();
        failed_since_drain_ = true;
        --outstanding_;
        done_cv_.notify_all();
      }
    }
  }

  Executor *ex_;
  Options opt_;
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  std::thread thread_;
  bool stopping_ = false;
  uint64_t next_ticket_ = 0;
  std::unordered_map<uint64_t, Req> reqs_;
  std::deque<uint64_t> pending_;
  std::deque<WorkTile> work_;
  std::vector<std::pair<int32_t, FrameIn>> new_descs_;
  std::vector<int32_t> free_descs_;
  std::vector<Slot> slots_;
  std::vector<Tile> tiles_;
  uint64_t inflight_bytes_ = 0, max_inflight_bytes_ = 0;
  int64_t outstanding_ = 0;
  int64_t n_launches_ = 0, n_mixed_launches_ = 0;
  bool failed_since_drain_ = false;
};

}  // namespace serve
}  // namespace gn
