// Frame-ring accounting of one serving-loop stream (pure C++, no HIP).
//
// The paper's input queue is a ring FIFO in GPU memory, fed in frame
// packets and drained in batches, sized so that it never overflows
// (Sec. II-B.1, Sec. III-A).  This class holds the bookkeeping of such a
// ring for windowed processing:
//   - frame f lives in ring slot f mod R; frames with f mod R < W - s are
//     also mirrored to slot R + (f mod R), so every window (which starts at a
//     multiple of the stride s, and R is a multiple of s) is contiguous;
//   - window j covers frames [j s, j s + W) and is complete once frame
//     j s + W - 1 has been pushed;
//   - windows complete on the device in launch order, so every frame below
//     done_windows * s is free; a push that would overwrite a frame at or
//     above that mark is refused (counted, never silent).
// The executor (GPU launches, or a fake in the CPU tests) drives it through
// take_ready() and mark_done().
#pragma once
#include <cstdint>
#include <mutex>
#include <vector>

namespace hvs {

struct Span {          // a contiguous run of frames in the ring
  int64_t first_frame;
  int slot;            // ring slot of first_frame
  int count;
};

struct WindowGroup {   // consecutive windows launched together
  int64_t first_window;
  int count;
  int slot;            // ring slot of the first window's first frame
  int64_t last_arrival_ns;  // arrival of the last frame of the last window
};

class RingLogic {
 public:
  RingLogic(int ring_frames, int window, int stride, int max_group)
      : R_(ring_frames), W_(window), S_(stride), G_(max_group), arrival_(ring_frames, 0) {}

  bool valid() const { return R_ > 0 && W_ > 0 && S_ > 0 && S_ <= W_ && R_ % S_ == 0 && R_ >= W_ && G_ > 0; }
  int ring_frames() const { return R_; }
  int mirror_frames() const { return W_ - S_; }
  int slots_total() const { return R_ + W_ - S_; }

  enum class Push { ok, full, failed };

  // Reserve n frames; on success returns the spans to copy (primary and
  // mirror) and records the arrival times.  Returns full (and counts the
  // drop) when the ring has no room, failed (nothing counted) once the
  // stream has been marked failed.
  Push push(int n, const int64_t* arrival_ns, int64_t now_ns, std::vector<Span>& copies) {
    std::lock_guard<std::mutex> g(mu_);
    copies.clear();
    if (failed_) return Push::failed;
    if (n <= 0) return Push::ok;
    const int64_t need_from = done_windows_ * S_;
    if (pushed_ + n - need_from > R_) {
      dropped_ += n;
      return Push::full;
    }
    int64_t f = pushed_;
    int left = n;
    while (left > 0) {
      const int slot = (int)(f % R_);
      const int run = left < R_ - slot ? left : R_ - slot;
      copies.push_back({f, slot, run});
      // mirror of the slots below W - s
      if (slot < W_ - S_) {
        const int mr = run < (W_ - S_) - slot ? run : (W_ - S_) - slot;
        copies.push_back({f, R_ + slot, mr});
      }
      f += run;
      left -= run;
    }
    for (int i = 0; i < n; ++i) arrival_[(pushed_ + i) % R_] = arrival_ns ? arrival_ns[i] : now_ns;
    pushed_ += n;
    accepted_ += n;
    return Push::ok;
  }

  // Complete windows not yet launched, grouped so that a group never crosses
  // the end of the ring and holds at most max_group windows.  Nothing is
  // handed out once the stream has failed.
  bool take_ready(WindowGroup& out) {
    std::lock_guard<std::mutex> g(mu_);
    if (failed_) return false;
    const int64_t complete = pushed_ >= W_ ? (pushed_ - W_) / S_ + 1 : 0;
    if (launched_ >= complete) return false;
    const int slot = (int)((launched_ * S_) % R_);
    // windows starting at slots slot, slot + s, ... up to R - s
    const int64_t room = (R_ - slot) / S_;
    int64_t cnt = complete - launched_;
    if (cnt > G_) cnt = G_;
    if (cnt > room) cnt = room;
    out.first_window = launched_;
    out.count = (int)cnt;
    out.slot = slot;
    const int64_t last_frame = (launched_ + cnt - 1) * S_ + W_ - 1;
    out.last_arrival_ns = arrival_[last_frame % R_];
    launched_ += cnt;
    return true;
  }

  // Arrival time of the last frame of window j (must still be in the ring).
  int64_t window_arrival(int64_t j) const {
    std::lock_guard<std::mutex> g(mu_);
    return arrival_[(j * S_ + W_ - 1) % R_];
  }

  // The device finished windows [.., first + count); they complete in order.
  void mark_done(int64_t first, int count) {
    std::lock_guard<std::mutex> g(mu_);
    if (first == done_windows_) done_windows_ += count;
  }

  // The launch of group g (the last one taken) could not be issued: its
  // windows go back to "not launched" and the stream is marked failed, so
  // later pushes are refused as a failed stream instead of being counted
  // as drops of a ring that would never drain.
  void abandon(const WindowGroup& grp) {
    std::lock_guard<std::mutex> g(mu_);
    if (launched_ == grp.first_window + grp.count) launched_ = grp.first_window;
    failed_ = true;
  }
  // A device error was reported for work already launched.
  void set_failed() {
    std::lock_guard<std::mutex> g(mu_);
    failed_ = true;
  }
  bool failed() const { std::lock_guard<std::mutex> g(mu_); return failed_; }

  int64_t pushed() const { std::lock_guard<std::mutex> g(mu_); return pushed_; }
  int64_t dropped() const { std::lock_guard<std::mutex> g(mu_); return dropped_; }
  int64_t launched() const { std::lock_guard<std::mutex> g(mu_); return launched_; }
  int64_t done() const { std::lock_guard<std::mutex> g(mu_); return done_windows_; }
  int64_t windows_possible() const {
    std::lock_guard<std::mutex> g(mu_);
    return pushed_ >= W_ ? (pushed_ - W_) / S_ + 1 : 0;
  }

 private:
  const int R_, W_, S_, G_;
  mutable std::mutex mu_;
  std::vector<int64_t> arrival_;
  int64_t pushed_ = 0, accepted_ = 0, dropped_ = 0;
  int64_t launched_ = 0, done_windows_ = 0;
  bool failed_ = false;
};

// Latency samples with percentiles (nearest-rank).
class LatencyLog {
 public:
  void add(int64_t ns) {
    std::lock_guard<std::mutex> g(mu_);
    v_.push_back(ns);
  }
  void clear() {
    std::lock_guard<std::mutex> g(mu_);
    v_.clear();
  }
  size_t size() const {
    std::lock_guard<std::mutex> g(mu_);
    return v_.size();
  }
  // p in [0, 100]; nearest-rank percentile, 0 when empty
  int64_t percentile(double p) const;

 private:
  mutable std::mutex mu_;
  std::vector<int64_t> v_;
};

}  // namespace hvs

#include <algorithm>
#include <cmath>

inline int64_t hvs::LatencyLog::percentile(double p) const {
  std::vector<int64_t> c;
  {
    std::lock_guard<std::mutex> g(mu_);
    c = v_;
  }
  if (c.empty()) return 0;
  std::sort(c.begin(), c.end());
  size_t rank = (size_t)std::ceil(p / 100.0 * (double)c.size());
  if (rank < 1) rank = 1;
  if (rank > c.size()) rank = c.size();
  return c[rank - 1];
}
