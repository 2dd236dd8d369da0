// Host-only test of the serving-loop ring accounting (stream_ring.h) with a
// fake executor: no GPU, no HIP.  Built with g++ under AddressSanitizer +
// UndefinedBehaviorSanitizer and under ThreadSanitizer by
// tests/test_stream_logic.py.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "stream_ring.h"

using hvs::RingLogic;
using hvs::Span;
using hvs::WindowGroup;
using Push = hvs::RingLogic::Push;

static int failures = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "%s:%d CHECK failed: %s\n", __FILE__, __LINE__, #c); \
      ++failures;                                                  \
    }                                                              \
  } while (0)

// Device ring stand-in: slot -> frame id.
struct FakeRing {
  std::vector<int64_t> slot;
  explicit FakeRing(int n) : slot(n, -1) {}
  void apply(const std::vector<Span>& c) {
    for (const Span& s : c)
      for (int i = 0; i < s.count; ++i) slot[s.slot + i] = s.first_frame + i;
  }
};

static bool window_ok(const FakeRing& fr, int slot, int64_t first_frame, int W) {
  for (int i = 0; i < W; ++i)
    if (fr.slot[slot + i] != first_frame + i) return false;
  return true;
}

static void test_contiguity(int R, int W, int S, int G) {
  RingLogic r(R, W, S, G);
  CHECK(r.valid());
  FakeRing fr(r.slots_total());
  std::mt19937 rng(R * 31 + W * 7 + S);
  std::vector<Span> copies;
  int64_t windows = 0, refused = 0;
  for (int it = 0; it < 400; ++it) {
    const int n = 1 + (int)(rng() % (unsigned)(S + 5));
    if (r.push(n, nullptr, it, copies) != Push::ok) {
      refused += n;
      // drain everything launched, then retry
      WindowGroup g;
      while (r.take_ready(g)) {
        for (int k = 0; k < g.count; ++k) CHECK(window_ok(fr, g.slot + k * S, (g.first_window + k) * S, W));
        r.mark_done(g.first_window, g.count);
        windows += g.count;
      }
      CHECK(r.push(n, nullptr, it, copies) == Push::ok);
    }
    fr.apply(copies);
    if (rng() % 3 == 0) {
      WindowGroup g;
      while (r.take_ready(g)) {
        CHECK(g.count >= 1 && g.count <= G);
        CHECK(g.slot + (g.count - 1) * S <= R - S);  // never crosses the ring end
        for (int k = 0; k < g.count; ++k) CHECK(window_ok(fr, g.slot + k * S, (g.first_window + k) * S, W));
        r.mark_done(g.first_window, g.count);
        windows += g.count;
      }
    }
  }
  WindowGroup g;
  while (r.take_ready(g)) {
    for (int k = 0; k < g.count; ++k) CHECK(window_ok(fr, g.slot + k * S, (g.first_window + k) * S, W));
    r.mark_done(g.first_window, g.count);
    windows += g.count;
  }
  CHECK(windows == (r.pushed() - W) / S + 1);
  CHECK(r.dropped() == refused);
}

static void test_overflow_counted() {
  RingLogic r(32, 16, 16, 2);
  std::vector<Span> c;
  CHECK(r.push(40, nullptr, 0, c) == Push::full);  // larger than the ring
  CHECK(r.dropped() == 40 && r.pushed() == 0);
  CHECK(r.push(32, nullptr, 0, c) == Push::ok);
  CHECK(r.push(1, nullptr, 0, c) == Push::full);  // nothing consumed yet
  CHECK(r.dropped() == 41);
  WindowGroup g;
  CHECK(r.take_ready(g) && g.first_window == 0 && g.count == 2);
  CHECK(r.push(1, nullptr, 0, c) == Push::full);  // launched but not done: still needed
  r.mark_done(0, 1);
  CHECK(r.push(16, nullptr, 0, c) == Push::ok);  // window 0's frames are free now
  CHECK(r.push(1, nullptr, 0, c) == Push::full);
  r.mark_done(1, 1);
  CHECK(r.push(16, nullptr, 0, c) == Push::ok);
  CHECK(r.dropped() == 43);
}

static void test_arrival_and_percentiles() {
  RingLogic r(64, 16, 8, 4);
  std::vector<Span> c;
  std::vector<int64_t> arr(24);
  for (int i = 0; i < 24; ++i) arr[i] = 1000 + i;
  CHECK(r.push(24, arr.data(), 0, c) == Push::ok);
  WindowGroup g;
  CHECK(r.take_ready(g) && g.first_window == 0 && g.count == 2);
  CHECK(r.window_arrival(0) == 1015 && r.window_arrival(1) == 1023 && g.last_arrival_ns == 1023);
  hvs::LatencyLog l;
  for (int i = 1; i <= 100; ++i) l.add(i);
  CHECK(l.percentile(50) == 50 && l.percentile(99) == 99 && l.percentile(100) == 100);
  l.clear();
  CHECK(l.percentile(99) == 0);
  l.add(7);
  CHECK(l.percentile(1) == 7 && l.percentile(99) == 7);
}

// Producer and executor threads; the executor completes groups after a
// delay.  Every refused packet is counted exactly; with backpressure (the
// producer retries a refused packet) every frame is eventually processed,
// and a slow executor without backpressure makes the ring refuse packets.
static void test_threads(bool slow) {
  const int R = 64, W = 16, S = 16;
  RingLogic r(R, W, S, 3);
  FakeRing fr(r.slots_total());
  std::mutex fr_mu;
  std::atomic<bool> done{false};
  std::atomic<int64_t> refused{0}, accepted{0};
  std::atomic<int> bad{0};
  std::thread prod([&] {
    std::mt19937 rng(5);
    std::vector<Span> c;
    for (int it = 0; it < 3000; ++it) {
      const int n = 1 + (int)(rng() % 7u);
      for (;;) {
        bool ok;
        {
          std::lock_guard<std::mutex> g(fr_mu);
          ok = r.push(n, nullptr, it, c) == Push::ok;
          if (ok) {
            fr.apply(c);
            accepted += n;
          } else {
            refused += n;
          }
        }
        if (ok || slow) break;
        std::this_thread::sleep_for(std::chrono::microseconds(50));  // backpressure: retry
      }
    }
    done = true;
  });
  std::thread exec([&] {
    WindowGroup g;
    for (;;) {
      bool any = false;
      while (r.take_ready(g)) {
        any = true;
        std::this_thread::sleep_for(std::chrono::microseconds(slow ? 400 : 5));
        {
          std::lock_guard<std::mutex> lk(fr_mu);
          for (int k = 0; k < g.count; ++k)
            if (!window_ok(fr, g.slot + k * S, (g.first_window + k) * S, W)) bad++;
        }
        r.mark_done(g.first_window, g.count);
      }
      if (!any && done.load() && r.launched() == r.windows_possible()) break;
      if (!any) std::this_thread::sleep_for(std::chrono::microseconds(10));
    }
  });
  prod.join();
  exec.join();
  CHECK(bad.load() == 0);
  CHECK(r.dropped() == refused.load());
  CHECK(r.pushed() == accepted.load());
  CHECK(r.done() == r.windows_possible());
  if (slow) CHECK(refused.load() > 0);
  else CHECK(r.pushed() == accepted.load() && accepted.load() > 0);
}

// A launch that cannot be issued: the group goes back to "not launched",
// the stream is marked failed, and later pushes report the failure without
// being counted as drops; nothing more is handed to the executor.
static void test_launch_failure() {
  RingLogic r(64, 16, 16, 2);
  std::vector<Span> c;
  CHECK(r.push(32, nullptr, 0, c) == Push::ok);
  WindowGroup g;
  CHECK(r.take_ready(g) && g.first_window == 0 && g.count == 2);
  CHECK(r.launched() == 2);
  r.abandon(g);
  CHECK(r.failed() && r.launched() == 0);
  CHECK(r.push(16, nullptr, 0, c) == Push::failed);
  CHECK(r.dropped() == 0 && r.pushed() == 32);
  CHECK(!r.take_ready(g));
  // a device error on work already in flight also stops the stream
  RingLogic q(64, 16, 16, 2);
  CHECK(q.push(16, nullptr, 0, c) == Push::ok);
  CHECK(q.take_ready(g) && g.count == 1);
  q.set_failed();
  CHECK(q.push(16, nullptr, 0, c) == Push::failed && q.dropped() == 0);
  CHECK(!q.take_ready(g));
}

int main() {
  test_contiguity(64, 16, 16, 4);
  test_contiguity(48, 16, 8, 3);
  test_contiguity(60, 20, 5, 2);
  test_contiguity(192, 64, 64, 1);
  test_contiguity(128, 32, 1, 8);
  test_overflow_counted();
  test_arrival_and_percentiles();
  test_launch_failure();
  test_threads(false);
  test_threads(true);
  RingLogic bad_cfg(50, 16, 16, 1);
  CHECK(!bad_cfg.valid());
  if (failures) {
    std::fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  std::printf("stream logic: all checks passed\n");
  return 0;
}
