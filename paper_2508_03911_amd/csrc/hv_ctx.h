// Context, plans and workspaces behind the hv_ctx handle (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <string>
#include <memory>
#include <mutex>
#include <tuple>
#include <utility>
#include <vector>

#include "hv_internal.h"

namespace hvi {

// A device allocation that only grows.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf();
  void release();
  // Make room for `want` bytes (contents are not preserved); `accounted`
  // tracks the bytes held by the owner.
  hv_status ensure(size_t want, size_t* accounted);
  hv_status upload(const void* host, size_t n, size_t* accounted);
};

struct AsPlan {
  int ny = 0, nx = 0;
  double wavelength = 0, dx = 0, dy = 0, z = 0;
  double highpass = 0;  // radius in cycles per pixel, folded into the tables (0 = none)
  DevBuf ht;  // [nx][ny] float2: H_z(fx = column, fy) * mask / ny
  DevBuf hs;  // [2][nx/2][ny] float2: H_z(fx, fy) / ny, then H_z(-fx, fy) / ny (fx = 0: nx/2)
  const float2* ht_ptr() const { return (const float2*)ht.ptr; }
  const float2* hs_ptr() const { return (const float2*)hs.ptr; }
};

struct FresnelPlan {
  int ny = 0, nx = 0;
  double wavelength = 0, dx = 0, dy = 0, z = 0;
  DevBuf tables;  // float2: qx_in[nx], qy_in[ny], qx_out[nx], qy_out[ny]
};

struct DftPlan {
  int window = 0, mtiles = 0;
  std::vector<int> bins;
  std::vector<double> freqs;
  DevBuf a32, a16hi, a16lo, wts;
  // real-input fragments for the band-first order: A[2b + c][t] =
  // (cos, -sin)(2 pi k_b t / W), [mtiles][max(1, W/16)][64] fp16x8 (hi, lo)
  DevBuf ar_hi, ar_lo;
};

int band_bins(const hv_temporal& tp, std::vector<int>& bins, std::vector<double>& freqs);
// Positive wavelength and pitches, finite z, a known method, z != 0 for
// Fresnel, a high-pass radius in [0, 1) and only with the angular spectrum.
hv_status check_optics(const hv_optics* o);
const char* last_error();

struct ServeState;  // serving loop (stream.cpp)
void serve_shutdown(struct Ctx* c);

// Optional per-kernel timing with HIP events recorded around each launch on
// the caller's stream (no work is skipped or reordered).
struct Timing {
  bool on = false;
  struct Rec {
    const char* name;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  std::map<std::string, std::pair<double, long>> acc;  // total ms, launches
  hipEvent_t take();  // null if no event could be created
  void give_back(hipEvent_t e) {
    if (e) pool.push_back(e);
  }
  void collect();
  void reset();
  ~Timing();
};

struct Ctx {
  std::recursive_mutex mu;  // plans, workspaces and launches (the serving loop uses several threads)
  ServeState* serve = nullptr;
  Timing timing;
  int device = 0;
  size_t budget = 0;
  size_t held = 0;  // bytes of plans and workspaces
  int chunk_frames = 0;
  int stft_order = HV_ORDER_FRAMES_FIRST;  // HV_ORDER_*: the paper's per-frame order unless asked
  using OptKey = std::tuple<int, int, double, double, double, double, double>;
  std::map<OptKey, std::unique_ptr<AsPlan>> as_plans;
  std::map<OptKey, std::unique_ptr<FresnelPlan>> fr_plans;
  std::map<std::tuple<int, std::vector<int>, std::vector<double>>, std::unique_ptr<DftPlan>> dft_plans;
  std::map<std::pair<void*, int>, DevBuf> ws;
  std::map<std::string, DevBuf> misc;  // other float64-built tables (autofocus)

  // A second stream per caller stream.  The chunks of one call alternate
  // between the caller's stream and this one (fork and join by events,
  // default priority), so one chunk's kernels overlap the next chunk's.
  struct Lane2 {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    // The second stream waits for everything queued on `from` so far.
    hv_status fork_from(hipStream_t from);
    // `to` waits for everything queued on the second stream so far.
    hv_status join_into(hipStream_t to);
  };
  std::map<void*, Lane2> lanes;

  Ctx() = default;
  Ctx(const Ctx&) = delete;
  Ctx& operator=(const Ctx&) = delete;
  ~Ctx();
  Lane2* lane2(hipStream_t caller, hv_status* st);
  // Plans are built on first use; with build = false a missing plan is an
  // HV_ERR_STATE error instead (nothing is allocated).
  AsPlan* as_plan(int ny, int nx, const hv_optics& o, hv_status* st, bool build = true);
  FresnelPlan* fresnel_plan(int ny, int nx, const hv_optics& o, hv_status* st, bool build = true);
  DftPlan* dft_plan(const hv_temporal& tp, hv_status* st, bool build = true);
  DevBuf& work(hipStream_t s, int slot);
  int chunk_frames_for(int ny, int nx, bool mixed) const;
};

// Runs f() (a kernel launch), bracketed by timing events when enabled.
template <class F>
hv_status timed(Ctx* c, const char* name, hipStream_t st, F&& f) {
  if (!c->timing.on) return f();
  hipEvent_t a = c->timing.take(), b = c->timing.take();
  // timing is diagnostic: a launch whose events cannot be recorded runs
  // untimed
  const bool ra = a && b && hipEventRecord(a, st) == hipSuccess;
  hv_status s = f();
  if (ra && hipEventRecord(b, st) == hipSuccess) {
    c->timing.pending.push_back({name, a, b});
  } else {
    (void)hipGetLastError();
    c->timing.give_back(a);
    c->timing.give_back(b);
  }
  return s;
}

// Row C2C FFT of sign dir with an optional separable chirp (qx[m] qy[n]),
// transposed write [n][nx][ny]; input u8, u16 or c64.
hv_status launch_rows_c2c(const void* in, int in_t, void* out, bool half_out, const float2* qx, const float2* qy,
                          int dir, int n, int ny, int nx, float scale, hipStream_t st);
// Column pass for a full complex spectrum [n][nx][ny]: column FFT, multiply
// by ht[column][fy], inverse column FFT, write [n][ny][nx].
hv_status launch_col_full(const void* in, void* out, bool half_io, const float2* ht, int n, int ny, int nx,
                          hipStream_t st);

}  // namespace hvi

struct hv_ctx : hvi::Ctx {};

extern "C" hv_status hvi_stft_common(hv_ctx* ctx, const void* in, int in_t, int n, int ny, int nx,
                                     const hv_optics* optics, const hv_temporal* tp, int prec, float* m0, float* m1,
                                     float* m2, float2* spec, void* hip_stream);
