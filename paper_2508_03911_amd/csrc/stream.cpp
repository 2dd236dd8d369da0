// Multi-stream serving loop: device frame rings, HBM-budget admission,
// window launches and frame-to-image latency.
//
// The paper decouples acquisition from computation with a GPU-resident
// input ring fed packet by packet and drained batch by batch, uses separate
// streams for transfers and kernels, and requires zero frame loss
// (Sec. II-B.1, II-B.4, III-A; the zero-drop run of Sec. VIII).  Here each
// camera stream owns: a device ring of raw frames (accounting in
// stream_ring.h), its own HIP stream, preallocated workspaces, and a ring of
// output images.  A push copies a packet into the ring (device to device)
// and immediately launches every window it completes; a poller thread
// timestamps completions from HIP events and frees ring space in order.
// Admission charges each stream's ring, images and workspaces against the
// context's HBM budget.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "hv_ctx.h"
#include "hv_internal.h"
#include "stream_ring.h"

using hvi::fail;

static int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct hv_stream {
  hv_ctx* ctx = nullptr;
  int ny = 0, nx = 0, raw_t = 0, prec = 0;
  size_t frame_bytes = 0;
  hv_optics optics{};
  hv_temporal tp{};
  int out_slots = 0;     // output image slots (ring of windows)
  int keep_ready = 4;    // completed, unpopped images kept
  hvs::RingLogic ring;
  hipStream_t st = nullptr;
  hipStream_t up = nullptr;  // uploads of frames pushed from host memory
  void* ring_dev = nullptr;
  float* out_dev[3] = {nullptr, nullptr, nullptr};
  size_t admitted_bytes = 0;
  std::mutex push_mu;  // one pusher at a time
  struct Pending {
    hipEvent_t ev;
    hvs::WindowGroup g;
  };
  struct Ready {
    int64_t window, t_last, t_done;
  };
  std::mutex mu;  // pending / ready
  std::deque<Pending> pending;
  std::deque<Ready> ready;
  int64_t written_upto = 0;  // windows launched into output slots
  hv_stream(int r, int w, int s, int g) : ring(r, w, s, g) {}
};

namespace hvi {

struct ServeState {
  std::mutex mu;  // stream list
  std::vector<hv_stream*> streams;
  std::thread poller;
  std::atomic<bool> stop{false};
  std::atomic<int64_t> frames_in{0}, frames_dropped{0}, windows_done{0}, admitted{0}, refused{0},
      images_overwritten{0}, device_errors{0};
  std::atomic<int64_t> lat_after_ns{0};  // latencies of windows whose last frame arrived before are ignored
  size_t admitted_bytes = 0;
  hvs::LatencyLog lat;
  std::vector<hipEvent_t> ev_pool;
  std::mutex ev_mu;
  hipEvent_t take_event() {
    std::lock_guard<std::mutex> g(ev_mu);
    if (!ev_pool.empty()) {
      hipEvent_t e = ev_pool.back();
      ev_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return e;
  }
  void give_event(hipEvent_t e) {
    std::lock_guard<std::mutex> g(ev_mu);
    ev_pool.push_back(e);
  }
};

// Completions of one stream, in launch order.  Returns how many groups finished.
static int drain(ServeState* sv, hv_stream* s, bool wait) {
  int n = 0;
  for (;;) {
    hv_stream::Pending p;
    {
      std::lock_guard<std::mutex> g(s->mu);
      if (s->pending.empty()) break;
      p = s->pending.front();
    }
    hipError_t q = wait ? hipEventSynchronize(p.ev) : hipEventQuery(p.ev);
    if (q == hipErrorNotReady) break;
    if (q != hipSuccess) {
      // a device error: these windows are not complete and are not timed;
      // the stream is marked failed so pushes report it
      (void)hipGetLastError();
      s->ring.set_failed();
      sv->device_errors++;
      {
        std::lock_guard<std::mutex> g(s->mu);
        s->pending.pop_front();
      }
      (void)hipEventDestroy(p.ev);
      ++n;
      continue;
    }
    const int64_t t_done = now_ns();
    const int64_t after = sv->lat_after_ns.load();
    {
      std::lock_guard<std::mutex> g(s->mu);
      for (int i = 0; i < p.g.count; ++i) {
        const int64_t j = p.g.first_window + i;
        const int64_t t_last = s->ring.window_arrival(j);
        if (t_last >= after) sv->lat.add(t_done - t_last);
        s->ready.push_back({j, t_last, t_done});
        while ((int)s->ready.size() > s->keep_ready) {
          s->ready.pop_front();
          sv->images_overwritten++;
        }
      }
      s->pending.pop_front();
    }
    s->ring.mark_done(p.g.first_window, p.g.count);
    sv->windows_done += p.g.count;
    sv->give_event(p.ev);
    ++n;
  }
  return n;
}

static void poll_loop(hv_ctx* ctx) {
  ServeState* sv = ctx->serve;
  // the context's device was set successfully when the context was created
  (void)hipSetDevice(ctx->device);
  while (!sv->stop.load()) {
    int done = 0;
    {
      std::lock_guard<std::mutex> g(sv->mu);
      for (hv_stream* s : sv->streams) done += drain(sv, s, false);
    }
    if (!done) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

static ServeState* serve(hv_ctx* ctx) {
  std::lock_guard<std::recursive_mutex> lock(ctx->mu);
  if (!ctx->serve) {
    ctx->serve = new ServeState();
    ctx->serve->poller = std::thread(poll_loop, ctx);
  }
  return ctx->serve;
}

void serve_shutdown(Ctx* c) {
  hv_ctx* ctx = static_cast<hv_ctx*>(c);
  ServeState* sv = ctx->serve;
  if (!sv) return;
  std::vector<hv_stream*> left;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    left = sv->streams;
  }
  for (hv_stream* s : left) hv_stream_close(s);
  sv->stop = true;
  if (sv->poller.joinable()) sv->poller.join();
  for (hipEvent_t e : sv->ev_pool) (void)hipEventDestroy(e);
  delete sv;
  ctx->serve = nullptr;
}

// Launch every window the ring holds complete.
static hv_status launch_ready(hv_stream* s) {
  ServeState* sv = s->ctx->serve;
  hvs::WindowGroup g;
  const size_t npix = (size_t)s->ny * s->nx;
  while (s->ring.take_ready(g)) {
    // output slots j mod O, split where the slot ring wraps
    int64_t j = g.first_window;
    int left = g.count;
    int slot = g.slot;
    while (left > 0) {
      const int os = (int)(j % s->out_slots);
      const int run = std::min(left, s->out_slots - os);
      const int nf = (run - 1) * s->tp.stride + s->tp.window;
      const char* src = (const char*)s->ring_dev + (size_t)slot * s->frame_bytes;
      hv_status st = hvi_stft_common(s->ctx, src, s->raw_t, nf, s->ny, s->nx, &s->optics, &s->tp, s->prec,
                                     s->out_dev[0] + (size_t)os * npix, s->out_dev[1] + (size_t)os * npix,
                                     s->out_dev[2] + (size_t)os * npix, nullptr, s->st);
      if (st) {
        s->ring.abandon(g);
        return st;
      }
      j += run;
      left -= run;
      slot += run * s->tp.stride;
    }
    hipEvent_t ev = sv->take_event();
    if (!ev) {
      s->ring.abandon(g);
      return fail(HV_ERR_DEVICE, "could not create a completion event");
    }
    if (hipEventRecord(ev, s->st) != hipSuccess) {
      sv->give_event(ev);
      s->ring.abandon(g);
      return fail(HV_ERR_DEVICE, "event record failed: %s", hipGetErrorString(hipGetLastError()));
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->pending.push_back({ev, g});
  }
  return HV_OK;
}

}  // namespace hvi

using namespace hvi;

extern "C" {

hv_status hv_stream_open(hv_ctx* ctx, int ny, int nx, int raw_t, const hv_optics* optics,
                         const hv_temporal* temporal, int prec, int ring_frames, hv_stream** out) {
  if (!ctx || !optics || !temporal || !out) return fail(HV_ERR_ARG, "NULL argument");
  *out = nullptr;
  if (raw_t != HV_U8 && raw_t != HV_U16) return fail(HV_ERR_ARG, "stream frames must be HV_U8 or HV_U16");
  if (!pow2_in(nx, 64, 1024) || !pow2_in(ny, 64, 1024)) return fail(HV_ERR_SHAPE, "frame %dx%d not supported", nx, ny);
  const int w = temporal->window, s = temporal->stride;
  if (w != 8 && w != 16 && w != 32 && w != 64) return fail(HV_ERR_SHAPE, "window %d not supported", w);
  if (s <= 0 || s > w) return fail(HV_ERR_ARG, "stream stride must be in [1, window]");
  if (ring_frames <= 0) ring_frames = 8 * w;
  if (ring_frames % s || ring_frames < 2 * w)
    return fail(HV_ERR_ARG, "ring_frames must be a multiple of the stride and >= 2 W");
  if (prec != HV_PREC_FP32 && prec != HV_PREC_MIXED) return fail(HV_ERR_ARG, "unknown precision %d", prec);
  {
    hv_status e = check_optics(optics);
    if (e) return e;
  }
  if (!(temporal->fs_hz > 0)) return fail(HV_ERR_ARG, "fs must be positive");
  {
    // the band must keep at least one bin (the same check as the offline call)
    std::vector<int> bins;
    std::vector<double> freqs;
    if (band_bins(*temporal, bins, freqs) <= 0) return fail(HV_ERR_ARG, "the band holds no bin");
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(HV_ERR_DEVICE, "hipSetDevice failed");
  ServeState* sv = serve(ctx);
  const int group = std::max(1, std::min(8, ring_frames / (2 * s)));
  hv_stream* st = new hv_stream(ring_frames, w, s, group);
  st->ctx = ctx;
  st->ny = ny;
  st->nx = nx;
  st->raw_t = raw_t;
  st->prec = prec;
  st->optics = *optics;
  st->tp = *temporal;
  st->frame_bytes = (size_t)ny * nx * (raw_t == HV_U8 ? 1 : 2);
  // images in flight are at most ring_frames / stride; with keep_ready more
  // kept for pop, slot j mod out_slots is never reused while still wanted
  st->out_slots = ring_frames / s + st->keep_ready + 1;
  const size_t npix = (size_t)ny * nx;
  const size_t ring_b = (size_t)st->ring.slots_total() * st->frame_bytes;
  const size_t out_b = (size_t)st->out_slots * npix * 4;
  // workspace of one launch of `group` windows: spectra (and a field when not fused)
  const size_t nf = (size_t)(group - 1) * s + w;
  const size_t cplx = prec == HV_PREC_MIXED ? 4 : 8;
  const bool fused = optics->method == HV_AS && rowinv_coef_fits(nx, w);
  const size_t ws0 = nf * npix * cplx;  // row pass output (upper bound)
  size_t ws1 = nf * npix * cplx;
  if (optics->method == HV_AS && band_first_fits(ny, nx, raw_t)) {
    // room for the band-first order too: `group` windows of nb bin fields
    std::vector<int> bins;
    std::vector<double> freqs;
    const size_t nb = (size_t)band_bins(*temporal, bins, freqs);
    ws1 = std::max(ws1, (size_t)group * nb * npix * cplx);
  }
  const size_t ws2 = fused ? 0 : nf * npix * cplx;
  const size_t table_b = npix * 8 + 4 * (size_t)(nx + ny) * 8;
  const size_t total = ring_b + 3 * out_b + ws0 + ws1 + ws2 + table_b;
  {
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    if (ctx->budget && sv->admitted_bytes + total > ctx->budget) {
      sv->refused++;
      delete st;
      return fail(HV_ERR_BUDGET, "stream needs %zu bytes; %zu of %zu admitted", total, sv->admitted_bytes,
                  ctx->budget);
    }
    sv->admitted_bytes += total;
  }
  st->admitted_bytes = total;
  auto undo = [&](hv_status e) {
    {
      std::lock_guard<std::recursive_mutex> lock(ctx->mu);
      sv->admitted_bytes -= total;
    }
    if (st->ring_dev) (void)hipFree(st->ring_dev);
    for (float* p : st->out_dev)
      if (p) (void)hipFree(p);
    if (st->st) (void)hipStreamDestroy(st->st);
    if (st->up) (void)hipStreamDestroy(st->up);
    delete st;
    return e;
  };
  if (hipStreamCreateWithFlags(&st->st, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&st->up, hipStreamNonBlocking) != hipSuccess)
    return undo(fail(HV_ERR_DEVICE, "hipStreamCreate failed"));
  if (hipMalloc(&st->ring_dev, ring_b) != hipSuccess) return undo(fail(HV_ERR_NOMEM, "ring allocation failed"));
  for (int i = 0; i < 3; ++i)
    if (hipMalloc(&st->out_dev[i], out_b) != hipSuccess) return undo(fail(HV_ERR_NOMEM, "output allocation failed"));
  {
    // preallocate workspaces and tables so the loop never allocates; the
    // allocations and the float64 table builds run outside the context lock
    hv_status e;
    const size_t want[3] = {ws0, ws1, ws2};
    for (int slot = 0; slot < 3; ++slot) {
      if (!want[slot]) continue;
      void* p = nullptr;
      if (hipMalloc(&p, want[slot]) != hipSuccess) return undo(fail(HV_ERR_NOMEM, "workspace allocation failed"));
      std::lock_guard<std::recursive_mutex> lock(ctx->mu);
      DevBuf& b = ctx->ws[std::make_pair((void*)st->st, slot)];
      b.ptr = p;
      b.bytes = want[slot];
      ctx->held += want[slot];
    }
    if (optics->method == HV_AS) {
      if (!ctx->as_plan(ny, nx, *optics, &e)) return undo(e);
    } else if (!ctx->fresnel_plan(ny, nx, *optics, &e)) {
      return undo(e);
    }
    if (!ctx->dft_plan(*temporal, &e)) return undo(e);
  }
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->streams.push_back(st);
  }
  sv->admitted++;
  *out = st;
  return HV_OK;
}

hv_status hv_stream_push(hv_stream* s, const void* frames, int n_frames, const int64_t* arrival_ns) {
  if (!s || (!frames && n_frames > 0)) return fail(HV_ERR_ARG, "NULL argument");
  if (n_frames < 0) return fail(HV_ERR_ARG, "negative frame count");
  ServeState* sv = s->ctx->serve;
  std::lock_guard<std::mutex> lk(s->push_mu);
  std::vector<hvs::Span> copies;
  const int64_t first = s->ring.pushed();
  const hvs::RingLogic::Push pr = s->ring.push(n_frames, arrival_ns, now_ns(), copies);
  if (pr == hvs::RingLogic::Push::failed)
    return fail(HV_ERR_STATE, "stream failed on an earlier launch or device error; close it");
  if (pr == hvs::RingLogic::Push::full) {
    sv->frames_dropped += n_frames;
    return fail(HV_ERR_OVERFLOW, "ring full: %d frames refused", n_frames);
  }
  // Device frames are copied on the stream's own queue, ahead of the
  // windows they complete.  Host frames (pinned, or pageable at a lower
  // rate) go up on the upload queue and are waited for, so the caller may
  // reuse the buffer on return and the windows launched below see them.
  // Either way the slots written hold no frame of an unfinished window.
  bool on_host = true;
  if (!copies.empty()) {
    hipPointerAttribute_t pa{};
    if (hipPointerGetAttributes(&pa, frames) == hipSuccess)
      on_host = !(pa.type == hipMemoryTypeDevice || pa.type == hipMemoryTypeManaged);
    else
      (void)hipGetLastError();  // not known to HIP: pageable host memory
  }
  for (const hvs::Span& c : copies) {
    const char* src = (const char*)frames + (size_t)(c.first_frame - first) * s->frame_bytes;
    char* dst = (char*)s->ring_dev + (size_t)c.slot * s->frame_bytes;
    if (hipMemcpyAsync(dst, src, (size_t)c.count * s->frame_bytes,
                       on_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, on_host ? s->up : s->st) !=
        hipSuccess) {
      s->ring.set_failed();
      return fail(HV_ERR_DEVICE, "ring copy failed");
    }
  }
  if (on_host && !copies.empty() && hipStreamSynchronize(s->up) != hipSuccess) {
    s->ring.set_failed();
    return fail(HV_ERR_DEVICE, "ring upload failed: %s", hipGetErrorString(hipGetLastError()));
  }
  sv->frames_in += n_frames;
  return launch_ready(s);
}

hv_status hv_stream_pop(hv_stream* s, float* m0, float* m1, float* m2, int64_t* t_last_arrival_ns,
                        int64_t* t_done_ns) {
  if (!s) return fail(HV_ERR_ARG, "NULL stream");
  hv_stream::Ready r;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->ready.empty()) return fail(HV_ERR_STATE, "no completed window");
    r = s->ready.front();
    s->ready.pop_front();
  }
  const size_t npix = (size_t)s->ny * s->nx;
  const int os = (int)(r.window % s->out_slots);
  float* dst[3] = {m0, m1, m2};
  for (int i = 0; i < 3; ++i)
    if (dst[i] && hipMemcpyAsync(dst[i], s->out_dev[i] + (size_t)os * npix, npix * 4, hipMemcpyDeviceToDevice,
                                 s->st) != hipSuccess)
      return fail(HV_ERR_DEVICE, "image copy failed");
  if (hipStreamSynchronize(s->st) != hipSuccess) return fail(HV_ERR_DEVICE, "stream sync failed");
  if (t_last_arrival_ns) *t_last_arrival_ns = r.t_last;
  if (t_done_ns) *t_done_ns = r.t_done;
  return HV_OK;
}

hv_status hv_stream_close(hv_stream* s) {
  if (!s) return fail(HV_ERR_ARG, "NULL stream");
  hv_ctx* ctx = s->ctx;
  ServeState* sv = ctx->serve;
  // A device error is reported, but the stream is released all the same.
  hv_status res = HV_OK;
  const bool on_dev = hipSetDevice(ctx->device) == hipSuccess;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->streams.erase(std::remove(sv->streams.begin(), sv->streams.end(), s), sv->streams.end());
  }
  if (!on_dev || hipStreamSynchronize(s->st) != hipSuccess)
    res = fail(HV_ERR_DEVICE, "device error while closing a stream: %s", hipGetErrorString(hipGetLastError()));
  drain(sv, s, true);
  std::vector<void*> to_free;
  std::vector<std::unique_ptr<AsPlan>> dead_as;
  std::vector<std::unique_ptr<FresnelPlan>> dead_fr;
  {
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    for (int slot = 0; slot < 3; ++slot) {
      auto it = ctx->ws.find(std::make_pair((void*)s->st, slot));
      if (it != ctx->ws.end()) {
        ctx->held -= it->second.bytes;
        to_free.push_back(it->second.ptr);
        it->second.ptr = nullptr;  // freed below, outside the lock
        it->second.bytes = 0;
        ctx->ws.erase(it);
      }
    }
    sv->admitted_bytes -= s->admitted_bytes;
    // drop this stream's propagation tables unless another open stream uses them
    bool shared = false;
    {
      std::lock_guard<std::mutex> g(sv->mu);
      for (hv_stream* o : sv->streams)
        shared |= o->ny == s->ny && o->nx == s->nx && o->optics.method == s->optics.method &&
                  o->optics.z_m == s->optics.z_m && o->optics.wavelength_m == s->optics.wavelength_m &&
                  o->optics.pitch_x_m == s->optics.pitch_x_m && o->optics.pitch_y_m == s->optics.pitch_y_m &&
                  o->optics.highpass_cpp == s->optics.highpass_cpp;
    }
    if (!shared) {
      auto key = std::make_tuple(s->ny, s->nx, s->optics.wavelength_m, s->optics.pitch_x_m, s->optics.pitch_y_m,
                                 s->optics.z_m, s->optics.method == HV_AS ? s->optics.highpass_cpp : 0.0);
      auto ia = ctx->as_plans.find(key);
      if (s->optics.method == HV_AS && ia != ctx->as_plans.end()) {
        ctx->held -= ia->second->ht.bytes + ia->second->hs.bytes;
        dead_as.push_back(std::move(ia->second));
        ctx->as_plans.erase(ia);
      }
      auto ifr = ctx->fr_plans.find(key);
      if (s->optics.method == HV_FRESNEL && ifr != ctx->fr_plans.end()) {
        ctx->held -= ifr->second->tables.bytes;
        dead_fr.push_back(std::move(ifr->second));
        ctx->fr_plans.erase(ifr);
      }
    }
  }
  // teardown of a closed stream: failures here cannot be acted on
  for (void* p : to_free) (void)hipFree(p);
  dead_as.clear();
  dead_fr.clear();
  (void)hipFree(s->ring_dev);
  for (float* p : s->out_dev) (void)hipFree(p);
  (void)hipStreamDestroy(s->st);
  (void)hipStreamDestroy(s->up);
  delete s;
  return res;
}

hv_status hv_stream_frames(const hv_stream* s, int64_t* pushed, int64_t* dropped, int64_t* windows_done) {
  if (!s) return fail(HV_ERR_ARG, "NULL stream");
  if (pushed) *pushed = s->ring.pushed();
  if (dropped) *dropped = s->ring.dropped();
  if (windows_done) *windows_done = s->ring.done();
  return HV_OK;
}

hv_status hv_ctx_stats(hv_ctx* ctx, hv_stats* out) {
  if (!ctx || !out) return fail(HV_ERR_ARG, "NULL argument");
  std::memset(out, 0, sizeof *out);
  ServeState* sv = ctx->serve;
  if (!sv) return HV_OK;
  out->frames_in = sv->frames_in;
  out->frames_dropped = sv->frames_dropped;
  out->windows_done = sv->windows_done;
  out->streams_admitted = sv->admitted;
  out->streams_refused = sv->refused;
  out->images_overwritten = sv->images_overwritten;
  out->latency_samples = (int64_t)sv->lat.size();
  out->lat_p50_ns = sv->lat.percentile(50.0);
  out->lat_p99_ns = sv->lat.percentile(99.0);
  out->lat_max_ns = sv->lat.percentile(100.0);
  {
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    out->admitted_bytes = (int64_t)sv->admitted_bytes;
  }
  out->device_errors = sv->device_errors;
  return HV_OK;
}

hv_status hv_ctx_stats_reset(hv_ctx* ctx) {
  if (!ctx) return fail(HV_ERR_ARG, "NULL argument");
  ServeState* sv = serve(ctx);
  sv->lat.clear();
  sv->lat_after_ns = now_ns();
  sv->frames_in = 0;
  sv->frames_dropped = 0;
  sv->windows_done = 0;
  sv->admitted = 0;
  sv->refused = 0;
  sv->images_overwritten = 0;
  sv->device_errors = 0;
  return HV_OK;
}

// ---------------------------------------------------------------- replay driver

hv_status hv_replay_run(hv_ctx* ctx, const hv_replay_config* cfg, hv_replay_result* res) {
  if (!ctx || !cfg || !res) return fail(HV_ERR_ARG, "NULL argument");
  if (cfg->nclass <= 0 || cfg->nclass > HV_REPLAY_MAX_CLASSES) return fail(HV_ERR_ARG, "nclass out of range");
  for (int c = 0; c < cfg->nclass; ++c) {
    const hv_replay_class& k = cfg->cls[c];
    if (!k.block || k.block_frames <= 0 || !(k.fps > 0) || k.max_active <= 0)
      return fail(HV_ERR_ARG, "class %d: block, fps and max_active are required", c);
  }
  if (!(cfg->duration_s > 0) || !(cfg->arrival_hz > 0) || !(cfg->mean_life_s > 0))
    return fail(HV_ERR_ARG, "duration, arrival rate and lifetime must be positive");
  std::memset(res, 0, sizeof *res);
  hv_status e = hv_ctx_stats_reset(ctx);
  if (e) return e;
  ServeState* sv = ctx->serve;
  std::mt19937_64 rng(cfg->seed);
  std::exponential_distribution<double> gap(cfg->arrival_hz), life(1.0 / cfg->mean_life_s);
  std::uniform_int_distribution<int> pick(0, cfg->nclass - 1);
  std::uniform_real_distribution<double> zdist(cfg->z_lo_m, cfg->z_hi_m);
  const int packet = cfg->packet_frames > 0 ? cfg->packet_frames : 8;
  const int64_t t0 = now_ns();
  const int64_t t_end = t0 + (int64_t)(cfg->duration_s * 1e9);
  sv->lat_after_ns = t0 + (int64_t)(cfg->warmup_s * 1e9);
  std::vector<std::thread> workers;
  std::vector<std::atomic<int>> active(HV_REPLAY_MAX_CLASSES);
  for (auto& a : active) a = 0;
  std::atomic<int64_t> offered{0}, consumed{0};
  std::atomic<int> errors{0};
  int64_t t_next = t0;
  uint64_t stream_id = 0;
  while (true) {
    t_next += (int64_t)(gap(rng) * 1e9);
    if (t_next >= t_end) break;
    std::this_thread::sleep_until(std::chrono::steady_clock::time_point(std::chrono::nanoseconds(t_next)));
    const int c = pick(rng);
    const double lifetime = life(rng);
    const double z = zdist(rng);
    const hv_replay_class k = cfg->cls[c];
    if (active[c].load() >= k.max_active) {
      sv->refused++;
      continue;
    }
    hv_optics op{cfg->wavelength_m, cfg->pitch_m, cfg->pitch_m, -z, HV_AS};
    hv_temporal tp{k.window, k.stride, k.fps, k.f_lo_hz, k.f_hi_hz, 0};
    hv_stream* s = nullptr;
    int ring = k.ring_frames;
    if (ring <= 0) {  // at least 8 windows and 20 ms of frames, a multiple of the stride
      const int by_time = (int)std::ceil(0.02 * k.fps);
      ring = std::max(8 * k.window, by_time);
      ring = (ring + k.stride - 1) / k.stride * k.stride;
    }
    hv_status st = hv_stream_open(ctx, k.ny, k.nx, k.raw_t, &op, &tp, cfg->prec, ring, &s);
    if (st == HV_ERR_BUDGET) continue;  // counted as refused by hv_stream_open
    if (st) {
      errors++;
      continue;
    }
    active[c]++;
    const int64_t t_start = t_next;
    const int64_t t_stop = std::min(t_end, t_start + (int64_t)(lifetime * 1e9));
    const uint64_t sid = stream_id++;
    workers.emplace_back([&, s, c, k, t_start, t_stop, sid]() {
      (void)hipSetDevice(ctx->device);  // set successfully when the context was created
      const size_t fb = (size_t)k.ny * k.nx * (k.raw_t == HV_U8 ? 1 : 2);
      std::vector<int64_t> arr(packet);
      int64_t f = 0;
      int64_t boff = (int64_t)((sid * 7919) % (uint64_t)k.block_frames);
      for (;;) {
        const int64_t t_pkt = t_start + (int64_t)((double)(f + packet) * 1e9 / k.fps);  // last frame of the packet
        if (t_pkt > t_stop) break;
        std::this_thread::sleep_until(std::chrono::steady_clock::time_point(std::chrono::nanoseconds(t_pkt)));
        int sent = 0;
        while (sent < packet) {
          const int64_t b = (boff + f + sent) % k.block_frames;
          const int run = (int)std::min<int64_t>(packet - sent, k.block_frames - b);
          for (int i = 0; i < run; ++i) arr[i] = t_start + (int64_t)((double)(f + sent + i + 1) * 1e9 / k.fps);
          const hv_status ps = hv_stream_push(s, (const char*)k.block + (size_t)b * fb, run, arr.data());
          if (ps && ps != HV_ERR_OVERFLOW) errors++;
          offered += run;
          sent += run;
        }
        f += packet;
      }
      hv_stream_close(s);
      active[c]--;
    });
  }
  for (auto& t : workers) t.join();
  const int64_t t1 = now_ns();
  hv_stats stt;
  hv_ctx_stats(ctx, &stt);
  res->frames_offered = offered.load();
  res->frames_in = stt.frames_in;
  res->frames_dropped = stt.frames_dropped;
  res->windows_done = stt.windows_done;
  res->streams_admitted = stt.streams_admitted;
  res->streams_refused = stt.streams_refused;
  res->lat_p50_ns = stt.lat_p50_ns;
  res->lat_p99_ns = stt.lat_p99_ns;
  res->lat_max_ns = stt.lat_max_ns;
  res->latency_samples = stt.latency_samples;
  res->seconds = (t1 - t0) * 1e-9;
  res->frames_per_s = stt.frames_in / res->seconds;
  res->errors = errors.load();
  return errors.load() ? fail(HV_ERR_DEVICE, "%d push/open errors during replay", errors.load()) : HV_OK;
}

}  // extern "C"
