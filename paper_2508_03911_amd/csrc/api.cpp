// C-ABI entry points, context, plan cache and workspaces.
//
// Plans hold tables computed once in float64 on the host and stored on the
// device as float32: the angular-spectrum transfer function (its phase
// 2 pi z sqrt(1/lambda^2 - f^2) reaches ~1e6 rad, far beyond what float32
// can carry), the Fresnel chirps with the centring checkerboard folded in,
// and the MFMA fragments of the DFT coefficient matrix.  Workspaces are
// per stream and grow only when a larger shape arrives (allocation is kept
// out of the steady state, Sec. VII-C).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "hv_ctx.h"
#include "hv_internal.h"

namespace hvi {

static thread_local char g_err[512] = "";

hv_status fail(hv_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return st;
}

const char* last_error() { return g_err; }

// ---------------------------------------------------------------- device buffers

DevBuf::~DevBuf() { release(); }
void DevBuf::release() {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  bytes = 0;
}
hv_status DevBuf::ensure(size_t want, size_t* accounted) {
  if (want <= bytes) return HV_OK;
  if (accounted) *accounted -= bytes;
  // queued work may still read the old buffer
  if (ptr && hipDeviceSynchronize() != hipSuccess)
    return fail(HV_ERR_DEVICE, "device error before regrowing a workspace: %s",
                hipGetErrorString(hipGetLastError()));
  release();
  if (hipMalloc(&ptr, want) != hipSuccess) {
    (void)hipGetLastError();
    ptr = nullptr;
    return fail(HV_ERR_NOMEM, "hipMalloc of %zu bytes failed", want);
  }
  bytes = want;
  if (accounted) *accounted += bytes;
  return HV_OK;
}
hv_status DevBuf::upload(const void* host, size_t n, size_t* accounted) {
  hv_status st = ensure(n, accounted);
  if (st) return st;
  if (hipMemcpy(ptr, host, n, hipMemcpyHostToDevice) != hipSuccess)
    return fail(HV_ERR_DEVICE, "table upload failed: %s", hipGetErrorString(hipGetLastError()));
  return HV_OK;
}

// ---------------------------------------------------------------- timing

hipEvent_t Timing::take() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}
void Timing::collect() {
  for (auto& r : pending) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      auto& slot = acc[r.name];
      slot.first += ms;
      slot.second += 1;
    } else {
      (void)hipGetLastError();  // a sample that cannot be read is left out
    }
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  pending.clear();
}
void Timing::reset() {
  collect();
  acc.clear();
}
Timing::~Timing() {
  collect();
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

// ---------------------------------------------------------------- band

int band_bins(const hv_temporal& tp, std::vector<int>& bins, std::vector<double>& freqs) {
  bins.clear();
  freqs.clear();
  const int w = tp.window;
  long lo = (long)std::ceil(tp.f_lo_hz * w / tp.fs_hz);
  long hi = (long)std::floor(tp.f_hi_hz * w / tp.fs_hz);
  if (lo < 0) lo = 0;
  if (hi > w / 2) hi = w / 2;
  for (long k = lo; k <= hi; ++k) {
    bins.push_back((int)k);
    freqs.push_back((double)k * tp.fs_hz / w);
  }
  if (tp.symmetric_band) {
    const size_t npos = bins.size();
    for (size_t i = 0; i < npos; ++i) {
      const int k = bins[i];
      if (k > 0 && 2 * k != w) {
        bins.push_back(w - k);
        freqs.push_back((double)k * tp.fs_hz / w);
      }
    }
  }
  return (int)bins.size();
}

// ---------------------------------------------------------------- table builders (float64)

static hv_status build_as_table(size_t* held, AsPlan& p) {
  const int ny = p.ny, nx = p.nx;
  std::vector<float2> h((size_t)nx * ny);
  const double inv_l2 = 1.0 / (p.wavelength * p.wavelength);
  for (int cx = 0; cx < nx; ++cx) {
    const double fx = (cx < (nx + 1) / 2 ? cx : cx - nx) / (nx * p.dx);
    for (int cy = 0; cy < ny; ++cy) {
      const double fy = (cy < (ny + 1) / 2 ? cy : cy - ny) / (ny * p.dy);
      const double rad = inv_l2 - fx * fx - fy * fy;
      double re = 0.0, im = 0.0;
      const double ux = (cx < (nx + 1) / 2 ? cx : cx - nx) / (double)nx;  // cycles per pixel
      const double uy = (cy < (ny + 1) / 2 ? cy : cy - ny) / (double)ny;
      const bool keep = p.highpass <= 0 || ux * ux + uy * uy >= p.highpass * p.highpass;
      if (rad > 0 && keep) {
        const double ph = 2.0 * M_PI * p.z * std::sqrt(rad);
        re = std::cos(ph) / ny;
        im = std::sin(ph) / ny;
      }
      h[(size_t)cx * ny + cy] = make_float2((float)re, (float)im);
    }
  }
  // the column pass's order: +fx columns, then the -fx column of each fx
  std::vector<float2> hs((size_t)nx * ny);
  for (int fx = 0; fx < nx / 2; ++fx) {
    const int neg = fx == 0 ? nx / 2 : nx - fx;
    std::copy_n(&h[(size_t)fx * ny], ny, &hs[(size_t)fx * ny]);
    std::copy_n(&h[(size_t)neg * ny], ny, &hs[(size_t)(nx / 2 + fx) * ny]);
  }
  hv_status s = p.ht.upload(h.data(), h.size() * sizeof(float2), held);
  return s ? s : p.hs.upload(hs.data(), hs.size() * sizeof(float2), held);
}

static hv_status build_fresnel_tables(size_t* held, FresnelPlan& p) {
  const int ny = p.ny, nx = p.nx;
  const double lz = p.wavelength * p.z;
  const double opx = p.wavelength * std::fabs(p.z) / (nx * p.dx);
  const double opy = p.wavelength * std::fabs(p.z) / (ny * p.dy);
  std::vector<float2> t(2 * (size_t)(nx + ny));
  auto chirp = [&](double r, int idx) {
    const double ph = M_PI * r * r / lz;
    const double sg = (idx & 1) ? -1.0 : 1.0;  // (-1)^index: centring of the DFT
    return make_float2((float)(sg * std::cos(ph)), (float)(sg * std::sin(ph)));
  };
  for (int m = 0; m < nx; ++m) t[m] = chirp((m - nx / 2) * p.dx, m);
  for (int n = 0; n < ny; ++n) t[nx + n] = chirp((n - ny / 2) * p.dy, n);
  for (int m = 0; m < nx; ++m) t[nx + ny + m] = chirp((m - nx / 2) * opx, m);
  for (int n = 0; n < ny; ++n) t[2 * nx + ny + n] = chirp((n - ny / 2) * opy, n);
  return p.tables.upload(t.data(), t.size() * sizeof(float2), held);
}

static hv_status build_dft_plan(size_t* held, DftPlan& p) {
  const int w = p.window;
  const int nb = (int)p.bins.size();
  p.mtiles = (nb + 15) / 16;
  const int mt = p.mtiles;
  auto coef = [&](int m, int k) -> double {
    const int b = m >> 1, t = k >> 1;
    if (b >= nb) return 0.0;
    const long prod = ((long)p.bins[b] * t) % w;
    const double th = 2.0 * M_PI * (double)prod / w;
    const double cs = std::cos(th), sn = std::sin(th);
    if ((m & 1) == 0) return (k & 1) == 0 ? cs : sn;
    return (k & 1) == 0 ? -sn : cs;
  };
  std::vector<float> a32((size_t)mt * w * 64);
  for (int m_t = 0; m_t < mt; ++m_t)
    for (int kk = 0; kk < w; ++kk)
      for (int lane = 0; lane < 64; ++lane)
        a32[((size_t)m_t * w + kk) * 64 + lane] = (float)coef(32 * m_t + (lane & 31), 2 * kk + (lane >> 5));
  std::vector<hv_h8> hi((size_t)mt * (w / 8) * 64), lo(hi.size());
  for (int m_t = 0; m_t < mt; ++m_t)
    for (int kk = 0; kk < w / 8; ++kk)
      for (int lane = 0; lane < 64; ++lane) {
        hv_h8 h, l;
        for (int e = 0; e < 8; ++e) {
          const float a = (float)coef(32 * m_t + (lane & 31), 16 * kk + 8 * (lane >> 5) + e);
          h[e] = (_Float16)a;
          l[e] = (_Float16)(a - (float)h[e]);
        }
        hi[((size_t)m_t * (w / 8) + kk) * 64 + lane] = h;
        lo[((size_t)m_t * (w / 8) + kk) * 64 + lane] = l;
      }
  std::vector<float> wts((size_t)3 * mt * 16, 0.f);
  for (int b = 0; b < nb; ++b) {
    wts[b] = 1.0f;
    wts[mt * 16 + b] = (float)p.freqs[b];
    wts[2 * mt * 16 + b] = (float)(p.freqs[b] * p.freqs[b]);
  }
  const int ks = w >= 16 ? w / 16 : 1;
  std::vector<hv_h8> rhi((size_t)mt * ks * 64), rlo(rhi.size());
  for (int m_t = 0; m_t < mt; ++m_t)
    for (int kk = 0; kk < ks; ++kk)
      for (int lane = 0; lane < 64; ++lane) {
        hv_h8 h, l;
        for (int e = 0; e < 8; ++e) {
          const int t = 16 * kk + 8 * (lane >> 5) + e;
          // real input: column 2t of the complex-input matrix
          const float a = t < w ? (float)coef(32 * m_t + (lane & 31), 2 * t) : 0.f;
          h[e] = (_Float16)a;
          l[e] = (_Float16)(a - (float)h[e]);
        }
        rhi[((size_t)m_t * ks + kk) * 64 + lane] = h;
        rlo[((size_t)m_t * ks + kk) * 64 + lane] = l;
      }
  hv_status st = p.a32.upload(a32.data(), a32.size() * sizeof(float), held);
  if (!st) st = p.ar_hi.upload(rhi.data(), rhi.size() * sizeof(hv_h8), held);
  if (!st) st = p.ar_lo.upload(rlo.data(), rlo.size() * sizeof(hv_h8), held);
  if (!st) st = p.a16hi.upload(hi.data(), hi.size() * sizeof(hv_h8), held);
  if (!st) st = p.a16lo.upload(lo.data(), lo.size() * sizeof(hv_h8), held);
  if (!st) st = p.wts.upload(wts.data(), wts.size() * sizeof(float), held);
  return st;
}

// ---------------------------------------------------------------- plan lookup

// Plans are looked up under the context lock but built outside it (the
// float64 tables of a large frame take milliseconds), so a stream being
// opened never stalls the launches of the streams already running.
template <class Map, class Key, class Make>
static auto* plan_lookup(Ctx* c, Map& m, const Key& key, Make make, hv_status* st, bool build) {
  {
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    auto it = m.find(key);
    if (it != m.end()) return it->second.get();
  }
  if (!build) {
    *st = fail(HV_ERR_STATE, "no plan for these settings in the context: one call of the allocating entry point "
                             "with the same frame shape, optics and temporal settings builds it");
    return (decltype(make(nullptr, nullptr).get())) nullptr;
  }
  size_t bytes = 0;
  auto p = make(&bytes, st);
  if (!p) return (decltype(p.get())) nullptr;
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  auto it = m.find(key);
  if (it != m.end()) return it->second.get();  // built meanwhile by another thread
  c->held += bytes;
  auto* raw = p.get();
  m[key] = std::move(p);
  return raw;
}

AsPlan* Ctx::as_plan(int ny, int nx, const hv_optics& o, hv_status* st, bool build) {
  auto key = std::make_tuple(ny, nx, o.wavelength_m, o.pitch_x_m, o.pitch_y_m, o.z_m, o.highpass_cpp);
  return plan_lookup(this, as_plans, key, [&](size_t* bytes, hv_status* e) {
    auto p = std::make_unique<AsPlan>();
    p->ny = ny;
    p->nx = nx;
    p->wavelength = o.wavelength_m;
    p->dx = o.pitch_x_m;
    p->dy = o.pitch_y_m;
    p->z = o.z_m;
    p->highpass = o.highpass_cpp;
    *e = build_as_table(bytes, *p);
    if (*e) p.reset();
    return p;
  }, st, build);
}

FresnelPlan* Ctx::fresnel_plan(int ny, int nx, const hv_optics& o, hv_status* st, bool build) {
  auto key = std::make_tuple(ny, nx, o.wavelength_m, o.pitch_x_m, o.pitch_y_m, o.z_m, 0.0);
  return plan_lookup(this, fr_plans, key, [&](size_t* bytes, hv_status* e) {
    auto p = std::make_unique<FresnelPlan>();
    p->ny = ny;
    p->nx = nx;
    p->wavelength = o.wavelength_m;
    p->dx = o.pitch_x_m;
    p->dy = o.pitch_y_m;
    p->z = o.z_m;
    *e = build_fresnel_tables(bytes, *p);
    if (*e) p.reset();
    return p;
  }, st, build);
}

DftPlan* Ctx::dft_plan(const hv_temporal& tp, hv_status* st, bool build) {
  std::vector<int> bins;
  std::vector<double> freqs;
  band_bins(tp, bins, freqs);
  if (bins.empty()) {
    *st = fail(HV_ERR_ARG, "band [%g, %g] Hz holds no DFT bin at W=%d fs=%g", tp.f_lo_hz, tp.f_hi_hz, tp.window,
               tp.fs_hz);
    return nullptr;
  }
  auto key = std::make_tuple(tp.window, bins, freqs);
  return plan_lookup(this, dft_plans, key, [&](size_t* bytes, hv_status* e) {
    auto p = std::make_unique<DftPlan>();
    p->window = tp.window;
    p->bins = bins;
    p->freqs = freqs;
    *e = build_dft_plan(bytes, *p);
    if (*e) p.reset();
    return p;
  }, st, build);
}

Ctx::~Ctx() {
  for (auto& kv : lanes) {
    if (kv.second.s) (void)hipStreamDestroy(kv.second.s);
    if (kv.second.fork) (void)hipEventDestroy(kv.second.fork);
    if (kv.second.join) (void)hipEventDestroy(kv.second.join);
  }
}

Ctx::Lane2* Ctx::lane2(hipStream_t caller, hv_status* st) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  Lane2& l = lanes[(void*)caller];
  if (!l.s) {
    hipStream_t s2 = nullptr;
    hipEvent_t f = nullptr, j = nullptr;
    if (hipStreamCreateWithFlags(&s2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&f, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&j, hipEventDisableTiming) != hipSuccess) {
      const hipError_t e = hipGetLastError();
      if (j) (void)hipEventDestroy(j);
      if (f) (void)hipEventDestroy(f);
      if (s2) (void)hipStreamDestroy(s2);
      lanes.erase((void*)caller);  // a later call tries again from scratch
      *st = fail(HV_ERR_DEVICE, "could not create the second stream: %s", hipGetErrorString(e));
      return nullptr;
    }
    l.s = s2;
    l.fork = f;
    l.join = j;
  }
  return &l;
}

hv_status Ctx::Lane2::fork_from(hipStream_t from) {
  hipError_t e = hipEventRecord(fork, from);
  if (e == hipSuccess) e = hipStreamWaitEvent(s, fork, 0);
  if (e == hipSuccess) return HV_OK;
  (void)hipGetLastError();
  return fail(HV_ERR_DEVICE, "could not order the second stream after the caller's: %s", hipGetErrorString(e));
}

hv_status Ctx::Lane2::join_into(hipStream_t to) {
  hipError_t e = hipEventRecord(join, s);
  if (e == hipSuccess) e = hipStreamWaitEvent(to, join, 0);
  if (e == hipSuccess) return HV_OK;
  (void)hipGetLastError();
  return fail(HV_ERR_DEVICE, "could not order the caller's stream after the second one: %s", hipGetErrorString(e));
}

int persistent_blocks(const void* kernel, int threads) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) (void)hipGetLastError();
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_pair(kernel, dev);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int cus = 0, per = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    cus = 0;
  }
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess) {
    (void)hipGetLastError();
    per = 1;
  }
  const int b = (cus > 0 ? cus : 256) * (per > 0 ? per : 1);
  cache[key] = b;
  return b;
}

DevBuf& Ctx::work(hipStream_t s, int slot) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  return ws[std::make_pair((void*)s, slot)];
}

int Ctx::chunk_frames_for(int ny, int nx, bool mixed) const {
  if (chunk_frames > 0) return chunk_frames;
  // about 96 MiB of intermediate spectra per chunk (half spectrum + full
  // spectrum = 1.5 complex values per pixel), at least 64 frames: 128 frames
  // (FP32) and 256 (fp16) at 256 x 256, the fastest measured with two
  // streams in flight
  const long per = (long)ny * nx * (mixed ? 4 : 8) * 3 / 2;
  long f = (96L << 20) / per;
  if (f < 64) f = 64;
  if (f > 2048) f = 2048;
  return (int)f;
}

}  // namespace hvi

using namespace hvi;

// ---------------------------------------------------------------- validation helpers

// Frame sides: powers of two in [64, 1024], or the mixed-radix sides of the
// paper's Table IV frames (1280 x 800, 512 x 320, 384 x 384).
static bool side_ok(int n) { return pow2_in(n, 64, 1024) || n == 320 || n == 384 || n == 800 || n == 1280; }

static hv_status check_frame(int n, int ny, int nx) {
  if (n < 0) return fail(HV_ERR_SHAPE, "negative frame count");
  if (!side_ok(nx) || !side_ok(ny))
    return fail(HV_ERR_SHAPE, "frame %dx%d: sides must be powers of two in [64, 1024] or 320, 384, 800, 1280", nx,
                ny);
  return HV_OK;
}

hv_status hvi::check_optics(const hv_optics* o) {
  if (!o) return fail(HV_ERR_ARG, "optics is NULL");
  if (!(o->wavelength_m > 0) || !(o->pitch_x_m > 0) || !(o->pitch_y_m > 0) || !std::isfinite(o->z_m))
    return fail(HV_ERR_ARG, "wavelength and pitches must be positive, z finite");
  if (o->method != HV_AS && o->method != HV_FRESNEL) return fail(HV_ERR_ARG, "unknown method %d", o->method);
  if (o->method == HV_FRESNEL && o->z_m == 0.0) return fail(HV_ERR_ARG, "Fresnel transform needs z != 0");
  if (!(o->highpass_cpp >= 0 && o->highpass_cpp < 1)) return fail(HV_ERR_ARG, "high-pass radius outside [0, 1)");
  if (o->method == HV_FRESNEL && o->highpass_cpp > 0)
    return fail(HV_ERR_ARG, "the high-pass filter belongs to the angular-spectrum path");
  return HV_OK;
}

static hv_status check_dtype(int t, bool allow_field) {
  if (t == HV_U8 || t == HV_U16) return HV_OK;
  if (t == HV_C64 && allow_field) return HV_OK;
  return fail(HV_ERR_ARG, "input dtype %d not allowed here", t);
}

static size_t in_elem(int t) { return t == HV_U8 ? 1 : t == HV_U16 ? 2 : 8; }

// The kernels read their inputs in 8- and 16-byte vectors.
static hv_status check_aligned(const void* p) {
  if (reinterpret_cast<uintptr_t>(p) % 16)
    return fail(HV_ERR_ARG, "input pointer %p is not 16-byte aligned", p);
  return HV_OK;
}

static hv_status enter(hv_ctx* ctx) {
  if (!ctx) return fail(HV_ERR_ARG, "context is NULL");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(HV_ERR_DEVICE, "hipSetDevice(%d) failed", ctx->device);
  return HV_OK;
}

// Power-of-two scale that keeps a unitary transform of the input inside the
// fp16 range: |U| <= ||x||_2 <= sqrt(P) * max input value.
static float fp16_field_scale(int in_t, int ny, int nx) {
  if (in_t == HV_C64) return 1.0f;  // a field input is taken as |u| < 32768
  const double maxv = in_t == HV_U8 ? 255.0 : 65535.0;
  const double bound = std::sqrt((double)ny * nx) * maxv;
  int k = 0;
  while (bound * std::ldexp(1.0, -k) > 32768.0) ++k;
  return (float)std::ldexp(1.0, -k);
}

// Power-of-two scale of the row-pass output when spectra are stored as fp16.
// After the row transform |X| <= nx * maxv; the angular-spectrum column pass
// is unitary along y, so one column can gather into a single value of at
// most sqrt(ny) * nx * maxv (a coherent full-scale input).  The scale keeps
// that below 32768 (fp16 max 65504): 1/nx for 8-bit frames at every side up
// to 1280, and 2^-k / nx for 16-bit frames (k = 6 at ny = 1024).
static float fp16_row_scale(int in_t, int ny, int nx) {
  const double maxv = in_t == HV_U16 ? 65535.0 : 255.0;
  const double bound = std::sqrt((double)ny) * maxv;
  int k = 0;
  while (bound * std::ldexp(1.0, -k) > 32768.0) ++k;
  return (float)(std::ldexp(1.0, -k) / nx);
}

// ---------------------------------------------------------------- spatial driver

namespace hvi {

// Spatial transform of nf frames starting at `in` into either the AS column
// output Z (as_z_only, real AS input: row inverse left to the caller) or the
// field F.  Returns the buffers used through zbuf/fbuf.
// Fixed workspaces for the entry point that allocates nothing: regions of
// the library's static device scratch, one per workspace slot.
struct FixedWs {
  static constexpr int kSlots = 3;
  void* ptr[kSlots];
  size_t cap[kSlots];
};

struct SpatialOut {
  void* z = nullptr;   // [nf][ny][nx] after the AS column pass (AS only)
  void* f = nullptr;   // [nf][ny][nx] field
  bool half = false;
  float z_to_field = 1.f;  // field = z_to_field * IDFT_x(z)
  float f_scale = 1.f;     // stored field = f_scale * U
};

// A workspace of `bytes` for `slot`: the context's per-stream buffer (grown
// on demand), or, for the entry point that allocates nothing, a fixed region
// of the library's static device scratch (too small: HV_ERR_SHAPE).
static hv_status ws_get(Ctx* c, hipStream_t st, int slot, size_t bytes, const FixedWs* fixed, void** out) {
  if (fixed) {
    if (slot < 0 || slot >= FixedWs::kSlots || bytes > fixed->cap[slot])
      return fail(HV_ERR_SHAPE, "workspace slot %d needs %zu bytes, the fixed scratch holds %zu", slot, bytes,
                  slot >= 0 && slot < FixedWs::kSlots ? fixed->cap[slot] : (size_t)0);
    *out = fixed->ptr[slot];
    return HV_OK;
  }
  DevBuf& b = c->work(st, slot);
  hv_status s = b.ensure(bytes, &c->held);
  if (s) return s;
  *out = b.ptr;
  return HV_OK;
}

// A launch, timed by events when timing is on, untimed with fixed
// workspaces (that path creates no events).
template <class F>
static hv_status run(Ctx* c, const char* name, hipStream_t st, const FixedWs* fixed, F&& f) {
  return fixed ? f() : timed(c, name, st, std::forward<F>(f));
}

hv_status spatial(Ctx* c, const void* in, int in_t, int nf, int ny, int nx, const hv_optics& o, bool mixed,
                  bool want_field, float f_scale, hipStream_t st, SpatialOut& out, const FixedWs* fixed = nullptr) {
  const size_t cplx = mixed ? 4 : 8;
  const size_t frame = (size_t)ny * nx;
  const float s1 = mixed ? fp16_row_scale(in_t, ny, nx) : 1.0f;
  const bool build = fixed == nullptr;
  out.half = mixed;
  out.f_scale = f_scale;
  hv_status s;
  if (o.method == HV_AS) {
    AsPlan* p = c->as_plan(ny, nx, o, &s, build);
    if (!p) return s;
    void *zb = nullptr, *tb = nullptr;
    if ((s = ws_get(c, st, 1, (size_t)nf * frame * cplx, fixed, &zb))) return s;
    if (in_t == HV_C64 || !pow2_in(nx, 64, 1024) || !pow2_in(ny, 64, 1024)) {
      // complex rows (no real-input packing), full columns: any supported side
      if ((s = ws_get(c, st, 0, (size_t)nf * frame * cplx, fixed, &tb))) return s;
      if ((s = run(c, "rows_c2c", st, fixed, [&] { return launch_rows_c2c(in, in_t, tb, mixed, nullptr, nullptr, -1, nf, ny, nx, s1, st); }))) return s;
      if ((s = run(c, "col_full", st, fixed, [&] { return launch_col_full(tb, zb, mixed, p->ht_ptr(), nf, ny, nx, st); }))) return s;
    } else {
      if ((s = ws_get(c, st, 0, (size_t)nf * (frame / 2) * cplx, fixed, &tb))) return s;
      if ((s = run(c, "row_r2c", st, fixed, [&] { return launch_row_r2c(in, (hv_dtype)in_t, tb, mixed, nf, ny, nx, s1, st); }))) return s;
      if ((s = run(c, "col_as", st, fixed, [&] { return launch_col_as(tb, zb, mixed, p->hs_ptr(), nf, ny, nx, st); }))) return s;
    }
    out.z = zb;
    out.z_to_field = 1.0f / (nx * s1);
    if (want_field) {
      void* fb = nullptr;
      if ((s = ws_get(c, st, 2, (size_t)nf * frame * cplx, fixed, &fb))) return s;
      if ((s = run(c, "row_inv", st, fixed, [&] { return launch_row_inv(zb, mixed, fb, mixed, nf, ny, nx, out.z_to_field * f_scale, st); }))) return s;
      out.f = fb;
    }
    return HV_OK;
  }
  FresnelPlan* p = c->fresnel_plan(ny, nx, o, &s, build);
  if (!p) return s;
  const int dir = o.z_m > 0 ? -1 : +1;
  void *tb = nullptr, *fb = nullptr;
  if ((s = ws_get(c, st, 0, (size_t)nf * frame * cplx, fixed, &tb))) return s;
  if ((s = ws_get(c, st, 2, (size_t)nf * frame * cplx, fixed, &fb))) return s;
  const float2* q = (const float2*)p->tables.ptr;
  if ((s = run(c, "fresnel_rows", st, fixed, [&] { return launch_rows_c2c(in, in_t, tb, mixed, q, q + nx, dir, nf, ny, nx, s1, st); })))
    return s;
  const float unit = (float)(1.0 / std::sqrt((double)nx * ny));
  if ((s = run(c, "fresnel_cols", st, fixed, [&] {
         return launch_fresnel_cols(tb, mixed, fb, mixed, q + nx + ny, q + 2 * nx + ny, dir, nf, ny, nx,
                                    unit / s1 * f_scale, st);
       })))
    return s;
  out.f = fb;
  return HV_OK;
}

}  // namespace hvi

// ---------------------------------------------------------------- static scratch

// Static device scratch of hv_stft_moments_noalloc.  In host code the name
// `scratch` is a host-side stand-in, not a device address: the address of
// each GPU's copy is taken once per device by hipGetSymbolAddress at
// context creation (that device current), kept in g_scratch, and used
// wherever host code needs the array.
static constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
struct ScratchAddr {
  void* ptr = nullptr;
  hipError_t err = hipSuccess;
};
std::mutex g_scratch_mu;
std::map<int, ScratchAddr> g_scratch;  // device -> its copy of the scratch
}  // namespace

static void scratch_setup(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch.count(device) && g_scratch[device].ptr) return;
  ScratchAddr a;
  a.err = hipGetSymbolAddress(&a.ptr, HIP_SYMBOL(scratch));
  if (a.err != hipSuccess) {
    (void)hipGetLastError();
    a.ptr = nullptr;
  }
  g_scratch[device] = a;
}

static hv_status scratch_of(int device, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find(device);
  if (it == g_scratch.end() || !it->second.ptr)
    return fail(HV_ERR_DEVICE, "the static scratch of device %d could not be located: %s", device,
                it == g_scratch.end() ? "no context was created on it" : hipGetErrorString(it->second.err));
  *out = it->second.ptr;
  return HV_OK;
}

// ---------------------------------------------------------------- C-ABI

extern "C" {

const char* hv_last_error(void) { return hvi::last_error(); }

hv_status hv_ctx_create(int device, size_t hbm_budget_bytes, hv_ctx** out) {
  if (!out) return fail(HV_ERR_ARG, "out is NULL");
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    return fail(HV_ERR_DEVICE, "no HIP device available");
  }
  if (device < 0 || device >= count) return fail(HV_ERR_ARG, "device %d out of range (%d devices)", device, count);
  if (hipSetDevice(device) != hipSuccess) return fail(HV_ERR_DEVICE, "hipSetDevice(%d) failed", device);
  hv_ctx* c = new (std::nothrow) hv_ctx();
  if (!c) return fail(HV_ERR_NOMEM, "host allocation failed");
  c->device = device;
  c->budget = hbm_budget_bytes;
  if (const char* e = std::getenv("HV_CHUNK_FRAMES")) c->chunk_frames = std::atoi(e);
  if (const char* e = std::getenv("HV_STFT_ORDER")) {
    const int o = std::atoi(e);
    if (o == HV_ORDER_AUTO || o == HV_ORDER_FRAMES_FIRST || o == HV_ORDER_BAND_FIRST) c->stft_order = o;
  }
  // the device address of this device's static scratch (no-allocation entry point)
  scratch_setup(device);
  *out = c;
  return HV_OK;
}

void hv_ctx_destroy(hv_ctx* ctx) {
  if (!ctx) return;
  // teardown cannot report: a failing device still has its host state freed
  (void)hipSetDevice(ctx->device);
  serve_shutdown(ctx);
  (void)hipDeviceSynchronize();
  (void)hipGetLastError();
  delete ctx;
}

size_t hv_ctx_workspace_bytes(const hv_ctx* ctx) { return ctx ? ctx->held : 0; }

hv_status hv_ctx_set_chunk_frames(hv_ctx* ctx, int frames) {
  if (!ctx) return fail(HV_ERR_ARG, "context is NULL");
  if (frames < 0) return fail(HV_ERR_ARG, "negative chunk");
  ctx->chunk_frames = frames;
  return HV_OK;
}

hv_status hv_ctx_set_stft_order(hv_ctx* ctx, int order) {
  if (!ctx) return fail(HV_ERR_ARG, "context is NULL");
  if (order != HV_ORDER_AUTO && order != HV_ORDER_FRAMES_FIRST && order != HV_ORDER_BAND_FIRST)
    return fail(HV_ERR_ARG, "unknown order %d", order);
  ctx->stft_order = order;
  return HV_OK;
}

hv_status hv_ctx_set_timing(hv_ctx* ctx, int on) {
  if (!ctx) return fail(HV_ERR_ARG, "context is NULL");
  ctx->timing.reset();
  ctx->timing.on = on != 0;
  return HV_OK;
}

hv_status hv_ctx_kernel_time(hv_ctx* ctx, const char* name, double* total_ms, long* launches) {
  if (!ctx || !name || !total_ms || !launches) return fail(HV_ERR_ARG, "NULL argument");
  ctx->timing.collect();
  auto it = ctx->timing.acc.find(name);
  *total_ms = it == ctx->timing.acc.end() ? 0.0 : it->second.first;
  *launches = it == ctx->timing.acc.end() ? 0 : it->second.second;
  return HV_OK;
}

hv_status hv_band_bins(const hv_temporal* tp, int* nbins, int* bins, double* freqs) {
  if (!tp || !nbins) return fail(HV_ERR_ARG, "NULL argument");
  if (tp->window <= 0 || !(tp->fs_hz > 0)) return fail(HV_ERR_ARG, "window and fs must be positive");
  std::vector<int> b;
  std::vector<double> f;
  *nbins = band_bins(*tp, b, f);
  for (size_t i = 0; i < b.size(); ++i) {
    if (bins) bins[i] = b[i];
    if (freqs) freqs[i] = f[i];
  }
  return HV_OK;
}

hv_status hv_field_scale(int in_t, int ny, int nx, float* scale) {
  if (!scale) return fail(HV_ERR_ARG, "NULL argument");
  if (ny <= 0 || nx <= 0) return fail(HV_ERR_SHAPE, "frame %d x %d", ny, nx);
  hv_status s;
  if ((s = check_dtype(in_t, true))) return s;
  *scale = fp16_field_scale(in_t, ny, nx);
  return HV_OK;
}

hv_status hv_propagate(hv_ctx* ctx, const void* in, int in_t, int n, int ny, int nx, const hv_optics* optics,
                       int prec, int out_t, void* out, void* hip_stream) {
  hv_status s;
  if ((s = enter(ctx))) return s;
  std::lock_guard<std::recursive_mutex> lock(ctx->mu);
  if ((s = check_frame(n, ny, nx)) || (s = check_optics(optics)) || (s = check_dtype(in_t, true))) return s;
  if (prec != HV_PREC_FP32 && prec != HV_PREC_MIXED) return fail(HV_ERR_ARG, "unknown precision %d", prec);
  if (out_t != HV_C64 && out_t != HV_C32H) return fail(HV_ERR_ARG, "output dtype %d is not a field type", out_t);
  if (n == 0) return HV_OK;
  if (!in || !out) return fail(HV_ERR_ARG, "NULL data pointer");
  if ((s = check_aligned(in))) return s;
  hipStream_t st = (hipStream_t)hip_stream;
  const bool mixed = prec == HV_PREC_MIXED;
  // an fp16 field holds U * osc, a power of two that keeps every field the
  // input type can give inside the fp16 range
  const bool half_out = out_t == HV_C32H;
  const float osc = half_out ? fp16_field_scale(in_t, ny, nx) : 1.f;
  const size_t out_elem = half_out ? 4 : 8;
  const int chunk = ctx->chunk_frames_for(ny, nx, mixed);
  const size_t frame = (size_t)ny * nx;
  for (int f0 = 0; f0 < n; f0 += chunk) {
    const int nf = n - f0 < chunk ? n - f0 : chunk;
    const char* src = (const char*)in + (size_t)f0 * frame * in_elem(in_t);
    void* dst = (char*)out + (size_t)f0 * frame * out_elem;
    SpatialOut so;
    if (optics->method == HV_AS) {
      if ((s = spatial(ctx, src, in_t, nf, ny, nx, *optics, mixed, false, 1.f, st, so))) return s;
      if ((s = timed(ctx, "row_inv", st, [&] {
             return launch_row_inv(so.z, so.half, dst, half_out, nf, ny, nx, so.z_to_field * osc, st);
           })))
        return s;
    } else {
      // Fresnel writes the field straight from its column pass
      const bool mix = mixed;
      const int dir = optics->z_m > 0 ? -1 : +1;
      FresnelPlan* p = ctx->fresnel_plan(ny, nx, *optics, &s);
      if (!p) return s;
      DevBuf& tb = ctx->work(st, 0);
      if ((s = tb.ensure((size_t)nf * frame * (mix ? 4 : 8), &ctx->held))) return s;
      const float s1 = mix ? fp16_row_scale(in_t, ny, nx) : 1.0f;
      const float2* q = (const float2*)p->tables.ptr;
      if ((s = timed(ctx, "fresnel_rows", st, [&] {
             return launch_rows_c2c(src, in_t, tb.ptr, mix, q, q + nx, dir, nf, ny, nx, s1, st);
           })))
        return s;
      const float unit = (float)(1.0 / std::sqrt((double)nx * ny));
      if ((s = timed(ctx, "fresnel_cols", st, [&] {
             return launch_fresnel_cols(tb.ptr, mix, dst, half_out, q + nx + ny, q + 2 * nx + ny, dir, nf, ny, nx,
                                        unit / s1 * osc, st);
           })))
        return s;
    }
  }
  return HV_OK;
}

// Bytes per pixel and window of the two orders of the AS moments path
// (camera values read, intermediate spectra written and read, three f32
// images written): frames first moves every frame through the row pass
// (in + half spectrum), the column pass (half spectrum in, full out) and
// the fused temporal kernel (W full spectra); band first reads the window's
// raw frames once and moves nb bin fields through three passes.
static bool band_first_cheaper(int w, int stride, int nb, int in_bytes, bool mixed) {
  const double e = mixed ? 4.0 : 8.0;
  const double frames_first = stride * (in_bytes + 2.0 * e) + w * e;
  const double band_first = w * (double)in_bytes + 4.0 * nb * e;
  return band_first < frames_first;
}

// Windows per band-first chunk: about 96 MiB of bin fields (13 windows of
// 14 bins at 256 x 256 FP32), or the frames set by hv_ctx_set_chunk_frames.
static int band_chunk_windows(const Ctx* c, int ny, int nx, int nb, int w, int stride, bool mixed) {
  long g;
  if (c->chunk_frames > 0) {
    g = c->chunk_frames >= w ? (c->chunk_frames - w) / stride + 1 : 1;
  } else {
    g = (96L << 20) / ((long)nb * ny * nx * (mixed ? 4 : 8));
  }
  return g < 1 ? 1 : g > 4096 ? 4096 : (int)g;
}

// Band-first AS moments: per chunk of windows, the bins' row spectra from
// the raw frames (KA), the AS column pass in place (KB), the inverse row
// pass with the weighted powers (KC).  Chunks alternate between two
// streams like the frames-first driver.
static hv_status stft_band_first(Ctx* ctx, const void* in, int in_t, int ny, int nx, const hv_optics& o,
                                 const DftPlan& dp, int w, int stride, int nwin_total, int gw, bool mixed,
                                 float* m0, float* m1, float* m2, float2* spec, hipStream_t caller,
                                 bool two_lanes) {
  hv_status s;
  AsPlan* p = ctx->as_plan(ny, nx, o, &s);
  if (!p) return s;
  const int nb = (int)dp.bins.size();
  const size_t frame = (size_t)ny * nx;
  const size_t per_win = (size_t)nb * frame * (mixed ? 4 : 8);
  // fp16 storage: values scaled so that the worst case (every camera value
  // at full scale, coherent) stays below the fp16 maximum through the passes
  // (a bin sums W frames, hence the extra 1/W)
  const float s1 = fp16_row_scale(in_t, ny, nx);
  const float sc = mixed ? s1 / w : 1.0f;
  const float amp = 1.0f / (nx * sc);
  Ctx::Lane2* l2 = nullptr;
  hipStream_t st = caller;
  if (two_lanes && nwin_total > gw) {
    if (!(l2 = ctx->lane2(caller, &s))) return s;
    if ((s = l2->fork_from(caller))) return s;
  }
  hv_status res = HV_OK;
  for (int j0 = 0, c = 0; j0 < nwin_total && res == HV_OK; j0 += gw, ++c) {
    st = (l2 && (c & 1)) ? l2->s : caller;
    res = [&]() -> hv_status {
      const int g_n = nwin_total - j0 < gw ? nwin_total - j0 : gw;
      const char* src = (const char*)in + (size_t)j0 * stride * frame * in_elem(in_t);
      DevBuf& b = ctx->work(st, 1);
      if ((s = b.ensure((size_t)g_n * per_win, &ctx->held))) return s;
      float* o0 = m0 ? m0 + (size_t)j0 * frame : nullptr;
      float* o1 = m1 ? m1 + (size_t)j0 * frame : nullptr;
      float* o2 = m2 ? m2 + (size_t)j0 * frame : nullptr;
      float2* os = spec ? spec + (size_t)j0 * nb * frame : nullptr;
      if ((s = timed(ctx, "band_rows", st, [&] {
             return launch_band_rows(src, in_t, b.ptr, mixed, ny, nx, stride, g_n, w, nb, dp.mtiles,
                                     (const hv_h8*)dp.ar_hi.ptr, (const hv_h8*)dp.ar_lo.ptr, sc, st);
           })))
        return s;
      if ((s = timed(ctx, "band_cols", st, [&] {
             return launch_band_cols(b.ptr, mixed, p->ht_ptr(), g_n * nb, ny, nx, st);
           })))
        return s;
      return timed(ctx, "band_power", st, [&] {
        return launch_band_power(b.ptr, mixed, ny, nx, g_n, nb, dp.mtiles, (const float*)dp.wts.ptr, amp, o0, o1,
                                 o2, os, st);
      });
    }();
  }
  if (l2) {
    const hv_status j = l2->join_into(caller);
    if (res == HV_OK) res = j;
  }
  return res;
}

// One chunk of the frames-first order: windows j0 .. j0 + g_n - 1 of the
// call (frames from j0 * stride), spatial passes then the temporal GEMM with
// the moment epilogue; outputs at window j0 of m0/m1/m2/spec.
static hv_status frames_first_chunk(Ctx* ctx, const void* in, int in_t, int ny, int nx, const hv_optics& o,
                                    const CoefGemm& g, int nb, int w, int stride, int j0, int g_n, bool mixed,
                                    float* m0, float* m1, float* m2, float2* spec, hipStream_t st,
                                    const FixedWs* fixed) {
  hv_status s;
  const size_t frame = (size_t)ny * nx;
  const float fsc = mixed ? fp16_field_scale(in_t, ny, nx) : 1.f;
  const int nf = (g_n - 1) * stride + w;
  const char* src = (const char*)in + (size_t)j0 * stride * frame * in_elem(in_t);
  float* o0 = m0 ? m0 + (size_t)j0 * frame : nullptr;
  float* o1 = m1 ? m1 + (size_t)j0 * frame : nullptr;
  float* o2 = m2 ? m2 + (size_t)j0 * frame : nullptr;
  float2* os = spec ? spec + (size_t)j0 * nb * frame : nullptr;
  const bool fused = o.method == HV_AS && rowinv_coef_fits(nx, w);
  SpatialOut so;
  if ((s = spatial(ctx, src, in_t, nf, ny, nx, o, mixed, !fused, fsc, st, so, fixed))) return s;
  if (fused) {
    // B = z_to_field * IDFT_x(z) * bsc with bsc keeping fp16 in range
    const float bsc = mixed ? so.z_to_field * fsc : 1.f;
    const float amp = mixed ? 1.f / fsc : so.z_to_field;
    return run(ctx, "rowinv_coef", st, fixed, [&] {
      return launch_rowinv_coef(so.z, so.half, ny, nx, stride, g_n, g, mixed, bsc, amp, o0, o1, o2, os, st);
    });
  }
  return run(ctx, "field_coef", st, fixed, [&] {
    return launch_field_coef(so.f, so.half, (long)frame, stride, g_n, g, mixed, 1.f, 1.f / so.f_scale, o0, o1, o2,
                             os, st);
  });
}

// Shared driver of hv_stft_moments and hv_stft_bins.
static hv_status stft_impl(hv_ctx* ctx, const void* in, int in_t, int n, int ny, int nx, const hv_optics* optics,
                           const hv_temporal* tp, int prec, float* m0, float* m1, float* m2, float2* spec,
                           void* hip_stream, bool two_lanes, bool fixed_ws = false);

// The serving loop's entry: one stream per call, on workspaces allocated
// at admission (fixed_ws: nothing grows here).
hv_status hvi_stft_common(hv_ctx* ctx, const void* in, int in_t, int n, int ny, int nx, const hv_optics* optics,
                          const hv_temporal* tp, int prec, float* m0, float* m1, float* m2, float2* spec,
                          void* hip_stream) {
  return stft_impl(ctx, in, in_t, n, ny, nx, optics, tp, prec, m0, m1, m2, spec, hip_stream, false, true);
}

static hv_status stft_impl(hv_ctx* ctx, const void* in, int in_t, int n, int ny, int nx, const hv_optics* optics,
                           const hv_temporal* tp, int prec, float* m0, float* m1, float* m2, float2* spec,
                           void* hip_stream, bool two_lanes, bool fixed_ws) {
  hv_status s;
  if ((s = enter(ctx))) return s;
  std::lock_guard<std::recursive_mutex> lock(ctx->mu);
  if ((s = check_frame(n, ny, nx))) return s;
  if (!tp) return fail(HV_ERR_ARG, "temporal is NULL");
  const int w = tp->window, stride = tp->stride;
  if (w != 8 && w != 16 && w != 32 && w != 64) return fail(HV_ERR_SHAPE, "window %d: use 8, 16, 32 or 64", w);
  if (stride <= 0) return fail(HV_ERR_ARG, "stride must be positive");
  if (!(tp->fs_hz > 0)) return fail(HV_ERR_ARG, "fs must be positive");
  if (prec != HV_PREC_FP32 && prec != HV_PREC_MIXED) return fail(HV_ERR_ARG, "unknown precision %d", prec);
  if (optics) {
    if ((s = check_optics(optics)) || (s = check_dtype(in_t, true))) return s;
  } else if (in_t != HV_C64) {
    return fail(HV_ERR_ARG, "without optics the input must be a field (HV_C64)");
  }
  if (n < w) return fail(HV_ERR_SHAPE, "%d frames hold no complete window of %d", n, w);
  if (!in) return fail(HV_ERR_ARG, "input is NULL");
  if ((s = check_aligned(in))) return s;
  if (!m0 && !m1 && !m2 && !spec) return fail(HV_ERR_ARG, "no output requested");
  DftPlan* dp = ctx->dft_plan(*tp, &s);
  if (!dp) return s;
  const int nwin_total = (n - w) / stride + 1;
  const bool mixed = prec == HV_PREC_MIXED;
  const size_t frame = (size_t)ny * nx;
  hipStream_t st = (hipStream_t)hip_stream;
  CoefGemm g{w, dp->mtiles, (int)dp->bins.size(), (const float*)dp->a32.ptr, (const hv_h8*)dp->a16hi.ptr,
             (const hv_h8*)dp->a16lo.ptr, (const float*)dp->wts.ptr, 3};
  const int nb = (int)dp->bins.size();
  if (!optics) {
    const float bsc = mixed ? fp16_field_scale(HV_C64, ny, nx) : 1.f;
    return launch_field_coef(in, false, (long)frame, stride, nwin_total, g, mixed, bsc, mixed ? 1.f / bsc : 1.f, m0,
                             m1, m2, spec, st);
  }
  if (optics->method == HV_AS && band_first_fits(ny, nx, in_t) && ctx->stft_order != HV_ORDER_FRAMES_FIRST &&
      (ctx->stft_order == HV_ORDER_BAND_FIRST || band_first_cheaper(w, stride, nb, (int)in_elem(in_t), mixed))) {
    int gb = band_chunk_windows(ctx, ny, nx, nb, w, stride, mixed);
    if (gb > nwin_total) gb = nwin_total;
    // the serving loop's streams run on workspaces sized at admission (for
    // either order): take this order there only when it fits the one held
    const bool fits = !fixed_ws || ctx->work(st, 1).bytes >= (size_t)gb * nb * frame * (mixed ? 4 : 8);
    if (fits)
      return stft_band_first(ctx, in, in_t, ny, nx, *optics, *dp, w, stride, nwin_total, gb, mixed, m0, m1, m2,
                             spec, st, two_lanes);
  }
  const int chunk = ctx->chunk_frames_for(ny, nx, mixed);
  int gw = chunk >= w ? (chunk - w) / stride + 1 : 1;
  if (gw < 1) gw = 1;
  // Chunks alternate between the caller's stream and a second one (per-kernel
  // timing events, when on, bracket each launch on its own stream and so
  // time it as it runs beside the other stream's work).
  Ctx::Lane2* l2 = nullptr;
  if (two_lanes && nwin_total > gw) {
    if (!(l2 = ctx->lane2(st, &s))) return s;
    if ((s = l2->fork_from(st))) return s;
  }
  hv_status res = HV_OK;
  const hipStream_t caller = st;
  for (int j0 = 0, c = 0; j0 < nwin_total && res == HV_OK; j0 += gw, ++c) {
    st = (l2 && (c & 1)) ? l2->s : caller;
    const int g_n = nwin_total - j0 < gw ? nwin_total - j0 : gw;
    res = frames_first_chunk(ctx, in, in_t, ny, nx, *optics, g, nb, w, stride, j0, g_n, mixed, m0, m1, m2, spec, st,
                             nullptr);
  }
  if (l2) {  // join, also after an error, so no work of this call outlives it on the second stream
    const hv_status j = l2->join_into(caller);
    if (res == HV_OK) res = j;
  }
  return res;
}

hv_status hv_stft_moments(hv_ctx* ctx, const void* in, int in_t, int n, int ny, int nx, const hv_optics* optics,
                          const hv_temporal* temporal, int prec, float* m0, float* m1, float* m2,
                          void* hip_stream) {
  return stft_impl(ctx, in, in_t, n, ny, nx, optics, temporal, prec, m0, m1, m2, nullptr, hip_stream, true);
}

// ---------------------------------------------------------------- the entry point that allocates nothing

hv_status hv_stft_moments_noalloc(hv_ctx* ctx, const void* in, int in_t, int n, int ny, int nx,
                                  const hv_optics* optics, const hv_temporal* tp, int prec, float* m0, float* m1,
                                  float* m2, void* hip_stream) {
  hv_status s;
  if ((s = enter(ctx))) return s;
  std::lock_guard<std::recursive_mutex> lock(ctx->mu);
  if ((s = check_frame(n, ny, nx))) return s;
  if (!tp) return fail(HV_ERR_ARG, "temporal is NULL");
  const int w = tp->window, stride = tp->stride;
  if (w != 8 && w != 16 && w != 32 && w != 64) return fail(HV_ERR_SHAPE, "window %d: use 8, 16, 32 or 64", w);
  if (stride <= 0) return fail(HV_ERR_ARG, "stride must be positive");
  if (!(tp->fs_hz > 0)) return fail(HV_ERR_ARG, "fs must be positive");
  if (prec != HV_PREC_FP32 && prec != HV_PREC_MIXED) return fail(HV_ERR_ARG, "unknown precision %d", prec);
  if (optics) {
    if ((s = check_optics(optics)) || (s = check_dtype(in_t, true))) return s;
  } else if (in_t != HV_C64) {
    return fail(HV_ERR_ARG, "without optics the input must be a field (HV_C64)");
  }
  if (n < w) return fail(HV_ERR_SHAPE, "%d frames hold no complete window of %d", n, w);
  if (!in) return fail(HV_ERR_ARG, "input is NULL");
  if ((s = check_aligned(in))) return s;
  if (!m0 && !m1 && !m2) return fail(HV_ERR_ARG, "no output requested");
  DftPlan* dp = ctx->dft_plan(*tp, &s, false);
  if (!dp) return s;
  const int nwin_total = (n - w) / stride + 1;
  const bool mixed = prec == HV_PREC_MIXED;
  const size_t frame = (size_t)ny * nx;
  hipStream_t st = (hipStream_t)hip_stream;
  CoefGemm g{w, dp->mtiles, (int)dp->bins.size(), (const float*)dp->a32.ptr, (const hv_h8*)dp->a16hi.ptr,
             (const hv_h8*)dp->a16lo.ptr, (const float*)dp->wts.ptr, 3};
  const int nb = (int)dp->bins.size();
  if (!optics) {  // a field in memory: the temporal kernel alone, no workspace
    const float bsc = mixed ? fp16_field_scale(HV_C64, ny, nx) : 1.f;
    return launch_field_coef(in, false, (long)frame, stride, nwin_total, g, mixed, bsc, mixed ? 1.f / bsc : 1.f, m0,
                             m1, m2, nullptr, st);
  }
  void* base = nullptr;
  if ((s = scratch_of(ctx->device, &base))) return s;
  // bytes per frame of the three workspaces of the frames-first order (the
  // same sizes the spatial passes ask for)
  const size_t cplx = mixed ? 4 : 8;
  const bool as = optics->method == HV_AS;
  const bool real_rows = as && in_t != HV_C64 && pow2_in(nx, 64, 1024) && pow2_in(ny, 64, 1024);
  const bool fused = as && rowinv_coef_fits(nx, w);
  const size_t per[3] = {real_rows ? frame / 2 * cplx : frame * cplx, as ? frame * cplx : 0,
                         fused ? 0 : frame * cplx};
  const size_t per_frame = per[0] + per[1] + per[2];
  auto fits = [&](long frames) {
    size_t used = 0;
    for (size_t b : per) used += (b * (size_t)frames + 255) / 256 * 256;
    return used <= kScratchBytes;
  };
  if (!fits(w))
    return fail(HV_ERR_SHAPE,
                "one window of %d frames of %dx%d needs %zu bytes of workspace; the fixed scratch holds %zu", w, nx,
                ny, per_frame * (size_t)w, kScratchBytes);
  int gw = 1;
  while (gw < nwin_total && fits((long)gw * stride + w)) ++gw;  // windows per chunk
  const long nf_max = (long)(gw - 1) * stride + w;
  FixedWs fx{};
  char* at = (char*)base;
  for (int k = 0; k < FixedWs::kSlots; ++k) {
    fx.ptr[k] = at;
    fx.cap[k] = per[k] * (size_t)nf_max;
    at += (fx.cap[k] + 255) / 256 * 256;
  }
  for (int j0 = 0; j0 < nwin_total; j0 += gw) {
    const int g_n = nwin_total - j0 < gw ? nwin_total - j0 : gw;
    if ((s = frames_first_chunk(ctx, in, in_t, ny, nx, *optics, g, nb, w, stride, j0, g_n, mixed, m0, m1, m2,
                                nullptr, st, &fx)))
      return s;
  }
  return HV_OK;
}

hv_status hv_stft_bins(hv_ctx* ctx, const void* in, int in_t, int n, int ny, int nx, const hv_optics* optics,
                       const hv_temporal* temporal, int prec, void* spec, void* hip_stream) {
  return stft_impl(ctx, in, in_t, n, ny, nx, optics, temporal, prec, nullptr, nullptr, nullptr, (float2*)spec,
                   hip_stream, true);
}

hv_status hv_stft_moments_host(hv_ctx* ctx, const void* host_in, int in_t, int n, int ny, int nx,
                               const hv_optics* optics, const hv_temporal* tp, int prec, float* host_m0,
                               float* host_m1, float* host_m2, void* hip_stream) {
  hv_status s;
  if ((s = enter(ctx))) return s;
  std::lock_guard<std::recursive_mutex> lock(ctx->mu);
  if ((s = check_frame(n, ny, nx)) || (s = check_optics(optics)) || (s = check_dtype(in_t, false))) return s;
  if (!tp) return fail(HV_ERR_ARG, "temporal is NULL");
  const int w = tp->window, stride = tp->stride;
  if (stride <= 0 || w <= 0) return fail(HV_ERR_ARG, "window and stride must be positive");
  if (n < w) return fail(HV_ERR_SHAPE, "%d frames hold no complete window of %d", n, w);
  if (!host_in) return fail(HV_ERR_ARG, "input is NULL");
  if (!host_m0 && !host_m1 && !host_m2) return fail(HV_ERR_ARG, "no output requested");
  const bool mixed = prec == HV_PREC_MIXED;
  const int nwin_total = (n - w) / stride + 1;
  const size_t frame = (size_t)ny * nx, fbytes = frame * in_elem(in_t);
  const int chunk = std::max(ctx->chunk_frames_for(ny, nx, mixed), w);
  const int gw = (chunk - w) / stride + 1;
  const int cf = (gw - 1) * stride + w;  // frames staged per chunk
  hipStream_t st = (hipStream_t)hip_stream;
  float* const host_out[3] = {host_m0, host_m1, host_m2};
  // staging per stream: raw frames in, moment images out
  auto stage = [&](hipStream_t cs, void** in_dev, float** out_dev) -> hv_status {
    DevBuf& bi = ctx->work(cs, 20);
    hv_status e = bi.ensure((size_t)cf * fbytes, &ctx->held);
    if (e) return e;
    *in_dev = bi.ptr;
    for (int k = 0; k < 3; ++k) {
      out_dev[k] = nullptr;
      if (!host_out[k]) continue;
      DevBuf& bo = ctx->work(cs, 21 + k);
      if ((e = bo.ensure((size_t)gw * frame * 4, &ctx->held))) return e;
      out_dev[k] = (float*)bo.ptr;
    }
    return HV_OK;
  };
  void* in_dev[2];
  float* out_dev[2][3];
  if ((s = stage(st, &in_dev[0], out_dev[0]))) return s;
  Ctx::Lane2* l2 = nullptr;
  if (nwin_total > gw) {
    if (!(l2 = ctx->lane2(st, &s))) return s;
    if ((s = stage(l2->s, &in_dev[1], out_dev[1]))) return s;
    if ((s = l2->fork_from(st))) return s;
  }
  // Each chunk is copied in, processed and copied out on its own stream;
  // with two streams one chunk's copies overlap the other chunk's kernels.
  hv_status res = HV_OK;
  for (int j0 = 0, c = 0; j0 < nwin_total && res == HV_OK; j0 += gw, ++c) {
    const int lane = (l2 && (c & 1)) ? 1 : 0;
    const hipStream_t cs = lane ? l2->s : st;
    const int g_n = nwin_total - j0 < gw ? nwin_total - j0 : gw;
    const int nf = (g_n - 1) * stride + w;
    if (hipMemcpyAsync(in_dev[lane], (const char*)host_in + (size_t)j0 * stride * fbytes, (size_t)nf * fbytes,
                       hipMemcpyHostToDevice, cs) != hipSuccess) {
      res = fail(HV_ERR_DEVICE, "frame upload failed");
      break;
    }
    res = stft_impl(ctx, in_dev[lane], in_t, nf, ny, nx, optics, tp, prec, out_dev[lane][0], out_dev[lane][1],
                    out_dev[lane][2], nullptr, cs, false);
    for (int k = 0; k < 3 && res == HV_OK; ++k)
      if (host_out[k] && hipMemcpyAsync(host_out[k] + (size_t)j0 * frame, out_dev[lane][k],
                                        (size_t)g_n * frame * 4, hipMemcpyDeviceToHost, cs) != hipSuccess)
        res = fail(HV_ERR_DEVICE, "image download failed");
  }
  if (l2) {  // join, also after an error
    const hv_status j = l2->join_into(st);
    if (res == HV_OK) res = j;
  }
  return res;
}

hv_status hv_stft_volume(hv_ctx* ctx, const void* in, int in_t, int n, int ny, int nx, const hv_optics* optics,
                         int window, int stride, int prec, float* power, void* hip_stream) {
  hv_status s;
  if ((s = enter(ctx))) return s;
  std::lock_guard<std::recursive_mutex> lock(ctx->mu);
  if ((s = check_frame(n, ny, nx))) return s;
  if (window != 128 && window != 256 && window != 512)
    return fail(HV_ERR_SHAPE, "volume window %d: use 128, 256 or 512", window);
  if (stride <= 0) return fail(HV_ERR_ARG, "stride must be positive");
  if (prec != HV_PREC_FP32 && prec != HV_PREC_MIXED) return fail(HV_ERR_ARG, "unknown precision %d", prec);
  if (optics) {
    if ((s = check_optics(optics)) || (s = check_dtype(in_t, true))) return s;
  } else if (in_t != HV_C64) {
    return fail(HV_ERR_ARG, "without optics the input must be a field (HV_C64)");
  }
  if (n < window) return fail(HV_ERR_SHAPE, "%d frames hold no complete window of %d", n, window);
  if (!in || !power) return fail(HV_ERR_ARG, "NULL data pointer");
  if ((s = check_aligned(in))) return s;
  const bool mixed = prec == HV_PREC_MIXED;
  const int w = window;
  const int nwin_total = (n - w) / stride + 1;
  const size_t frame = (size_t)ny * nx;
  hipStream_t st = (hipStream_t)hip_stream;
  if (!optics)
    return timed(ctx, "time_fft", st, [&] {
      return launch_time_fft(in, false, (long)frame, stride, nwin_total, w, 1.f, power, st);
    });
  const int chunk = std::max(ctx->chunk_frames_for(ny, nx, mixed), w);
  const int gw = (chunk - w) / stride + 1;
  const float fsc = mixed ? fp16_field_scale(in_t, ny, nx) : 1.f;
  // chunks alternate between the caller's stream and a second one
  Ctx::Lane2* l2 = nullptr;
  if (nwin_total > gw) {
    if (!(l2 = ctx->lane2(st, &s))) return s;
    if ((s = l2->fork_from(st))) return s;
  }
  hv_status res = HV_OK;
  const hipStream_t caller = st;
  for (int j0 = 0, c = 0; j0 < nwin_total && res == HV_OK; j0 += gw, ++c) {
    st = (l2 && (c & 1)) ? l2->s : caller;
    const int g_n = nwin_total - j0 < gw ? nwin_total - j0 : gw;
    const int nf = (g_n - 1) * stride + w;
    const char* src = (const char*)in + (size_t)j0 * stride * frame * in_elem(in_t);
    SpatialOut so;
    res = spatial(ctx, src, in_t, nf, ny, nx, *optics, mixed, true, fsc, st, so);
    if (res == HV_OK)
      res = timed(ctx, "time_fft", st, [&] {
        return launch_time_fft(so.f, so.half, (long)frame, stride, g_n, w, 1.f / (so.f_scale * so.f_scale),
                               power + (size_t)j0 * w * frame, st);
      });
  }
  if (l2) {  // join, also after an error
    const hv_status j = l2->join_into(caller);
    if (res == HV_OK) res = j;
  }
  return res;
}

// Sweep limit of the FP64 Jacobi eigensolver (cyclic sweeps converge
// quadratically; W = 64 windows of camera data take well under 20).
static constexpr int kJacobiSweeps = 40;

// Outputs of the eigen-decomposition paths (each nullable except as noted).
struct EigOut {
  float *m0, *m1, *m2;  // PCA: m0 (required) = projection energy; SSA: the moments
  double *eigvals, *cov, *offdiag;
};

// Shared driver of the PCA and SSA + FFT paths (Sec. III-B.1: covariance of
// the window, eigen-decomposition, projection onto a sub-basis).  Per chunk
// of windows: the field (spatial passes), the Gram partials and their FP64
// reduction, the FP64 Jacobi; then, for PCA (ssa == nullptr), the
// projection energy of components comp_lo..comp_hi, and for SSA the
// coefficients of "project onto those components and back, then the DFT of
// the band bins" and the coefficient GEMM with the moment epilogue.
static hv_status eig_path(hv_ctx* ctx, const void* in, int in_t, int n, int ny, int nx, const hv_optics* optics,
                          int w, int stride, int comp_lo, int comp_hi, bool mixed, const DftPlan* ssa,
                          const EigOut& o, hipStream_t st) {
  hv_status s;
  const int nwin_total = (n - w) / stride + 1;
  const size_t frame = (size_t)ny * nx;
  const int npair = ssa ? (int)ssa->bins.size() : comp_hi - comp_lo + 1;
  const int mtiles = ssa ? ssa->mtiles : (npair + 15) / 16;
  const int nblk = (int)std::max<long>(1, std::min<long>(256, (long)frame / 4096));
  // The eigensolve runs one workgroup per window, so a chunk should carry
  // many windows: up to 64 windows, within about 2 GiB of field per stream.
  int chunk = ctx->chunk_frames_for(ny, nx, mixed);
  if (ctx->chunk_frames <= 0) {
    const long by_mem = (2L << 30) / (long)(frame * (mixed ? 4 : 8));
    const long want = std::min<long>((long)63 * stride + w, by_mem);
    if (want > chunk) chunk = (int)want;
  }
  int gw = chunk >= w ? (chunk - w) / stride + 1 : 1;
  if (gw < 1) gw = 1;
  // per-window scratch of one chunk, one set per stream
  struct Scratch {
    void *part, *cv, *ev, *vec, *a32, *a16h, *a16l;
  };
  const size_t M = 2 * (size_t)w;
  auto scratch = [&](hipStream_t cs, Scratch* x) -> hv_status {
    const size_t bytes[7] = {(size_t)gw * nblk * M * M * 4, (size_t)gw * w * w * 16, (size_t)gw * w * 8,
                             (size_t)gw * w * w * 16, (size_t)gw * mtiles * w * 64 * 4,
                             (size_t)gw * mtiles * (w / 8) * 64 * 16, (size_t)gw * mtiles * (w / 8) * 64 * 16};
    void** dst[7] = {&x->part, &x->cv, &x->ev, &x->vec, &x->a32, &x->a16h, &x->a16l};
    for (int i = 0; i < 7; ++i) {
      DevBuf& b = ctx->work(cs, 10 + i);
      hv_status e = b.ensure(bytes[i], &ctx->held);
      if (e) return e;
      *dst[i] = b.ptr;
    }
    return HV_OK;
  };
  const float* wts = nullptr;
  if (ssa) {
    wts = (const float*)ssa->wts.ptr;  // f_k^n of the band bins, as the STFT path
  } else {
    DevBuf& wb = ctx->work(st, 17);  // read-only, shared by both streams
    std::vector<float> hw((size_t)3 * mtiles * 16, 0.f);
    for (int i = 0; i < npair; ++i) hw[i] = 1.f;
    if ((s = wb.upload(hw.data(), hw.size() * 4, &ctx->held))) return s;
    wts = (const float*)wb.ptr;
  }
  const float fsc = mixed ? fp16_field_scale(optics ? in_t : HV_C64, ny, nx) : 1.f;
  // Chunks alternate between the caller's stream and a second one: one
  // chunk's eigensolve (one workgroup per window) overlaps the next chunk's
  // transforms.
  Ctx::Lane2* l2 = nullptr;
  Scratch sc[2];
  if ((s = scratch(st, &sc[0]))) return s;
  if (nwin_total > gw) {
    if (!(l2 = ctx->lane2(st, &s))) return s;
    if ((s = scratch(l2->s, &sc[1]))) return s;
    if ((s = l2->fork_from(st))) return s;
  }
  hv_status res = HV_OK;
  const hipStream_t caller = st;
  for (int j0 = 0, c = 0; j0 < nwin_total && res == HV_OK; j0 += gw, ++c) {
    const bool second = l2 && (c & 1);
    st = second ? l2->s : caller;
    const Scratch& x = sc[second ? 1 : 0];
    res = [&]() -> hv_status {
      const int g_n = nwin_total - j0 < gw ? nwin_total - j0 : gw;
      const int f0 = j0 * stride;
      const int nf = (g_n - 1) * stride + w;
      const void* field;
      bool half;
      float fs;
      if (optics) {
        const char* src = (const char*)in + (size_t)f0 * frame * in_elem(in_t);
        SpatialOut so;
        if ((s = spatial(ctx, src, in_t, nf, ny, nx, *optics, mixed, true, fsc, st, so))) return s;
        field = so.f;
        half = so.half;
        fs = so.f_scale;
      } else {
        field = (const float2*)in + (size_t)f0 * frame;
        half = false;
        fs = fsc;
      }
      if ((s = timed(ctx, "gram", st, [&] {
             return launch_gram_partials(field, half, (long)frame, stride, g_n, w, mixed, half ? 1.f : fs,
                                         (float*)x.part, nblk, st);
           })))
        return s;
      if ((s = launch_gram_reduce((const float*)x.part, g_n, nblk, w, 1.0 / ((double)fs * fs), (double*)x.cv, st)))
        return s;
      if ((s = timed(ctx, "jacobi", st, [&] {
             return launch_jacobi((const double*)x.cv, g_n, w, (double*)x.ev, (double*)x.vec,
                                  o.offdiag ? o.offdiag + j0 : nullptr, kJacobiSweeps, st);
           })))
        return s;
      const size_t at = (size_t)j0 * frame;
      if (ssa) {
        if ((s = launch_ssa_coefs((const double*)x.vec, g_n, w, comp_lo, comp_hi, ssa->bins.data(), npair, mtiles,
                                  (float*)x.a32, (hv_h8*)x.a16h, (hv_h8*)x.a16l, st)))
          return s;
        if ((s = timed(ctx, "ssa_moments", st, [&] {
               return launch_coef_moments(field, half, (long)frame, stride, g_n, w, mtiles, npair,
                                          (const float*)x.a32, (const hv_h8*)x.a16h, (const hv_h8*)x.a16l, wts,
                                          mixed, half ? 1.f : fs, 1.f / fs, o.m0 ? o.m0 + at : nullptr,
                                          o.m1 ? o.m1 + at : nullptr, o.m2 ? o.m2 + at : nullptr, st);
             })))
          return s;
      } else {
        if ((s = launch_proj_coefs((const double*)x.vec, g_n, w, comp_lo, comp_hi, mtiles, (float*)x.a32,
                                   (hv_h8*)x.a16h, (hv_h8*)x.a16l, st)))
          return s;
        if ((s = timed(ctx, "proj_energy", st, [&] {
               return launch_proj_energy(field, half, (long)frame, stride, g_n, w, mtiles, npair,
                                         (const float*)x.a32, (const hv_h8*)x.a16h, (const hv_h8*)x.a16l, wts,
                                         mixed, half ? 1.f : fs, 1.f / fs, o.m0 + at, st);
             })))
          return s;
      }
      if (o.eigvals && hipMemcpyAsync(o.eigvals + (size_t)j0 * w, x.ev, (size_t)g_n * w * 8,
                                      hipMemcpyDeviceToDevice, st) != hipSuccess)
        return fail(HV_ERR_DEVICE, "eigenvalue copy failed");
      if (o.cov && hipMemcpyAsync(o.cov + (size_t)j0 * w * w * 2, x.cv, (size_t)g_n * w * w * 16,
                                  hipMemcpyDeviceToDevice, st) != hipSuccess)
        return fail(HV_ERR_DEVICE, "covariance copy failed");
      return HV_OK;
    }();
  }
  if (l2) {  // join, also after an error
    const hv_status j = l2->join_into(caller);
    if (res == HV_OK) res = j;
  }
  return res;
}

// Checks shared by hv_pca and hv_ssa_moments.
static hv_status check_eig_call(int n, int ny, int nx, const hv_optics* optics, int in_t, const void* in, int window,
                                int stride, int comp_lo, int comp_hi, int prec) {
  hv_status s;
  if ((s = check_frame(n, ny, nx))) return s;
  if (window != 16 && window != 32 && window != 64) return fail(HV_ERR_SHAPE, "window %d: use 16, 32 or 64", window);
  if (stride <= 0) return fail(HV_ERR_ARG, "stride must be positive");
  if (!(0 <= comp_lo && comp_lo <= comp_hi && comp_hi < window))
    return fail(HV_ERR_ARG, "component range [%d, %d] outside [0, %d)", comp_lo, comp_hi, window);
  if (prec != HV_PREC_FP32 && prec != HV_PREC_MIXED) return fail(HV_ERR_ARG, "unknown precision %d", prec);
  if (optics) {
    if ((s = check_optics(optics)) || (s = check_dtype(in_t, true))) return s;
  } else if (in_t != HV_C64) {
    return fail(HV_ERR_ARG, "without optics the input must be a field (HV_C64)");
  }
  if (n < window) return fail(HV_ERR_SHAPE, "%d frames hold no complete window of %d", n, window);
  if (!in) return fail(HV_ERR_ARG, "input is NULL");
  return check_aligned(in);
}

hv_status hv_pca(hv_ctx* ctx, const void* in, int in_t, int n, int ny, int nx, const hv_optics* optics, int window,
                 int stride, int comp_lo, int comp_hi, int prec, float* m0, double* eigvals, double* cov,
                 double* offdiag, void* hip_stream) {
  hv_status s;
  if ((s = enter(ctx))) return s;
  std::lock_guard<std::recursive_mutex> lock(ctx->mu);
  if ((s = check_eig_call(n, ny, nx, optics, in_t, in, window, stride, comp_lo, comp_hi, prec))) return s;
  if (!m0) return fail(HV_ERR_ARG, "m0 is NULL");
  return eig_path(ctx, in, in_t, n, ny, nx, optics, window, stride, comp_lo, comp_hi, prec == HV_PREC_MIXED, nullptr,
                  EigOut{m0, nullptr, nullptr, eigvals, cov, offdiag}, (hipStream_t)hip_stream);
}

hv_status hv_ssa_moments(hv_ctx* ctx, const void* in, int in_t, int n, int ny, int nx, const hv_optics* optics,
                         const hv_temporal* temporal, int comp_lo, int comp_hi, int prec, float* m0, float* m1,
                         float* m2, double* eigvals, double* offdiag, void* hip_stream) {
  hv_status s;
  if ((s = enter(ctx))) return s;
  std::lock_guard<std::recursive_mutex> lock(ctx->mu);
  if (!temporal) return fail(HV_ERR_ARG, "temporal is NULL");
  if ((s = check_eig_call(n, ny, nx, optics, in_t, in, temporal->window, temporal->stride, comp_lo, comp_hi, prec)))
    return s;
  if (!(temporal->fs_hz > 0)) return fail(HV_ERR_ARG, "fs must be positive");
  if (!m0 && !m1 && !m2) return fail(HV_ERR_ARG, "no output requested");
  DftPlan* dp = ctx->dft_plan(*temporal, &s);
  if (!dp) return s;
  return eig_path(ctx, in, in_t, n, ny, nx, optics, temporal->window, temporal->stride, comp_lo, comp_hi,
                  prec == HV_PREC_MIXED, dp, EigOut{m0, m1, m2, eigvals, nullptr, offdiag}, (hipStream_t)hip_stream);
}

}  // extern "C"
