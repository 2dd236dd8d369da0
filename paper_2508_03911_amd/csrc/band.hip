// Band-first order of the angular-spectrum + short-time DFT moments, an
// alternative to the paper's per-frame order that callers ask for with
// hv_ctx_set_stft_order.
//
// The angular spectrum applies one linear operator to every frame
// (Sec. II-B.3), and each bin of the short-time DFT is a fixed linear
// combination of a window's frames (Sec. III-B.1).  The two commute: the
// bin-k field of a window is the angular spectrum of the bin-k combination
// of its raw frames.  When the band holds fewer bins than the window holds
// frames, propagating the band's combinations instead of the frames moves
// fewer bytes and runs fewer FFTs.  (The bins are complex, so the real-input
// row pass of the per-frame order has no counterpart here; that order needs
// the full spectrum after its column pass all the same.)
//
//   KA band rows : the W raw rows of one row index of a window are reduced
//                  to the band's bins on MFMA (camera values are exact in
//                  fp16, the coefficients are split into fp16 high and low
//                  parts), then every bin's row gets a forward row FFT;
//                  out [window][bin][ny][nx] (complex, c64 or fp16);
//   KB band cols : per bin field, column FFT, multiply by H_z / ny, inverse
//                  column FFT, in place;
//   KC band power: per (window, row), inverse row FFT of every bin's row,
//                  then |.|^2 summed with the weights f^0, f^1, f^2 (and the
//                  bins written out when asked for).
//
// MFMA layout (v_mfma_f32_32x32x16_f16, wave64): lane l holds
// A[l%32][k0 + 8(l/32) + e] and B[k0 + 8(l/32) + e][l%32], e = 0..7; the
// result register r of lane l is row 8(r/4) + 4(l/32) + r%4 of column l%32.
// Rows of A come in (real, imaginary) pairs, one pair per bin; k is the
// frame index t within the window.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fft_lds.h"
#include "gmem.h"
#include "hv_internal.h"

using namespace hvk;
using hvi::persistent_grid;

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ inline void store_c(float2* p, float2 v) { *p = v; }
__device__ inline void store_c(hv_h2* p, float2 v) {
  hv_h2 h;
  h.x = (_Float16)v.x;
  h.y = (_Float16)v.y;
  *p = h;
}
__device__ inline float2 load_c(const float2* p) { return *p; }
__device__ inline float2 load_c(const hv_h2* p) {
  hv_h2 h = *p;
  return make_float2((float)h.x, (float)h.y);
}

// Two neighbouring camera values of type TIN read as one word.
template <typename TIN>
using Raw2 = std::conditional_t<sizeof(TIN) == 1, uint16_t, uint32_t>;

template <typename TIN>
__device__ inline uint32_t pick(uint32_t w, int q) {
  constexpr int BITS = 8 * sizeof(TIN);
  return (w >> (BITS * q)) & ((1u << BITS) - 1u);
}

// ------------------------------------------------------------------ KA
// Unit u = (window u / ny, row u % ny); persistent workgroups of NX
// threads take units u = blockIdx.x, + gridDim.x, ... and load the next
// unit's camera values into registers while the current one is
// transformed.  Wave v owns pixels [64 v, 64 v + 64); lane (c, h) loads the
// two neighbouring pixels 64 v + 2c + q (q = 0, 1) of frames
// t = 16 kk + 8 h + e, which make its B fragments of the two column tiles
// (tile q, column c).  u16 values are split into two exact bytes, reduced
// separately and recombined as lo + 256 hi.
template <int NX, int W, typename TIN, typename TOUT>
__global__ __launch_bounds__(NX) void k_band_rows(const TIN* __restrict__ in, TOUT* __restrict__ out, int ny,
                                                  int stride, int nb, int mtiles, const hv_h8* __restrict__ ahi,
                                                  const hv_h8* __restrict__ alo, float scale, int nunits) {
  constexpr int NT = NX, PL = 2;
  static_assert(NX % 64 == 0 && NX <= 512, "row width: whole waves of 64 pixels");
  constexpr int KS = W >= 16 ? W / 16 : 1;
  constexpr int S = lds_stride(NX);
  constexpr bool U16 = sizeof(TIN) == 2;
  using R = Raw2<TIN>;
  __shared__ float2 buf[16 * S];
  __shared__ float2 tw[tw_size(NX) > 0 ? tw_size(NX) : 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5, c = lane & 31;
  fill_twiddles<NX>(tw, tid, NT);
  const long npix = (long)ny * NX;
  const int xb = wave * 32 * PL + PL * c;
  // frame j*stride + t, row y: wave-uniform base + lane offset (8h frames, pixel xb)
  const uint32_t off = (uint32_t)((8 * h) * npix + xb) * (uint32_t)sizeof(TIN);
  R raw[KS][8];
  auto fetch = [&](int u) {
    const TIN* base = in + ((long)(u / ny) * stride * ny + u % ny) * NX;
#pragma unroll
    for (int kk = 0; kk < KS; ++kk)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        if (W >= 16 || h == 0)
          raw[kk][e] = ld_off(reinterpret_cast<const R*>(base + (long)(16 * kk + e) * npix), off);
        else
          raw[kk][e] = 0;
      }
  };
  int u = blockIdx.x;
  if (u < nunits) fetch(u);
  for (; u < nunits; u += gridDim.x) {
    TOUT* dst0 = out + ((long)(u / ny) * nb * ny + u % ny) * NX;
    for (int mt = 0; mt < mtiles; ++mt) {
      hv_h8 fh[KS], fl[KS];
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) {
        fh[kk] = ahi[(mt * KS + kk) * 64 + lane];
        fl[kk] = alo[(mt * KS + kk) * 64 + lane];
      }
#pragma unroll
      for (int q = 0; q < PL; ++q) {
        f32x16 acc, acc2;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = acc2[r] = 0.f;
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
          hv_h8 b, bh;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const uint32_t v = pick<TIN>(raw[kk][e], q);
            b[e] = (_Float16)(float)(v & 0xffu);
            if constexpr (U16) bh[e] = (_Float16)(float)(v >> 8);
          }
          acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(fh[kk], b, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(fl[kk], b, acc, 0, 0, 0);
          if constexpr (U16) {
            acc2 = __builtin_amdgcn_mfma_f32_32x32x16_f16(fh[kk], bh, acc2, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f32_32x32x16_f16(fl[kk], bh, acc2, 0, 0, 0);
          }
        }
        if constexpr (U16) {
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[r] += 256.f * acc2[r];
        }
        const int xs = skew(xb + q);
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
          for (int p = 0; p < 2; ++p)
            buf[(4 * g + 2 * h + p) * S + xs] = make_float2(acc[4 * g + 2 * p], acc[4 * g + 2 * p + 1]);
      }
      // the camera values are consumed: fetch the next unit's
      if (mt == mtiles - 1 && u + (int)gridDim.x < nunits) fetch(u + gridDim.x);
      __syncthreads();
      fft_lds<NX, 16, NT, -1>(buf, tw, tid);
      const int live = nb - 16 * mt < 16 ? nb - 16 * mt : 16;
      TOUT* dst = dst0 + (long)16 * mt * npix;
      for (int q = tid; q < live * NX; q += NT) {
        const int b = q / NX, x = q % NX;
        TOUT v;
        store_c(&v, c2::scale(buf[b * S + skew(x)], scale));
        st_off(dst, (uint32_t)(b * npix + x) * (uint32_t)sizeof(TOUT), v);
      }
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------------ KB
// Unit u = (field u / groups, column group u % groups): columns
// [x0, x0 + BC) of one bin field [ny][nx], transformed in place.  Persistent
// workgroups take units u = blockIdx.x, + gridDim.x, ... with gridDim.x a
// multiple of groups, so a workgroup keeps one column group: its H_z values
// stay in registers, and the next unit's columns load into registers while
// the current one is transformed.  ht is column-major [nx][ny]:
// H_z(fx, fy) / ny with the high-pass mask folded in.
template <int NY, int BC, int NTK, typename TIO>
__global__ __launch_bounds__(NTK) void k_band_cols(TIO* __restrict__ io, const float2* __restrict__ ht, int nx,
                                                   int nunits) {
  constexpr int S = lds_stride(NY);
  constexpr int U = BC * NY / NTK;
  constexpr int RS = NTK / BC;  // rows per pass of the threads
  static_assert(BC * NY % NTK == 0 && NTK % BC == 0 && NY % RS == 0, "column tile split");
  __shared__ float2 buf[BC * S];
  __shared__ float2 tw[tw_size(NY) > 0 ? tw_size(NY) : 1];
  const int tid = threadIdx.x;
  const int groups = nx / BC;
  const int x0 = (blockIdx.x % groups) * BC;
  fill_twiddles<NY>(tw, tid, NTK);
  // H_z of the outputs this thread writes in the last forward FFT pass,
  // where the multiply is applied (the table run of one column is
  // contiguous, and so are the lanes' positions)
  constexpr int UL = fft_last_slots<NY, BC, NTK>(), RL = radix_of_pass(NY, num_passes(NY) - 1);
  const float2* hcol = ht + (long)x0 * NY;
  float2 hv[UL][RL];
#pragma unroll
  for (int u = 0; u < UL; ++u)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      int b, i;
      hv[u][r] = fft_last_index<NY, BC, NTK>(tid, u, r, &b, &i) ? hcol[b * NY + i] : make_float2(0.f, 0.f);
    }
  // load / store element u: column s, row yr + u * RS
  const int s = tid % BC, yr = tid / BC;
  const uint32_t off = (uint32_t)(yr * nx + s) * (uint32_t)sizeof(TIO);
  auto base_of = [&](int unit) { return io + (long)(unit / groups) * NY * nx + x0; };
  TIO pre[U];
  auto fetch = [&](int unit) {
    const TIO* base = base_of(unit);
#pragma unroll
    for (int u = 0; u < U; ++u) pre[u] = ld_off(base + (long)u * RS * nx, off);
  };
  int unit = blockIdx.x;
  if (unit < nunits) fetch(unit);
  for (; unit < nunits; unit += gridDim.x) {
    TIO* base = base_of(unit);
#pragma unroll
    for (int u = 0; u < U; ++u) buf[s * S + skew(yr + u * RS)] = load_c(&pre[u]);
    __syncthreads();
    if (unit + (int)gridDim.x < nunits) fetch(unit + gridDim.x);
    fft_lds_io<NY, BC, NTK, -1, true>(buf, tw, tid, nullptr, [&](int u, int r, int b, int i, float2 v) {
      buf[b * S + skew(i)] = c2::mul(v, hv[u][r]);
    });
    fft_lds<NY, BC, NTK, +1>(buf, tw, tid);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      TIO v;
      store_c(&v, buf[s * S + skew(yr + u * RS)]);
      st_off(base + (long)u * RS * nx, off, v);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ KC
// Unit u = (window u / ny, row u % ny), persistent workgroups of NX
// threads: bins in groups of 16, each group's rows inverse-transformed in
// LDS while the next group's (or next unit's) rows load into registers;
// thread tid owns pixel tid.
template <int NX, typename TIN>
__global__ __launch_bounds__(NX) void k_band_power(const TIN* __restrict__ in, int ny, int nb, int mtiles,
                                                   const float* __restrict__ wts, float amp,
                                                   float* __restrict__ o0, float* __restrict__ o1,
                                                   float* __restrict__ o2, float2* __restrict__ spec, int nunits) {
  constexpr int NT = NX;
  constexpr int S = lds_stride(NX);
  __shared__ float2 buf[16 * S];
  __shared__ float2 tw[tw_size(NX) > 0 ? tw_size(NX) : 1];
  const int tid = threadIdx.x;
  fill_twiddles<NX>(tw, tid, NT);
  const long npix = (long)ny * NX;
  const int ws = 16 * mtiles;
  // the elements this thread reads in the first inverse FFT pass: slot u,
  // element r is bin pb[u] at pixel pi[u][r] (16 lanes read 16 consecutive
  // pixels of one bin row)
  constexpr int UF = fft_first_slots<NX, 16, NT>(), RF = radix_of_pass(NX, 0);
  int pb[UF];
  uint32_t po[UF][RF];
#pragma unroll
  for (int u = 0; u < UF; ++u)
#pragma unroll
    for (int r = 0; r < RF; ++r) {
      int b = 16, i = 0;
      if (!fft_first_index<NX, 16, NT>(tid, u, r, &b, &i)) b = 16;
      if (r == 0) pb[u] = b;
      po[u][r] = (uint32_t)(b * npix + i) * (uint32_t)sizeof(TIN);
    }
  TIN pre[UF][RF];
  auto live_of = [&](int mt) { return nb - 16 * mt < 16 ? nb - 16 * mt : 16; };
  auto fetch = [&](int u, int mt) {
    const TIN* s0 = in + (((long)(u / ny) * nb + 16 * mt) * ny + u % ny) * NX;
    const int live = live_of(mt);
#pragma unroll
    for (int uu = 0; uu < UF; ++uu)
#pragma unroll
      for (int r = 0; r < RF; ++r)
        if (pb[uu] < live) pre[uu][r] = ld_off(s0, po[uu][r]);
  };
  float e0 = 0.f, e1 = 0.f, e2 = 0.f;
  int u = blockIdx.x, mt = 0;
  if (u < nunits) fetch(u, 0);
  while (u < nunits) {
    const int live = live_of(mt);
    float2 cur[UF][RF];
#pragma unroll
    for (int uu = 0; uu < UF; ++uu)
#pragma unroll
      for (int r = 0; r < RF; ++r) cur[uu][r] = pb[uu] < live ? load_c(&pre[uu][r]) : make_float2(0.f, 0.f);
    int nu = u, nm = mt + 1;
    if (nm == mtiles) {
      nu = u + gridDim.x;
      nm = 0;
    }
    if (nu < nunits) fetch(nu, nm);
    fft_lds_io<NX, 16, NT, +1>(buf, tw, tid, [&](int uu, int r, int, int) { return cur[uu][r]; }, nullptr);
    const long pix = (long)(u % ny) * NX + tid;
    for (int b = 0; b < live; ++b) {
      const int wi = 16 * mt + b;
      const float w0 = wts[wi], w1 = wts[ws + wi], w2 = wts[2 * ws + wi];
      const float2 v = c2::scale(buf[b * S + skew(tid)], amp);
      const float pw = v.x * v.x + v.y * v.y;
      e0 += w0 * pw;
      e1 += w1 * pw;
      e2 += w2 * pw;
      if (spec) spec[((long)(u / ny) * nb + wi) * npix + pix] = v;
    }
    if (mt == mtiles - 1) {
      const long o = (long)(u / ny) * npix + pix;
      if (o0) o0[o] = e0;
      if (o1) o1[o] = e1;
      if (o2) o2[o] = e2;
      e0 = e1 = e2 = 0.f;
    }
    __syncthreads();
    u = nu;
    mt = nm;
  }
}

hv_status launched(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hvi::fail(HV_ERR_DEVICE, "%s launch failed: %s", what, hipGetErrorString(e));
  return HV_OK;
}

template <int NX, typename TIN, typename TOUT>
hv_status go_rows(const void* in, void* out, int ny, int stride, int nwin, int window, int nb, int mtiles,
                  const hv_h8* ahi, const hv_h8* alo, float scale, hipStream_t st) {
  const int nunits = nwin * ny;
  const dim3 block(NX);
  dim3 grid;
  switch (window) {
    case 8: grid = dim3(persistent_grid(k_band_rows<NX, 8, TIN, TOUT>, NX, nunits)); break;
    case 16: grid = dim3(persistent_grid(k_band_rows<NX, 16, TIN, TOUT>, NX, nunits)); break;
    case 32: grid = dim3(persistent_grid(k_band_rows<NX, 32, TIN, TOUT>, NX, nunits)); break;
    case 64: grid = dim3(persistent_grid(k_band_rows<NX, 64, TIN, TOUT>, NX, nunits)); break;
    default: return hvi::fail(HV_ERR_SHAPE, "window %d not supported", window);
  }
  switch (window) {
    case 8: hipLaunchKernelGGL((k_band_rows<NX, 8, TIN, TOUT>), grid, block, 0, st, (const TIN*)in, (TOUT*)out, ny, stride, nb, mtiles, ahi, alo, scale, nunits); break;
    case 16: hipLaunchKernelGGL((k_band_rows<NX, 16, TIN, TOUT>), grid, block, 0, st, (const TIN*)in, (TOUT*)out, ny, stride, nb, mtiles, ahi, alo, scale, nunits); break;
    case 32: hipLaunchKernelGGL((k_band_rows<NX, 32, TIN, TOUT>), grid, block, 0, st, (const TIN*)in, (TOUT*)out, ny, stride, nb, mtiles, ahi, alo, scale, nunits); break;
    case 64: hipLaunchKernelGGL((k_band_rows<NX, 64, TIN, TOUT>), grid, block, 0, st, (const TIN*)in, (TOUT*)out, ny, stride, nb, mtiles, ahi, alo, scale, nunits); break;
    default: return hvi::fail(HV_ERR_SHAPE, "window %d not supported", window);
  }
  return launched("band_rows");
}

template <int NY, typename TIO>
hv_status go_cols(void* io, const float2* ht, int nfields, int nx, hipStream_t st) {
  // 128-byte runs per row of the column tile (64-byte fp16 runs above
  // 256 rows, where 32 columns would not leave room for two tiles per CU);
  // 16 (above 256 rows 32) column elements per thread
  constexpr int BC = (sizeof(TIO) == 4 && NY <= 256) ? 32 : 16;
  constexpr int NTK = BC * (NY <= 256 ? 16 : 32);
  const int groups = nx / BC, nunits = groups * nfields;
  auto kern = k_band_cols<NY, BC, NTK, TIO>;
  int grid = persistent_grid(kern, NTK, nunits);
  if (grid < nunits) grid = grid / groups * groups;  // a whole number of column-group sets
  hipLaunchKernelGGL(kern, dim3(grid), dim3(NTK), 0, st, (TIO*)io, ht, nx, nunits);
  return launched("band_cols");
}

template <int NX, typename TIN>
hv_status go_power(const void* in, int ny, int nwin, int nb, int mtiles, const float* wts, float amp, float* o0,
                   float* o1, float* o2, float2* spec, hipStream_t st) {
  const int nunits = nwin * ny;
  auto kern = k_band_power<NX, TIN>;
  hipLaunchKernelGGL(kern, dim3(persistent_grid(kern, NX, nunits)), dim3(NX), 0, st, (const TIN*)in, ny, nb, mtiles,
                     wts, amp, o0, o1, o2, spec, nunits);
  return launched("band_power");
}

}  // namespace

namespace hvi {

bool band_first_fits(int ny, int nx, int in_t) {
  if (in_t != HV_U8 && in_t != HV_U16) return false;
  if (!pow2_in(nx, 64, 512)) return false;
  switch (ny) {
    case 64: case 128: case 256: case 320: case 384: case 512: return true;
    default: return false;
  }
}

hv_status launch_band_rows(const void* in, int in_t, void* out, bool half_out, int ny, int nx, int stride, int nwin,
                           int window, int nb, int mtiles, const hv_h8* ahi, const hv_h8* alo, float scale,
                           hipStream_t st) {
  if (!band_first_fits(ny, nx, in_t)) return fail(HV_ERR_SHAPE, "band-first rows: %dx%d type %d", nx, ny, in_t);
  if (nb <= 0 || nb > 16 * mtiles || mtiles > 4) return fail(HV_ERR_ARG, "band-first rows: %d bins", nb);
  if (nwin <= 0) return HV_OK;
#define HV_ROWS(NX_)                                                                                        \
  if (in_t == HV_U8)                                                                                        \
    return half_out ? go_rows<NX_, uint8_t, hv_h2>(in, out, ny, stride, nwin, window, nb, mtiles, ahi, alo, scale, st) \
                    : go_rows<NX_, uint8_t, float2>(in, out, ny, stride, nwin, window, nb, mtiles, ahi, alo, scale, st); \
  return half_out ? go_rows<NX_, uint16_t, hv_h2>(in, out, ny, stride, nwin, window, nb, mtiles, ahi, alo, scale, st) \
                  : go_rows<NX_, uint16_t, float2>(in, out, ny, stride, nwin, window, nb, mtiles, ahi, alo, scale, st);
  switch (nx) {
    case 64: { HV_ROWS(64) }
    case 128: { HV_ROWS(128) }
    case 256: { HV_ROWS(256) }
    default: { HV_ROWS(512) }
  }
#undef HV_ROWS
}

hv_status launch_band_cols(void* io, bool half_io, const float2* ht, int nfields, int ny, int nx, hipStream_t st) {
  if (nfields <= 0) return HV_OK;
  if (nx % 32 || !band_first_fits(ny, 256, HV_U8)) return fail(HV_ERR_SHAPE, "band-first columns: nx %d", nx);
#define HV_COLS(NY_) \
  case NY_: return half_io ? go_cols<NY_, hv_h2>(io, ht, nfields, nx, st) : go_cols<NY_, float2>(io, ht, nfields, nx, st);
  switch (ny) {
    HV_COLS(64) HV_COLS(128) HV_COLS(256) HV_COLS(320) HV_COLS(384) HV_COLS(512)
    default: return fail(HV_ERR_SHAPE, "band-first columns: ny %d", ny);
  }
#undef HV_COLS
}

hv_status launch_band_power(const void* in, bool half_in, int ny, int nx, int nwin, int nb, int mtiles,
                            const float* wts, float amp, float* o0, float* o1, float* o2, float2* spec,
                            hipStream_t st) {
  if (nwin <= 0) return HV_OK;
#define HV_POWER(NX_)                                                                          \
  case NX_:                                                                                    \
    return half_in ? go_power<NX_, hv_h2>(in, ny, nwin, nb, mtiles, wts, amp, o0, o1, o2, spec, st) \
                   : go_power<NX_, float2>(in, ny, nwin, nb, mtiles, wts, amp, o0, o1, o2, spec, st);
  switch (nx) {
    HV_POWER(64) HV_POWER(128) HV_POWER(256) HV_POWER(512)
    default: return fail(HV_ERR_SHAPE, "band-first power: nx %d", nx);
  }
#undef HV_POWER
}

}  // namespace hvi
