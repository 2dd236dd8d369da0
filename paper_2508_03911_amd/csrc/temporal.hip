// Temporal transforms on MFMA: the short-time DFT as a dense GEMM with a
// Doppler-moment epilogue, and the PCA projection energy, which has the same
// shape (Sec. III-B.1: temporal transform over a window of consecutive
// reconstructed frames, then a moment over a range of temporal indices).
//
// A window of W frames at P pixels is read as the real matrix
// B [2W x P] with row 2t + c = component c (0 real, 1 imaginary) of frame t.
// A coefficient matrix A [2M x 2W] whose rows come in (real, imaginary)
// pairs turns B into M complex outputs per pixel:
//   DFT:  pair b is bin k_b: Re = sum_t (ur cos + ui sin), Im = sum_t
//         (ui cos - ur sin) with angle 2 pi k_b t / W;
//   PCA:  pair c is component c: Y_c = sum_t X_t V[t, c].
// The epilogue forms |.|^2 of every pair and sums them with up to three
// weight vectors (f^0, f^1, f^2 for the moments; 1 for the PCA energy).
//
// MFMA layouts (gfx950, wave64).  v_mfma_f32_32x32x2f32: lane l holds
// A[l%32][k0 + l/32] and B[k0 + l/32][l%32].  v_mfma_f32_32x32x16_f16: lane l
// holds A[l%32][k0 + 8(l/32) + e] and B[k0 + 8(l/32) + e][l%32], e = 0..7
// (any k assignment works as long as A and B agree).  Both write the 32x32
// result with lane l, register r holding row 8(r/4) + 4(l/32) + r%4 of
// column l%32, so a lane owns both rows of 8 (re, im) pairs of one pixel.
#include <hip/hip_runtime.h>

#include "fft_lds.h"
#include "gmem.h"
#include "hv_internal.h"

using namespace hvk;
using hvi::persistent_grid;

typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {

constexpr int NT = 512;  // threads per block: 8 waves
constexpr int MT_MAX = 4;  // up to 64 (re, im) pairs

__device__ inline float2 load_c(const float2* p) { return *p; }
__device__ inline float2 load_c(const hv_h2* p) {
  hv_h2 h = *p;
  return make_float2((float)h.x, (float)h.y);
}

// This lane's A fragments of one 32-row tile (FP32: W floats; mixed: W/8
// fp16x8 hi and lo parts), held in registers so that their loads can be
// issued long before the MFMAs need them.
template <int W, bool MIXED>
struct AFrag;
template <int W>
struct AFrag<W, false> {
  float a[W];
};
template <int W>
struct AFrag<W, true> {
  hv_h8 hi[W / 8], lo[W / 8];
};

// One 32x32 output tile: A from registers, B from the LDS tile
// buf[t * S + skew(x)].
template <int W, bool MIXED, bool EXACT_B>
__device__ inline f32x16 coef_tile(const AFrag<W, MIXED>& f, const float2* buf, int S, int x0, int lane,
                                   float bsc) {
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  const int h = lane >> 5;
  const int xs = skew(x0 + (lane & 31));
  if constexpr (!MIXED) {
    const float* col = reinterpret_cast<const float*>(buf + xs) + h;
#pragma unroll
    for (int kk = 0; kk < W; ++kk) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(f.a[kk], col[2 * kk * S], acc, 0, 0, 0);
  } else {
#pragma unroll
    for (int kk = 0; kk < W / 8; ++kk) {
      hv_h8 bh, bl;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float2 v = buf[(8 * kk + 4 * h + i) * S + xs];
        float x = v.x * bsc, y = v.y * bsc;
        bh[2 * i] = (_Float16)x;
        bh[2 * i + 1] = (_Float16)y;
        if constexpr (!EXACT_B) {
          bl[2 * i] = (_Float16)(x - (float)bh[2 * i]);
          bl[2 * i + 1] = (_Float16)(y - (float)bh[2 * i + 1]);
        }
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(f.hi[kk], bh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(f.lo[kk], bh, acc, 0, 0, 0);
      if constexpr (!EXACT_B) acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(f.hi[kk], bl, acc, 0, 0, 0);
    }
  }
  return acc;
}

struct CoefArgs {
  const float* a32;
  const hv_h8* a16hi;
  const hv_h8* a16lo;
  long a_win_stride;  // elements of a32 (and of a16) per window; 0 = shared
  const float* wts;   // [3][mtiles*16]
  int mtiles, npair, nout;
  float bsc;          // scale applied to B before the fp16 split
  float amp;          // scale applied to every output amplitude
  float* out[3];
  float2* spec;       // [nwin][npair][npix] or null
};

template <int W, bool MIXED>
__device__ inline void load_afrag(AFrag<W, MIXED>& f, const CoefArgs& g, long jj, int mt, int lane) {
  const long aw = g.a_win_stride * jj;
  if constexpr (!MIXED) {
    const float* p = g.a32 + aw + (long)mt * W * 64;
#pragma unroll
    for (int kk = 0; kk < W; ++kk) f.a[kk] = p[kk * 64 + lane];
  } else {
    const long o = (aw >> 3) + (long)mt * (W / 8) * 64;
#pragma unroll
    for (int kk = 0; kk < W / 8; ++kk) {
      f.hi[kk] = g.a16hi[o + kk * 64 + lane];
      f.lo[kk] = g.a16lo[o + kk * 64 + lane];
    }
  }
}

// GEMM + epilogue for the wave's pixel tile [x0, x0+32) of the LDS tile.
// Writes outputs at out[k][obase + x0 + lane] and spec[(jj*npair + pair)*npix + obase + x0 + lane].
// PRE: f0 holds the fragments of tile 0, loaded by the caller; otherwise
// every tile's fragments are loaded here.
// PIPE (with PRE): the next tile's fragments are loaded into a second set of
// registers before the current tile's MFMAs, so their latency hides behind
// them (W more VGPRs: for kernels with registers to spare).
template <int W, bool MIXED, bool EXACT_B, bool PRE, bool PIPE = false>
__device__ inline void coef_pixels(const CoefArgs& g, const float* wts_lds, const float2* buf, int S, int x0,
                                   int lane, long jj, long obase, long npix, const AFrag<W, MIXED>& f0) {
  static_assert(!PIPE || PRE, "the pipelined form starts from the caller's first fragments");
  const int h = lane >> 5;
  float e0 = 0.f, e1 = 0.f, e2 = 0.f;
  AFrag<W, MIXED> cur;
  if constexpr (PIPE) cur = f0;
  for (int mt = 0; mt < g.mtiles; ++mt) {
    f32x16 acc;
    if constexpr (PIPE) {
      AFrag<W, MIXED> nxt;
      if (mt + 1 < g.mtiles) load_afrag(nxt, g, jj, mt + 1, lane);
      acc = coef_tile<W, MIXED, EXACT_B>(cur, buf, S, x0, lane, g.bsc);
      cur = nxt;
    } else if (PRE && mt == 0) {
      acc = coef_tile<W, MIXED, EXACT_B>(f0, buf, S, x0, lane, g.bsc);
    } else {
      AFrag<W, MIXED> f;
      load_afrag(f, g, jj, mt, lane);
      acc = coef_tile<W, MIXED, EXACT_B>(f, buf, S, x0, lane, g.bsc);
    }
#pragma unroll
    for (int gq = 0; gq < 4; ++gq) {
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const int pair = 16 * mt + 4 * gq + 2 * h + p;
        const float re = acc[4 * gq + 2 * p], im = acc[4 * gq + 2 * p + 1];
        const float pw = re * re + im * im;
        const int wi = 16 * mt + 4 * gq + 2 * h + p;
        e0 += wts_lds[wi] * pw;
        e1 += wts_lds[MT_MAX * 16 + wi] * pw;
        e2 += wts_lds[2 * MT_MAX * 16 + wi] * pw;
        if (g.spec && pair < g.npair)
          g.spec[(jj * g.npair + pair) * npix + obase + x0 + (lane & 31)] =
              make_float2(re * g.amp, im * g.amp);
      }
    }
  }
  e0 += __shfl_xor(e0, 32);
  e1 += __shfl_xor(e1, 32);
  e2 += __shfl_xor(e2, 32);
  if (lane < 32) {
    const float a2 = g.amp * g.amp;
    const long o = jj * npix + obase + x0 + lane;
    if (g.out[0]) g.out[0][o] = e0 * a2;
    if (g.nout > 1 && g.out[1]) g.out[1][o] = e1 * a2;
    if (g.nout > 2 && g.out[2]) g.out[2][o] = e2 * a2;
  }
}

__device__ inline void load_wts(float* wts_lds, const CoefArgs& g, int tid, int nthreads = NT) {
  for (int i = tid; i < 3 * MT_MAX * 16; i += nthreads) {
    const int k = i / (MT_MAX * 16), m = i % (MT_MAX * 16);
    wts_lds[i] = (m < g.mtiles * 16 && k < g.nout) ? g.wts[k * g.mtiles * 16 + m] : 0.f;
  }
}

// ------------------------------------------------------------------ fused row inverse + GEMM
// Unit u = (window u / ny, row u % ny): the W rows y of the window's frames
// are inverse-transformed in LDS and reduced by the coefficient GEMM.
//
// FP16 input: persistent blocks with a register prefetch of the next unit's
// rows (16 VGPRs) while the current unit is transformed and reduced.
// FP32 input: one unit per block.  A 32-VGPR prefetch would lift the kernel
// past 128 VGPRs and halve the resident blocks per CU, which costs more than
// the prefetch gains (measured at 256 x 256, W = 32).
template <int NX, int W, bool MIXED, typename TIN>
__global__ __launch_bounds__(NT) void k_rowinv_coef(const TIN* __restrict__ z, int ny, int stride, int nunits,
                                                    CoefArgs g) {
  constexpr bool PF = sizeof(TIN) == 4;
  constexpr int S = lds_stride(NX);
  __shared__ float2 buf[W * S];
  __shared__ float2 tw[tw_size(NX) > 0 ? tw_size(NX) : 1];
  __shared__ float wts_lds[3 * MT_MAX * 16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  fill_twiddles<NX>(tw, tid, NT);
  load_wts(wts_lds, g, tid);
  const long npix = (long)ny * NX;
  // The row inverse FFT's first pass reads straight from registers: element
  // (u, r) of this thread is frame b_u of the window at pixel i_u + r * SP
  // (16 lanes take 16 consecutive pixels of one frame row), so the rows are
  // loaded into exactly those registers and skip the LDS staging.
  // (small tiles leave some threads without a first-pass butterfly)
  constexpr int UF = fft_first_slots<NX, W, NT>(), RF = radix_of_pass(NX, 0), SP = NX / RF;
  uint32_t po[UF];  // byte offset of element (u, 0) in the field (W * ny * NX * 8 B < 4 GiB)
  bool act[UF];
#pragma unroll
  for (int u = 0; u < UF; ++u) {
    int b, i;
    act[u] = fft_first_index<NX, W, NT>(tid, u, 0, &b, &i);
    po[u] = act[u] ? (uint32_t)(b * npix + i) * (uint32_t)sizeof(TIN) : 0u;
  }
  // first element of unit u = (window u / ny, row u % ny): wave-uniform
  auto rows = [&](int u) { return z + (((long)(u / ny) * stride) * (long)ny + u % ny) * NX; };
  auto load = [&](int u, TIN (&v)[UF][RF]) {
    const TIN* src = rows(u);
#pragma unroll
    for (int uu = 0; uu < UF; ++uu)
#pragma unroll
      for (int r = 0; r < RF; ++r)
        if (act[uu]) v[uu][r] = ld_off(src + r * SP, po[uu]);
  };
  // FP32 input: the A fragments are loaded before the FFT and consumed
  // after it.  FP16 input: they are loaded in the GEMM (measured faster
  // there: the 32 extra VGPRs across the FFT cost more than they hide).
  auto reduce = [&](int u, const AFrag<W, MIXED>& af, const auto& src) {
    fft_lds_io<NX, W, NT, +1>(buf, tw, tid, [&](int uu, int r, int, int) { return load_c(&src[uu][r]); }, nullptr);
    for (int nt = wave; nt < NX / 32; nt += NT / 64)
      coef_pixels<W, MIXED, false, !PF>(g, wts_lds, buf, S, nt * 32, lane, u / ny, (long)(u % ny) * NX, npix,
                                        af);
  };
  if constexpr (PF) {
    TIN pre[UF][RF];
    int u = blockIdx.x;
    if (u < nunits) load(u, pre);
    for (; u < nunits; u += gridDim.x) {
      TIN cur[UF][RF];
#pragma unroll
      for (int uu = 0; uu < UF; ++uu)
#pragma unroll
        for (int r = 0; r < RF; ++r) cur[uu][r] = pre[uu][r];
      if (u + (int)gridDim.x < nunits) load(u + gridDim.x, pre);
      AFrag<W, MIXED> unused;
      reduce(u, unused, cur);
      __syncthreads();
    }
  } else {
    const int u = blockIdx.x;
    TIN v[UF][RF];
    load(u, v);
    AFrag<W, MIXED> af;
    load_afrag(af, g, u / ny, 0, lane);
    reduce(u, af, v);
  }
}

// ------------------------------------------------------------------ GEMM from a field in memory
constexpr int TPIX = NT / 2;  // pixel counts must be a multiple of this

// Threads per block: one 32-pixel tile per wave, so a block covers
// threads / 2 pixels.  A W = 64 tile of 256 pixels fills 140 KB of LDS and
// leaves one block per CU, its loads and its MFMAs in turn.  DIV = 2 halves it
// (128 pixels, four waves, 67 KB) so that two blocks share a CU and one's
// loads run under the other's MFMAs.  Measured on 1024^2 fields: the STFT
// GEMM 0.50 -> 0.445 ms per window with it; the PCA projection ran faster
// too, but its pass slower (it shares the chip with the other stream's
// eigensolve and covariance), so that one keeps the full tile.
template <int W, int DIV>
constexpr int coef_threads() {
  return W >= 64 ? NT / DIV : NT;
}

template <int W, bool MIXED, typename TIN, int DIV>
__global__ __launch_bounds__((coef_threads<W, DIV>())) void k_field_coef(const TIN* __restrict__ u, long npix,
                                                                        int stride, CoefArgs g) {
  constexpr int NTB = coef_threads<W, DIV>(), TP = NTB / 2;
  constexpr int S = lds_stride(TP);
  constexpr bool EXACT = MIXED && sizeof(TIN) == 4;  // fp16 storage is exact in fp16
  __shared__ float2 buf[W * S];
  __shared__ float wts_lds[3 * MT_MAX * 16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long p0 = (long)blockIdx.x * TP;
  const long jj = blockIdx.y;
  load_wts(wts_lds, g, tid, NTB);
  AFrag<W, MIXED> af;
  load_afrag(af, g, jj, 0, lane);
  const TIN* src = u + (jj * stride) * npix + p0;
  // element i of this thread: frame RPI * i + tid / TP, pixel tid % TP;
  // loads go out in batches of 8 so that several are in flight at once
  constexpr int RPI = NTB / TP, PER = W * TP / NTB, BATCH = PER < 8 ? PER : 8;
  static_assert(PER % BATCH == 0, "load batches");
  const int tr = tid / TP, x = tid % TP;
  const uint32_t off = (uint32_t)(tr * npix + x) * (uint32_t)sizeof(TIN);
  float2* lds = buf + tr * S + skew(x);
#pragma unroll
  for (int i0 = 0; i0 < PER; i0 += BATCH) {
    TIN v[BATCH];
#pragma unroll
    for (int i = 0; i < BATCH; ++i) v[i] = ld_off(src + (long)RPI * (i0 + i) * npix, off);
#pragma unroll
    for (int i = 0; i < BATCH; ++i) lds[RPI * (i0 + i) * S] = load_c(&v[i]);
  }
  __syncthreads();
  coef_pixels<W, MIXED, EXACT, true, true>(g, wts_lds, buf, S, wave * 32, lane, jj, p0, npix, af);
}

// ------------------------------------------------------------------ full-band STFT power (temporal FFT)
// The paper's STFT benchmark transforms whole windows of W = 128..512 frames
// and renders every bin (Sec. VI-B.1).  Block (pixel tile, window j): the W
// samples of PT = 8192 / W pixels sit in LDS as PT sequences; a radix FFT
// transforms them and |S_k|^2 * amp2 goes out for every bin k:
// out[(j * W + k) * npix + p].  Element i of a thread is pixel pt and time
// (or bin) tt + i * TPI, TPI = NT / PT.
template <int W, typename TIN>
__global__ __launch_bounds__(NT) void k_time_fft(const TIN* __restrict__ u, int npix, int stride, float amp2,
                                                 float* __restrict__ out) {
  constexpr int PT = 8192 / W;
  constexpr int TPI = NT / PT;
  constexpr int PER = W / TPI;
  constexpr int S = lds_stride(W);
  static_assert(NT % PT == 0 && W % TPI == 0, "tile split");
  __shared__ float2 buf[PT * S];
  __shared__ float2 tw[tw_size(W)];
  const int tid = threadIdx.x;
  // Workgroups go to the 8 XCDs round-robin by linear index; tiles 2m and
  // 2m + 1 (whose 64-byte output runs share 128-byte lines) are given
  // indices of one residue mod 8, so the lines merge in one L2.
  const int tiles = npix / PT;  // a multiple of 16
  const int lin = blockIdx.x % tiles, q = lin >> 3;
  const long p0 = (long)(16 * (q >> 1) + 2 * (lin & 7) + (q & 1)) * PT;
  const long jj = blockIdx.x / tiles;
  fill_twiddles<W>(tw, tid, NT);
  const int pt = tid % PT, tt = tid / PT;
  float2* lds = buf + pt * S + skew(tt);
  const TIN* src = u + (jj * stride) * (long)npix + p0;
  const uint32_t off_in = (uint32_t)(tt * npix + pt) * (uint32_t)sizeof(TIN);
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const TIN v = ld_off(src + (long)i * TPI * npix, off_in);
    lds[skew(i * TPI)] = load_c(&v);
  }
  __syncthreads();
  fft_lds<W, PT, NT, -1>(buf, tw, tid);
  float* dst = out + jj * W * (long)npix + p0;
  const uint32_t off_out = (uint32_t)(tt * npix + pt) * 4u;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const float2 v = lds[skew(i * TPI)];
    st_off(dst + (long)i * TPI * npix, off_out, (v.x * v.x + v.y * v.y) * amp2);
  }
}

// ------------------------------------------------------------------ Gram partials (PCA covariance)
// Block (blk, jj) accumulates G = B^T B over its pixel range for window jj.
// LDS holds the tile transposed, L[m][p] with m = 2t + c, so both MFMA
// operands read contiguous pixel runs of one row.  Each thread loads runs
// of 4 pixels of one frame (16 bytes of fp16 pairs, 32 of float pairs), and
// the next tile's runs are loaded into registers before the current tile's
// MFMAs, so the loads are in flight while the matrix cores work.  Pixel
// ranges are multiples of GP and frames a multiple of 4 pixels, so a run
// lies wholly inside or wholly outside the range.
constexpr int GP = 64;  // pixels per LDS tile

template <typename TIN> struct Run4;
template <> struct Run4<hv_h2> {  // 4 fp16 pairs: re/im of 4 pixels
  uint4 w;
  __device__ void load(const hv_h2* p) { w = *reinterpret_cast<const uint4*>(p); }
  __device__ void zero() { w = make_uint4(0u, 0u, 0u, 0u); }
  __device__ hv_h2 pair(int e) const {
    const uint32_t v = e == 0 ? w.x : e == 1 ? w.y : e == 2 ? w.z : w.w;
    hv_h2 h;
    __builtin_memcpy(&h, &v, 4);
    return h;
  }
  __device__ float2 get(int e) const {
    const hv_h2 h = pair(e);
    return make_float2((float)h.x, (float)h.y);
  }
  // the re (c = 0) or im (c = 1) halves of the 4 pixels, as bit copies
  __device__ uint2 part4(int c) const {
    const hv_h2 a = pair(0), b = pair(1), d = pair(2), e = pair(3);
    hv_h2 lo, hi;
    lo.x = c ? a.y : a.x;
    lo.y = c ? b.y : b.x;
    hi.x = c ? d.y : d.x;
    hi.y = c ? e.y : e.x;
    uint2 r;
    __builtin_memcpy(&r.x, &lo, 4);
    __builtin_memcpy(&r.y, &hi, 4);
    return r;
  }
};
template <> struct Run4<float2> {  // 4 float pairs
  float4 a, b;
  __device__ void load(const float2* p) {
    a = reinterpret_cast<const float4*>(p)[0];
    b = reinterpret_cast<const float4*>(p)[1];
  }
  __device__ void zero() { a = b = make_float4(0.f, 0.f, 0.f, 0.f); }
  __device__ float2 get(int e) const {
    return e == 0 ? make_float2(a.x, a.y) : e == 1 ? make_float2(a.z, a.w) : e == 2 ? make_float2(b.x, b.y)
                                                                                   : make_float2(b.z, b.w);
  }
};

template <int W, bool MIXED, typename TIN>
__global__ __launch_bounds__(NT) void k_gram(const TIN* __restrict__ u, long npix, int stride, long pix_per_blk,
                                             float bsc, float* __restrict__ part, int nblk) {
  constexpr int M = 2 * W;
  constexpr int T = M / 32;             // tiles per dimension
  constexpr int NW = NT / 64;
  constexpr int TPW = (T * T + NW - 1) / NW;  // tiles per wave
  constexpr int LS32 = GP + 1;          // f32 row stride (odd)
  constexpr int LS16 = GP + 8;          // fp16 row stride (keeps 16-byte reads aligned)
  constexpr int RUNS = W * GP / 4;      // 4-pixel runs per tile
  constexpr int PER = (RUNS + NT - 1) / NT;
  // fp16 pairs at unit scale go to LDS as bit copies
  constexpr bool COPY16 = MIXED && sizeof(TIN) == 4;
  __shared__ float l32[MIXED ? 1 : M * LS32];
  __shared__ __attribute__((aligned(16))) _Float16 l16[MIXED ? M * LS16 : 8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5;
  const long jj = blockIdx.y;
  const int blk = blockIdx.x;
  const long pbeg = (long)blk * pix_per_blk;
  const long pend = pbeg + pix_per_blk < npix ? pbeg + pix_per_blk : npix;
  f32x16 acc[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[i][r] = 0.f;
  const TIN* src = u + (jj * stride) * npix;
  // run q = tid + i * NT of a tile: frame q / (GP / 4), pixels 4 (q % (GP / 4)) + 0..3
  Run4<TIN> nxt[PER];
  auto fetch = [&](long p0) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int q = tid + i * NT;
      if (RUNS % NT == 0 || q < RUNS) {
        const int t = q / (GP / 4), x = 4 * (q % (GP / 4));
        if (p0 + x < pend)
          nxt[i].load(src + (long)t * npix + p0 + x);
        else
          nxt[i].zero();
      }
    }
  };
  if (pbeg < pend) fetch(pbeg);
  for (long p0 = pbeg; p0 < pend; p0 += GP) {
    __syncthreads();  // every wave is done reading the previous tile
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int q = tid + i * NT;
      if (RUNS % NT == 0 || q < RUNS) {
        const int t = q / (GP / 4), x = 4 * (q % (GP / 4));
        if constexpr (COPY16) {
          *reinterpret_cast<uint2*>(&l16[(2 * t) * LS16 + x]) = nxt[i].part4(0);
          *reinterpret_cast<uint2*>(&l16[(2 * t + 1) * LS16 + x]) = nxt[i].part4(1);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float2 v = nxt[i].get(e);
            if constexpr (MIXED) {
              l16[(2 * t) * LS16 + x + e] = (_Float16)(v.x * bsc);
              l16[(2 * t + 1) * LS16 + x + e] = (_Float16)(v.y * bsc);
            } else {
              l32[(2 * t) * LS32 + x + e] = v.x;
              l32[(2 * t + 1) * LS32 + x + e] = v.y;
            }
          }
        }
      }
    }
    __syncthreads();
    if (p0 + GP < pend) fetch(p0 + GP);
    if constexpr (MIXED) {
#pragma unroll
      for (int i = 0; i < TPW; ++i) {
        const int tile = wave + NW * i;
        if (tile < T * T) {
          const int mt = tile / T, nt = tile % T;
          const int ma = 32 * mt + (lane & 31), nb = 32 * nt + (lane & 31);
#pragma unroll
          for (int kk = 0; kk < GP / 16; ++kk) {
            hv_h8 a = *reinterpret_cast<const hv_h8*>(&l16[ma * LS16 + 16 * kk + 8 * h]);
            hv_h8 b = *reinterpret_cast<const hv_h8*>(&l16[nb * LS16 + 16 * kk + 8 * h]);
            acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc[i], 0, 0, 0);
          }
        }
      }
    } else {
      // the wave's tiles interleaved per k-step (independent accumulators),
      // each step's operands read from LDS one step ahead of its MFMAs; each
      // accumulator sees its k-steps in the same order as one tile at a time
      const float* ap[TPW];
      const float* bp[TPW];
#pragma unroll
      for (int i = 0; i < TPW; ++i) {
        const int tile = min(wave + NW * i, T * T - 1), mt = tile / T, nt = tile % T;
        ap[i] = l32 + (32 * mt + (lane & 31)) * LS32 + h;
        bp[i] = l32 + (32 * nt + (lane & 31)) * LS32 + h;
      }
      float a[TPW], b[TPW];
#pragma unroll
      for (int i = 0; i < TPW; ++i) {
        a[i] = ap[i][0];
        b[i] = bp[i][0];
      }
#pragma unroll
      for (int kk = 0; kk < GP / 2; ++kk) {
        float an[TPW], bn[TPW];
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
          an[i] = kk + 1 < GP / 2 ? ap[i][2 * (kk + 1)] : 0.f;
          bn[i] = kk + 1 < GP / 2 ? bp[i][2 * (kk + 1)] : 0.f;
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < TPW; ++i)
          if (wave + NW * i < T * T) acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[i], acc[i], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
          a[i] = an[i];
          b[i] = bn[i];
        }
      }
    }
  }
  float* dst = part + (jj * nblk + blk) * (long)M * M;
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int tile = wave + NW * i;
    if (tile < T * T) {
      const int mt = tile / T, nt = tile % T;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = 32 * mt + 8 * (r / 4) + 4 * h + (r % 4);
        const int n = 32 * nt + (lane & 31);
        dst[m * M + n] = acc[i][r];
      }
    }
  }
}

// C[a][b] = sum_blk G[2a][2b] + G[2a+1][2b+1] + i (G[2a][2b+1] - G[2a+1][2b]),
// summed in f64 in block order (deterministic).
__global__ void k_gram_reduce(const float* __restrict__ part, int nblk, int W, double cscale,
                              double* __restrict__ cov) {
  const long jj = blockIdx.y;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= W * W) return;
  const int a = idx / W, b = idx % W;
  const int M = 2 * W;
  double re = 0.0, im = 0.0;
  for (int blk = 0; blk < nblk; ++blk) {
    const float* g = part + (jj * nblk + blk) * (long)M * M;
    re += (double)g[(2 * a) * M + 2 * b] + (double)g[(2 * a + 1) * M + 2 * b + 1];
    im += (double)g[(2 * a) * M + 2 * b + 1] - (double)g[(2 * a + 1) * M + 2 * b];
  }
  cov[(jj * W * W + idx) * 2] = re * cscale;
  cov[(jj * W * W + idx) * 2 + 1] = im * cscale;
}

// ------------------------------------------------------------------ FP64 Jacobi
// Cyclic Jacobi for a Hermitian W x W matrix, one block per window, with the
// round-robin (circle) ordering: in each of the W-1 steps of a sweep, W/2
// disjoint pairs rotate at once, the matrix in independent 2x2 blocks (the
// column and the row rotation together) and the eigenvector columns in one
// pass between two barriers.  Pair (p, q) with a = A_pp,
// d = A_qq, b = A_pq = |b| e^{i phi}: J = [[c, s], [-s e^{-i phi}, c e^{-i phi}]]
// with t = sgn(th)/(|th| + sqrt(th^2 + 1)), th = (d - a)/(2|b|),
// c = 1/sqrt(t^2 + 1), s = t c zeroes A_pq in J^H A J.
struct dc {
  double x, y;
};
__device__ inline dc dmul(dc a, dc b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline dc dadd(dc a, dc b) { return {a.x + b.x, a.y + b.y}; }
__device__ inline dc dscale(dc a, double s) { return {a.x * s, a.y * s}; }
__device__ inline dc dconj(dc a) { return {a.x, -a.y}; }

// JT = W^2 / 2 threads per window (one per eigenvector-pair update of a
// rotation step; the (W/2)^2 matrix blocks take a half or a quarter of
// them), at most 1024.  A and V sit in LDS with a padded row stride W + 1, so
// lanes walking down a column spread over the banks.  The
// rotation parameters use reciprocal square roots: 1/|b| once, then t and
// c = 1/sqrt(t^2 + 1).
template <int W>
constexpr int jacobi_threads() {
  return W * W / 2 > 1024 ? 1024 : W * W / 2;
}

template <int W>
__device__ inline double jacobi_sum(double v, double* red) {
  constexpr int JT = jacobi_threads<W>();
  const int tid = threadIdx.x;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if constexpr (JT <= 64) {
    return v;
  } else {
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < JT / 64; ++i) r += red[i];
    __syncthreads();
    return r;
  }
}

template <int W>
__global__ __launch_bounds__(jacobi_threads<W>()) void k_jacobi(const double* __restrict__ cov,
                                                                double* __restrict__ evals,
                                                                double* __restrict__ evecs,
                                                                double* __restrict__ offdiag, int max_sweeps) {
  constexpr int JT = jacobi_threads<W>();
  constexpr int WP = W + 1;  // padded row stride
  __shared__ dc A[W * WP];
  __shared__ dc V[W * WP];
  __shared__ int pp[W / 2], qq[W / 2];
  __shared__ double rc[W / 2], rs[W / 2];  // c, s
  __shared__ dc re[W / 2];                  // e^{-i phi}
  __shared__ double red[JT / 64 > 0 ? JT / 64 : 1];
  __shared__ int perm[W];
  const int tid = threadIdx.x;
  const long jj = blockIdx.x;
  const dc* src = reinterpret_cast<const dc*>(cov) + jj * W * W;
  for (int i = tid; i < W * W; i += JT) {
    const int r = i / W, c = i % W;
    A[r * WP + c] = src[i];
    V[r * WP + c] = {r == c ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  for (int sweep = 0;; ++sweep) {
    // convergence: off-diagonal energy relative to the total; at exit the
    // ratio sqrt(off / total) is reported, so a window that reached the
    // sweep limit unconverged is visible to the caller
    double off = 0.0, tot = 0.0;
    for (int i = tid; i < W * W; i += JT) {
      const int r = i / W, c = i % W;
      const dc v = A[r * WP + c];
      const double m2 = v.x * v.x + v.y * v.y;
      tot += m2;
      if (r != c) off += m2;
    }
    const double off_all = jacobi_sum<W>(off, red);
    const double tot_all = jacobi_sum<W>(tot, red);
    if (!(off_all > 1e-30 * tot_all) || sweep >= max_sweeps) {
      if (offdiag && tid == 0) offdiag[jj] = tot_all > 0 ? sqrt(off_all / tot_all) : 0.0;
      break;
    }
    for (int step = 0; step < W - 1; ++step) {
      if (tid < W / 2) {
        const int k = tid;
        auto player = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + step) % (W - 1); };
        int p = player(k), q = player(W - 1 - k);
        if (p > q) {
          int t = p;
          p = q;
          q = t;
        }
        pp[k] = p;
        qq[k] = q;
        const double a = A[p * WP + p].x, d = A[q * WP + q].x;
        const dc b = A[p * WP + q];
        const double b2 = b.x * b.x + b.y * b.y;
        if (b2 == 0.0 || b2 < 1e-300 * (a * a + d * d)) {  // |b| negligible: no rotation
          rc[k] = 1.0;
          rs[k] = 0.0;
          re[k] = {1.0, 0.0};
        } else {
          const double inv = rsqrt(b2);  // 1 / |b|
          const double th = 0.5 * (d - a) * inv;
          const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          const double c = rsqrt(t * t + 1.0);
          rc[k] = c;
          rs[k] = t * c;
          re[k] = {b.x * inv, -b.y * inv};  // e^{-i phi}
        }
      }
      __syncthreads();
      // The step's rotations act on disjoint index pairs that cover 0..W-1,
      // so A' = J^H A J splits into independent 2x2 blocks: rows {p_i, q_i}
      // by columns {p_j, q_j} take the column rotation of pair j,
      //   A[:,p] = c A[:,p] - s e A[:,q],  A[:,q] = s A[:,p] + c e A[:,q],
      // then the row rotation of pair i,
      //   A[p,:] = c A[p,:] - s conj(e) A[q,:],  A[q,:] = s A[p,:] + c conj(e) A[q,:],
      // in registers, with one read and one write of each element.
      for (int b = tid; b < (W / 2) * (W / 2); b += JT) {
        const int i = b / (W / 2), j = b % (W / 2);
        const int pi = pp[i], qi = qq[i], pj = pp[j], qj = qq[j];
        const double cj = rc[j], sj = rs[j], ci = rc[i], si = rs[i];
        const dc ej = re[j], eci = dconj(re[i]);
        const dc a_pp = A[pi * WP + pj], a_pq = A[pi * WP + qj];
        const dc a_qp = A[qi * WP + pj], a_qq = A[qi * WP + qj];
        dc t = dmul(ej, a_pq);
        const dc n_pp = dadd(dscale(a_pp, cj), dscale(t, -sj));
        const dc n_pq = dadd(dscale(a_pp, sj), dscale(t, cj));
        t = dmul(ej, a_qq);
        const dc n_qp = dadd(dscale(a_qp, cj), dscale(t, -sj));
        const dc n_qq = dadd(dscale(a_qp, sj), dscale(t, cj));
        t = dmul(eci, n_qp);
        A[pi * WP + pj] = dadd(dscale(n_pp, ci), dscale(t, -si));
        A[qi * WP + pj] = dadd(dscale(n_pp, si), dscale(t, ci));
        t = dmul(eci, n_qq);
        A[pi * WP + qj] = dadd(dscale(n_pq, ci), dscale(t, -si));
        A[qi * WP + qj] = dadd(dscale(n_pq, si), dscale(t, ci));
      }
      // V = V J: the column rotation of every pair on every row
      for (int i = tid; i < (W / 2) * W; i += JT) {
        const int k = i / W, r = i % W;
        const int p = pp[k], q = qq[k];
        const double c = rc[k], sn = rs[k];
        const dc e = re[k];
        dc vp = V[r * WP + p], vq = V[r * WP + q];
        dc ev = dmul(e, vq);
        V[r * WP + p] = dadd(dscale(vp, c), dscale(ev, -sn));
        V[r * WP + q] = dadd(dscale(vp, sn), dscale(ev, c));
      }
      __syncthreads();
    }
  }
  // descending order, ties keep the lower index
  if (tid == 0) {
    for (int i = 0; i < W; ++i) perm[i] = i;
    for (int i = 0; i < W; ++i) {
      int best = i;
      for (int j = i + 1; j < W; ++j) {
        const double vj = A[perm[j] * WP + perm[j]].x, vb = A[perm[best] * WP + perm[best]].x;
        if (vj > vb || (vj == vb && perm[j] < perm[best])) best = j;
      }
      int t = perm[i];
      perm[i] = perm[best];
      perm[best] = t;
    }
  }
  __syncthreads();
  if (tid < W) evals[jj * W + tid] = A[perm[tid] * WP + perm[tid]].x;
  dc* dst = reinterpret_cast<dc*>(evecs) + jj * W * W;
  for (int i = tid; i < W * W; i += JT) {
    const int r = i / W, c = i % W;
    dst[i] = V[r * WP + perm[c]];
  }
}

// ------------------------------------------------------------------ PCA projection coefficients
// Pair i = component c1 + i: rows 2i (Re Y), 2i+1 (Im Y); columns 2t + comp:
// A[2i][2t] = Vr, A[2i][2t+1] = -Vi, A[2i+1][2t] = Vi, A[2i+1][2t+1] = Vr.
__device__ inline float proj_coef(const dc* v, int W, int c1, int npair, int m, int k) {
  const int i = m >> 1, t = k >> 1;
  if (i >= npair) return 0.f;
  const dc e = v[t * W + c1 + i];
  const int rm = m & 1, ck = k & 1;
  double val = rm == 0 ? (ck == 0 ? e.x : -e.y) : (ck == 0 ? e.y : e.x);
  return (float)val;
}

__global__ void k_proj_coefs(const double* __restrict__ evecs, int W, int c1, int npair, int mtiles,
                             float* __restrict__ a32, hv_h8* __restrict__ a16hi, hv_h8* __restrict__ a16lo) {
  const long jj = blockIdx.x;
  const dc* v = reinterpret_cast<const dc*>(evecs) + jj * W * W;
  const long per_win = (long)mtiles * W * 64;
  for (int i = threadIdx.x; i < mtiles * W * 64; i += blockDim.x) {
    const int lane = i % 64, kk = (i / 64) % W, mt = i / (64 * W);
    a32[jj * per_win + i] = proj_coef(v, W, c1, npair, 32 * mt + (lane & 31), 2 * kk + (lane >> 5));
  }
  for (int i = threadIdx.x; i < mtiles * (W / 8) * 64; i += blockDim.x) {
    const int lane = i % 64, kk = (i / 64) % (W / 8), mt = i / (64 * (W / 8));
    hv_h8 hi, lo;
    for (int e = 0; e < 8; ++e) {
      float a = proj_coef(v, W, c1, npair, 32 * mt + (lane & 31), 16 * kk + 8 * (lane >> 5) + e);
      hi[e] = (_Float16)a;
      lo[e] = (_Float16)(a - (float)hi[e]);
    }
    a16hi[jj * (per_win / 8) + i] = hi;
    a16lo[jj * (per_win / 8) + i] = lo;
  }
}

// ------------------------------------------------------------------ SSA + FFT coefficients
// The SSA filter keeps components c1..c2 of the window, X_f = X V_S V_S^H,
// and the FFT follows, S_k = sum_t d_k[t] X_f[:, t] with d_k[t] =
// exp(-2 pi i k t / W).  Both steps are linear in the window's frames, so
// S_k = sum_t' A[k][t'] X[:, t'] with A[k][t'] = sum_i V_S[t', i] G[k][i]
// and G[k][i] = sum_t conj(V_S[t, i]) d_k[t]; A (FP64) goes into the same
// MFMA fragment layout as the DFT coefficients, one set per window, and
// the field is read once by the coefficient GEMM with the moment epilogue.
struct SsaBins {
  int n;
  int k[64];
};

template <int W>
__global__ __launch_bounds__(256) void k_ssa_coefs(const double* __restrict__ evecs, int c1, int ns, SsaBins bins,
                                                   int mtiles, float* __restrict__ a32, hv_h8* __restrict__ a16hi,
                                                   hv_h8* __restrict__ a16lo) {
  __shared__ dc G[W * W];  // [bin][component]
  __shared__ dc A[W * W];  // [bin][frame]
  const long jj = blockIdx.x;
  const dc* v = reinterpret_cast<const dc*>(evecs) + jj * W * W;  // v[t * W + c]
  const int nb = bins.n;
  for (int e = threadIdx.x; e < nb * ns; e += blockDim.x) {
    const int b = e / ns, i = e % ns;
    const int k = bins.k[b];
    dc acc = {0.0, 0.0};
    for (int t = 0; t < W; ++t) {
      double sn, cs;
      sincospi(2.0 * (double)((k * t) % W) / W, &sn, &cs);
      acc = dadd(acc, dmul(dconj(v[t * W + c1 + i]), dc{cs, -sn}));
    }
    G[b * W + i] = acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nb * W; e += blockDim.x) {
    const int b = e / W, t = e % W;
    dc acc = {0.0, 0.0};
    for (int i = 0; i < ns; ++i) acc = dadd(acc, dmul(v[t * W + c1 + i], G[b * W + i]));
    A[b * W + t] = acc;
  }
  __syncthreads();
  // row m = 2b + (0: Re S, 1: Im S), column q = 2t + (0: Re u, 1: Im u)
  auto coef = [&](int m, int q) -> float {
    const int b = m >> 1, t = q >> 1;
    if (b >= nb) return 0.f;
    const dc a = A[b * W + t];
    const double val = (m & 1) == 0 ? ((q & 1) == 0 ? a.x : -a.y) : ((q & 1) == 0 ? a.y : a.x);
    return (float)val;
  };
  const long per_win = (long)mtiles * W * 64;
  for (int i = threadIdx.x; i < mtiles * W * 64; i += blockDim.x) {
    const int lane = i % 64, kk = (i / 64) % W, mt = i / (64 * W);
    a32[jj * per_win + i] = coef(32 * mt + (lane & 31), 2 * kk + (lane >> 5));
  }
  for (int i = threadIdx.x; i < mtiles * (W / 8) * 64; i += blockDim.x) {
    const int lane = i % 64, kk = (i / 64) % (W / 8), mt = i / (64 * (W / 8));
    hv_h8 hi, lo;
    for (int e = 0; e < 8; ++e) {
      const float a = coef(32 * mt + (lane & 31), 16 * kk + 8 * (lane >> 5) + e);
      hi[e] = (_Float16)a;
      lo[e] = (_Float16)(a - (float)hi[e]);
    }
    a16hi[jj * (per_win / 8) + i] = hi;
    a16lo[jj * (per_win / 8) + i] = lo;
  }
}

hv_status launched(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hvi::fail(HV_ERR_DEVICE, "%s launch failed: %s", what, hipGetErrorString(e));
  return HV_OK;
}

CoefArgs make_args(const hvi::CoefGemm& g, long a_win_stride, float bsc, float amp, float* o0, float* o1,
                   float* o2, float2* spec) {
  CoefArgs a;
  a.a32 = g.a32;
  a.a16hi = g.a16hi;
  a.a16lo = g.a16lo;
  a.a_win_stride = a_win_stride;
  a.wts = g.wts;
  a.mtiles = g.mtiles;
  a.npair = g.npair;
  a.nout = g.nout;
  a.bsc = bsc;
  a.amp = amp;
  a.out[0] = o0;
  a.out[1] = o1;
  a.out[2] = o2;
  a.spec = spec;
  return a;
}

template <int NX, int W, bool MIXED>
hv_status go_rowinv(const void* z, bool half_in, int ny, int stride, int nwin, const CoefArgs& a,
                    hipStream_t st) {
  if constexpr (W * NX <= 8192 && (W * NX) % NT == 0) {
    const int nunits = ny * nwin;
    if (half_in) {
      auto kern = k_rowinv_coef<NX, W, MIXED, hv_h2>;
      hipLaunchKernelGGL(kern, dim3(persistent_grid(kern, NT, nunits)), dim3(NT), 0, st, (const hv_h2*)z, ny, stride,
                         nunits, a);
    } else {
      hipLaunchKernelGGL((k_rowinv_coef<NX, W, MIXED, float2>), dim3(nunits), dim3(NT), 0, st, (const float2*)z,
                         ny, stride, nunits, a);
    }
    return launched("rowinv_coef");
  } else {
    return hvi::fail(HV_ERR_SHAPE, "fused row-inverse GEMM does not fit nx=%d W=%d", NX, W);
  }
}

template <int W>
hv_status go_rowinv_w(const void* z, bool half_in, int ny, int nx, int stride, int nwin, const CoefArgs& a,
                      bool mixed, hipStream_t st) {
  switch (nx) {
    case 64: return mixed ? go_rowinv<64, W, true>(z, half_in, ny, stride, nwin, a, st)
                          : go_rowinv<64, W, false>(z, half_in, ny, stride, nwin, a, st);
    case 128: return mixed ? go_rowinv<128, W, true>(z, half_in, ny, stride, nwin, a, st)
                           : go_rowinv<128, W, false>(z, half_in, ny, stride, nwin, a, st);
    case 256: return mixed ? go_rowinv<256, W, true>(z, half_in, ny, stride, nwin, a, st)
                           : go_rowinv<256, W, false>(z, half_in, ny, stride, nwin, a, st);
    case 512: return mixed ? go_rowinv<512, W, true>(z, half_in, ny, stride, nwin, a, st)
                           : go_rowinv<512, W, false>(z, half_in, ny, stride, nwin, a, st);
    case 1024: return mixed ? go_rowinv<1024, W, true>(z, half_in, ny, stride, nwin, a, st)
                            : go_rowinv<1024, W, false>(z, half_in, ny, stride, nwin, a, st);
  }
  return hvi::fail(HV_ERR_SHAPE, "nx=%d not supported", nx);
}

template <int W, bool MIXED, int DIV = 1>
void go_field(const void* u, bool half_in, long npix, int stride, int nwin, const CoefArgs& a, hipStream_t st) {
  constexpr int NTB = coef_threads<W, DIV>();
  dim3 grid((unsigned)(npix / (NTB / 2)), nwin);
  if (half_in)
    hipLaunchKernelGGL((k_field_coef<W, MIXED, hv_h2, DIV>), grid, dim3(NTB), 0, st, (const hv_h2*)u, npix,
                       stride, a);
  else
    hipLaunchKernelGGL((k_field_coef<W, MIXED, float2, DIV>), grid, dim3(NTB), 0, st, (const float2*)u, npix,
                       stride, a);
}

template <int W, bool MIXED>
void go_gram(const void* u, bool half_in, long npix, int stride, int nwin, long ppb, float bsc, float* part,
             int nblk, hipStream_t st) {
  dim3 grid(nblk, nwin);
  if (half_in)
    hipLaunchKernelGGL((k_gram<W, MIXED, hv_h2>), grid, dim3(NT), 0, st, (const hv_h2*)u, npix, stride, ppb, bsc,
                       part, nblk);
  else
    hipLaunchKernelGGL((k_gram<W, MIXED, float2>), grid, dim3(NT), 0, st, (const float2*)u, npix, stride, ppb,
                       bsc, part, nblk);
}

}  // namespace

namespace hvi {

bool rowinv_coef_fits(int nx, int window) {
  return (nx & (nx - 1)) == 0 && (long)nx * window <= 8192 && ((long)nx * window) % NT == 0;
}

hv_status launch_rowinv_coef(const void* z, bool half_in, int ny, int nx, int stride, int nwin, const CoefGemm& g,
                             bool mixed, float b_scale, float out_scale, float* out0, float* out1, float* out2,
                             float2* spec, hipStream_t st) {
  if (nwin <= 0) return HV_OK;
  CoefArgs a = make_args(g, 0, b_scale, out_scale, out0, out1, out2, spec);
  switch (g.window) {
    case 8: return go_rowinv_w<8>(z, half_in, ny, nx, stride, nwin, a, mixed, st);
    case 16: return go_rowinv_w<16>(z, half_in, ny, nx, stride, nwin, a, mixed, st);
    case 32: return go_rowinv_w<32>(z, half_in, ny, nx, stride, nwin, a, mixed, st);
    case 64: return go_rowinv_w<64>(z, half_in, ny, nx, stride, nwin, a, mixed, st);
  }
  return fail(HV_ERR_SHAPE, "window %d not supported", g.window);
}

// half_tile: W = 64 runs two 128-pixel blocks per CU (the STFT GEMM) rather
// than one of 256 pixels (the PCA projection).
static hv_status field_coef(const void* u, bool half_in, long npix, int stride, int nwin, const CoefArgs& a,
                            int window, bool mixed, bool half_tile, hipStream_t st) {
  if (nwin <= 0) return HV_OK;
  if (npix % TPIX) return fail(HV_ERR_SHAPE, "pixel count %ld not a multiple of %d", npix, TPIX);
  switch (window) {
    case 8: mixed ? go_field<8, true>(u, half_in, npix, stride, nwin, a, st)
                  : go_field<8, false>(u, half_in, npix, stride, nwin, a, st); break;
    case 16: mixed ? go_field<16, true>(u, half_in, npix, stride, nwin, a, st)
                   : go_field<16, false>(u, half_in, npix, stride, nwin, a, st); break;
    case 32: mixed ? go_field<32, true>(u, half_in, npix, stride, nwin, a, st)
                   : go_field<32, false>(u, half_in, npix, stride, nwin, a, st); break;
    case 64:
      if (half_tile)
        mixed ? go_field<64, true, 2>(u, half_in, npix, stride, nwin, a, st)
              : go_field<64, false, 2>(u, half_in, npix, stride, nwin, a, st);
      else
        mixed ? go_field<64, true>(u, half_in, npix, stride, nwin, a, st)
              : go_field<64, false>(u, half_in, npix, stride, nwin, a, st);
      break;
    default: return fail(HV_ERR_SHAPE, "window %d not supported", window);
  }
  return launched("field_coef");
}

hv_status launch_field_coef(const void* u, bool half_in, long npix, int stride, int nwin, const CoefGemm& g,
                            bool mixed, float b_scale, float out_scale, float* out0, float* out1, float* out2,
                            float2* spec, hipStream_t st) {
  CoefArgs a = make_args(g, 0, b_scale, out_scale, out0, out1, out2, spec);
  return field_coef(u, half_in, npix, stride, nwin, a, g.window, mixed, true, st);
}

hv_status launch_gram_partials(const void* u, bool half_in, long npix, int stride, int nwin, int window,
                               bool mixed, float b_scale, float* part, int nblk, hipStream_t st) {
  if (nwin <= 0) return HV_OK;
  if (npix % 4) return fail(HV_ERR_SHAPE, "frame of %ld pixels: a multiple of 4 is needed", npix);
  // pixel ranges in whole tiles (the last blocks may get fewer pixels, or none)
  const long ppb = ((npix + nblk - 1) / nblk + GP - 1) / GP * GP;
  switch (window) {
    case 16: mixed ? go_gram<16, true>(u, half_in, npix, stride, nwin, ppb, b_scale, part, nblk, st)
                   : go_gram<16, false>(u, half_in, npix, stride, nwin, ppb, b_scale, part, nblk, st); break;
    case 32: mixed ? go_gram<32, true>(u, half_in, npix, stride, nwin, ppb, b_scale, part, nblk, st)
                   : go_gram<32, false>(u, half_in, npix, stride, nwin, ppb, b_scale, part, nblk, st); break;
    case 64: mixed ? go_gram<64, true>(u, half_in, npix, stride, nwin, ppb, b_scale, part, nblk, st)
                   : go_gram<64, false>(u, half_in, npix, stride, nwin, ppb, b_scale, part, nblk, st); break;
    default: return fail(HV_ERR_SHAPE, "PCA window %d not supported (16, 32 or 64)", window);
  }
  return launched("gram");
}

hv_status launch_gram_reduce(const float* part, int nwin, int nblk, int window, double cscale, double* cov,
                             hipStream_t st) {
  if (nwin <= 0) return HV_OK;
  dim3 grid((window * window + 255) / 256, nwin);
  hipLaunchKernelGGL(k_gram_reduce, grid, dim3(256), 0, st, part, nblk, window, cscale, cov);
  return launched("gram_reduce");
}

hv_status launch_jacobi(const double* cov, int nwin, int window, double* evals, double* evecs, double* offdiag,
                        int max_sweeps, hipStream_t st) {
  if (nwin <= 0) return HV_OK;
  switch (window) {
    case 16:
      hipLaunchKernelGGL(k_jacobi<16>, dim3(nwin), dim3(jacobi_threads<16>()), 0, st, cov, evals, evecs, offdiag,
                         max_sweeps);
      break;
    case 32:
      hipLaunchKernelGGL(k_jacobi<32>, dim3(nwin), dim3(jacobi_threads<32>()), 0, st, cov, evals, evecs, offdiag,
                         max_sweeps);
      break;
    case 64:
      hipLaunchKernelGGL(k_jacobi<64>, dim3(nwin), dim3(jacobi_threads<64>()), 0, st, cov, evals, evecs, offdiag,
                         max_sweeps);
      break;
    default: return fail(HV_ERR_SHAPE, "PCA window %d not supported", window);
  }
  return launched("jacobi");
}

hv_status launch_proj_coefs(const double* evecs, int nwin, int window, int c1, int c2, int mtiles, float* a32,
                            hv_h8* a16hi, hv_h8* a16lo, hipStream_t st) {
  if (nwin <= 0) return HV_OK;
  hipLaunchKernelGGL(k_proj_coefs, dim3(nwin), dim3(256), 0, st, evecs, window, c1, c2 - c1 + 1, mtiles, a32,
                     a16hi, a16lo);
  return launched("proj_coefs");
}

hv_status launch_ssa_coefs(const double* evecs, int nwin, int window, int c1, int c2, const int* bins, int nb,
                           int mtiles, float* a32, hv_h8* a16hi, hv_h8* a16lo, hipStream_t st) {
  if (nwin <= 0) return HV_OK;
  if (nb <= 0 || nb > window || mtiles * 16 < nb) return fail(HV_ERR_ARG, "SSA band of %d bins", nb);
  if (!(0 <= c1 && c1 <= c2 && c2 < window)) return fail(HV_ERR_ARG, "component range [%d, %d]", c1, c2);
  SsaBins b{};
  b.n = nb;
  for (int i = 0; i < nb; ++i) {
    if (bins[i] < 0 || bins[i] >= window) return fail(HV_ERR_ARG, "bin %d outside the window", bins[i]);
    b.k[i] = bins[i];
  }
  const int ns = c2 - c1 + 1;
  switch (window) {
    case 16: hipLaunchKernelGGL(k_ssa_coefs<16>, dim3(nwin), dim3(256), 0, st, evecs, c1, ns, b, mtiles, a32, a16hi, a16lo); break;
    case 32: hipLaunchKernelGGL(k_ssa_coefs<32>, dim3(nwin), dim3(256), 0, st, evecs, c1, ns, b, mtiles, a32, a16hi, a16lo); break;
    case 64: hipLaunchKernelGGL(k_ssa_coefs<64>, dim3(nwin), dim3(256), 0, st, evecs, c1, ns, b, mtiles, a32, a16hi, a16lo); break;
    default: return fail(HV_ERR_SHAPE, "SSA window %d not supported (16, 32 or 64)", window);
  }
  return launched("ssa_coefs");
}

hv_status launch_coef_moments(const void* u, bool half_in, long npix, int stride, int nwin, int window, int mtiles,
                              int npair, const float* a32, const hv_h8* a16hi, const hv_h8* a16lo, const float* wts,
                              bool mixed, float b_scale, float out_scale, float* m0, float* m1, float* m2,
                              hipStream_t st) {
  CoefGemm g{window, mtiles, npair, a32, a16hi, a16lo, wts, 3};
  CoefArgs a = make_args(g, (long)mtiles * window * 64, b_scale, out_scale, m0, m1, m2, nullptr);
  return field_coef(u, half_in, npix, stride, nwin, a, window, mixed, false, st);
}

hv_status launch_proj_energy(const void* u, bool half_in, long npix, int stride, int nwin, int window, int mtiles,
                             int npair, const float* a32, const hv_h8* a16hi, const hv_h8* a16lo,
                             const float* wts, bool mixed, float b_scale, float out_scale, float* m0,
                             hipStream_t st) {
  CoefGemm g{window, mtiles, npair, a32, a16hi, a16lo, wts, 1};
  CoefArgs a = make_args(g, (long)mtiles * window * 64, b_scale, out_scale, m0, nullptr, nullptr, nullptr);
  return field_coef(u, half_in, npix, stride, nwin, a, window, mixed, false, st);
}

hv_status launch_time_fft(const void* u, bool half_in, long npix, int stride, int nwin, int window, float amp2,
                          float* out, hipStream_t st) {
  if (nwin <= 0) return HV_OK;
  if (npix % (16L * (8192 / window)) != 0 || npix > (1L << 24)) return fail(HV_ERR_SHAPE, "pixel count %ld", npix);
  const dim3 grid((unsigned)(npix / (8192 / window) * nwin));
#define HV_TFFT(WV)                                                                                          \
  if (half_in)                                                                                                \
    hipLaunchKernelGGL((k_time_fft<WV, hv_h2>), grid, dim3(NT), 0, st, (const hv_h2*)u, (int)npix, stride,  \
                       amp2, out);                                                                            \
  else                                                                                                        \
    hipLaunchKernelGGL((k_time_fft<WV, float2>), grid, dim3(NT), 0, st, (const float2*)u, (int)npix, stride, \
                       amp2, out);
  switch (window) {
    case 128: HV_TFFT(128) break;
    case 256: HV_TFFT(256) break;
    case 512: HV_TFFT(512) break;
    default: return fail(HV_ERR_SHAPE, "volume window %d: use 128, 256 or 512", window);
  }
#undef HV_TFFT
  return launched("time_fft");
}

}  // namespace hvi
