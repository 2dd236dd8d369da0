// Spatial demodulation kernels: angular spectrum and single-FFT Fresnel.
//
// Angular spectrum (Abstract; Sec. II-B.3): U = IDFT2(H_z DFT2(x)).  The 2D
// transforms are split into a row pass and a column pass so that each pass
// holds whole sequences in LDS:
//   K1 row R2C  : unpack u8/u16 in the load, two real rows packed as one
//                 complex FFT, half spectrum written transposed
//                 [t][nx/2][ny] (column 0 packs the real DC and Nyquist
//                 columns);
//   K2 column   : column FFT, the -fx column from Hermitian symmetry,
//                 multiply by H_z, inverse column FFT, write [t][ny][nx];
//   K3 row inv  : inverse row FFT to the field (or fused with the temporal
//                 GEMM elsewhere).
// Fresnel (Abstract; Sec. VI-B.2): chirp * centred DFT * chirp, the
// centring folded into the chirps as a (-1)^(m+n) checkerboard.
#include <hip/hip_runtime.h>

#include "fft_lds.h"
#include "gmem.h"
#include "hv_ctx.h"
#include "hv_internal.h"

using namespace hvk;
using hvi::persistent_grid;

namespace {

constexpr int NT = 512;  // threads per block: 8 waves

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

// 8 consecutive camera values as floats (exact).
__device__ inline void load8(const uint8_t* p, float* f) {
  uint2 w = *reinterpret_cast<const uint2*>(p);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    f[e] = (float)((w.x >> (8 * e)) & 0xffu);
    f[e + 4] = (float)((w.y >> (8 * e)) & 0xffu);
  }
}
__device__ inline void load8(const uint16_t* p, float* f) {
  uint4 w = *reinterpret_cast<const uint4*>(p);
  uint32_t a[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    f[2 * e] = (float)(a[e] & 0xffffu);
    f[2 * e + 1] = (float)(a[e] >> 16);
  }
}

// 8 consecutive inputs of a row as complex values.
__device__ inline void load8c(const uint8_t* p, float2* v) {
  float f[8];
  load8(p, f);
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = make_float2(f[e], 0.f);
}
__device__ inline void load8c(const uint16_t* p, float2* v) {
  float f[8];
  load8(p, f);
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = make_float2(f[e], 0.f);
}
__device__ inline void load8c(const float2* p, float2* v) {
  const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    float4 a = q[e];
    v[2 * e] = make_float2(a.x, a.y);
    v[2 * e + 1] = make_float2(a.z, a.w);
  }
}

// ------------------------------------------------------------------ K1
// Persistent: block b handles units b, b + gridDim.x, ... (unit = frame x
// row tile) and prefetches the next unit's camera bytes into registers while
// it transforms the current one.
template <typename TIN> struct Raw8;
template <> struct Raw8<uint8_t> {
  uint2 w;
  __device__ void load(const uint8_t* p) { w = *reinterpret_cast<const uint2*>(p); }
  __device__ float get(int e) const { return (float)(((e < 4 ? w.x : w.y) >> (8 * (e & 3))) & 0xffu); }
};
template <> struct Raw8<uint16_t> {
  uint4 w;
  __device__ void load(const uint16_t* p) { w = *reinterpret_cast<const uint4*>(p); }
  __device__ float get(int e) const {
    const uint32_t v = e < 2 ? w.x : e < 4 ? w.y : e < 6 ? w.z : w.w;
    return (float)((v >> (16 * (e & 1))) & 0xffffu);
  }
};

// Two consecutive outputs of one column of the transposed half spectrum
// (rows 2b and 2b + 1) as one store.
__device__ inline void store_pair(float2* p, float2 a, float2 b) {
  *reinterpret_cast<float4*>(p) = make_float4(a.x, a.y, b.x, b.y);
}
__device__ inline void store_pair(hv_h2* p, float2 a, float2 b) {
  typedef _Float16 h4 __attribute__((ext_vector_type(4)));
  h4 h;
  h[0] = (_Float16)a.x;
  h[1] = (_Float16)a.y;
  h[2] = (_Float16)b.x;
  h[3] = (_Float16)b.y;
  *reinterpret_cast<h4*>(p) = h;
}

template <int NX, int ROWS, typename TIN, typename TOUT>
__global__ __launch_bounds__(NT) void k_row_r2c(const TIN* __restrict__ in, TOUT* __restrict__ out, int ny,
                                                int nunits, float scale) {
  constexpr int NB = ROWS / 2;
  constexpr int S = lds_stride(NX);
  constexpr int CH = NB * (NX / 8);  // 8-element chunks of row pairs
  constexpr int PER = (CH + NT - 1) / NT;
  __shared__ float2 buf[NB * S];
  __shared__ float2 tw[tw_size(NX) > 0 ? tw_size(NX) : 1];
  const int tid = threadIdx.x;
  const int tiles = ny / ROWS;
  fill_twiddles<NX>(tw, tid, NT);
  // load: chunk q = tid + i * NT is row pair b, columns 8c .. 8c + 7
  using TL = TileSplit<NX / 8, NT>;
  const int bt = TL::row_thr(tid), ctl = TL::col_thr(tid);
  const uint32_t off_in = (uint32_t)(2 * bt * NX + 8 * ctl) * (uint32_t)sizeof(TIN);
  // store: item q = tid + k * NT is row pair b = q % NB of column fx = q / NB
  constexpr int FPK = NT / NB;  // columns per pass of the threads
  static_assert(NT % NB == 0 && (NX / 2) % FPK == 0, "store split");
  const int bs = tid % NB, fs = tid / NB;
  const uint32_t off_out = (uint32_t)(fs * ny + 2 * bs) * (uint32_t)sizeof(TOUT);
  const float2* prow = buf + bs * S;
  Raw8<TIN> ra[PER], rb[PER];
  auto fetch = [&](int u) {
    const TIN* src = in + ((long)(u / tiles) * ny + (long)(u % tiles) * ROWS) * NX;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      if (CH % NT == 0 || tid + i * NT < CH) {
        const TIN* p = src + 2 * TL::row_i(i) * NX + 8 * TL::col_i(i);
        ra[i].load(reinterpret_cast<const TIN*>(reinterpret_cast<const char*>(p) + off_in));
        rb[i].load(reinterpret_cast<const TIN*>(reinterpret_cast<const char*>(p + NX) + off_in));
      }
    }
  };
  // One unit.  The next unit's loads are issued on every pass (the last one
  // re-reads a unit) and the stores are unrolled; with the first pass peeled
  // off the loop, the loop is entered with the same operations in flight as
  // on its back edge, so the wait for the loads at the top of a pass counts
  // them exactly and leaves the previous pass's stores in flight.
  auto pass = [&](int u) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      if (CH % NT == 0 || tid + i * NT < CH) {
        float2* dst = buf + (bt + TL::row_i(i)) * S;
        const int c = ctl + TL::col_i(i);
#pragma unroll
        for (int e = 0; e < 8; ++e) dst[skew(8 * c + e)] = make_float2(ra[i].get(e), rb[i].get(e));
      }
    }
    __syncthreads();
    fetch(u + (int)gridDim.x < nunits ? u + (int)gridDim.x : nunits - 1);
    fft_lds<NX, NB, NT, -1>(buf, tw, tid);
    // The complex FFT Z of rows x (real part) and y (imaginary part) gives
    // X(f) = (Z(f) + conj Z(-f)) / 2 and Y(f) = (Z(f) - conj Z(-f)) / 2i.
    TOUT* dst = out + (long)(u / tiles) * (NX / 2) * ny + (u % tiles) * ROWS;
#pragma unroll
    for (int k = 0; k < (NX / 2) / FPK; ++k) {
      const int fx = fs + k * FPK;
      const float2 z1 = prow[skew(fx)];
      float2 ve, vo;
      if (fx == 0) {
        const float2 zn = prow[skew(NX / 2)];
        ve = make_float2(z1.x, zn.x);
        vo = make_float2(z1.y, zn.y);
      } else {
        const float2 z2 = c2::conj(prow[skew(NX - fx)]);
        ve = c2::scale(c2::add(z1, z2), 0.5f);
        const float2 d = c2::sub(z1, z2);
        vo = make_float2(0.5f * d.y, -0.5f * d.x);
      }
      store_pair(reinterpret_cast<TOUT*>(reinterpret_cast<char*>(dst + (long)k * FPK * ny) + off_out),
                 c2::scale(ve, scale), c2::scale(vo, scale));
    }
    __syncthreads();
  };
  int u = blockIdx.x;
  if (u >= nunits) return;
  fetch(u);
  pass(u);
  for (u += gridDim.x; u < nunits; u += gridDim.x) pass(u);
}

// ------------------------------------------------------------------ K2
// Block (f0 / BC, t): half-spectrum columns fx in [f0, f0 + BC) of frame t.
// Column fx yields output columns fx and -fx (= nx - fx); fx = 0 packs the
// real DC and Nyquist columns.  hs holds H_z in the order this kernel reads
// it: hs[0][fx][fy] = H(fx, fy), hs[1][fx][fy] = H(-fx, fy) (H(nx/2, fy) for
// fx = 0), both / ny.
template <int NY, int BC, typename TIO>
__global__ __launch_bounds__(NT) void k_col_as(const TIO* __restrict__ in, TIO* __restrict__ out,
                                               const float2* __restrict__ hs, int nx, bool frames8) {
  constexpr int S = lds_stride(NY);
  constexpr int U = BC * NY / NT;
  static_assert(BC * NY % NT == 0, "column tile must split evenly");
  __shared__ float2 buf[2 * BC * S];
  __shared__ float2 tw[tw_size(NY) > 0 ? tw_size(NY) : 1];
  const int tid = threadIdx.x;
  // Workgroups go to the 8 XCDs round-robin by linear index.  The mirrored
  // runs of neighbouring column groups of one frame share 128-byte lines,
  // so when the frame count allows, all groups of a frame are given indices
  // of one residue mod 8 (one XCD, one L2) and the partial lines merge there.
  const int groups = nx / 2 / BC;
  const int lin = blockIdx.x;
  int gx, tf;
  if (frames8) {
    const int r = lin >> 3;
    tf = 8 * (r / groups) + (lin & 7);
    gx = r % groups;
  } else {
    tf = lin / groups;
    gx = lin % groups;
  }
  const int f0 = gx * BC;
  const long t = tf;
  const int half = nx / 2;
  fill_twiddles<NY>(tw, tid, NT);
  // element u of this thread in the BC x NY tile: column s = st + row_i(u),
  // frequency fy = yt + col_i(u)
  using TS = TileSplit<NY, NT>;
  const int st = TS::row_thr(tid), yt = TS::col_thr(tid);
  const uint32_t off_h = (uint32_t)(st * NY + yt) * 8u;
  const TIO* src = in + (t * half + f0) * (long)NY;
  const float2* hpos = hs + (long)f0 * NY;
  const float2* hneg = hs + ((long)half + f0) * NY;
  float2* lds = buf + st * S + skew(yt);
  // The forward column FFT's first pass reads straight from registers:
  // element (u, r) of this thread is column b_u at frequency i_u + r * SP
  // (16 lanes take 16 consecutive values of one column), so the input is
  // loaded into exactly those registers and skips the LDS staging.
  constexpr int UF = fft_first_slots<NY, BC, NT>(), RF = radix_of_pass(NY, 0), SP = NY / RF;
  TIO v0[UF][RF];
#pragma unroll
  for (int u = 0; u < UF; ++u) {
    int b, i;
    if (fft_first_index<NY, BC, NT>(tid, u, 0, &b, &i)) {
      const uint32_t o = (uint32_t)(b * NY + i) * (uint32_t)sizeof(TIO);
#pragma unroll
      for (int r = 0; r < RF; ++r) v0[u][r] = ld_off(src + r * SP, o);
    }
  }
  // transfer-function values of this thread's outputs (+fx and -fx
  // tables; for the packed column fx = 0 the -fx partner is the Nyquist
  // column), fetched now so that their latency hides behind the column FFT.
  // Both are loaded unconditionally: a copy of one into the other where
  // they are equal would wait for every load issued before it.
  float2 ha[U], hb[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    ha[u] = ld_off(hpos + TS::row_i(u) * NY + TS::col_i(u), off_h);
    hb[u] = ld_off(hneg + TS::row_i(u) * NY + TS::col_i(u), off_h);
  }
  fft_lds_io<NY, BC, NT, -1>(buf, tw, tid, [&](int u, int r, int, int) { return load_c(&v0[u][r]); }, nullptr);
  // Sequences BC..2BC-1 are free until the inverse transform: the -fx
  // products go there at once, the +fx products after every read of the
  // forward spectrum is done.
  float2 va[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int s = st + TS::row_i(u), fy = yt + TS::col_i(u);
    const float2* col = buf + s * S;
    float2 z1 = col[skew(fy)];
    float2 z2 = c2::conj(col[skew((NY - fy) & (NY - 1))]);
    float2 a, b;
    if (f0 + s == 0) {
      a = c2::scale(c2::add(z1, z2), 0.5f);
      float2 d = c2::sub(z1, z2);
      b = make_float2(0.5f * d.y, -0.5f * d.x);
    } else {
      a = z1;
      b = z2;
    }
    va[u] = c2::mul(a, ha[u]);
    lds[(BC + TS::row_i(u)) * S + skew(TS::col_i(u))] = c2::mul(b, hb[u]);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < U; ++u) lds[TS::row_i(u) * S + skew(TS::col_i(u))] = va[u];
  __syncthreads();
  fft_lds<NY, 2 * BC, NT, +1>(buf, tw, tid);
  // output row y = yo + k * RPK, sequence i: +fx column f0 + i for i < BC,
  // else the -fx column of fx = f0 + i - BC
  constexpr int RPK = NT / (2 * BC);
  static_assert(NT % (2 * BC) == 0 && NY % RPK == 0, "store split");
  const int i = tid % (2 * BC), yo = tid / (2 * BC);
  int c = f0 + i;
  if (i >= BC) c = f0 + i - BC == 0 ? half : nx - (f0 + i - BC);
  const uint32_t off_out = (uint32_t)(yo * nx + c) * (uint32_t)sizeof(TIO);
  TIO* dst = out + t * (long)NY * nx;
  const float2* row = buf + i * S + skew(yo);
#pragma unroll 4
  for (int k = 0; k < NY / RPK; ++k) {
    TIO v;
    store_c(&v, row[skew(k * RPK)]);
    st_off(dst + (long)k * RPK * nx, off_out, v);
  }
}

// A tile of E elements from src (element q at src + q, sequence-major) into
// the LDS rows buf[(q / N) * S + skew(q % N)].  The trip count is fixed at
// compile time, so every load is issued before the first LDS write.
template <int N, int E, typename TIN>
__device__ inline void load_tile(float2* buf, const TIN* __restrict__ src, int tid) {
  constexpr int S = lds_stride(N), PER = (E + NT - 1) / NT;
  TIN v[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int q = tid + i * NT;
    if (E % NT == 0 || q < E) v[i] = src[q];
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int q = tid + i * NT;
    if (E % NT == 0 || q < E) buf[(q / N) * S + skew(q % N)] = load_c(&v[i]);
  }
}

// ------------------------------------------------------------------ K3
template <int NX, int ROWS, typename TIN, typename TOUT>
__global__ __launch_bounds__(NT) void k_row_inv(const TIN* __restrict__ in, TOUT* __restrict__ out, int ny,
                                                float scale) {
  constexpr int S = lds_stride(NX);
  __shared__ float2 buf[ROWS * S];
  __shared__ float2 tw[tw_size(NX) > 0 ? tw_size(NX) : 1];
  const int tid = threadIdx.x;
  const long base = ((long)blockIdx.y * ny + (long)blockIdx.x * ROWS) * NX;
  fill_twiddles<NX>(tw, tid, NT);
  load_tile<NX, ROWS * NX>(buf, in + base, tid);
  __syncthreads();
  fft_lds<NX, ROWS, NT, +1>(buf, tw, tid);
  for (int q = tid; q < ROWS * NX; q += NT)
    store_c(out + base + q, c2::scale(buf[(q / NX) * S + skew(q % NX)], scale));
}

// Workgroups go to the 8 XCDs round-robin by linear index.  The tiles of a
// frame below write runs of 8 or 16 values, so neighbouring tiles 2m and
// 2m + 1 share 128-byte lines; when the tile count is a multiple of 16 this
// numbering gives the two of a pair indices of one residue mod 8 (one XCD,
// one L2), where the partial lines merge before they reach HBM.
__device__ inline int xcd_paired(int bx, int tiles) {
  return (tiles & 15) ? bx : 16 * (bx >> 4) + 2 * (bx & 7) + ((bx >> 3) & 1);
}

// ------------------------------------------------------------------ K4 rows / complex rows
// Row FFT of sign DIR of (input * qx[m] * qy[n]) (no chirp when qx is
// null), transposed write [t][nx][ny].
template <int NX, int ROWS, typename TIN, typename TOUT, int DIR>
__global__ __launch_bounds__(NT) void k_rows_c2c(const TIN* __restrict__ in, TOUT* __restrict__ out,
                                                 const float2* __restrict__ qx, const float2* __restrict__ qy,
                                                 int ny, float scale) {
  constexpr int S = lds_stride(NX);
  __shared__ float2 buf[ROWS * S];
  __shared__ float2 tw[tw_size(NX) > 0 ? tw_size(NX) : 1];
  const int tid = threadIdx.x;
  const int y0 = xcd_paired(blockIdx.x, gridDim.x) * ROWS;
  const long t = blockIdx.y;
  fill_twiddles<NX>(tw, tid, NT);
  const TIN* src = in + (t * ny + y0) * (long)NX;
  // Runs of 8 values; every run of the tile is loaded before the first LDS
  // write.
  constexpr int E8 = ROWS * (NX / 8), PER = (E8 + NT - 1) / NT;
  float2 v[PER][8];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int q = tid + k * NT;
    if (E8 % NT == 0 || q < E8) load8c(src + (q / (NX / 8)) * NX + 8 * (q % (NX / 8)), v[k]);
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int q = tid + k * NT;
    if (E8 % NT != 0 && q >= E8) continue;
    const int r = q / (NX / 8), c = q % (NX / 8);
    if (qx) {
      const float2 cy = qy[y0 + r];
#pragma unroll
      for (int e = 0; e < 8; ++e) v[k][e] = c2::mul(v[k][e], c2::mul(qx[8 * c + e], cy));
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) buf[r * S + skew(8 * c + e)] = v[k][e];
  }
  __syncthreads();
  fft_lds<NX, ROWS, NT, DIR>(buf, tw, tid);
  TOUT* dst = out + t * (long)NX * ny + y0;
  for (int q = tid; q < NX * ROWS; q += NT) {
    const int p = q / ROWS, r = q % ROWS;
    store_c(dst + (long)p * ny + r, c2::scale(buf[r * S + skew(p)], scale));
  }
}

// ------------------------------------------------------------------ complex AS columns
// Column FFT, multiply by ht[column][fy], inverse column FFT; in [t][nx][ny],
// out [t][ny][nx].
template <int NY, int BC, typename TIO>
__global__ __launch_bounds__(NT) void k_col_full(const TIO* __restrict__ in, TIO* __restrict__ out,
                                                 const float2* __restrict__ ht, int nx) {
  constexpr int S = lds_stride(NY);
  __shared__ float2 buf[BC * S];
  __shared__ float2 tw[tw_size(NY) > 0 ? tw_size(NY) : 1];
  const int tid = threadIdx.x;
  const int p0 = xcd_paired(blockIdx.x, gridDim.x) * BC;
  const long t = blockIdx.y;
  fill_twiddles<NY>(tw, tid, NT);
  const TIO* src = in + (t * nx + p0) * (long)NY;
  load_tile<NY, BC * NY>(buf, src, tid);
  // The tile's transfer-function values are one contiguous run
  // ht[p0 * NY + q], fetched here so they arrive during the forward FFT.
  // For 1024-point columns the extra registers would cost the second
  // workgroup per CU, so there they are read after the FFT.
  constexpr int E = BC * NY, PER = (E + NT - 1) / NT;
  constexpr bool PRE = NY < 1024;
  const float2* hp = ht + (long)p0 * NY;
  float2 h[PRE ? PER : 1];
  if constexpr (PRE) {
#pragma unroll
    for (int k = 0; k < PER; ++k)
      if (E % NT == 0 || tid + k * NT < E) h[k] = hp[tid + k * NT];
  }
  __syncthreads();
  fft_lds<NY, BC, NT, -1>(buf, tw, tid);
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int q = tid + k * NT;
    if (E % NT != 0 && q >= E) continue;
    float2* e = &buf[(q / NY) * S + skew(q % NY)];
    *e = c2::mul(*e, PRE ? h[PRE ? k : 0] : hp[q]);
  }
  __syncthreads();
  fft_lds<NY, BC, NT, +1>(buf, tw, tid);
  TIO* dst = out + t * (long)NY * nx;
  for (int q = tid; q < BC * NY; q += NT) {
    const int y = q / BC, i = q % BC;
    store_c(dst + (long)y * nx + p0 + i, buf[i * S + skew(y)]);
  }
}

// ------------------------------------------------------------------ K4 columns
template <int NY, int BC, typename TIN, typename TOUT, int DIR>
__global__ __launch_bounds__(NT) void k_fresnel_cols(const TIN* __restrict__ in, TOUT* __restrict__ out,
                                                     const float2* __restrict__ qx,
                                                     const float2* __restrict__ qy, int nx, float scale) {
  constexpr int S = lds_stride(NY);
  __shared__ float2 buf[BC * S];
  __shared__ float2 tw[tw_size(NY) > 0 ? tw_size(NY) : 1];
  const int tid = threadIdx.x;
  const int p0 = xcd_paired(blockIdx.x, gridDim.x) * BC;
  const long t = blockIdx.y;
  fill_twiddles<NY>(tw, tid, NT);
  const TIN* src = in + (t * nx + p0) * (long)NY;
  load_tile<NY, BC * NY>(buf, src, tid);
  // Output element q = tid + k * NT is (y, i) = (q / BC, q % BC); NT is a
  // multiple of BC, so each thread keeps one column i and steps y by NT / BC.
  // Its chirp values are fetched here and arrive during the FFT.
  constexpr int E = BC * NY, PER = (E + NT - 1) / NT, YS = NT / BC;
  static_assert(NT % BC == 0, "a thread keeps one column");
  const int i = tid % BC, yt = tid / BC;
  const float2 cx = qx[p0 + i];
  float2 cy[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (E % NT == 0 || yt + k * YS < NY) cy[k] = qy[yt + k * YS];
  __syncthreads();
  fft_lds<NY, BC, NT, DIR>(buf, tw, tid);
  TOUT* dst = out + t * (long)NY * nx + p0 + i;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int y = yt + k * YS;
    if (E % NT != 0 && y >= NY) continue;
    float2 v = c2::mul(buf[i * S + skew(y)], c2::mul(cx, cy[k]));
    store_c(dst + (long)y * nx, c2::scale(v, scale));
  }
}

// ------------------------------------------------------------------ dispatch helpers

constexpr int cap64(int r) { return r > 64 ? 64 : r; }
constexpr int cap32(int r) { return r > 32 ? 32 : r; }
constexpr int p2floor(int r) {
  int p = 1;
  while (2 * p <= r) p *= 2;
  return p;
}

template <int NX, typename TIN, typename TOUT>
void go_r2c(const void* in, void* out, int n, int ny, float scale, hipStream_t st) {
  constexpr int ROWS = cap64(16384 / NX);
  const int nunits = n * (ny / ROWS);
  auto kern = k_row_r2c<NX, ROWS, TIN, TOUT>;
  hipLaunchKernelGGL(kern, dim3(persistent_grid(kern, NT, nunits)), dim3(NT), 0, st, (const TIN*)in, (TOUT*)out, ny,
                     nunits, scale);
}

template <int NY, typename TIO>
void go_col_as(const void* in, void* out, const float2* hs, int n, int nx, hipStream_t st) {
  constexpr int BC = cap32(4096 / NY);  // nx/2 >= 32 >= BC, so BC divides nx/2
  hipLaunchKernelGGL((k_col_as<NY, BC, TIO>), dim3((nx / 2) / BC * n), dim3(NT), 0, st, (const TIO*)in,
                     (TIO*)out, hs, nx, n % 8 == 0);
}

template <int NX, typename TIN, typename TOUT>
void go_row_inv(const void* in, void* out, int n, int ny, float scale, hipStream_t st) {
  constexpr int ROWS = cap64(p2floor(8192 / NX));
  hipLaunchKernelGGL((k_row_inv<NX, ROWS, TIN, TOUT>), dim3(ny / ROWS, n), dim3(NT), 0, st, (const TIN*)in,
                     (TOUT*)out, ny, scale);
}

template <int NX, typename TIN, typename TOUT>
void go_rows(const void* in, void* out, const float2* qx, const float2* qy, int dir, int n, int ny, float scale,
             hipStream_t st) {
  constexpr int ROWS = cap64(p2floor(8192 / NX));
  if (dir < 0)
    hipLaunchKernelGGL((k_rows_c2c<NX, ROWS, TIN, TOUT, -1>), dim3(ny / ROWS, n), dim3(NT), 0, st,
                       (const TIN*)in, (TOUT*)out, qx, qy, ny, scale);
  else
    hipLaunchKernelGGL((k_rows_c2c<NX, ROWS, TIN, TOUT, +1>), dim3(ny / ROWS, n), dim3(NT), 0, st,
                       (const TIN*)in, (TOUT*)out, qx, qy, ny, scale);
}

template <int NY, typename TIO>
void go_col_full(const void* in, void* out, const float2* ht, int n, int nx, hipStream_t st) {
  constexpr int BC = cap32(p2floor(8192 / NY));
  hipLaunchKernelGGL((k_col_full<NY, BC, TIO>), dim3(nx / BC, n), dim3(NT), 0, st, (const TIO*)in, (TIO*)out, ht,
                     nx);
}

template <int NY, typename TIN, typename TOUT>
void go_fr_cols(const void* in, void* out, const float2* qx, const float2* qy, int dir, int n, int nx,
                float scale, hipStream_t st) {
  constexpr int BC = cap32(p2floor(8192 / NY));
  if (dir < 0)
    hipLaunchKernelGGL((k_fresnel_cols<NY, BC, TIN, TOUT, -1>), dim3(nx / BC, n), dim3(NT), 0, st,
                       (const TIN*)in, (TOUT*)out, qx, qy, nx, scale);
  else
    hipLaunchKernelGGL((k_fresnel_cols<NY, BC, TIN, TOUT, +1>), dim3(nx / BC, n), dim3(NT), 0, st,
                       (const TIN*)in, (TOUT*)out, qx, qy, nx, scale);
}

hv_status launched(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hvi::fail(HV_ERR_DEVICE, "%s launch failed: %s", what, hipGetErrorString(e));
  return HV_OK;
}

// Calls F<N>(args...) for N in {64, 128, 256, 512, 1024} (the real-input
// row pass, the column pass of the angular spectrum and the fused temporal
// kernel, which rely on power-of-two sides).
#define HV_SWITCH_N(n, CALL)          \
  switch (n) {                        \
    case 64: { constexpr int N_ = 64; CALL; } break;     \
    case 128: { constexpr int N_ = 128; CALL; } break;   \
    case 256: { constexpr int N_ = 256; CALL; } break;   \
    case 512: { constexpr int N_ = 512; CALL; } break;   \
    case 1024: { constexpr int N_ = 1024; CALL; } break; \
    default: return hvi::fail(HV_ERR_SHAPE, "size %d not supported", n); \
  }
// The complex row and column passes also take the mixed-radix sides of the
// paper's Table IV frames: 320, 384, 800 and 1280.
#define HV_SWITCH_NG(n, CALL)         \
  switch (n) {                        \
    case 64: { constexpr int N_ = 64; CALL; } break;     \
    case 128: { constexpr int N_ = 128; CALL; } break;   \
    case 256: { constexpr int N_ = 256; CALL; } break;   \
    case 320: { constexpr int N_ = 320; CALL; } break;   \
    case 384: { constexpr int N_ = 384; CALL; } break;   \
    case 512: { constexpr int N_ = 512; CALL; } break;   \
    case 800: { constexpr int N_ = 800; CALL; } break;   \
    case 1024: { constexpr int N_ = 1024; CALL; } break; \
    case 1280: { constexpr int N_ = 1280; CALL; } break; \
    default: return hvi::fail(HV_ERR_SHAPE, "size %d not supported", n); \
  }

}  // namespace

namespace hvi {

hv_status launch_row_r2c(const void* in, hv_dtype in_t, void* out, bool half_out, int n, int ny, int nx,
                         float scale, hipStream_t st) {
  if (n <= 0) return HV_OK;
  if (in_t == HV_U8) {
    if (half_out) { HV_SWITCH_N(nx, (go_r2c<N_, uint8_t, hv_h2>(in, out, n, ny, scale, st))); }
    else { HV_SWITCH_N(nx, (go_r2c<N_, uint8_t, float2>(in, out, n, ny, scale, st))); }
  } else {
    if (half_out) { HV_SWITCH_N(nx, (go_r2c<N_, uint16_t, hv_h2>(in, out, n, ny, scale, st))); }
    else { HV_SWITCH_N(nx, (go_r2c<N_, uint16_t, float2>(in, out, n, ny, scale, st))); }
  }
  return launched("row_r2c");
}

hv_status launch_col_as(const void* in, void* out, bool half_io, const float2* hs, int n, int ny, int nx,
                        hipStream_t st) {
  if (n <= 0) return HV_OK;
  if (half_io) { HV_SWITCH_N(ny, (go_col_as<N_, hv_h2>(in, out, hs, n, nx, st))); }
  else { HV_SWITCH_N(ny, (go_col_as<N_, float2>(in, out, hs, n, nx, st))); }
  return launched("col_as");
}

hv_status launch_row_inv(const void* in, bool half_in, void* out, bool half_out, int n, int ny, int nx,
                         float scale, hipStream_t st) {
  if (n <= 0) return HV_OK;
  if (half_in) {
    if (half_out) { HV_SWITCH_NG(nx, (go_row_inv<N_, hv_h2, hv_h2>(in, out, n, ny, scale, st))); }
    else { HV_SWITCH_NG(nx, (go_row_inv<N_, hv_h2, float2>(in, out, n, ny, scale, st))); }
  } else {
    if (half_out) { HV_SWITCH_NG(nx, (go_row_inv<N_, float2, hv_h2>(in, out, n, ny, scale, st))); }
    else { HV_SWITCH_NG(nx, (go_row_inv<N_, float2, float2>(in, out, n, ny, scale, st))); }
  }
  return launched("row_inv");
}

hv_status launch_rows_c2c(const void* in, int in_t, void* out, bool half_out, const float2* qx, const float2* qy,
                          int dir, int n, int ny, int nx, float scale, hipStream_t st) {
  if (n <= 0) return HV_OK;
#define HV_ROWS_T(TIN)                                                                                     \
  if (half_out) { HV_SWITCH_NG(nx, (go_rows<N_, TIN, hv_h2>(in, out, qx, qy, dir, n, ny, scale, st))); }   \
  else { HV_SWITCH_NG(nx, (go_rows<N_, TIN, float2>(in, out, qx, qy, dir, n, ny, scale, st))); }
  if (in_t == HV_U8) {
    HV_ROWS_T(uint8_t)
  } else if (in_t == HV_U16) {
    HV_ROWS_T(uint16_t)
  } else {
    HV_ROWS_T(float2)
  }
#undef HV_ROWS_T
  return launched("rows_c2c");
}

hv_status launch_col_full(const void* in, void* out, bool half_io, const float2* ht, int n, int ny, int nx,
                          hipStream_t st) {
  if (n <= 0) return HV_OK;
  if (half_io) { HV_SWITCH_NG(ny, (go_col_full<N_, hv_h2>(in, out, ht, n, nx, st))); }
  else { HV_SWITCH_NG(ny, (go_col_full<N_, float2>(in, out, ht, n, nx, st))); }
  return launched("col_full");
}

hv_status launch_fresnel_cols(const void* in, bool half_in, void* out, bool half_out, const float2* qx,
                              const float2* qy, int dir, int n, int ny, int nx, float scale, hipStream_t st) {
  if (n <= 0) return HV_OK;
  if (half_in) {
    if (half_out) { HV_SWITCH_NG(ny, (go_fr_cols<N_, hv_h2, hv_h2>(in, out, qx, qy, dir, n, nx, scale, st))); }
    else { HV_SWITCH_NG(ny, (go_fr_cols<N_, hv_h2, float2>(in, out, qx, qy, dir, n, nx, scale, st))); }
  } else {
    if (half_out) { HV_SWITCH_NG(ny, (go_fr_cols<N_, float2, hv_h2>(in, out, qx, qy, dir, n, nx, scale, st))); }
    else { HV_SWITCH_NG(ny, (go_fr_cols<N_, float2, float2>(in, out, qx, qy, dir, n, nx, scale, st))); }
  }
  return launched("fresnel_cols");
}

}  // namespace hvi
