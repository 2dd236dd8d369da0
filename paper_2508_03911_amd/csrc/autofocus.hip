// Learned autofocus with a brute-force z-scan as fallback and as a check.
//
// The paper lists machine-learning inference as a plug-in for the real-time
// pipeline (Sec. VIII, future work).  Built here for 256 x 256 holograms:
//   - spectrum crop: log(1 + |DFT2(h - mean)|), 64 x 64 centred on DC,
//     standardised per crop (the network input, stored fp16);
//   - z-scan: the +1-order sub-band (64 x 64 bins around the carrier at
//     (-1/4, -1/4) cycles/pixel, masked to radius 0.1 cycles/pixel) times
//     H_{-z_c} at the demodulated object frequencies, inverse FFT at 64 x 64,
//     sharpness = variance of the forward-difference gradient magnitude of
//     the amplitude, argmax over the candidates (ties to the lowest z);
//   - CNN: conv3x3(1->32) ReLU, 3 x [conv3x3(32->32) ReLU], global average
//     pooling, FC(32->64) ReLU, FC(64->2) = (z, log sigma^2); Gaussian NLL;
//     Adam.  Forward, backward-data, backward-weight, head and optimizer are
//     hand-written FP32 kernels; weight-gradient partial sums are reduced in
//     a fixed order (deterministic);
//   - training holograms synthesised on the GPU: counter-based noise
//     (Philox4x32-10, Salmon et al., SC'11) band-limited by a circular pupil
//     through the library's own FFT passes, a disk mask, propagation by
//     hv_propagate, an off-axis reference, and photon noise.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <random>
#include <string>
#include <vector>

#include "fft_lds.h"
#include "hv_ctx.h"
#include "hv_internal.h"

using namespace hvk;
using hvi::fail;

namespace {

constexpr int AN = 256;   // hologram side
constexpr int CROP = 64;  // network input side
constexpr int SUB = 64;   // scan sub-band side
constexpr int NCH = 32;   // conv channels
constexpr int HW = CROP * CROP;
constexpr int NPARAM = 30306;
constexpr int OFF_W[4] = {0, 320, 9568, 18816};
constexpr int OFF_B[4] = {288, 9536, 18784, 28032};
constexpr int OFF_FC1W = 28064, OFF_FC1B = 30112, OFF_FC2W = 30176, OFF_FC2B = 30304;
constexpr int HEAD_N = 2048 + 64 + 128 + 2;  // fc1 w, fc1 b, fc2 w, fc2 b

__device__ inline float to_f(float v) { return v; }
__device__ inline float to_f(_Float16 v) { return (float)v; }

// ------------------------------------------------------------------ block reduction (double)
template <int NT>
__device__ inline double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// ------------------------------------------------------------------ spectrum crop and sub-band
// Straight from the camera bytes, one hologram per unit: CR, the network's
// crop, from the 2-D spectrum X at columns kx = 0 .. 32 and rows
// ky = -32 .. 32; SB, the +1-order sub-band, from columns and rows
// 33 .. 96.  The 256 rows are taken in eight interleaved groups
// (y = 8 m + g, m < 32), 32 rows = 16 complex FFTs of two real rows each
// (the next group's bytes load into registers meanwhile); the two rows'
// spectra are separated at the needed columns, a 32-point FFT along m
// gives Y_g(ky mod 32, kx), and X(ky, kx) = sum_g W256^(g ky) Y_g(ky mod 32,
// kx) is accumulated in registers, one output per (thread, slot) -- the
// column transform split as 256 = 8 x 32, so that LDS holds one row group
// rather than all 256 rows.  Then
//   crop: log(1 + |X(fy, fx)|) for fy, fx in [-32, 32) (fx < 0 through
//         X(fy, fx) = conj X(-fy, -fx), the DC bin zero as for h - mean),
//         standardised over the crop (mean and variance in FP64);
//   sub-band: bins ky = i - 96, kx = j - 96 (i, j < 64), read as
//         conj X(96 - i, 96 - j), zero beyond 0.1 cycles/pixel of the
//         carrier.
template <bool CR, bool SB, typename TOUT>
__global__ __launch_bounds__(256) void k_af_spec(const uint8_t* __restrict__ holo, int n, TOUT* __restrict__ crop,
                                                 float2* __restrict__ sub) {
  constexpr int NT = 256, S = lds_stride(AN), RG = 32, NBR = RG / 2, NG = AN / RG;
  constexpr int S32 = lds_stride(RG);
  constexpr int NCC = CR ? 33 : 0, NSC = SB ? 64 : 0, NSLOT = NCC + NSC;  // column slots
  constexpr int NOC = CR ? 33 * 65 : 0, NOS = SB ? 64 * 64 : 0, NOUT = NOC + NOS;
  constexpr int PERT = (NOUT + NT - 1) / NT;  // outputs per thread
  static_assert(NBR * S * 8 >= NOC * 4 + NT * 8, "the crop's staging fits in the row buffer");
  __shared__ float2 rb[NBR * S];  // a row group; the crop's staging after the last group
  __shared__ float2 cb[NSLOT * S32];
  __shared__ float2 tw[tw_size(AN)];
  __shared__ float2 tw32[tw_size(RG)];
  __shared__ float2 w256[AN];  // W256^k = exp(-2 pi i k / 256)
  const int tid = threadIdx.x;
  fill_twiddles<AN>(tw, tid, NT);
  fill_twiddles<RG>(tw32, tid, NT);
  {
    float sn, cs;
    sincospif(-2.0f * (float)tid / AN, &sn, &cs);
    w256[tid] = make_float2(cs, sn);
  }
  // load slot: row pair lb (rows 16 lb + g and 16 lb + 8 + g: m = 2 lb and
  // 2 lb + 1), bytes lx .. lx + 15
  const int lb = tid >> 4, lx = (tid & 15) * 16;
  uint4 w0, w1;
  auto fetch = [&](long u, int g) {
    const uint8_t* p = holo + u * (AN * AN) + (long)(16 * lb + g) * AN + lx;
    w0 = *reinterpret_cast<const uint4*>(p);
    w1 = *reinterpret_cast<const uint4*>(p + 8 * AN);
  };
  auto byte_of = [](const uint4& w, int e) {
    const uint32_t v = e < 4 ? w.x : e < 8 ? w.y : e < 12 ? w.z : w.w;
    return (float)((v >> (8 * (e & 3))) & 0xffu);
  };
  // output o of this thread: slot (column) and row ky
  auto out_slot = [](int o) { return o < NOC ? o / 65 : NCC + (o - NOC) / 64; };
  auto out_ky = [](int o) { return o < NOC ? o % 65 - 32 : 33 + (o - NOC) % 64; };
  auto slot_kx = [](int sl) { return sl < NCC ? sl : 33 + (sl - NCC); };
  if ((long)blockIdx.x < n) fetch(blockIdx.x, 0);
  for (long u = blockIdx.x; u < n; u += gridDim.x) {
    float2 acc[PERT];
#pragma unroll
    for (int j = 0; j < PERT; ++j) acc[j] = make_float2(0.f, 0.f);
    for (int g = 0; g < NG; ++g) {
      float2* dst = rb + lb * S;
#pragma unroll
      for (int e = 0; e < 16; ++e) dst[skew(lx + e)] = make_float2(byte_of(w0, e), byte_of(w1, e));
      __syncthreads();
      if (g + 1 < NG)
        fetch(u, g + 1);
      else if (u + gridDim.x < n)
        fetch(u + gridDim.x, 0);
      fft_lds<AN, NBR, NT, -1>(rb, tw, tid);
      // Z of rows x (real part) and y (imaginary part): X(f) = (Z(f) +
      // conj Z(-f)) / 2, Y(f) = (Z(f) - conj Z(-f)) / 2i; column 0 is the
      // real DC column alone
      for (int q = tid; q < NBR * NSLOT; q += NT) {
        const int b = q % NBR, sl = q / NBR, fx = slot_kx(sl);
        const float2* prow = rb + b * S;
        const float2 z1 = prow[skew(fx)];
        float2 xe, xo;
        if (fx == 0) {
          xe = make_float2(z1.x, 0.f);
          xo = make_float2(z1.y, 0.f);
        } else {
          const float2 z2 = c2::conj(prow[skew(AN - fx)]);
          xe = c2::scale(c2::add(z1, z2), 0.5f);
          const float2 d = c2::sub(z1, z2);
          xo = make_float2(0.5f * d.y, -0.5f * d.x);
        }
        float2* col = cb + sl * S32;
        col[skew(2 * b)] = xe;
        col[skew(2 * b + 1)] = xo;
      }
      __syncthreads();
      fft_lds<RG, NSLOT, NT, -1>(cb, tw32, tid);
#pragma unroll
      for (int j = 0; j < PERT; ++j) {
        const int o = tid + NT * j;
        if (NOUT % NT == 0 || o < NOUT) {
          const int ky = out_ky(o);
          const float2 y = cb[out_slot(o) * S32 + skew(ky & (RG - 1))];
          const float2 w = w256[(g * ky) & (AN - 1)];
          acc[j] = make_float2(acc[j].x + (y.x * w.x - y.y * w.y), acc[j].y + (y.x * w.y + y.y * w.x));
        }
      }
    }
    const long h = u;
    if constexpr (SB) {
#pragma unroll
      for (int j = 0; j < PERT; ++j) {
        const int o = tid + NT * j;
        if (o >= NOC && o < NOUT) {
          const int i = 96 - out_ky(o), jj = 96 - slot_kx(out_slot(o));
          const int di = i - SUB / 2, dj = jj - SUB / 2;
          const bool in_band = 100 * (di * di + dj * dj) <= AN * AN;  // radius 0.1 cycles/pixel
          sub[h * SUB * SUB + i * SUB + jj] = in_band ? make_float2(acc[j].x, -acc[j].y) : make_float2(0.f, 0.f);
        }
      }
    }
    if constexpr (CR) {
      // log-magnitudes of the 33 x 65 outputs, then the crop through the symmetry
      float* lm = reinterpret_cast<float*>(rb);
#pragma unroll
      for (int j = 0; j < PERT; ++j) {
        const int o = tid + NT * j;
        if (o < NOC) {
          const float mag = o == 32 ? 0.f : sqrtf(acc[j].x * acc[j].x + acc[j].y * acc[j].y);  // DC removed with the mean
          lm[o] = log1pf(mag);
        }
      }
      __syncthreads();
      constexpr int PQ = HW / NT;
      float v[PQ];
      double s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int j = 0; j < PQ; ++j) {
        const int q = tid + NT * j;
        const int fy = q / CROP - CROP / 2, fx = q % CROP - CROP / 2;
        v[j] = fx >= 0 ? lm[fx * 65 + fy + 32] : lm[-fx * 65 - fy + 32];
        s1 += v[j];
        s2 += (double)v[j] * v[j];
      }
      double* red = reinterpret_cast<double*>(lm + NOC + 1);  // 8-byte aligned past the staging
      s1 = block_sum<NT>(s1, red);
      s2 = block_sum<NT>(s2, red);
      const double mean = s1 / HW;
      const double sd = sqrt(fmax(s2 / HW - mean * mean, 1e-30));
      const float m = (float)mean, inv = (float)(1.0 / sd);
#pragma unroll
      for (int j = 0; j < PQ; ++j) crop[h * HW + tid + NT * j] = (TOUT)((v[j] - m) * inv);
    }
  }
}

// Sharpness of the reconstruction for CPB candidates per block.  Transfer
// functions: from htab [nc][SUB][SUB] (candidates shared by every hologram),
// or, with RANGES, candidate c of hologram n at
// z = zlo[n] + (zhi[n] - zlo[n]) c / (nc - 1), H = exp(-i z kz) with
// kz = 2 pi sqrt(1/lambda^2 - |f|^2) from the FP64 table kz (negative:
// evanescent, H = 0).  The candidates of a block are equally spaced, so H
// of the first one and the step factor exp(-i dz kz) are formed once per
// pixel (phase reduced modulo 2 pi in FP64, sine and cosine of the reduced
// angle in FP32) and H advances by one complex product per candidate.
template <int CPB, bool RANGES>
__global__ __launch_bounds__(256) void k_af_scan(const float2* __restrict__ sub, const float2* __restrict__ htab,
                                                 const double* __restrict__ kz, const float* __restrict__ zlo,
                                                 const float* __restrict__ zhi, int nc, float* __restrict__ scores) {
  constexpr int NT = 256, S = lds_stride(SUB), QT = SUB * SUB / NT;
  __shared__ float2 A[SUB * S];
  __shared__ float2 B[SUB * S];
  __shared__ float2 tw[tw_size(SUB) > 0 ? tw_size(SUB) : 1];
  __shared__ double red[NT];
  const int tid = threadIdx.x;
  const long n = blockIdx.x;
  fill_twiddles<SUB>(tw, tid, NT);
  const float2* sv = sub + n * SUB * SUB;
  // RANGES: H of this block's current candidate and the step factor at the
  // pixels q = tid + NT j of this thread
  float2 hcur[RANGES ? QT : 1], hstep[RANGES ? QT : 1];
  if constexpr (RANGES) {
    const double z0 = zlo[n], z1 = zhi[n];
    const double dz = (z1 - z0) / (nc - 1);
    const double zc = z0 + dz * (blockIdx.y * CPB);
    auto unit = [](double ph) {
      const double r = ph - 6.283185307179586 * rint(ph * 0.15915494309189535);
      float sn, cs;
      sincosf((float)r, &sn, &cs);
      return make_float2(cs, sn);
    };
#pragma unroll
    for (int j = 0; j < QT; ++j) {
      const double k = kz[tid + NT * j];
      hcur[j] = k >= 0.0 ? unit(-zc * k) : make_float2(0.f, 0.f);
      hstep[j] = k >= 0.0 ? unit(-dz * k) : make_float2(0.f, 0.f);
    }
  }
  for (int cc = 0; cc < CPB; ++cc) {
    const int c = blockIdx.y * CPB + cc;
    if (c >= nc) break;
    if constexpr (RANGES) {
#pragma unroll
      for (int j = 0; j < QT; ++j) {
        const int q = tid + NT * j;
        A[(q / SUB) * S + skew(q % SUB)] = c2::mul(sv[q], hcur[j]);
        hcur[j] = c2::mul(hcur[j], hstep[j]);
      }
    } else {
      const float2* h = htab + (long)c * SUB * SUB;
      for (int q = tid; q < SUB * SUB; q += NT) A[(q / SUB) * S + skew(q % SUB)] = c2::mul(sv[q], h[q]);
    }
    __syncthreads();
    fft_lds<SUB, SUB, NT, +1>(A, tw, tid);  // rows
    for (int q = tid; q < SUB * SUB; q += NT) {
      const int i = q / SUB, j = q % SUB;
      B[j * S + skew(i)] = A[i * S + skew(j)];
    }
    __syncthreads();
    fft_lds<SUB, SUB, NT, +1>(B, tw, tid);  // columns
    constexpr float inv = 1.0f / (SUB * SUB);
    double s1 = 0.0, s2 = 0.0;
    for (int q = tid; q < (SUB - 1) * (SUB - 1); q += NT) {
      const int i = q / (SUB - 1), j = q % (SUB - 1);
      const float2 u = B[j * S + skew(i)], ux = B[(j + 1) * S + skew(i)], uy = B[j * S + skew(i + 1)];
      const float a = sqrtf(u.x * u.x + u.y * u.y) * inv;
      const float ax = sqrtf(ux.x * ux.x + ux.y * ux.y) * inv;
      const float ay = sqrtf(uy.x * uy.x + uy.y * uy.y) * inv;
      const float gx = ax - a, gy = ay - a;
      const double g = sqrt((double)gx * gx + (double)gy * gy);
      s1 += g;
      s2 += g * g;
    }
    s1 = block_sum<NT>(s1, red);
    s2 = block_sum<NT>(s2, red);
    if (tid == 0) {
      const double m = s1 / ((SUB - 1) * (SUB - 1));
      scores[n * nc + c] = (float)(s2 / ((SUB - 1) * (SUB - 1)) - m * m);
    }
    __syncthreads();
  }
}

// Argmax over each hologram's candidates (ties to the lowest z); the range
// is [z_lo, z_hi] for all, or [zlo[i], zhi[i]] when zlo is not null.  With
// `refine`, [zlo, zhi] is then narrowed to one candidate step on each side
// of the best (within the old range) for a finer scan.
__global__ void k_af_argmax(const float* __restrict__ scores, int n, int nc, double z_lo, double z_hi,
                            float* __restrict__ zlo, float* __restrict__ zhi, float* __restrict__ z_out,
                            float* __restrict__ best, int refine) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int arg = 0;
  float bs = scores[(long)i * nc];
  for (int c = 1; c < nc; ++c) {
    const float s = scores[(long)i * nc + c];
    if (s > bs) {
      bs = s;
      arg = c;
    }
  }
  const double a = zlo ? (double)zlo[i] : z_lo, b = zlo ? (double)zhi[i] : z_hi;
  const double step = (b - a) / (nc - 1);
  z_out[i] = (float)(a + step * arg);
  if (best) best[i] = bs;
  if (refine && zlo) {
    zlo[i] = (float)(a + step * (arg > 0 ? arg - 1 : 0));
    zhi[i] = (float)(a + step * (arg < nc - 1 ? arg + 1 : nc - 1));
  }
}

// Local scan ranges from the network: [z - k sigma, z + k sigma] clipped to
// [lo, hi], at least `minw` wide.
__global__ void k_af_ranges(const float* __restrict__ z, const float* __restrict__ sigma, int n, float k, float lo,
                            float hi, float minw, float* __restrict__ zlo, float* __restrict__ zhi) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float half = fmaxf(k * sigma[i], 0.5f * minw);
  float a = z[i] - half, b = z[i] + half;
  if (a < lo) {
    b = fminf(hi, b + (lo - a));
    a = lo;
  }
  if (b > hi) {
    a = fmaxf(lo, a - (b - hi));
    b = hi;
  }
  zlo[i] = a;
  zhi[i] = b;
}

// ------------------------------------------------------------------ CNN: convolution
// First layer of training's forward pass (1 -> 32 channels: nine taps, too
// few for the matrix cores): direct 3x3 convolution, zero padding 1, on one
// 16 x 16 output tile of one sample; wave w produces output channels
// 8w..8w+7 (weights are wave-uniform and come through the scalar cache),
// each lane 4 pixels: out = ReLU(b + W * in).
template <int CIN, typename TIN>
__global__ __launch_bounds__(256) void k_conv(const TIN* __restrict__ in, const float* __restrict__ params, int woff,
                                              int boff, float* __restrict__ out) {
  __shared__ float tile[CIN][18][19];
  const int tid = threadIdx.x;
  const int ty0 = (blockIdx.x >> 2) * 16, tx0 = (blockIdx.x & 3) * 16;
  const long b = blockIdx.y;
  for (int q = tid; q < CIN * 324; q += 256) {
    const int c = q / 324, r = (q % 324) / 18, col = q % 18;
    const int y = ty0 + r - 1, x = tx0 + col - 1;
    float v = 0.f;
    if (y >= 0 && y < CROP && x >= 0 && x < CROP) v = to_f(in[((b * CIN + c) * CROP + y) * CROP + x]);
    tile[c][r][col] = v;
  }
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  float acc[8][4];
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int p = 0; p < 4; ++p) acc[k][p] = 0.f;
  for (int c = 0; c < CIN; ++c) {
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        float xv[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const int idx = lane + 64 * p;
          xv[p] = tile[c][(idx >> 4) + dy][(idx & 15) + dx];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int o = 8 * wave + k;
          const float w = params[woff + ((o * CIN + c) * 3 + dy) * 3 + dx];
#pragma unroll
          for (int p = 0; p < 4; ++p) acc[k][p] += w * xv[p];
        }
      }
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int o = 8 * wave + k;
    const float bias = params[boff + o];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int idx = lane + 64 * p;
      const int y = ty0 + (idx >> 4), x = tx0 + (idx & 15);
      out[((b * NCH + o) * CROP + y) * CROP + x] = fmaxf(acc[k][p] + bias, 0.f);
    }
  }
}

// ------------------------------------------------------------------ CNN: inference on MFMA
// The forward pass again, for prediction only, as implicit GEMMs on the
// matrix cores: per layer, [256 pixels of a 16 x 16 output tile] x [9 CIN]
// times [9 CIN] x [32 output channels] with fp16 operands and FP32
// accumulation (v_mfma_f32_32x32x16_f16; lane l holds A[l%32][k0 + 8(l/32)
// + e] and B[k0 + 8(l/32) + e][l%32], and result register r is row
// 8(r/4) + 4(l/32) + r%4 of column l%32).  Activations are stored NHWC in
// fp16.  The k index runs over taps, then channels: k = 32 tap + c for the
// 32-channel layers, k = tap (padded to 16) for the first.

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef _Float16 h8v __attribute__((ext_vector_type(8)));

constexpr int IKS = 1 + 3 * 18;  // k-steps of the four layers' B fragments

// B fragments of all layers from the FP32 parameters: wf[(kstep) * 64 + lane].
__global__ void k_pack_weights(const float* __restrict__ params, h8v* __restrict__ wf) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= IKS * 64) return;
  const int ks = q / 64, lane = q % 64, o = lane & 31, h = lane >> 5;
  h8v v;
  if (ks == 0) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 8 * h + e;
      v[e] = (_Float16)(k < 9 ? params[OFF_W[0] + o * 9 + k] : 0.f);
    }
  } else {
    const int l = 1 + (ks - 1) / 18, s = (ks - 1) % 18;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 16 * s + 8 * h + e, tap = k / NCH, c = k % NCH;
      v[e] = (_Float16)params[OFF_W[l] + (o * NCH + c) * 9 + tap];
    }
  }
  wf[q] = v;
}

// A 32-channel layer of the inference pass as an implicit GEMM on the
// matrix cores: per 16 x 16 output tile, [256 pixels] x [288 = 9 taps x 32
// channels] times [288] x [32 output channels], NHWC fp16 activations.
// Persistent: workgroup g takes units g, g + gridDim.x, ... (unit = one
// output tile of one sample) with the layer's weight fragments held in
// registers across units, and loads the next unit's input tile into
// registers while the current unit's MFMAs run.  Wave w owns tile pixels
// [64 w, 64 w + 64) as two 32-pixel tiles.  The product is formed as
// (channels x pixels) = W x X^T, so that a lane holds 16 output channels
// of one pixel (channels 8 q + 4 h + j, q, j < 4) and stores them as four
// 8-byte runs; LAST forms pixels x channels instead, a lane holding one
// channel of 16 pixels, and stores no activation: the ReLU outputs of the
// tile are summed per channel into pooled[sample][tile][32] (the global
// average pool, finished in the head in a fixed order).  FIRST: `in` is
// the crop, and the first layer (1 -> 32 channels, nine taps: one k-step
// with the fragment wf0 and the biases at boff0) is evaluated on the
// 18 x 18 input tile, one tile row per product (lanes 18 .. 31 idle), from
// a 20 x 20 crop tile, rounded to fp16 after its ReLU and kept in LDS (zero
// outside the image: the second layer's padding), so that the first
// layer's activations never reach HBM.
template <bool LAST, bool FIRST>
__global__ __launch_bounds__(256) void k_conv_mfma(const _Float16* __restrict__ in, const h8v* __restrict__ wf,
                                                   const float* __restrict__ params, int boff,
                                                   _Float16* __restrict__ out, float* __restrict__ pooled,
                                                   int nunits, const h8v* __restrict__ wf0, int boff0) {
  typedef _Float16 h4v __attribute__((ext_vector_type(4)));
  constexpr int PS = NCH + 8;  // halves per LDS pixel (80 B: 16-B reads of 16 lanes hit distinct banks)
  constexpr int KS = 9 * NCH / 16;
  constexpr int CT = 34;       // crop tile row stride (columns 20 .. 33 zero)
  // input items per unit: 18 x 18 pixels of NCH/8 chunks of 8 channels, or
  // (FIRST) 20 x 20 crop pixels
  constexpr int ITEMS = FIRST ? 400 : 324 * (NCH / 8);
  constexpr int PER = (ITEMS + 255) / 256;
  using Item = typename std::conditional<FIRST, _Float16, h8v>::type;
  // tile and ctile end in a dummy row that takes the fill of items past the
  // tile, so that the fill has no branch and each load is used where it is
  // issued
  constexpr int TN = 18 * 18 * PS, CN = 20 * CT;
  __shared__ __attribute__((aligned(16))) _Float16 tile[TN + (FIRST ? 0 : 8 * 256)];
  __shared__ _Float16 ctile[FIRST ? CN + 256 : 1];
  __shared__ float red[4][32];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5, c = lane & 31;
  h8v bw[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) bw[s] = wf[s * 64 + lane];
  // biases of the channels this lane produces
  float bias[LAST ? 1 : 16];
  if constexpr (LAST) {
    bias[0] = params[boff + c];
  } else {
#pragma unroll
    for (int r = 0; r < 16; ++r) bias[r] = params[boff + 8 * (r >> 2) + 4 * h + (r & 3)];
  }
  h8v bw0;
  float bias0[FIRST ? 16 : 1];
  if constexpr (FIRST) {
    bw0 = wf0[lane];
#pragma unroll
    for (int r = 0; r < 16; ++r) bias0[r] = params[boff0 + 8 * (r >> 2) + 4 * h + (r & 3)];
    for (int q = tid; q < CN; q += 256)
      if (q % CT >= 20) ctile[q] = (_Float16)0.f;
  }
  // The next unit's input tile in registers.  Every lane issues every load
  // (items outside the image or past the tile read a clamped in-range
  // address and are zeroed when stored to LDS), so the wait for them at the
  // top of the next unit counts exactly the loads and leaves the previous
  // unit's stores in flight.
  Item nxt[PER];
  uint32_t nmask = 0;  // bit i: item i is inside the image
  auto fetch = [&](int u) {
    u = u < nunits ? u : nunits - 1;
    const long b = u >> 4;
    const int ty0 = ((u & 15) >> 2) * 16, tx0 = (u & 3) * 16;
    nmask = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int q = min(tid + 256 * i, ITEMS - 1);
      int y, x, ch = 0;
      if constexpr (FIRST) {
        y = ty0 + q / 20 - 2;
        x = tx0 + q % 20 - 2;
      } else {
        const int pix = q / (NCH / 8);
        ch = q % (NCH / 8);
        y = ty0 + pix / 18 - 1;
        x = tx0 + pix % 18 - 1;
      }
      const bool inside = y >= 0 && y < CROP && x >= 0 && x < CROP;
      nmask |= (uint32_t)inside << i;
      const long at = (b * CROP + min(max(y, 0), CROP - 1)) * CROP + min(max(x, 0), CROP - 1);
      if constexpr (FIRST)
        nxt[i] = in[at];
      else
        nxt[i] = *reinterpret_cast<const h8v*>(in + at * NCH + 8 * ch);
    }
  };
  // the fetched tile into LDS (ctile or tile), zero outside the image
  auto fill = [&]() {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int q = tid + 256 * i;
      const bool valid = ITEMS % 256 == 0 || q < ITEMS;
      const bool inside = (nmask >> i) & 1;
      if constexpr (FIRST) {
        ctile[valid ? (q / 20) * CT + q % 20 : CN + tid] = inside ? nxt[i] : (_Float16)0.f;
      } else {
        h8v v = nxt[i];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = inside ? v[e] : (_Float16)0.f;
        *reinterpret_cast<h8v*>(tile + (valid ? (q / (NCH / 8)) * PS + 8 * (q % (NCH / 8)) : TN + 8 * tid)) = v;
      }
    }
  };
  int u = blockIdx.x;
  if (u < nunits) {
    fetch(u);
    if constexpr (FIRST) fill();
  }
  for (; u < nunits; u += gridDim.x) {
    const long b = u >> 4;
    const int t16 = u & 15, ty0 = (t16 >> 2) * 16, tx0 = (t16 & 3) * 16;
    __syncthreads();  // the previous unit's reads of tile and red are done; ctile is filled
    if constexpr (!FIRST) {
      fill();
      __syncthreads();
      fetch(u + gridDim.x);
      __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the MFMAs
    }
    if constexpr (FIRST) {
      // tile row mt = wave + 4 i (< 18): pixel (mt, c), k = tap for k < 9
      // (lanes h = 1 hold k = 8 .. 15: tap 8, then zeros)
      const unsigned xin = tx0 + c - 1;
#pragma unroll 1
      for (int i = 0; i < 5; ++i) {
        const int mt = wave + 4 * i;
        if (mt < 18) {
          const _Float16* cp = ctile + mt * CT + c;
          h8v a;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const _Float16 v = cp[h ? 2 * CT + 2 : (e / 3) * CT + e % 3];
            a[e] = h && e > 0 ? (_Float16)0.f : v;
          }
          f32x16 acc0;
#pragma unroll
          for (int r = 0; r < 16; ++r) acc0[r] = 0.f;
          acc0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(bw0, a, acc0, 0, 0, 0);
          if (c < 18) {
            const bool inside = (unsigned)(ty0 + mt - 1) < (unsigned)CROP && xin < (unsigned)CROP;
            _Float16* dst = tile + (mt * 18 + c) * PS + 4 * h;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              h4v v;
#pragma unroll
              for (int j = 0; j < 4; ++j)
                v[j] = inside ? (_Float16)fmaxf(acc0[4 * q + j] + bias0[4 * q + j], 0.f) : (_Float16)0.f;
              *reinterpret_cast<h4v*>(dst + 8 * q) = v;
            }
          }
        }
      }
      __syncthreads();
      fetch(u + gridDim.x);  // the next crop tile loads under the second layer's MFMAs
      __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the MFMAs
    }
    // the two 32-pixel tiles' products interleaved, each k-step's A
    // fragments read from LDS one step ahead of their MFMAs
    f32x16 acc[2];
    const _Float16* ap[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[mt][r] = 0.f;
      const int p = (2 * wave + mt) * 32 + c;
      ap[mt] = tile + ((p >> 4) * 18 + (p & 15)) * PS + 8 * h;
    }
    auto afrag = [&](int mt, int s) {
      const int tap = s >> 1;
      return *reinterpret_cast<const h8v*>(ap[mt] + ((tap / 3) * 18 + tap % 3) * PS + 16 * (s & 1));
    };
    h8v a_cur[2] = {afrag(0, 0), afrag(1, 0)};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      h8v a_nxt[2];
      if (s + 1 < KS) {
        a_nxt[0] = afrag(0, s + 1);
        a_nxt[1] = afrag(1, s + 1);
      }
      __builtin_amdgcn_sched_barrier(0);  // the reads stay one k-step ahead
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        if constexpr (LAST)
          acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a_cur[mt], bw[s], acc[mt], 0, 0, 0);
        else
          acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_f16(bw[s], a_cur[mt], acc[mt], 0, 0, 0);
      }
      if (s + 1 < KS) {
        a_cur[0] = a_nxt[0];
        a_cur[1] = a_nxt[1];
      }
    }
    // FIRST: ctile is not read again before the next unit's first barrier,
    // so the next crop tile goes there now, ahead of this unit's stores
    if constexpr (FIRST) fill();
    if constexpr (!LAST) {
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        const int p = (2 * wave + mt) * 32 + c;
        _Float16* dst = out + ((b * CROP + ty0 + (p >> 4)) * CROP + tx0 + (p & 15)) * NCH + 4 * h;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          h4v v;
#pragma unroll
          for (int j = 0; j < 4; ++j) v[j] = (_Float16)fmaxf(acc[mt][4 * q + j] + bias[4 * q + j], 0.f);
          *reinterpret_cast<h4v*>(dst + 8 * q) = v;
        }
      }
    } else {
      float sum = 0.f;
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int r = 0; r < 16; ++r) sum += fmaxf(acc[mt][r] + bias[0], 0.f);
      sum += __shfl_xor(sum, 32);
      if (h == 0) red[wave][c] = sum;
      __syncthreads();
      if (tid < 32) pooled[(b * 16 + t16) * NCH + tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
    }
  }
}

// Head for the inference pass, one wave per sample (four per workgroup):
// lane c < 32 sums channel c's 16 tile sums in tile order and divides by
// HW, lane j forms hidden unit j of FC(32->64) + ReLU, and lanes 0 and 1
// form the two outputs of FC(64->2) over j in order -- each value with the
// operations, in the order, of a single-thread evaluation.
__global__ __launch_bounds__(256) void k_head_pooled(const float* __restrict__ pooled,
                                                     const float* __restrict__ params, int bsz,
                                                     float* __restrict__ out) {
  __shared__ float g[4][NCH];
  __shared__ float hid[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const long b = (long)blockIdx.x * 4 + w;
  const bool live = b < bsz;
  if (live && lane < NCH) {
    float s = 0.f;
    for (int t = 0; t < 16; ++t) s += pooled[(b * 16 + t) * NCH + lane];
    g[w][lane] = s / HW;
  }
  __syncthreads();
  if (live) {
    float hj = params[OFF_FC1B + lane];
#pragma unroll
    for (int c = 0; c < NCH; ++c) hj += params[OFF_FC1W + lane * NCH + c] * g[w][c];
    hid[w][lane] = fmaxf(hj, 0.f);
  }
  __syncthreads();
  if (live && lane < 2) {
    float o = params[OFF_FC2B + lane];
    for (int j = 0; j < 64; ++j) o += params[OFF_FC2W + 64 * lane + j] * hid[w][j];
    out[2 * b + lane] = o;
  }
}

// A 32-channel convolution of training as an implicit GEMM on the matrix
// cores (FP32 operands, v_mfma_f32_32x32x2f32): per 16 x 16 output tile,
// [256 pixels] x [288 = 9 c + tap] times [288] x [32 output channels], with
// NCHW FP32 activations, in two modes:
//   MODE 0 (forward):    out = ReLU(b + W * in)
//   MODE 1 (input grad): out = W^T(flipped) * in, with in = dZ (the output
//                        gradient already masked by the ReLU)
// MODE 1 with relu_of (the activation A of the layer below): the stored
// gradient is already taken through that layer's ReLU, out [A > 0].
// Persistent: the layer's weights sit in LDS as B[k][o] for all of the
// block's units; wave w owns the 32-pixel M tiles 2w and 2w + 1; the
// outputs are staged in LDS so that each channel's 16-pixel rows are stored
// contiguously.
template <int MODE>
__global__ __launch_bounds__(256, 2) void k_conv_f32mfma(const float* __restrict__ in, const float* __restrict__ params,
                                                         int woff, int boff, float* __restrict__ out, int nunits,
                                                         const float* __restrict__ relu_of) {
  constexpr int K = NCH * 9, KH = K / 2;  // lanes 0-31 take k < 144, lanes 32-63 k >= 144
  constexpr int XC = 18 * 19;              // floats per channel of the input tile
  constexpr int OS = 257;                  // staging row stride
  static_assert(NCH * OS <= NCH * XC, "output staging fits in the input tile");
  static_assert(KH % 9 == 0, "each half of k holds whole channels");
  __shared__ float xt[NCH][18][19];
  __shared__ float wl[K * NCH];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, n = lane & 31, kb = lane >> 5;
  for (int q = tid; q < K * NCH; q += 256) {
    const int k = q / NCH, o = q % NCH, c = k / 9, tap = k % 9;
    wl[q] = MODE == 0 ? params[woff + (o * NCH + c) * 9 + tap] : params[woff + (c * NCH + o) * 9 + (8 - tap)];
  }
  const float bias = MODE == 0 ? params[boff + n] : 0.f;
  float* ot = &xt[0][0][0];
  // per-lane bases: step ks reads k = ks + KH kb, i.e. channel ks / 9 + 16 kb
  // and tap ks % 9, at offsets that are constants of ks
  const float* xa[2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    const int p = (2 * w + mt) * 32 + n;
    xa[mt] = &xt[0][0][0] + kb * (KH / 9) * XC + (p >> 4) * 19 + (p & 15);
  }
  const float* wb = wl + kb * KH * NCH + n;
  // the unit's input tile: every lane issues every load (clamped address,
  // zeroed when stored to LDS)
  constexpr int PER = (NCH * 324 + 255) / 256;
  float v[PER];
  uint64_t vmask = 0;
  auto fetch = [&](int u) {
    u = u < nunits ? u : nunits - 1;
    const float* bp = in + (long)(u >> 4) * (NCH * HW);  // wave-uniform base, 32-bit lane offsets
    const int ty0 = ((u & 15) >> 2) * 16, tx0 = (u & 3) * 16;
    vmask = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int q = min(tid + 256 * i, NCH * 324 - 1);
      const int c = q / 324, r = (q % 324) / 18, col = q % 18;
      const int y = ty0 + r - 1, x = tx0 + col - 1;
      vmask |= (uint64_t)(y >= 0 && y < CROP && x >= 0 && x < CROP) << i;
      v[i] = bp[(c * CROP + min(max(y, 0), CROP - 1)) * CROP + min(max(x, 0), CROP - 1)];
    }
  };
  for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
    const long b = u >> 4;
    const int ty0 = ((u & 15) >> 2) * 16, tx0 = (u & 3) * 16;
    fetch(u);  // every load of the tile is issued before the first LDS write
    __syncthreads();  // the previous unit's staged outputs are stored
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int q = tid + 256 * i;
      if (q < NCH * 324) xt[q / 324][(q % 324) / 18][q % 18] = (vmask >> i) & 1 ? v[i] : 0.f;
    }
    __syncthreads();
    // the two 32-pixel products interleaved, operands read one step ahead
    f32x16 acc[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[mt][r] = 0.f;
    auto xoff = [](int ks) { return (ks / 9) * XC + ((ks % 9) / 3) * 19 + (ks % 9) % 3; };
    float a0 = xa[0][xoff(0)], a1 = xa[1][xoff(0)], bv = wb[0];
#pragma unroll
    for (int ks = 0; ks < KH; ++ks) {
      float a0n = 0.f, a1n = 0.f, bn = 0.f;
      if (ks + 1 < KH) {
        a0n = xa[0][xoff(ks + 1)];
        a1n = xa[1][xoff(ks + 1)];
        bn = wb[(ks + 1) * NCH];
      }
      __builtin_amdgcn_sched_barrier(0);
      acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, bv, acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, bv, acc[1], 0, 0, 0);
      a0 = a0n;
      a1 = a1n;
      bv = bn;
    }
    __syncthreads();  // every read of the input tile is done
    // result register r of lane l: pixel 8 (r / 4) + 4 (l / 32) + r % 4 of the M tile, output channel l % 32
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int p = (2 * w + mt) * 32 + 8 * (r >> 2) + 4 * kb + (r & 3);
        float o = acc[mt][r] + bias;
        if (MODE == 0) o = fmaxf(o, 0.f);
        ot[n * OS + p] = o;
      }
    __syncthreads();
    // thread tid stores pixel tid of every channel, eight channels at a time
    // (with relu_of, the eight activations are loaded together first)
    float* op = out + (b * NCH * CROP + ty0 + (tid >> 4)) * CROP + tx0 + (tid & 15);
#pragma unroll
    for (int o0 = 0; o0 < NCH; o0 += 8) {
      float keep[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) keep[e] = 1.f;
      if (MODE == 1 && relu_of) {
        const float* ap = relu_of + (op - out);
#pragma unroll
        for (int e = 0; e < 8; ++e) keep[e] = ap[(o0 + e) * HW];
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float o_v = ot[(o0 + e) * OS + tid];
        op[(o0 + e) * HW] = keep[e] > 0.f ? o_v : 0.f;
      }
    }
  }
}

// Weight and bias gradients of a conv layer as a GEMM on the matrix cores:
// dW[o][k] = sum_n dZ[n][o] X[n][k] over n = (sample, pixel), k = 9 c + tap,
// X[n][k] the input at pixel n moved by the tap (zero outside the image),
// dZ = dA [A > 0] (masked beforehand).  Workgroup g accumulates the units
// (sample, 16 x 16 tile) g, g + G, ... in registers and writes its partial
// sums; k_wgrad_reduce adds the G partials in workgroup order, so the
// result does not depend on scheduling.
//
// k_wgrad1, the first layer (nine taps of the fp16 crop), on
// v_mfma_f32_32x32x2f32: the nine k columns padded to 32, the 128 pixel
// pairs of a tile split over four waves whose partials are added in wave
// order; threads 0..31 sum the bias gradient of their output channel over
// the workgroup's pixels in order.  Each step's operands are read from LDS
// one step ahead of its MFMA.
__global__ __launch_bounds__(256) void k_wgrad1(const _Float16* __restrict__ x, const float* __restrict__ dz,
                                                int nunits, float* __restrict__ part_w,
                                                float* __restrict__ part_b) {
  constexpr int NK = 9, KS = 32;  // k columns; pixel pairs per wave and unit
  constexpr int DS = 257;          // dz row stride: the 32 rows of an A read fall on distinct banks
  __shared__ float xt[18][19];
  __shared__ float dzt[NCH * DS];  // dZ of the unit, [o][pixel]
  __shared__ float red[3 * 16 * 64];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, n = lane & 31, kb = lane >> 5;
  const bool kval = n < NK;
  const int tap = kval ? n : 0;
  const float* xb = &xt[tap / 3][tap % 3];
  const int ks0 = KS * w;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  float accb = 0.f;
  for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
    const long b = u >> 4;
    const int ty0 = ((u & 15) >> 2) * 16, tx0 = (u & 3) * 16;
    // the loads of each array are all issued before its first LDS write
    constexpr int PX = (324 + 255) / 256, PZ = NCH;
    {
      float vx[PX];
#pragma unroll
      for (int i = 0; i < PX; ++i) {
        const int q = tid + 256 * i, y = ty0 + q / 18 - 1, xx = tx0 + q % 18 - 1;
        vx[i] = (q < 324 && y >= 0 && y < CROP && xx >= 0 && xx < CROP) ? (float)x[(b * CROP + y) * CROP + xx] : 0.f;
      }
      __syncthreads();  // the previous unit's reads are done
#pragma unroll
      for (int i = 0; i < PX; ++i) {
        const int q = tid + 256 * i;
        if (q < 324) xt[q / 18][q % 18] = vx[i];
      }
    }
    {
      const float* pz = dz + ((b * NCH) * CROP + ty0 + (tid >> 4)) * CROP + tx0 + (tid & 15);
      float vz[PZ];
#pragma unroll
      for (int o = 0; o < PZ; ++o) vz[o] = pz[o * HW];
#pragma unroll
      for (int o = 0; o < PZ; ++o) dzt[o * DS + tid] = vz[o];
    }
    __syncthreads();
    if (tid < NCH)
      for (int pp = 0; pp < 256; ++pp) accb += dzt[tid * DS + pp];
    // step ks takes the pixel pair 2 ks, 2 ks + 1: lane half kb reads pixel
    // 2 ks + kb, at offsets that are constants of ks from per-lane bases
    const float* ap = dzt + n * DS + kb;
    const float* bp = xb + kb;
    auto boff = [](int ks) { return ((2 * ks) >> 4) * 19 + ((2 * ks) & 15); };
    float a = ap[2 * ks0], bv = kval ? bp[boff(ks0)] : 0.f;
#pragma unroll
    for (int j = 0; j < KS; ++j) {
      const int ks = ks0 + j;
      float an = 0.f, bn = 0.f;
      if (j + 1 < KS) {
        an = ap[2 * (ks + 1)];
        bn = kval ? bp[boff(ks + 1)] : 0.f;
      }
      __builtin_amdgcn_sched_barrier(0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bv, acc, 0, 0, 0);
      a = an;
      bv = bn;
    }
  }
  // result register r of lane l: output channel 8 (r / 4) + 4 (l / 32) + r % 4, k column n
  if (w > 0)
#pragma unroll
    for (int r = 0; r < 16; ++r) red[((w - 1) * 16 + r) * 64 + lane] = acc[r];
  __syncthreads();
  if (w == 0 && kval)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float v = ((acc[r] + red[r * 64 + lane]) + red[(16 + r) * 64 + lane]) + red[(32 + r) * 64 + lane];
      const int o = 8 * (r >> 2) + 4 * kb + (r & 3);
      part_w[((long)blockIdx.x * NCH + o) * NK + n] = v;
    }
  if (tid < NCH) part_b[blockIdx.x * NCH + tid] = accb;
}

// k_wgrad32, a 32-channel layer, in 16 x 16 tiles
// (v_mfma_f32_16x16x4f32): [32 outputs] x
// [288 k columns] is 2 x 18 tiles, nine per wave, so the four waves of a
// workgroup (one per SIMD) carry equal work and two workgroups share a CU.
// Step s takes pixels 4 s .. 4 s + 3 of the unit; every operand read is a
// constant offset from a per-lane base, and the operands of step s + 1 are
// read before the MFMAs of step s.  The bias gradient as eight fixed
// partial sums per channel (pixels t / 32, t / 32 + 8, ... of channel
// t % 32 for thread t), added in order.
typedef float f32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256, 2) void k_wgrad32(const float* __restrict__ x, const float* __restrict__ dz,
                                                    int nunits, float* __restrict__ part_w,
                                                    float* __restrict__ part_b) {
  constexpr int NK = NCH * 9, DS = 257, XC = 18 * 19, NTW = 9, NS = 64;
  __shared__ float xt[NCH * XC];
  __shared__ float dzt[NCH * DS];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, i16 = lane & 15, kk = lane >> 4;
  const int mt = w & 1, nt0 = NTW * (w >> 1);
  // A (16 x 4): lane l holds dZ[pixel 4 s + l / 16][output 16 mt + l % 16];
  // B (4 x 16): lane l holds X[pixel 4 s + l / 16][k column 16 nt + l % 16]
  const float* ap = dzt + (16 * mt + i16) * DS + kk;
  int xb[NTW];
#pragma unroll
  for (int j = 0; j < NTW; ++j) {
    const int kcol = 16 * (nt0 + j) + i16, c = kcol / 9, tap = kcol % 9;
    xb[j] = c * XC + (tap / 3) * 19 + tap % 3 + kk;
  }
  f32x4 acc[NTW];
#pragma unroll
  for (int j = 0; j < NTW; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[j][r] = 0.f;
  float accb = 0.f;
  for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
    const int ty0 = ((u & 15) >> 2) * 16, tx0 = (u & 3) * 16;
    const float* xp = x + (long)(u >> 4) * (NCH * HW);
    const float* zp = dz + (long)(u >> 4) * (NCH * HW);
    // The input tile (pixel tid of every channel; then the 68 x 32 items of
    // pixels 256 .. 323) and dZ (pixel tid of every channel), each batch of
    // loads issued (clamped address, zeroed when stored) before its LDS
    // writes; offsets are a per-lane value plus a constant per channel.
    __syncthreads();  // the previous unit's reads are done
    {
      const int r0 = tid / 18, c0 = tid % 18, y = ty0 + r0 - 1, xx = tx0 + c0 - 1;
      const bool in0 = y >= 0 && y < CROP && xx >= 0 && xx < CROP;
      const float* p0 = xp + min(max(y, 0), CROP - 1) * CROP + min(max(xx, 0), CROP - 1);
      float v[NCH];
#pragma unroll
      for (int c = 0; c < NCH; ++c) v[c] = p0[c * HW];
#pragma unroll
      for (int c = 0; c < NCH; ++c) xt[c * XC + r0 * 19 + c0] = in0 ? v[c] : 0.f;
    }
    {
      constexpr int N1 = NCH * 68, P1 = (N1 + 255) / 256;
      float v[P1];
      uint32_t m = 0;
#pragma unroll
      for (int k = 0; k < P1; ++k) {
        const int j = min(tid + 256 * k, N1 - 1), c = j / 68, pp = 256 + j % 68;
        const int y = ty0 + pp / 18 - 1, xx = tx0 + pp % 18 - 1;
        m |= (uint32_t)(y >= 0 && y < CROP && xx >= 0 && xx < CROP) << k;
        v[k] = xp[(c * CROP + min(max(y, 0), CROP - 1)) * CROP + min(max(xx, 0), CROP - 1)];
      }
#pragma unroll
      for (int k = 0; k < P1; ++k) {
        const int j = tid + 256 * k, c = j / 68, pp = 256 + j % 68;
        if (j < N1) xt[c * XC + (pp / 18) * 19 + pp % 18] = (m >> k) & 1 ? v[k] : 0.f;
      }
    }
    {
      const float* pz = zp + (ty0 + (tid >> 4)) * CROP + tx0 + (tid & 15);
      float v[NCH];
#pragma unroll
      for (int o = 0; o < NCH; ++o) v[o] = pz[o * HW];
#pragma unroll
      for (int o = 0; o < NCH; ++o) dzt[o * DS + tid] = v[o];
    }
    __syncthreads();
    // bias: thread t sums pixels t / 32, t / 32 + 8, ... of channel t % 32
    for (int pp = tid / NCH; pp < 256; pp += 256 / NCH) accb += dzt[(tid % NCH) * DS + pp];
    auto boff = [](int st) { return ((4 * st) >> 4) * 19 + ((4 * st) & 15); };
    float a = ap[0], bv[NTW];
#pragma unroll
    for (int j = 0; j < NTW; ++j) bv[j] = xt[xb[j] + boff(0)];
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      float an = 0.f, bn[NTW];
#pragma unroll
      for (int j = 0; j < NTW; ++j) bn[j] = 0.f;
      if (st + 1 < NS) {
        an = ap[4 * (st + 1)];
#pragma unroll
        for (int j = 0; j < NTW; ++j) bn[j] = xt[xb[j] + boff(st + 1)];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < NTW; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv[j], acc[j], 0, 0, 0);
      a = an;
#pragma unroll
      for (int j = 0; j < NTW; ++j) bv[j] = bn[j];
    }
  }
  // D of lane l: row 4 (l / 16) + r = output channel 16 mt + 4 kk + r, column l % 16 = k column 16 nt + i16
#pragma unroll
  for (int j = 0; j < NTW; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      part_w[((long)blockIdx.x * NCH + 16 * mt + 4 * kk + r) * NK + 16 * (nt0 + j) + i16] = acc[j][r];
  __syncthreads();
  dzt[tid] = accb;  // the 256 partial bias sums, [part][channel]
  __syncthreads();
  if (tid < NCH) {
    float sb = 0.f;
    for (int q = 0; q < 256 / NCH; ++q) sb += dzt[q * NCH + tid];
    part_b[blockIdx.x * NCH + tid] = sb;
  }
}

// Sum of the per-workgroup partials into the gradient vector, in a fixed
// order (eight interleaved running sums over the workgroups, s_j over
// workgroups j, j + 8, ..., then ((s0 + s1) + (s2 + s3)) + ((s4 + s5) +
// (s6 + s7))), so the result does not depend on scheduling.  A workgroup
// of 256 threads takes 32 outputs; thread t runs sum t / 32 of output t % 32.
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* __restrict__ part_w,
                                                      const float* __restrict__ part_b, int splits, int cin,
                                                      int woff, int boff, float* __restrict__ grad) {
  __shared__ float red[8][32];
  const int t = threadIdx.x, j = t >> 5, i = blockIdx.x * 32 + (t & 31);
  const int nw = NCH * cin * 9;
  const bool live = i < nw + NCH;
  const float* src = i < nw ? part_w + i : part_b + (i - nw);
  const long stride = i < nw ? nw : NCH;
  float sj = 0.f;
  if (live)
    for (int k0 = j; k0 < splits; k0 += 64) {
      float v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = k0 + 8 * e < splits ? src[(long)(k0 + 8 * e) * stride] : 0.f;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (k0 + 8 * e < splits) sj += v[e];
    }
  red[j][t & 31] = sj;
  __syncthreads();
  if (j == 0 && live) {
    const int c = t & 31;
    const float r = ((red[0][c] + red[1][c]) + (red[2][c] + red[3][c])) + ((red[4][c] + red[5][c]) + (red[6][c] + red[7][c]));
    if (i < nw)
      grad[woff + i] = r;
    else
      grad[boff + i - nw] = r;
  }
}

// ------------------------------------------------------------------ CNN: head
// Global average pooling, FC(32->64) ReLU, FC(64->2), and for training the
// Gaussian NLL, the head gradients (per sample) and dg4[b][c] = dL/dg_c / HW,
// the gradient of every pixel of channel c of the last activation.
template <bool TRAIN>
__global__ __launch_bounds__(256) void k_head(const float* __restrict__ a4, const float* __restrict__ params,
                                              const float* __restrict__ zn, int bsize, float* __restrict__ out,
                                              float* __restrict__ loss_b, float* __restrict__ hpart,
                                              float* __restrict__ dg4) {
  __shared__ float red[256][NCH + 1];
  __shared__ float g[NCH], h1[64], dh1[64], outs[2], dout[2];
  const int tid = threadIdx.x;
  const long b = blockIdx.x;
  float acc[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) acc[c] = 0.f;
  for (int p = tid; p < HW; p += 256)
#pragma unroll
    for (int c = 0; c < NCH; ++c) acc[c] += a4[(b * NCH + c) * HW + p];
#pragma unroll
  for (int c = 0; c < NCH; ++c) red[tid][c] = acc[c];
  __syncthreads();
  if (tid < NCH) {
    // in thread order, sixteen reads issued ahead of their additions
    float s = 0.f;
    for (int t0 = 0; t0 < 256; t0 += 16) {
      float v[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = red[t0 + j][tid];
#pragma unroll
      for (int j = 0; j < 16; ++j) s += v[j];
    }
    g[tid] = s / HW;
  }
  __syncthreads();
  if (tid < 64) {
    float h = params[OFF_FC1B + tid];
    for (int c = 0; c < NCH; ++c) h += params[OFF_FC1W + tid * NCH + c] * g[c];
    h1[tid] = fmaxf(h, 0.f);
  }
  __syncthreads();
  if (tid < 2) {
    float o = params[OFF_FC2B + tid];
    for (int k = 0; k < 64; ++k) o += params[OFF_FC2W + tid * 64 + k] * h1[k];
    outs[tid] = o;
    out[b * 2 + tid] = o;
  }
  __syncthreads();
  if (!TRAIN) return;
  if (tid == 0) {
    const float zh = outs[0], s = outs[1];
    const float r = zn[b] - zh, e = expf(-s);
    loss_b[b] = 0.5f * (s + r * r * e);
    dout[0] = -r * e / bsize;
    dout[1] = 0.5f * (1.f - r * r * e) / bsize;
  }
  __syncthreads();
  float* hp = hpart + b * HEAD_N;
  if (tid < 128) hp[2048 + 64 + tid] = dout[tid / 64] * h1[tid % 64];
  if (tid < 2) hp[2048 + 64 + 128 + tid] = dout[tid];
  if (tid < 64) {
    const float d = (dout[0] * params[OFF_FC2W + tid] + dout[1] * params[OFF_FC2W + 64 + tid]) *
                    (h1[tid] > 0.f ? 1.f : 0.f);
    dh1[tid] = d;
    hp[2048 + tid] = d;
  }
  __syncthreads();
  for (int q = tid; q < 2048; q += 256) hp[q] = dh1[q / NCH] * g[q % NCH];
  if (tid < NCH) {
    float d = 0.f;
    for (int o = 0; o < 64; ++o) d += dh1[o] * params[OFF_FC1W + o * NCH + tid];
    dg4[b * NCH + tid] = d / HW;
  }
}

// dZ of the last layer: dA = dg4[b][c] at every pixel of channel c, taken
// through the layer's ReLU: dz = [A > 0] dg4.
__global__ void k_dz_last(const float4* __restrict__ a, const float* __restrict__ dg4, float4* __restrict__ dz,
                          long n4) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n4; i += (long)gridDim.x * blockDim.x) {
    const float d = dg4[(i * 4) / HW];  // four consecutive pixels of one channel
    const float4 m = a[i];
    dz[i] = make_float4(m.x > 0.f ? d : 0.f, m.y > 0.f ? d : 0.f, m.z > 0.f ? d : 0.f, m.w > 0.f ? d : 0.f);
  }
}

__global__ void k_head_reduce(const float* __restrict__ hpart, const float* __restrict__ loss_b, int bsize,
                              float* __restrict__ grad, float* __restrict__ loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < HEAD_N) {
    // in sample order, sixteen loads issued ahead of their additions
    float s = 0.f;
    for (int b0 = 0; b0 < bsize; b0 += 16) {
      float v[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = b0 + j < bsize ? hpart[(long)(b0 + j) * HEAD_N + i] : 0.f;
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (b0 + j < bsize) s += v[j];
    }
    grad[OFF_FC1W + i] = s;  // fc1 w, fc1 b, fc2 w, fc2 b are contiguous
  } else if (i == HEAD_N && loss) {
    float s = 0.f;
    for (int b = 0; b < bsize; ++b) s += loss_b[b];
    *loss = s / bsize;
  }
}

__global__ void k_normalize(const float* __restrict__ z, int n, float mean, float inv_scale, float* __restrict__ zn) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) zn[i] = (z[i] - mean) * inv_scale;
}

// Adam; om1 = 1 - beta1 and om2 = 1 - beta2 come in already rounded from
// float64 (1 - 0.999f in float32 would be off by 1.3e-5 relative).
__global__ void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int n, float lr, float b1, float b2, float om1, float om2,
                       float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + om1 * gi;
  const float vi = b2 * v[i] + om2 * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Prediction in metres: z = mean + scale * z_n, sigma = scale * exp(s / 2).
__global__ void k_af_denorm(const float* __restrict__ out, int n, float mean, float scale, float* __restrict__ z,
                            float* __restrict__ sigma) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  z[i] = mean + scale * out[2 * i];
  if (sigma) sigma[i] = scale * expf(0.5f * out[2 * i + 1]);
}

__global__ void k_af_scatter(const float* __restrict__ zs, const int* __restrict__ idx, int m, float* __restrict__ z,
                             int* __restrict__ used) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  z[idx[i]] = zs[i];
  if (used) used[idx[i]] = 1;
}

__global__ void k_af_gather(const uint8_t* __restrict__ holo, const int* __restrict__ idx, int m,
                            uint8_t* __restrict__ dst) {
  const long n = (long)m * AN * AN / 16;
  for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
    const long e = q * 16;
    const long i = e / (AN * AN), off = e % (AN * AN);
    *reinterpret_cast<uint4*>(dst + e) = *reinterpret_cast<const uint4*>(holo + (long)idx[i] * AN * AN + off);
  }
}

// ------------------------------------------------------------------ training-data synthesis
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11): 10 rounds of two 32x32->64 multiplies with the
// Weyl key schedule.
__device__ inline uint4 philox(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t h0 = (uint32_t)(p0 >> 32), l0 = (uint32_t)p0, h1 = (uint32_t)(p1 >> 32), l1 = (uint32_t)p1;
    c = make_uint4(h1 ^ c.y ^ k.x, l1, h0 ^ c.w ^ k.y, l0);
    k.x += 0x9E3779B9u;
    k.y += 0xBB67AE85u;
  }
  return c;
}

// Two standard normals from two 32-bit integers (Box-Muller).
__device__ inline float2 box_muller(uint32_t a, uint32_t b) {
  const float u1 = ((float)a + 0.5f) * 2.3283064365386963e-10f;
  const float u2 = ((float)b + 0.5f) * 2.3283064365386963e-10f;
  const float r = sqrtf(-2.f * logf(u1));
  float s, c;
  sincospif(2.f * u2, &s, &c);
  return make_float2(r * c, r * s);
}

__global__ void k_af_noise(float2* __restrict__ out, int n, uint64_t seed, long base) {
  const long total = (long)n * AN * AN;
  const uint2 key = make_uint2((uint32_t)seed, (uint32_t)(seed >> 32));
  for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < total; q += (long)gridDim.x * blockDim.x) {
    const long h = base + q / (AN * AN);
    const uint4 r = philox(make_uint4((uint32_t)(q % (AN * AN)), (uint32_t)h, (uint32_t)(h >> 32), 0u), key);
    out[q] = box_muller(r.x, r.y);
  }
}

// Multiply by the union of soft disks: mask = max_d 1 / (1 + exp((|r - c_d| - r_d) / 1.5)).
__global__ void k_af_mask(float2* __restrict__ field, const float* __restrict__ disks, int n) {
  const long total = (long)n * AN * AN;
  for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < total; q += (long)gridDim.x * blockDim.x) {
    const long h = q / (AN * AN);
    const int p = (int)(q % (AN * AN));
    const float y = (float)(p / AN), x = (float)(p % AN);
    const float* d = disks + h * 25;
    const int nd = (int)d[0];
    float m = 0.f;
    for (int i = 0; i < nd; ++i) {
      const float dy = y - d[1 + 3 * i], dx = x - d[2 + 3 * i];
      const float dist = sqrtf(dy * dy + dx * dx);
      m = fmaxf(m, 1.f / (1.f + expf((dist - d[3 + 3 * i]) / 1.5f)));
    }
    field[q] = make_float2(field[q].x * m, field[q].y * m);
  }
}

// Off-axis hologram of one propagated object wave: reference amplitude
// 3 x rms, tilt of 1/4 cycle per pixel on both axes, mean 64 DN, photon
// noise with the normal approximation N(lambda, lambda), clipped to 8 bits.
__global__ __launch_bounds__(256) void k_af_holo(const float2* __restrict__ w, uint8_t* __restrict__ out,
                                                 uint64_t seed, long base) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const long h = blockIdx.x;
  const float2* src = w + h * AN * AN;
  double e = 0.0;
  for (int p = tid; p < AN * AN; p += 256) e += (double)src[p].x * src[p].x + (double)src[p].y * src[p].y;
  e = block_sum<256>(e, red);
  const float ra = 3.f * (float)sqrt(e / (AN * AN));
  double it = 0.0;
  for (int p = tid; p < AN * AN; p += 256) {
    float s, c;
    sincospif(0.5f * (float)((p / AN + p % AN) & 3), &s, &c);
    const float re = ra * c + src[p].x, im = ra * s + src[p].y;
    it += (double)re * re + (double)im * im;
  }
  it = block_sum<256>(it, red);
  const float scale = (float)(64.0 * (AN * AN) / it);
  const uint2 key = make_uint2((uint32_t)(seed ^ 0x5bd1e995u), (uint32_t)(seed >> 32));
  for (int p = tid; p < AN * AN; p += 256) {
    float s, c;
    sincospif(0.5f * (float)((p / AN + p % AN) & 3), &s, &c);
    const float re = ra * c + src[p].x, im = ra * s + src[p].y;
    const float lam = (re * re + im * im) * scale;
    const long hh = base + h;
    const uint4 r = philox(make_uint4((uint32_t)p, (uint32_t)hh, (uint32_t)(hh >> 32), 1u), key);
    const float nrm = box_muller(r.x, r.y).x;
    const float v = rintf(lam + sqrtf(lam) * nrm);
    out[h * AN * AN + p] = (uint8_t)fminf(fmaxf(v, 0.f), 255.f);
  }
}

hv_status launched(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HV_ERR_DEVICE, "%s launch failed: %s", what, hipGetErrorString(e));
  return HV_OK;
}

}  // namespace

// ------------------------------------------------------------------ model object

struct hv_af_model {
  hv_ctx* ctx = nullptr;
  int max_batch = 0;
  double z_mean = 0, z_scale = 1;
  int64_t step = 0;
  float *params = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
  float* act[4] = {nullptr, nullptr, nullptr, nullptr};
  float *d1 = nullptr, *d2 = nullptr;
  float *part_w = nullptr, *part_b = nullptr, *hpart = nullptr, *loss_b = nullptr, *out = nullptr, *zn = nullptr;
  float* dg4 = nullptr;  // [max_batch][32]: the last activation's gradient per channel
  float* loss_tmp = nullptr;
  int infer_batch = 0;                       // batch of the inference kernels (>= max_batch)
  _Float16* act16[2] = {nullptr, nullptr};  // inference activations, NHWC fp16 [infer_batch]
  float* pooled = nullptr;                   // [infer_batch][16 tiles][32]
  float* iout = nullptr;                     // [infer_batch][2] inference outputs
  void* wfrag = nullptr;                     // B fragments of the inference pass
  int64_t version = 0, packed = -1;          // parameter version, and the one wfrag was packed from
  std::vector<void*> owned;
};

namespace {

constexpr int WG_BLOCKS = 512;  // workgroups (and partial sums) of the weight gradients

hv_status dev_alloc(hv_af_model* md, void** p, size_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) return fail(HV_ERR_NOMEM, "autofocus allocation of %zu bytes failed", bytes);
  md->owned.push_back(*p);
  return HV_OK;
}

// Forward through the four conv layers and the head.
hv_status forward(hv_af_model* md, const _Float16* crops, int bsz, bool train, hipStream_t st) {
  const dim3 grid(16, bsz);
  hipLaunchKernelGGL((k_conv<1, _Float16>), grid, dim3(256), 0, st, crops, md->params, OFF_W[0], OFF_B[0],
                     md->act[0]);
  const int nu = 16 * bsz;
  const int gf = hvi::persistent_grid(k_conv_f32mfma<0>, 256, nu);
  for (int l = 1; l < 4; ++l)
    hipLaunchKernelGGL(k_conv_f32mfma<0>, dim3(gf), dim3(256), 0, st, md->act[l - 1], md->params, OFF_W[l], OFF_B[l],
                       md->act[l], nu, (const float*)nullptr);
  if (train)
    hipLaunchKernelGGL(k_head<true>, dim3(bsz), dim3(256), 0, st, md->act[3], md->params, md->zn, bsz, md->out,
                       md->loss_b, md->hpart, md->dg4);
  else
    hipLaunchKernelGGL(k_head<false>, dim3(bsz), dim3(256), 0, st, md->act[3], md->params, nullptr, bsz, md->out,
                       nullptr, nullptr, nullptr);
  return launched("af forward");
}

// The inference pass on MFMA (fp16 operands), same network and outputs as
// forward(.., false, ..) up to fp16 rounding.
hv_status infer(hv_af_model* md, const _Float16* crops, int bsz, hipStream_t st) {
  const h8v* wf = (const h8v*)md->wfrag;
  if (md->packed != md->version) {  // weights repacked only after they change
    hipLaunchKernelGGL(k_pack_weights, dim3((IKS * 64 + 255) / 256), dim3(256), 0, st, md->params, (h8v*)md->wfrag);
    md->packed = md->version;
  }
  const int nu = 16 * bsz;
  // layers 1 and 2 in one pass (the first layer's output stays in LDS)
  hipLaunchKernelGGL((k_conv_mfma<false, true>),
                     dim3(hvi::persistent_grid(k_conv_mfma<false, true>, 256, nu)), dim3(256), 0, st, crops,
                     wf + 64, md->params, OFF_B[1], md->act16[1], nullptr, nu, wf, OFF_B[0]);
  hipLaunchKernelGGL((k_conv_mfma<false, false>), dim3(hvi::persistent_grid(k_conv_mfma<false, false>, 256, nu)),
                     dim3(256), 0, st, md->act16[1], wf + 64 * 19, md->params, OFF_B[2], md->act16[0], nullptr, nu,
                     nullptr, 0);
  hipLaunchKernelGGL((k_conv_mfma<true, false>), dim3(hvi::persistent_grid(k_conv_mfma<true, false>, 256, nu)),
                     dim3(256), 0, st, md->act16[0], wf + 64 * 37, md->params, OFF_B[3], nullptr, md->pooled, nu,
                     nullptr, 0);
  hipLaunchKernelGGL(k_head_pooled, dim3((bsz + 3) / 4), dim3(256), 0, st, md->pooled, md->params, bsz, md->iout);
  return launched("af inference");
}

hv_status backward(hv_af_model* md, const _Float16* crops, int bsz, float* grad, float* loss, hipStream_t st) {
  hipLaunchKernelGGL(k_head_reduce, dim3((HEAD_N + 1 + 255) / 256), dim3(256), 0, st, md->hpart, md->loss_b, bsz,
                     grad, loss);
  float* dcur = md->d1;   // dA of the current layer's output
  float* dnext = md->d2;  // receives dA of its input
  const int nu = 16 * bsz, gw = std::min(nu, WG_BLOCKS);
  const long n4 = (long)bsz * NCH * HW / 4;
  // dZ of the last layer from the head's per-channel gradient; below it,
  // the input-gradient kernel applies the ReLU of the layer it feeds
  hipLaunchKernelGGL(k_dz_last, dim3((unsigned)std::min<long>(4096, (n4 + 255) / 256)), dim3(256), 0, st,
                     (const float4*)md->act[3], (const float*)md->dg4, (float4*)dcur, n4);
  for (int l = 3; l >= 0; --l) {
    if (l > 0) {
      hipLaunchKernelGGL(k_wgrad32, dim3(gw), dim3(256), 0, st, (const float*)md->act[l - 1], (const float*)dcur, nu,
                         md->part_w, md->part_b);
      hipLaunchKernelGGL(k_wgrad_reduce, dim3((NCH * NCH * 9 + NCH + 31) / 32), dim3(256), 0, st, md->part_w,
                         md->part_b, gw, NCH, OFF_W[l], OFF_B[l], grad);
      hipLaunchKernelGGL(k_conv_f32mfma<1>, dim3(hvi::persistent_grid(k_conv_f32mfma<1>, 256, nu)), dim3(256), 0,
                         st, dcur, md->params, OFF_W[l], 0, dnext, nu, (const float*)md->act[l - 1]);
      std::swap(dcur, dnext);
    } else {
      hipLaunchKernelGGL(k_wgrad1, dim3(gw), dim3(256), 0, st, crops, (const float*)dcur, nu, md->part_w,
                         md->part_b);
      hipLaunchKernelGGL(k_wgrad_reduce, dim3((NCH * 9 + NCH + 31) / 32), dim3(256), 0, st, md->part_w,
                         md->part_b, gw, 1, OFF_W[0], OFF_B[0], grad);
    }
  }
  return launched("af backward");
}

struct ScanPlan {
  hvi::DevBuf htab;
};

}  // namespace

// ------------------------------------------------------------------ C-ABI

using namespace hvi;

// The spectrum kernel reads the holograms in 16-byte words.
static hv_status check_holo(const uint8_t* holo) {
  return (reinterpret_cast<uintptr_t>(holo) & 15) ? fail(HV_ERR_ARG, "holograms must be 16-byte aligned") : HV_OK;
}

// Crops (fp16 or float) and/or +1-order sub-bands of n holograms in one
// launch; a null output is not produced.
template <bool CR, bool SB, typename TOUT>
static void launch_spec(const uint8_t* holo, int n, void* crop, float2* sub, hipStream_t st) {
  auto k = k_af_spec<CR, SB, TOUT>;
  hipLaunchKernelGGL(k, dim3(hvi::persistent_grid(k, 256, n)), dim3(256), 0, st, holo, n, (TOUT*)crop, sub);
}
static hv_status af_spectrum(const uint8_t* holo, int n, void* crop, bool half, float2* sub, hipStream_t st) {
  if (n <= 0 || (!crop && !sub)) return HV_OK;
  if (!crop)
    launch_spec<false, true, _Float16>(holo, n, nullptr, sub, st);
  else if (half)
    sub ? launch_spec<true, true, _Float16>(holo, n, crop, sub, st) : launch_spec<true, false, _Float16>(holo, n, crop, sub, st);
  else
    sub ? launch_spec<true, true, float>(holo, n, crop, sub, st) : launch_spec<true, false, float>(holo, n, crop, sub, st);
  return launched("af spectrum");
}

extern "C" {

int hv_af_nparams(void) { return NPARAM; }

hv_status hv_af_crops(hv_ctx* ctx, const uint8_t* holo, int n, int ny, int nx, void* out, int out_half,
                      void* hip_stream) {
  if (!ctx || !holo || !out) return fail(HV_ERR_ARG, "NULL argument");
  if (ny != AN || nx != AN) return fail(HV_ERR_SHAPE, "autofocus works on 256x256 holograms");
  if (n <= 0) return n == 0 ? HV_OK : fail(HV_ERR_ARG, "negative count");
  if (hv_status e = check_holo(holo)) return e;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(HV_ERR_DEVICE, "hipSetDevice failed");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  return af_spectrum(holo, n, out, out_half != 0, nullptr, (hipStream_t)hip_stream);
}

hv_status hv_af_scan(hv_ctx* ctx, const uint8_t* holo, int n, int ny, int nx, double wavelength_m, double pitch_m,
                     double z_lo_m, double z_hi_m, int n_candidates, float* z_out, float* scores_out,
                     void* hip_stream) {
  if (!ctx || !holo || !z_out) return fail(HV_ERR_ARG, "NULL argument");
  if (ny != AN || nx != AN) return fail(HV_ERR_SHAPE, "autofocus works on 256x256 holograms");
  if (n_candidates < 2 || !(z_hi_m > z_lo_m) || !(wavelength_m > 0) || !(pitch_m > 0))
    return fail(HV_ERR_ARG, "need >= 2 candidates, z_hi > z_lo, positive wavelength and pitch");
  if (n <= 0) return n == 0 ? HV_OK : fail(HV_ERR_ARG, "negative count");
  if (hv_status e = check_holo(holo)) return e;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(HV_ERR_DEVICE, "hipSetDevice failed");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  hipStream_t st = (hipStream_t)hip_stream;
  // transfer-function table per candidate, built in float64 once per setting
  char key[160];
  snprintf(key, sizeof key, "afscan %.17g %.17g %.17g %.17g %d", wavelength_m, pitch_m, z_lo_m, z_hi_m,
           n_candidates);
  DevBuf& tab = ctx->misc[key];
  hv_status s;
  if (!tab.ptr) {
    std::vector<float2> h((size_t)n_candidates * SUB * SUB);
    const double il2 = 1.0 / (wavelength_m * wavelength_m);
    for (int c = 0; c < n_candidates; ++c) {
      const double zc = z_lo_m + (z_hi_m - z_lo_m) * c / (n_candidates - 1);
      for (int i = 0; i < SUB; ++i)
        for (int j = 0; j < SUB; ++j) {
          const double fy = (i - SUB / 2) / (AN * pitch_m), fx = (j - SUB / 2) / (AN * pitch_m);
          const double rad = il2 - fx * fx - fy * fy;
          double re = 0, im = 0;
          if (rad > 0) {
            const double ph = -2.0 * M_PI * zc * std::sqrt(rad);
            re = std::cos(ph);
            im = std::sin(ph);
          }
          h[((size_t)c * SUB + i) * SUB + j] = make_float2((float)re, (float)im);
        }
    }
    if ((s = tab.upload(h.data(), h.size() * sizeof(float2), &ctx->held))) return s;
  }
  DevBuf& sb = ctx->work(st, 21);
  DevBuf& sc = ctx->work(st, 22);
  if ((s = sb.ensure((size_t)n * SUB * SUB * 8, &ctx->held))) return s;
  if ((s = sc.ensure((size_t)n * n_candidates * 4, &ctx->held))) return s;
  if ((s = af_spectrum(holo, n, nullptr, false, (float2*)sb.ptr, st))) return s;
  constexpr int CPB = 8;
  hipLaunchKernelGGL((k_af_scan<CPB, false>), dim3(n, (n_candidates + CPB - 1) / CPB), dim3(256), 0, st,
                     (const float2*)sb.ptr, (const float2*)tab.ptr, (const double*)nullptr, (const float*)nullptr,
                     (const float*)nullptr, n_candidates, (float*)sc.ptr);
  hipLaunchKernelGGL(k_af_argmax, dim3((n + 255) / 256), dim3(256), 0, st, (const float*)sc.ptr, n, n_candidates,
                     z_lo_m, z_hi_m, (float*)nullptr, (float*)nullptr, z_out, (float*)nullptr, 0);
  if (scores_out &&
      hipMemcpyAsync(scores_out, sc.ptr, (size_t)n * n_candidates * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return fail(HV_ERR_DEVICE, "score copy failed");
  return launched("af_scan");
}

}  // extern "C"

// kz = 2 pi sqrt(1/lambda^2 - |f|^2) at the demodulated object frequencies
// of the scan sub-band (FP64, -1 where evanescent), once per setting.
static hv_status af_kz_table(hv_ctx* ctx, double wavelength_m, double pitch_m, const double** out) {
  char key[96];
  snprintf(key, sizeof key, "afkz %.17g %.17g", wavelength_m, pitch_m);
  DevBuf& tab = ctx->misc[key];
  if (!tab.ptr) {
    std::vector<double> k((size_t)SUB * SUB);
    const double il2 = 1.0 / (wavelength_m * wavelength_m);
    for (int i = 0; i < SUB; ++i)
      for (int j = 0; j < SUB; ++j) {
        const double fy = (i - SUB / 2) / (AN * pitch_m), fx = (j - SUB / 2) / (AN * pitch_m);
        const double rad = il2 - fx * fx - fy * fy;
        k[(size_t)i * SUB + j] = rad > 0 ? 2.0 * M_PI * std::sqrt(rad) : -1.0;
      }
    hv_status s = tab.upload(k.data(), k.size() * sizeof(double), &ctx->held);
    if (s) return s;
  }
  *out = (const double*)tab.ptr;
  return HV_OK;
}

// Scan of the sub-bands sub [n][SUB][SUB] over per-hologram ranges
// [zlo[i], zhi[i]] with nc candidates; z_out[i] the best candidate.  With
// `refine`, zlo / zhi are narrowed to one step around the best on return.
static hv_status af_scan_ranges(hv_ctx* ctx, const float2* sub, int n, const double* kz, float* zlo, float* zhi,
                                int nc, float* z_out, float* scores_out, bool refine, hipStream_t st) {
  DevBuf& sc = ctx->work(st, 28);
  hv_status s;
  if ((s = sc.ensure((size_t)n * nc * 4, &ctx->held))) return s;
  constexpr int CPB = 8;
  hipLaunchKernelGGL((k_af_scan<CPB, true>), dim3(n, (nc + CPB - 1) / CPB), dim3(256), 0, st, sub, (const float2*)nullptr,
                     kz, (const float*)zlo, (const float*)zhi, nc, (float*)sc.ptr);
  hipLaunchKernelGGL(k_af_argmax, dim3((n + 255) / 256), dim3(256), 0, st, (const float*)sc.ptr, n, nc, 0.0, 0.0,
                     zlo, zhi, z_out, (float*)nullptr, refine ? 1 : 0);
  if (scores_out && hipMemcpyAsync(scores_out, sc.ptr, (size_t)n * nc * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return fail(HV_ERR_DEVICE, "score copy failed");
  return launched("af_scan_ranges");
}

extern "C" {

hv_status hv_af_scan_ranges(hv_ctx* ctx, const uint8_t* holo, int n, int ny, int nx, double wavelength_m,
                            double pitch_m, const float* z_lo, const float* z_hi, int n_candidates, float* z_out,
                            float* scores_out, void* hip_stream) {
  if (!ctx || !holo || !z_lo || !z_hi || !z_out) return fail(HV_ERR_ARG, "NULL argument");
  if (ny != AN || nx != AN) return fail(HV_ERR_SHAPE, "autofocus works on 256x256 holograms");
  if (n_candidates < 2 || !(wavelength_m > 0) || !(pitch_m > 0))
    return fail(HV_ERR_ARG, "need >= 2 candidates, positive wavelength and pitch");
  if (n <= 0) return n == 0 ? HV_OK : fail(HV_ERR_ARG, "negative count");
  if (hv_status e = check_holo(holo)) return e;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(HV_ERR_DEVICE, "hipSetDevice failed");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  hipStream_t st = (hipStream_t)hip_stream;
  hv_status s;
  const double* kz;
  if ((s = af_kz_table(ctx, wavelength_m, pitch_m, &kz))) return s;
  DevBuf& sb = ctx->work(st, 21);
  if ((s = sb.ensure((size_t)n * SUB * SUB * 8, &ctx->held))) return s;
  if ((s = af_spectrum(holo, n, nullptr, false, (float2*)sb.ptr, st))) return s;
  // the ranges are read, never written, on this path
  return af_scan_ranges(ctx, (const float2*)sb.ptr, n, kz, const_cast<float*>(z_lo), const_cast<float*>(z_hi),
                        n_candidates, z_out, scores_out, false, st);
}

hv_status hv_af_model_create(hv_ctx* ctx, const float* init_params, int max_batch, double z_mean, double z_scale,
                             hv_af_model** out) {
  if (!ctx || !init_params || !out) return fail(HV_ERR_ARG, "NULL argument");
  if (max_batch <= 0 || !(z_scale > 0)) return fail(HV_ERR_ARG, "max_batch and z_scale must be positive");
  *out = nullptr;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(HV_ERR_DEVICE, "hipSetDevice failed");
  auto* md = new hv_af_model();
  md->ctx = ctx;
  md->max_batch = max_batch;
  md->z_mean = z_mean;
  md->z_scale = z_scale;
  // inference runs in larger batches than training: its fp16 activations
  // are a quarter of the training set's per sample
  md->infer_batch = std::max(max_batch, 1024);
  const size_t ib = (size_t)md->infer_batch;
  hv_status s;
  const size_t act = (size_t)max_batch * NCH * HW * 4;
  // the weight gradients of any batch use at most WG_BLOCKS partial sums
  const int splits = WG_BLOCKS;
  auto fail_out = [&](hv_status e) {
    hv_af_model_destroy(md);
    return e;
  };
  if ((s = dev_alloc(md, (void**)&md->params, NPARAM * 4)) || (s = dev_alloc(md, (void**)&md->m, NPARAM * 4)) ||
      (s = dev_alloc(md, (void**)&md->v, NPARAM * 4)) || (s = dev_alloc(md, (void**)&md->grad, NPARAM * 4)))
    return fail_out(s);
  for (int l = 0; l < 4; ++l)
    if ((s = dev_alloc(md, (void**)&md->act[l], act))) return fail_out(s);
  if ((s = dev_alloc(md, (void**)&md->d1, act)) || (s = dev_alloc(md, (void**)&md->d2, act)) ||
      (s = dev_alloc(md, (void**)&md->part_w, (size_t)splits * NCH * NCH * 9 * 4)) ||
      (s = dev_alloc(md, (void**)&md->part_b, (size_t)splits * NCH * 4)) ||
      (s = dev_alloc(md, (void**)&md->hpart, (size_t)max_batch * HEAD_N * 4)) ||
      (s = dev_alloc(md, (void**)&md->loss_b, (size_t)max_batch * 4)) ||
      (s = dev_alloc(md, (void**)&md->dg4, (size_t)max_batch * NCH * 4)) ||
      (s = dev_alloc(md, (void**)&md->out, (size_t)max_batch * 8)) ||
      (s = dev_alloc(md, (void**)&md->zn, (size_t)max_batch * 4)) || (s = dev_alloc(md, (void**)&md->loss_tmp, 4)) ||
      (s = dev_alloc(md, (void**)&md->act16[0], ib * NCH * HW * 2)) ||
      (s = dev_alloc(md, (void**)&md->act16[1], ib * NCH * HW * 2)) ||
      (s = dev_alloc(md, (void**)&md->pooled, ib * 16 * NCH * 4)) || (s = dev_alloc(md, (void**)&md->iout, ib * 8)) ||
      (s = dev_alloc(md, &md->wfrag, (size_t)IKS * 64 * 16)))
    return fail_out(s);
  if (hipMemcpy(md->params, init_params, NPARAM * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(md->m, 0, NPARAM * 4) != hipSuccess || hipMemset(md->v, 0, NPARAM * 4) != hipSuccess)
    return fail_out(fail(HV_ERR_DEVICE, "model initialisation failed"));
  *out = md;
  return HV_OK;
}

void hv_af_model_destroy(hv_af_model* md) {
  if (!md) return;
  (void)hipSetDevice(md->ctx->device);  // teardown cannot report
  (void)hipDeviceSynchronize();
  for (void* p : md->owned) (void)hipFree(p);
  (void)hipGetLastError();
  delete md;
}

hv_status hv_af_model_state(hv_af_model* md, float* params, float* m, float* v, int64_t* step) {
  if (!md) return fail(HV_ERR_ARG, "NULL model");
  if (hipSetDevice(md->ctx->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
    return fail(HV_ERR_DEVICE, "device error: %s", hipGetErrorString(hipGetLastError()));
  if ((params && hipMemcpy(params, md->params, NPARAM * 4, hipMemcpyDeviceToHost) != hipSuccess) ||
      (m && hipMemcpy(m, md->m, NPARAM * 4, hipMemcpyDeviceToHost) != hipSuccess) ||
      (v && hipMemcpy(v, md->v, NPARAM * 4, hipMemcpyDeviceToHost) != hipSuccess))
    return fail(HV_ERR_DEVICE, "state copy failed");
  if (step) *step = md->step;
  return HV_OK;
}

hv_status hv_af_model_load(hv_af_model* md, const float* params, const float* m, const float* v, int64_t step) {
  if (!md || !params) return fail(HV_ERR_ARG, "NULL argument");
  if (hipSetDevice(md->ctx->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
    return fail(HV_ERR_DEVICE, "device error: %s", hipGetErrorString(hipGetLastError()));
  if (hipMemcpy(md->params, params, NPARAM * 4, hipMemcpyHostToDevice) != hipSuccess ||
      (m && hipMemcpy(md->m, m, NPARAM * 4, hipMemcpyHostToDevice) != hipSuccess) ||
      (v && hipMemcpy(md->v, v, NPARAM * 4, hipMemcpyHostToDevice) != hipSuccess))
    return fail(HV_ERR_DEVICE, "state upload failed");
  md->step = step;
  md->version += 1;
  return HV_OK;
}

hv_status hv_af_forward(hv_af_model* md, const void* crops, int batch, float* out, void* hip_stream) {
  if (!md || !crops || !out) return fail(HV_ERR_ARG, "NULL argument");
  if (batch <= 0 || batch > md->max_batch) return fail(HV_ERR_SHAPE, "batch %d outside [1, %d]", batch, md->max_batch);
  if (hipSetDevice(md->ctx->device) != hipSuccess) return fail(HV_ERR_DEVICE, "hipSetDevice failed");
  hipStream_t st = (hipStream_t)hip_stream;
  hv_status s = forward(md, (const _Float16*)crops, batch, false, st);
  if (s) return s;
  if (hipMemcpyAsync(out, md->out, (size_t)batch * 8, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return fail(HV_ERR_DEVICE, "output copy failed");
  return HV_OK;
}

hv_status hv_af_infer(hv_af_model* md, const void* crops, int batch, float* out, void* hip_stream) {
  if (!md || !crops || !out) return fail(HV_ERR_ARG, "NULL argument");
  if (batch <= 0 || batch > md->infer_batch)
    return fail(HV_ERR_SHAPE, "batch %d outside [1, %d]", batch, md->infer_batch);
  if (hipSetDevice(md->ctx->device) != hipSuccess) return fail(HV_ERR_DEVICE, "hipSetDevice failed");
  hipStream_t st = (hipStream_t)hip_stream;
  hv_status s = infer(md, (const _Float16*)crops, batch, st);
  if (s) return s;
  if (hipMemcpyAsync(out, md->iout, (size_t)batch * 8, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return fail(HV_ERR_DEVICE, "output copy failed");
  return HV_OK;
}

hv_status hv_af_loss_grad(hv_af_model* md, const void* crops, const float* z_m, int batch, float* loss, float* grad,
                          void* hip_stream) {
  if (!md || !crops || !z_m || !grad) return fail(HV_ERR_ARG, "NULL argument");
  if (batch <= 0 || batch > md->max_batch) return fail(HV_ERR_SHAPE, "batch %d outside [1, %d]", batch, md->max_batch);
  if (hipSetDevice(md->ctx->device) != hipSuccess) return fail(HV_ERR_DEVICE, "hipSetDevice failed");
  hipStream_t st = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(k_normalize, dim3((batch + 255) / 256), dim3(256), 0, st, z_m, batch, (float)md->z_mean,
                     (float)(1.0 / md->z_scale), md->zn);
  hv_status s = forward(md, (const _Float16*)crops, batch, true, st);
  if (s) return s;
  return backward(md, (const _Float16*)crops, batch, grad, loss, st);
}

hv_status hv_af_train_step(hv_af_model* md, const void* crops, const float* z_m, int batch, float lr, float* loss,
                           void* hip_stream) {
  hv_status s = hv_af_loss_grad(md, crops, z_m, batch, loss ? loss : md->loss_tmp, md->grad, hip_stream);
  if (s) return s;
  hipStream_t st = (hipStream_t)hip_stream;
  md->step += 1;
  md->version += 1;
  const float c1 = (float)(1.0 - std::pow(0.9, (double)md->step));
  const float c2 = (float)(1.0 - std::pow(0.999, (double)md->step));
  hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, st, md->params, md->m, md->v, md->grad,
                     NPARAM, lr, 0.9f, 0.999f, (float)(1.0 - 0.9), (float)(1.0 - 0.999), 1e-8f, c1, c2);
  return launched("adam");
}

hv_status hv_af_train_step_holo(hv_af_model* md, const uint8_t* holo, const float* z_m, int batch, float lr,
                                float* loss, void* hip_stream) {
  if (!md || !holo || !z_m) return fail(HV_ERR_ARG, "NULL argument");
  if (batch <= 0 || batch > md->max_batch) return fail(HV_ERR_SHAPE, "batch %d outside [1, %d]", batch, md->max_batch);
  hv_ctx* ctx = md->ctx;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(HV_ERR_DEVICE, "hipSetDevice failed");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  hipStream_t st = (hipStream_t)hip_stream;
  DevBuf& cb = ctx->work(st, 34);
  hv_status s;
  if ((s = cb.ensure((size_t)batch * HW * 2, &ctx->held))) return s;
  if ((s = hv_af_crops(ctx, holo, batch, AN, AN, cb.ptr, 1, st))) return s;
  return hv_af_train_step(md, cb.ptr, z_m, batch, lr, loss, hip_stream);
}

hv_status hv_af_predict(hv_af_model* md, const uint8_t* holo, int n, double wavelength_m, double pitch_m, float tau_m,
                        int refine_candidates, float refine_k, float* z_out, float* sigma_out, int* used_fallback,
                        int* n_fallback, void* hip_stream) {
  if (!md || !holo || !z_out) return fail(HV_ERR_ARG, "NULL argument");
  if (n <= 0) return n == 0 ? HV_OK : fail(HV_ERR_ARG, "negative count");
  if (hv_status e = check_holo(holo)) return e;
  const bool refine = refine_candidates > 0;
  if (refine && (refine_candidates < 4 || !(refine_k > 0)))
    return fail(HV_ERR_ARG, "a local scan needs >= 4 candidates and a positive width in sigma");
  hv_ctx* ctx = md->ctx;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(HV_ERR_DEVICE, "hipSetDevice failed");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  hipStream_t st = (hipStream_t)hip_stream;
  DevBuf& cb = ctx->work(st, 23);
  DevBuf& sg = ctx->work(st, 24);
  hv_status s;
  if ((s = cb.ensure((size_t)md->infer_batch * HW * 2, &ctx->held))) return s;
  if ((s = sg.ensure((size_t)n * 4, &ctx->held))) return s;
  float2* subs = nullptr;
  const double* kz = nullptr;
  if (refine) {
    DevBuf& sb = ctx->work(st, 29);
    if ((s = sb.ensure((size_t)n * SUB * SUB * 8, &ctx->held))) return s;
    subs = (float2*)sb.ptr;
    if ((s = af_kz_table(ctx, wavelength_m, pitch_m, &kz))) return s;
  }
  float* sigma = sigma_out ? sigma_out : (float*)sg.ptr;
  if (used_fallback && hipMemsetAsync(used_fallback, 0, (size_t)n * sizeof(int), st) != hipSuccess)
    return fail(HV_ERR_DEVICE, "memset failed");
  for (int b0 = 0; b0 < n; b0 += md->infer_batch) {
    const int bs = std::min(md->infer_batch, n - b0);
    // the crops and, for the local scan, the +1-order sub-bands in one pass
    if ((s = af_spectrum(holo + (size_t)b0 * AN * AN, bs, cb.ptr, true, refine ? subs + (size_t)b0 * SUB * SUB : nullptr,
                         st)))
      return s;
    if ((s = infer(md, (const _Float16*)cb.ptr, bs, st))) return s;
    hipLaunchKernelGGL(k_af_denorm, dim3((bs + 255) / 256), dim3(256), 0, st, md->iout, bs, (float)md->z_mean,
                       (float)md->z_scale, z_out + b0, sigma + b0);
  }
  if (refine) {
    // local scan seeded by the network: refine_candidates / 2 candidates over
    // z +- refine_k sigma, then the rest over one coarse step on each side
    // of the best
    DevBuf& rl = ctx->work(st, 30);
    DevBuf& rh = ctx->work(st, 31);
    DevBuf& rz = ctx->work(st, 32);
    if ((s = rl.ensure((size_t)n * 4, &ctx->held)) || (s = rh.ensure((size_t)n * 4, &ctx->held)) ||
        (s = rz.ensure((size_t)n * 4, &ctx->held)))
      return s;
    const int n1 = refine_candidates / 2, n2 = refine_candidates - n1;
    hipLaunchKernelGGL(k_af_ranges, dim3((n + 255) / 256), dim3(256), 0, st, (const float*)z_out,
                       (const float*)sigma, n, refine_k, 0.05f, 0.5f, 0.01f, (float*)rl.ptr, (float*)rh.ptr);
    if ((s = af_scan_ranges(ctx, subs, n, kz, (float*)rl.ptr, (float*)rh.ptr, n1, (float*)rz.ptr, nullptr, true, st)))
      return s;
    if ((s = af_scan_ranges(ctx, subs, n, kz, (float*)rl.ptr, (float*)rh.ptr, n2, z_out, nullptr, false, st)))
      return s;
  }
  // fallback: the full scan for every hologram whose predicted sigma exceeds tau
  std::vector<float> hs(n);
  if (hipMemcpyAsync(hs.data(), sigma, (size_t)n * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(HV_ERR_DEVICE, "sigma copy failed");
  std::vector<int> idx;
  for (int i = 0; i < n; ++i)
    if (!(hs[i] <= tau_m)) idx.push_back(i);
  if (n_fallback) *n_fallback = (int)idx.size();
  if (idx.empty()) return HV_OK;
  const int m = (int)idx.size();
  DevBuf& ib = ctx->work(st, 25);
  DevBuf& gb = ctx->work(st, 26);
  DevBuf& zb = ctx->work(st, 27);
  if ((s = ib.ensure((size_t)m * 4, &ctx->held)) || (s = gb.ensure((size_t)m * AN * AN, &ctx->held)) ||
      (s = zb.ensure((size_t)m * 4, &ctx->held)))
    return s;
  // a synchronous copy (m ints): the host vector may go out of scope on any
  // return below while nothing in flight still reads it
  if (hipMemcpy(ib.ptr, idx.data(), (size_t)m * 4, hipMemcpyHostToDevice) != hipSuccess)
    return fail(HV_ERR_DEVICE, "index copy failed");
  hipLaunchKernelGGL(k_af_gather, dim3(std::min(4096, (m * AN * AN / 16 + 255) / 256)), dim3(256), 0, st, holo,
                     (const int*)ib.ptr, m, (uint8_t*)gb.ptr);
  if ((s = hv_af_scan(ctx, (const uint8_t*)gb.ptr, m, AN, AN, wavelength_m, pitch_m, 0.05, 0.5, 128,
                      (float*)zb.ptr, nullptr, st)))
    return s;
  hipLaunchKernelGGL(k_af_scatter, dim3((m + 255) / 256), dim3(256), 0, st, (const float*)zb.ptr,
                     (const int*)ib.ptr, m, z_out, used_fallback);
  if ((s = launched("af_predict"))) return s;
  // z_out is complete on return, as on the path without fallback
  if (hipStreamSynchronize(st) != hipSuccess)
    return fail(HV_ERR_DEVICE, "af_predict: %s", hipGetErrorString(hipGetLastError()));
  return HV_OK;
}

hv_status hv_af_synthesize(hv_ctx* ctx, int n, const double* z_m, double wavelength_m, double pitch_m, uint64_t seed,
                           int64_t index_base, uint8_t* out, void* hip_stream) {
  if (!ctx || !z_m || !out) return fail(HV_ERR_ARG, "NULL argument");
  if (n <= 0) return n == 0 ? HV_OK : fail(HV_ERR_ARG, "negative count");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(HV_ERR_DEVICE, "hipSetDevice failed");
  hipStream_t st = (hipStream_t)hip_stream;
  constexpr int CH = 128;  // holograms per chunk
  hv_status s;
  DevBuf& fa = ctx->work(st, 30);
  DevBuf& fb = ctx->work(st, 31);
  DevBuf& db = ctx->work(st, 32);
  if ((s = fa.ensure((size_t)CH * AN * AN * 8, &ctx->held)) || (s = fb.ensure((size_t)CH * AN * AN * 8, &ctx->held)) ||
      (s = db.ensure((size_t)CH * 25 * 4, &ctx->held)))
    return s;
  // pupil of radius 0.09 cycles/pixel as a column-major transfer table (1/ny folded in)
  DevBuf& pup = ctx->misc["afpupil"];
  if (!pup.ptr) {
    std::vector<float2> t((size_t)AN * AN);
    for (int cx = 0; cx < AN; ++cx)
      for (int cy = 0; cy < AN; ++cy) {
        const double fx = (cx < AN / 2 ? cx : cx - AN) / (double)AN, fy = (cy < AN / 2 ? cy : cy - AN) / (double)AN;
        t[(size_t)cx * AN + cy] = make_float2(fx * fx + fy * fy <= 0.09 * 0.09 ? 1.0f / AN : 0.f, 0.f);
      }
    if ((s = pup.upload(t.data(), t.size() * 8, &ctx->held))) return s;
  }
  DevBuf& tb = ctx->work(st, 33);
  if ((s = tb.ensure((size_t)CH * AN * AN * 8, &ctx->held))) return s;
  std::vector<float> disks((size_t)CH * 25);
  for (int c0 = 0; c0 < n; c0 += CH) {
    const int cn = std::min(CH, n - c0);
    const long base = index_base + c0;
    for (int i = 0; i < cn; ++i) {
      std::mt19937_64 rng(seed * 0x9E3779B97F4A7C15ull + (uint64_t)(base + i));
      std::uniform_int_distribution<int> nd(3, 8);
      std::uniform_real_distribution<float> cpos(32.f, AN - 32.f), rad(8.f, 48.f);
      float* d = &disks[(size_t)i * 25];
      d[0] = (float)nd(rng);
      for (int k = 0; k < 8; ++k) {
        d[1 + 3 * k] = cpos(rng);
        d[2 + 3 * k] = cpos(rng);
        d[3 + 3 * k] = rad(rng);
      }
    }
    if (hipMemcpyAsync(db.ptr, disks.data(), (size_t)cn * 25 * 4, hipMemcpyHostToDevice, st) != hipSuccess)
      return fail(HV_ERR_DEVICE, "disk upload failed");
    hipLaunchKernelGGL(k_af_noise, dim3(2048), dim3(256), 0, st, (float2*)fa.ptr, cn, seed, base);
    // band-limit: row FFT, column FFT x pupil x inverse column FFT, inverse row FFT
    if ((s = launch_rows_c2c(fa.ptr, HV_C64, tb.ptr, false, nullptr, nullptr, -1, cn, AN, AN, 1.f, st))) return s;
    if ((s = launch_col_full(tb.ptr, fb.ptr, false, (const float2*)pup.ptr, cn, AN, AN, st))) return s;
    if ((s = launch_row_inv(fb.ptr, false, fa.ptr, false, cn, AN, AN, 1.f / AN, st))) return s;
    hipLaunchKernelGGL(k_af_mask, dim3(2048), dim3(256), 0, st, (float2*)fa.ptr, (const float*)db.ptr, cn);
    // propagate by +z, one call per run of equal distances
    for (int i = 0; i < cn;) {
      int j = i + 1;
      while (j < cn && z_m[c0 + j] == z_m[c0 + i]) ++j;
      hv_optics op{wavelength_m, pitch_m, pitch_m, z_m[c0 + i], HV_AS};
      if ((s = hv_propagate(ctx, (const float2*)fa.ptr + (size_t)i * AN * AN, HV_C64, j - i, AN, AN, &op,
                            HV_PREC_FP32, HV_C64, (float2*)fb.ptr + (size_t)i * AN * AN, st)))
        return s;
      i = j;
    }
    hipLaunchKernelGGL(k_af_holo, dim3(cn), dim3(256), 0, st, (const float2*)fb.ptr, out + (size_t)c0 * AN * AN,
                       seed, base);
    if ((s = launched("af_synthesize"))) return s;
    if (hipStreamSynchronize(st) != hipSuccess)  // the host disk table is reused by the next chunk
      return fail(HV_ERR_DEVICE, "af_synthesize: %s", hipGetErrorString(hipGetLastError()));
  }
  return HV_OK;
}

}  // extern "C"
