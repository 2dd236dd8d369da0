// LDS-resident batched radix FFT for gfx950 (wave64).
//
// A workgroup transforms NB sequences of length N that sit in LDS.  Each
// pass is a Stockham step of radix R: every butterfly reads R values at
// stride N/R, applies the twiddles, does an R-point DFT in registers and
// writes R values at stride Ns (the product of the earlier radices).  The
// transform is done in place: all reads of a pass complete before a
// workgroup barrier, then all writes, then another barrier.
//
// Layout of sequence b in LDS (float2 units): base b*STRIDE, element i at
// i + (i >> 4).  The skew of one slot every 16 elements and an odd row
// stride keep the strided butterfly writes and the transposed reads of the
// callers off the same LDS banks.
//
// Direction: DIR = -1 computes sum_m a[m] exp(-2 pi i k m / N) (forward),
// DIR = +1 the unnormalised inverse.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <type_traits>

namespace hvk {

struct c2 {
  __device__ static inline float2 add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
  __device__ static inline float2 sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
  __device__ static inline float2 mul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
  }
  __device__ static inline float2 conj(float2 a) { return make_float2(a.x, -a.y); }
  __device__ static inline float2 scale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
  // multiply by DIR*i : (x + iy) * (DIR i) = DIR * (-y + i x)
  template <int DIR>
  __device__ static inline float2 rot(float2 a) {
    return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
  }
};

// Skewed LDS index within one sequence.
__device__ __host__ constexpr inline int skew(int i) { return i + (i >> 4); }
// Row stride (float2 units) for sequences of length N: skewed length + 1 (odd).
__device__ __host__ constexpr inline int lds_stride(int n) { return n + (n >> 4) + 1; }

// ---------------------------------------------------------------- small DFTs

template <int DIR>
__device__ inline void dft2(float2& a, float2& b) {
  float2 t = a;
  a = c2::add(t, b);
  b = c2::sub(t, b);
}

template <int DIR>
__device__ inline void dft4(float2& v0, float2& v1, float2& v2, float2& v3) {
  float2 s02 = c2::add(v0, v2), d02 = c2::sub(v0, v2);
  float2 s13 = c2::add(v1, v3), d13 = c2::rot<DIR>(c2::sub(v1, v3));
  v0 = c2::add(s02, s13);
  v2 = c2::sub(s02, s13);
  v1 = c2::add(d02, d13);
  v3 = c2::sub(d02, d13);
}

// exp(DIR * 2 pi i m / 16) for m = 0..15 (cos and sin of multiples of pi/8).
__device__ inline float2 w16(int m, int dir) {
  constexpr float C1 = 0.92387953251128674f;   // cos(pi/8)
  constexpr float S1 = 0.38268343236508978f;   // sin(pi/8)
  constexpr float H = 0.70710678118654752f;    // cos(pi/4)
  const float cs[16] = {1.f, C1, H, S1, 0.f, -S1, -H, -C1, -1.f, -C1, -H, -S1, 0.f, S1, H, C1};
  const float sn[16] = {0.f, S1, H, C1, 1.f, C1, H, S1, 0.f, -S1, -H, -C1, -1.f, -C1, -H, -S1};
  return make_float2(cs[m & 15], dir * sn[m & 15]);
}

// R-point DFT of v[0..R) in registers, natural order in and out.
template <int R, int DIR>
__device__ inline void dft_reg(float2* v) {
  if constexpr (R == 2) {
    dft2<DIR>(v[0], v[1]);
  } else if constexpr (R == 3) {
    // X1,2 = a0 - (a1 + a2)/2 +- DIR i (sqrt(3)/2) (a1 - a2)
    constexpr float H3 = 0.86602540378443865f;  // sqrt(3)/2
    const float2 t = c2::add(v[1], v[2]);
    const float2 d = c2::rot<DIR>(c2::scale(c2::sub(v[1], v[2]), H3));
    const float2 m = make_float2(v[0].x - 0.5f * t.x, v[0].y - 0.5f * t.y);
    v[0] = c2::add(v[0], t);
    v[1] = c2::add(m, d);
    v[2] = c2::sub(m, d);
  } else if constexpr (R == 5) {
    // with t1 = a1 + a4, t2 = a2 + a3, t3 = a1 - a4, t4 = a2 - a3:
    // X1,4 = a0 + c1 t1 + c2 t2 +- DIR i (s1 t3 + s2 t4)
    // X2,3 = a0 + c2 t1 + c1 t2 +- DIR i (s2 t3 - s1 t4)
    constexpr float C1 = 0.30901699437494742f, C2 = -0.80901699437494742f;  // cos(2pi/5), cos(4pi/5)
    constexpr float S1 = 0.95105651629515357f, S2 = 0.58778525229247313f;   // sin(2pi/5), sin(4pi/5)
    const float2 t1 = c2::add(v[1], v[4]), t2 = c2::add(v[2], v[3]);
    const float2 t3 = c2::sub(v[1], v[4]), t4 = c2::sub(v[2], v[3]);
    const float2 m1 = make_float2(v[0].x + C1 * t1.x + C2 * t2.x, v[0].y + C1 * t1.y + C2 * t2.y);
    const float2 m2 = make_float2(v[0].x + C2 * t1.x + C1 * t2.x, v[0].y + C2 * t1.y + C1 * t2.y);
    const float2 r1 = c2::rot<DIR>(make_float2(S1 * t3.x + S2 * t4.x, S1 * t3.y + S2 * t4.y));
    const float2 r2 = c2::rot<DIR>(make_float2(S2 * t3.x - S1 * t4.x, S2 * t3.y - S1 * t4.y));
    v[0] = c2::add(v[0], c2::add(t1, t2));
    v[1] = c2::add(m1, r1);
    v[4] = c2::sub(m1, r1);
    v[2] = c2::add(m2, r2);
    v[3] = c2::sub(m2, r2);
  } else if constexpr (R == 4) {
    dft4<DIR>(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 8) {
    // X[k] = E[k] + w8^k O[k], X[k+4] = E[k] - w8^k O[k]
    float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<DIR>(e0, e1, e2, e3);
    dft4<DIR>(o0, o1, o2, o3);
    o1 = c2::mul(o1, w16(2, DIR));
    o2 = c2::rot<DIR>(o2);
    o3 = c2::mul(o3, w16(6, DIR));
    v[0] = c2::add(e0, o0); v[4] = c2::sub(e0, o0);
    v[1] = c2::add(e1, o1); v[5] = c2::sub(e1, o1);
    v[2] = c2::add(e2, o2); v[6] = c2::sub(e2, o2);
    v[3] = c2::add(e3, o3); v[7] = c2::sub(e3, o3);
  } else if constexpr (R == 16) {
    // n = 4 n2 + n1 ; k = k1 + 4 k2
    float2 y[4][4];
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) {
      y[n1][0] = v[n1]; y[n1][1] = v[n1 + 4]; y[n1][2] = v[n1 + 8]; y[n1][3] = v[n1 + 12];
      dft4<DIR>(y[n1][0], y[n1][1], y[n1][2], y[n1][3]);
#pragma unroll
      for (int k1 = 1; k1 < 4; ++k1)
        if (n1 > 0) y[n1][k1] = c2::mul(y[n1][k1], w16(n1 * k1, DIR));
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      float2 a = y[0][k1], b = y[1][k1], c = y[2][k1], d = y[3][k1];
      dft4<DIR>(a, b, c, d);
      v[k1] = a; v[k1 + 4] = b; v[k1 + 8] = c; v[k1 + 12] = d;
    }
  }
}

// ---------------------------------------------------------------- passes

// n = 5^c 3^b 2^L: first one radix-5 pass per factor 5 and one radix-3
// pass per factor 3, then 2^L split into P = ceil(L / 4) passes of nearly
// equal radix (exponents differ by at most one, the larger ones last):
// 256 = 16 x 16, 512 = 8 x 8 x 8, 1024 = 8 x 8 x 16, 128 = 8 x 16,
// 1280 = 5 x 16 x 16, 800 = 5 x 5 x 4 x 8, 384 = 3 x 8 x 16, 320 = 5 x 8 x 8.
// A lone radix-2 pass would cost a full LDS round trip for one add per
// element.
constexpr int log2_of(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}
constexpr int count_factor(int n, int f) {
  int c = 0;
  while (n % f == 0) {
    n /= f;
    ++c;
  }
  return c;
}
constexpr int pow2_part(int n) {
  while (n % 5 == 0) n /= 5;
  while (n % 3 == 0) n /= 3;
  return n;
}
constexpr int num_passes(int n) {
  const int m = pow2_part(n);
  return count_factor(n, 5) + count_factor(n, 3) + (m > 1 ? (log2_of(m) + 3) / 4 : 0);
}
constexpr int radix_of_pass(int n, int pass) {
  const int c5 = count_factor(n, 5), c3 = count_factor(n, 3);
  if (pass < c5) return 5;
  if (pass < c5 + c3) return 3;
  const int l = log2_of(pow2_part(n)), p = (l + 3) / 4;
  return 1 << ((l + pass - c5 - c3) / p);
}

// ---------------------------------------------------------------- twiddles
// One table per pass with Ns > 1, laid out [r][k] (k fastest): entry
// exp(-2 pi i k r / (Ns R)), k < Ns, r < R.  Lanes of a butterfly group read
// consecutive k for a fixed r, so the reads never collide on an LDS bank.
constexpr int ns_of_pass(int n, int pass) {
  int ns = 1;
  for (int p = 0; p < pass; ++p) ns *= radix_of_pass(n, p);
  return ns;
}
constexpr int tw_offset(int n, int pass) {
  int off = 0;
  for (int p = 0; p < pass; ++p) {
    const int ns = ns_of_pass(n, p);
    if (ns > 1) off += ns * radix_of_pass(n, p);
  }
  return off;
}
constexpr int tw_size(int n) { return tw_offset(n, num_passes(n)); }

template <int N>
__device__ inline void fill_twiddles(float2* tw, int tid, int nthreads) {
  constexpr int P = num_passes(N);
  for (int p = 1; p < P; ++p) {
    const int ns = ns_of_pass(N, p), r_ = radix_of_pass(N, p), off = tw_offset(N, p);
    for (int e = tid; e < ns * r_; e += nthreads) {
      const int r = e / ns, k = e % ns;
      float s, c;
      sincospif(-2.0f * (float)((k * r) % (ns * r_)) / (float)(ns * r_), &s, &c);
      tw[off + e] = make_float2(c, s);
    }
  }
}

// One Stockham pass of radix R over NB sequences of length N (in place).
// LD / ST replace the pass's LDS reads / writes when they are not
// std::nullptr_t: ld(u, r, b, i) returns element i of sequence b for
// element r of the thread's butterfly slot u, st(u, r, b, i, v) takes output
// element i of sequence b (u and r are compile-time after unrolling, so a
// hook can keep its data in registers).  ST_LDS: the store hook itself
// writes the buffer (in place of the plain write).  The barrier between the
// reads and the writes is kept when both touch LDS, the barrier after the
// writes when the writes touch LDS.
template <int N, int R, int NS, int NB, int NT, int DIR, int TWOFF, bool ST_LDS, class LD, class ST>
__device__ inline void stockham_pass_io(float2* buf, const float2* tw, int tid, const LD& ld, const ST& st) {
  constexpr int BF = NB * (N / R);             // butterflies in the pass
  constexpr int U = (BF + NT - 1) / NT;        // per thread
  constexpr int S = lds_stride(N);
  constexpr bool LDS_IN = std::is_same<LD, std::nullptr_t>::value;
  constexpr bool LDS_OUT = std::is_same<ST, std::nullptr_t>::value;
  float2 v[U][R];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    int q = tid + u * NT;
    if (BF % NT == 0 || q < BF) {
      int b = q / (N / R), j = q % (N / R);
      const float2* src = buf + b * S;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (LDS_IN)
          v[u][r] = src[skew(j + r * (N / R))];
        else
          v[u][r] = ld(u, r, b, j + r * (N / R));
      }
      int k = j % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = tw[TWOFF + r * NS + k];
          if (DIR > 0) w.y = -w.y;
          v[u][r] = c2::mul(v[u][r], w);
        }
      }
      dft_reg<R, DIR>(v[u]);
    }
  }
  if constexpr (LDS_IN && (LDS_OUT || ST_LDS)) __syncthreads();
#pragma unroll
  for (int u = 0; u < U; ++u) {
    int q = tid + u * NT;
    if (BF % NT == 0 || q < BF) {
      int b = q / (N / R), j = q % (N / R);
      int k = j % NS;
      float2* dst = buf + b * S;
      int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (LDS_OUT)
          dst[skew(base + r * NS)] = v[u][r];
        else
          st(u, r, b, base + r * NS, v[u][r]);
      }
    }
  }
  if constexpr (LDS_OUT || ST_LDS) __syncthreads();
}

template <int N, int R, int NS, int NB, int NT, int DIR, int TWOFF>
__device__ inline void stockham_pass(float2* buf, const float2* tw, int tid) {
  stockham_pass_io<N, R, NS, NB, NT, DIR, TWOFF, false>(buf, tw, tid, nullptr, nullptr);
}

template <int N, int PASS, int NS, int NB, int NT, int DIR>
__device__ inline void fft_passes(float2* buf, const float2* tw, int tid) {
  if constexpr (PASS < num_passes(N)) {
    constexpr int R = radix_of_pass(N, PASS);
    stockham_pass<N, R, NS, NB, NT, DIR, tw_offset(N, PASS)>(buf, tw, tid);
    fft_passes<N, PASS + 1, NS * R, NB, NT, DIR>(buf, tw, tid);
  }
}

template <int N, int PASS, int NS, int NB, int NT, int DIR, bool ST_LDS, class LD, class ST>
__device__ inline void fft_passes_io(float2* buf, const float2* tw, int tid, const LD& ld, const ST& st) {
  if constexpr (PASS < num_passes(N)) {
    constexpr int R = radix_of_pass(N, PASS);
    constexpr bool FIRST = PASS == 0, LAST = PASS + 1 == num_passes(N);
    if constexpr (FIRST && LAST)
      stockham_pass_io<N, R, NS, NB, NT, DIR, tw_offset(N, PASS), ST_LDS>(buf, tw, tid, ld, st);
    else if constexpr (FIRST)
      stockham_pass_io<N, R, NS, NB, NT, DIR, tw_offset(N, PASS), false>(buf, tw, tid, ld, nullptr);
    else if constexpr (LAST)
      stockham_pass_io<N, R, NS, NB, NT, DIR, tw_offset(N, PASS), ST_LDS>(buf, tw, tid, nullptr, st);
    else
      stockham_pass<N, R, NS, NB, NT, DIR, tw_offset(N, PASS)>(buf, tw, tid);
    fft_passes_io<N, PASS + 1, NS * R, NB, NT, DIR, ST_LDS>(buf, tw, tid, ld, st);
  }
}

// Placement of the elements of the first (read) and last (write) pass of
// fft_lds<N, NB, NT, .> for a thread: butterfly slot u, element r is
// position *i of sequence *b; false when the slot holds no butterfly.
template <int N, int NB, int NT>
__device__ inline bool fft_first_index(int tid, int u, int r, int* b, int* i) {
  constexpr int R = radix_of_pass(N, 0);
  const int q = tid + u * NT;
  *b = q / (N / R);
  *i = q % (N / R) + r * (N / R);
  return q < NB * (N / R);
}
template <int N, int NB, int NT>
__device__ inline bool fft_last_index(int tid, int u, int r, int* b, int* i) {
  constexpr int P = num_passes(N);
  constexpr int R = radix_of_pass(N, P - 1), NS = ns_of_pass(N, P - 1);
  const int q = tid + u * NT;
  const int j = q % (N / R);
  *b = q / (N / R);
  *i = (j / NS) * NS * R + j % NS + r * NS;
  return q < NB * (N / R);
}
// Butterfly slots per thread of the first and last pass.
template <int N, int NB, int NT>
constexpr int fft_first_slots() {
  return (NB * (N / radix_of_pass(N, 0)) + NT - 1) / NT;
}
template <int N, int NB, int NT>
constexpr int fft_last_slots() {
  return (NB * (N / radix_of_pass(N, num_passes(N) - 1)) + NT - 1) / NT;
}

// NB in-place FFTs of length N held in LDS at buf[b * lds_stride(N) + skew(i)].
// Requires a barrier before (data written) -- provided by the caller -- and
// leaves a barrier after.  tw (tw_size(N) entries) must hold fill_twiddles<N>.
template <int N, int NB, int NT, int DIR>
__device__ inline void fft_lds(float2* buf, const float2* tw, int tid) {
  fft_passes<N, 0, 1, NB, NT, DIR>(buf, tw, tid);
}

// fft_lds with the first pass reading through ld and/or the last pass
// writing through st (std::nullptr_t = LDS), see stockham_pass_io.  With a
// load hook no barrier is needed before the call for the data (the caller
// still orders earlier LDS reads of buf); with a store hook that does not
// write buf (ST_LDS false) the call ends without a barrier.
template <int N, int NB, int NT, int DIR, bool ST_LDS = false, class LD, class ST>
__device__ inline void fft_lds_io(float2* buf, const float2* tw, int tid, const LD& ld, const ST& st) {
  fft_passes_io<N, 0, 1, NB, NT, DIR, ST_LDS>(buf, tw, tid, ld, st);
}

}  // namespace hvk
