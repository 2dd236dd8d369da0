// Internal declarations shared by the library's translation units.
// Not part of the public C-ABI (that is include/hv.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hv.h"

typedef _Float16 hv_h2 __attribute__((ext_vector_type(2)));
typedef _Float16 hv_h8 __attribute__((ext_vector_type(8)));

namespace hvi {

// Sets the thread-local message returned by hv_last_error and returns st.
hv_status fail(hv_status st, const char* fmt, ...);

inline bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }

// Workgroups of a persistent kernel on the current device: every CU filled
// to the kernel's occupancy at `threads` per workgroup (computed once per
// kernel and device).
int persistent_blocks(const void* kernel, int threads);
template <class K>
int persistent_grid(K kernel, int threads, int nunits) {
  const int b = persistent_blocks(reinterpret_cast<const void*>(kernel), threads);
  return nunits < b ? nunits : b;
}

// ---------------------------------------------------------------- spatial kernels
// All launches are asynchronous on `stream`; shapes are validated by the caller.

// Row R2C FFT of real frames with the unpack fused into the load.
// in: [n][ny][nx] u8/u16; out: [n][nx/2][ny] complex (c64 or fp16 complex),
// column 0 packing (X(0,y), X(nx/2,y)) which are both real; values * scale.
hv_status launch_row_r2c(const void* in, hv_dtype in_t, void* out, bool half_out, int n, int ny, int nx,
                         float scale, hipStream_t st);

// Angular-spectrum column pass: column FFT, split into the +fx/-fx columns
// by Hermitian symmetry, multiply by ht (column-major [nx][ny], the
// transfer function divided by ny), inverse column FFT.
// in: [n][nx/2][ny] (from launch_row_r2c); out: [n][ny][nx].
hv_status launch_col_as(const void* in, void* out, bool half_io, const float2* hs, int n, int ny, int nx,
                        hipStream_t st);

// Row inverse FFT to the field: in [n][ny][nx] complex, out [n][ny][nx]
// complex (c64 or fp16), values * scale.
hv_status launch_row_inv(const void* in, bool half_in, void* out, bool half_out, int n, int ny, int nx,
                         float scale, hipStream_t st);

// Fresnel column pass: column FFT of sign dir, * (qx_out[p] qy_out[q]),
// write the field [n][ny][nx] complex (c64 or fp16), values * scale.
hv_status launch_fresnel_cols(const void* in, bool half_in, void* out, bool half_out, const float2* qx,
                              const float2* qy, int dir, int n, int ny, int nx, float scale, hipStream_t st);

// ---------------------------------------------------------------- temporal kernels

// Coefficient GEMM description shared by the DFT-moment and PCA kernels.
// Rows of the coefficient matrix come in (real, imaginary) pairs; npair
// pairs padded to mtiles * 16.  The B operand is the window's field as a
// [2W x pixels] real matrix with row 2t + c = component c of frame t.
struct CoefGemm {
  int window;          // W (8, 16, 32 or 64)
  int mtiles;          // 32-row tiles of the coefficient matrix
  int npair;           // live (re, im) pairs
  const float* a32;    // [mtiles][W][64] f32 MFMA A fragments
  const hv_h8* a16hi;  // [mtiles][W/8][64] f16 MFMA A fragments (high part)
  const hv_h8* a16lo;  // same, low part
  const float* wts;    // [3][mtiles*16] per-pair weights for the 3 outputs (0 = unused)
  int nout;            // outputs written (1..3)
};

// Fused: row inverse FFT of W frames of one row, then the coefficient GEMM
// and weighted power epilogue.  z: chunk [nf][ny][nx]; window jj starts at
// frame jj*stride of the chunk.  Outputs out[k] + jj*ny*nx + y*nx + x.
hv_status launch_rowinv_coef(const void* z, bool half_in, int ny, int nx, int stride, int nwin,
                             const CoefGemm& g, bool mixed, float b_scale, float out_scale, float* out0,
                             float* out1, float* out2, float2* spec, hipStream_t st);

// Unfused: field chunk [nf][P] (P = ny*nx) already in memory.
hv_status launch_field_coef(const void* u, bool half_in, long npix, int stride, int nwin,
                            const CoefGemm& g, bool mixed, float b_scale, float out_scale, float* out0,
                            float* out1, float* out2, float2* spec, hipStream_t st);

bool rowinv_coef_fits(int nx, int window);

// ---------------------------------------------------------------- PCA kernels

// Partial Gram matrices G = B^T B (B = [P x 2W], interleaved re/im columns)
// of each window over pixel blocks: part [nwin][nblk][2W][2W] f32.
hv_status launch_gram_partials(const void* u, bool half_in, long npix, int stride, int nwin, int window,
                               bool mixed, float b_scale, float* part, int nblk, hipStream_t st);
// Deterministic sum of the partials in fixed order, in f64, into the
// Hermitian covariance C [nwin][W][W] complex f64 (interleaved), scaled by cscale.
hv_status launch_gram_reduce(const float* part, int nwin, int nblk, int window, double cscale, double* cov,
                             hipStream_t st);
// FP64 cyclic Jacobi on each window's C: eigenvalues (descending) and
// eigenvectors (columns, complex f64 interleaved) [nwin][W][W]; offdiag
// (nullable) [nwin] receives sqrt(off-diagonal / total squared magnitude)
// when the window stops (converged below 1e-15, or max_sweeps reached).
hv_status launch_jacobi(const double* cov, int nwin, int window, double* evals, double* evecs, double* offdiag,
                        int max_sweeps, hipStream_t st);
// Build per-window projection coefficient fragments from eigenvectors
// columns c1..c2 (A = [Vr^T Vi^T ; ...]) for the coefficient GEMM.
hv_status launch_proj_coefs(const double* evecs, int nwin, int window, int c1, int c2, int mtiles,
                            float* a32, hv_h8* a16hi, hv_h8* a16lo, hipStream_t st);
// SSA + FFT: per-window coefficient fragments A[k][t'] = sum_t (V_S V_S^H)[t', t]
// exp(-2 pi i k t / W) for the nb band bins (bins[0..nb), host array) and
// components c1..c2, in the layout of the DFT coefficients (mtiles tiles).
hv_status launch_ssa_coefs(const double* evecs, int nwin, int window, int c1, int c2, const int* bins, int nb,
                           int mtiles, float* a32, hv_h8* a16hi, hv_h8* a16lo, hipStream_t st);
// Coefficient GEMM with per-window A and the three weighted-power outputs
// (wts [3][16 mtiles]) into m0/m1/m2 [nwin][npix] (each nullable).
hv_status launch_coef_moments(const void* u, bool half_in, long npix, int stride, int nwin, int window, int mtiles,
                              int npair, const float* a32, const hv_h8* a16hi, const hv_h8* a16lo, const float* wts,
                              bool mixed, float b_scale, float out_scale, float* m0, float* m1, float* m2,
                              hipStream_t st);
// Projection energy M0_pca per pixel per window, with per-window A.
hv_status launch_proj_energy(const void* u, bool half_in, long npix, int stride, int nwin, int window,
                             int mtiles, int npair, const float* a32, const hv_h8* a16hi, const hv_h8* a16lo,
                             const float* wts, bool mixed, float b_scale, float out_scale, float* m0,
                             hipStream_t st);

// Full-band STFT power of every complete window: a radix FFT over W frames
// (128, 256 or 512) per pixel, out [nwin][W][npix] f32 = |S_k|^2 * amp2.
hv_status launch_time_fft(const void* u, bool half_in, long npix, int stride, int nwin, int window, float amp2,
                          float* out, hipStream_t st);

// ---------------------------------------------------------------- band-first order
// (angular spectrum of each band bin's combination of raw frames)

// Frame shapes and input types the band-first kernels take: u8/u16 frames,
// nx a power of two in [64, 512], ny in {64, 128, 256, 320, 384, 512}.
bool band_first_fits(int ny, int nx, int in_t);
// Window jj of in (frames jj*stride ..) reduced to nb bins (real-input A
// fragments ahi/alo, mtiles tiles) and row-transformed:
// out [nwin][nb][ny][nx] complex (c64 or fp16), values * scale.
hv_status launch_band_rows(const void* in, int in_t, void* out, bool half_out, int ny, int nx, int stride, int nwin,
                           int window, int nb, int mtiles, const hv_h8* ahi, const hv_h8* alo, float scale,
                           hipStream_t st);
// In place on nfields fields [ny][nx]: column FFT, * ht (column-major
// [nx][ny]), inverse column FFT.
hv_status launch_band_cols(void* io, bool half_io, const float2* ht, int nfields, int ny, int nx, hipStream_t st);
// Inverse row FFT of [nwin][nb][ny][nx], values * amp, then the weighted
// powers (wts [3][16 mtiles]) into o0..o2 [nwin][ny][nx] and, when spec is
// not null, the values into spec [nwin][nb][ny*nx].
hv_status launch_band_power(const void* in, bool half_in, int ny, int nx, int nwin, int nb, int mtiles,
                            const float* wts, float amp, float* o0, float* o1, float* o2, float2* spec,
                            hipStream_t st);

}  // namespace hvi
