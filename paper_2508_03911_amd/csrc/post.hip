// Post-processing of rendered images (Sec. III-B.2): convolution with a
// given kernel, re-normalisation by the image mean, registration by circular
// cross-correlation with a masked mean reference (shift by the peak), and a
// moving average over an accumulation buffer, in that order.
//
// Images are float32 [count][ny][nx] in device memory.  The correlation uses
// the library's FFT passes: c = IDFT2(DFT2(img) conj(DFT2(ref))), computed as
// complex row FFT -> column FFT x table x inverse column FFT -> inverse row
// FFT, with the table conj(DFT2(ref)) / ny laid out like the angular-spectrum
// transfer function.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "hv_ctx.h"
#include "hv_internal.h"

using hvi::fail;

namespace {

constexpr int TILE = 32;   // output tile side of the convolution
constexpr int CT = 256;    // threads of the image kernels

__device__ inline double block_sum_d(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = CT / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// out[i, j] = sum_{m, n} k[m, n] in[i + r - m, j + r - n], zero outside the image.
__global__ __launch_bounds__(CT) void k_conv2d(const float* __restrict__ in, float* __restrict__ out,
                                               const float* __restrict__ kern, int ksize, int ny, int nx) {
  extern __shared__ float sm[];
  const int r = ksize / 2, side = TILE + ksize - 1;
  float* tile = sm;
  float* kw = sm + side * side;
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * TILE, y0 = blockIdx.y * TILE;
  const long img = blockIdx.z;
  const float* src = in + img * (long)ny * nx;
  for (int q = tid; q < ksize * ksize; q += CT) kw[q] = kern[q];
  for (int q = tid; q < side * side; q += CT) {
    const int yy = y0 - r + q / side, xx = x0 - r + q % side;
    tile[q] = (yy >= 0 && yy < ny && xx >= 0 && xx < nx) ? src[(long)yy * nx + xx] : 0.f;
  }
  __syncthreads();
  for (int q = tid; q < TILE * TILE; q += CT) {
    const int ty = q / TILE, tx = q % TILE;
    if (y0 + ty >= ny || x0 + tx >= nx) continue;
    float acc = 0.f;
    for (int m = 0; m < ksize; ++m)
      for (int n = 0; n < ksize; ++n) acc += kw[m * ksize + n] * tile[(ty + 2 * r - m) * side + (tx + 2 * r - n)];
    out[img * (long)ny * nx + (long)(y0 + ty) * nx + x0 + tx] = acc;
  }
}

// sums[img] = sum of the image (float64, fixed order within the block).
__global__ __launch_bounds__(CT) void k_image_sum(const float* __restrict__ in, long npix, double* __restrict__ sums) {
  __shared__ double red[CT];
  const long img = blockIdx.x;
  double v = 0.0;
  for (long p = threadIdx.x; p < npix; p += CT) v += in[img * npix + p];
  v = block_sum_d(v, red);
  if (threadIdx.x == 0) sums[img] = v;
}

__global__ void k_div_mean(const float* __restrict__ in, float* __restrict__ out, long npix,
                           const double* __restrict__ sums) {
  const long img = blockIdx.y;
  const float inv = (float)((double)npix / sums[img]);
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < npix; p += (long)gridDim.x * blockDim.x)
    out[img * npix + p] = in[img * npix + p] * inv;
}

// ref[p] = disk(p) * mean_{j < rc} img_j[p] as a complex value.
__global__ void k_ref_mean(const float* __restrict__ in, int rc, int ny, int nx, double radius,
                           float2* __restrict__ ref) {
  const long npix = (long)ny * nx;
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < npix; p += (long)gridDim.x * blockDim.x) {
    const double y = (double)(p / nx) - ny / 2.0, x = (double)(p % nx) - nx / 2.0;
    double v = 0.0;
    if (y * y + x * x <= radius * radius)
      for (int j = 0; j < rc; ++j) v += in[j * npix + p];
    ref[p] = make_float2((float)(v / rc), 0.f);
  }
}

__global__ void k_real_to_c64(const float* __restrict__ in, float2* __restrict__ out, long n) {
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < n; p += (long)gridDim.x * blockDim.x)
    out[p] = make_float2(in[p], 0.f);
}

// spec [ny][nx] -> table [nx][ny] = conj(spec) / ny
__global__ void k_conj_table(const float2* __restrict__ spec, float2* __restrict__ table, int ny, int nx) {
  const long npix = (long)ny * nx;
  const float s = 1.0f / ny;
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < npix; p += (long)gridDim.x * blockDim.x) {
    const int fy = (int)(p / nx), fx = (int)(p % nx);
    const float2 v = spec[p];
    table[(long)fx * ny + fy] = make_float2(v.x * s, -v.y * s);
  }
}

// Peak of the real part of each correlation: ties go to the lowest flat index.
__global__ __launch_bounds__(CT) void k_argmax(const float2* __restrict__ corr, long npix, int nx,
                                               int* __restrict__ shifts) {
  __shared__ float bv[CT];
  __shared__ long bi[CT];
  const long img = blockIdx.x;
  const int tid = threadIdx.x;
  float best = -INFINITY;
  long bidx = npix;
  for (long p = tid; p < npix; p += CT) {
    const float v = corr[img * npix + p].x;
    if (v > best) {  // p increases, so a tie keeps the earlier index
      best = v;
      bidx = p;
    }
  }
  bv[tid] = best;
  bi[tid] = bidx;
  __syncthreads();
  for (int s = CT / 2; s > 0; s >>= 1) {
    if (tid < s) {
      const float v = bv[tid + s];
      const long i = bi[tid + s];
      if (v > bv[tid] || (v == bv[tid] && i < bi[tid])) {
        bv[tid] = v;
        bi[tid] = i;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    shifts[2 * img] = (int)(bi[0] / nx);
    shifts[2 * img + 1] = (int)(bi[0] % nx);
  }
}

// out[y][x] = in[(y + dy) mod ny][(x + dx) mod nx]
__global__ void k_shift(const float* __restrict__ in, float* __restrict__ out, int ny, int nx,
                        const int* __restrict__ shifts) {
  const long img = blockIdx.y, npix = (long)ny * nx;
  const int dy = shifts[2 * img], dx = shifts[2 * img + 1];
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < npix; p += (long)gridDim.x * blockDim.x) {
    const int y = (int)(p / nx), x = (int)(p % nx);
    out[img * npix + p] = in[img * npix + (long)((y + dy) % ny) * nx + (x + dx) % nx];
  }
}

// out_j = mean(in_{max(0, j - A + 1)} .. in_j)
__global__ void k_moving_average(const float* __restrict__ in, float* __restrict__ out, long npix, int length) {
  const long j = blockIdx.y;
  const long j0 = j - length + 1 > 0 ? j - length + 1 : 0;
  const float inv = 1.0f / (float)(j - j0 + 1);
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < npix; p += (long)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (long i = j0; i <= j; ++i) s += in[i * npix + p];
    out[j * npix + p] = s * inv;
  }
}

// Magnitude or argument image of the windowed spectrum over a range of
// temporal indices (Sec. III-B.1): spec [J][nb][npix] c64 -> out [J][npix],
// magnitude sum_k |S_k|, argument arg(sum_k S_k).  Lanes walk the pixels, so
// every bin row is read once, coalesced.
template <bool ARG>
__global__ __launch_bounds__(CT) void k_bins_image(const float2* __restrict__ spec, int nb, long npix,
                                                   float* __restrict__ out) {
  const long j = blockIdx.y;
  const float2* sj = spec + j * nb * npix;
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < npix; p += (long)gridDim.x * blockDim.x) {
    float mag = 0.f, re = 0.f, im = 0.f;
    for (int k = 0; k < nb; ++k) {
      const float2 v = sj[k * npix + p];
      if (ARG) {
        re += v.x;
        im += v.y;
      } else {
        mag += hypotf(v.x, v.y);
      }
    }
    out[j * npix + p] = ARG ? atan2f(im, re) : mag;
  }
}

unsigned blocks_for(long n) { return (unsigned)std::min<long>((n + CT - 1) / CT, 4096); }

hv_status launched(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HV_ERR_DEVICE, "%s launch failed: %s", what, hipGetErrorString(e));
  return HV_OK;
}

}  // namespace

extern "C" hv_status hv_postprocess(hv_ctx* ctx, const float* in, int count, int ny, int nx, const hv_post* cfg,
                                   float* out, int* shifts, void* hip_stream) {
  using namespace hvi;
  if (!ctx || !cfg) return fail(HV_ERR_ARG, "NULL argument");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(HV_ERR_DEVICE, "hipSetDevice failed");
  std::lock_guard<std::recursive_mutex> lock(ctx->mu);
  if (count < 0 || ny < 16 || nx < 16) return fail(HV_ERR_SHAPE, "%d images of %dx%d", count, ny, nx);
  if (count == 0) return HV_OK;
  if (!in || !out) return fail(HV_ERR_ARG, "NULL image pointer");
  const int ks = cfg->kernel_size;
  if (ks < 0 || ks > 31 || (ks > 0 && ks % 2 == 0) || (ks > 0 && !cfg->kernel))
    return fail(HV_ERR_ARG, "convolution kernel size %d: odd, at most 31, with weights", ks);
  if (cfg->ref_count < 0 || cfg->ref_count > count) return fail(HV_ERR_ARG, "reference count %d", cfg->ref_count);
  if (cfg->ref_count > 0 && !(cfg->mask_radius > 0)) return fail(HV_ERR_ARG, "mask radius must be positive");
  const long npix = (long)ny * nx, total = npix * count;
  hipStream_t st = (hipStream_t)hip_stream;
  hv_status s;
  DevBuf& wa = ctx->work(st, 40);
  DevBuf& wb = ctx->work(st, 41);
  if ((s = wa.ensure((size_t)total * 4, &ctx->held)) || (s = wb.ensure((size_t)total * 4, &ctx->held))) return s;
  // the stage results alternate between the two buffers; `cur` is the latest
  const float* cur = in;
  float* bufs[2] = {(float*)wa.ptr, (float*)wb.ptr};
  int nb = 0;
  auto next = [&]() { return bufs[nb++ & 1]; };
  if (ks > 0) {
    DevBuf& kb = ctx->work(st, 42);
    if ((s = kb.upload(cfg->kernel, (size_t)ks * ks * 4, &ctx->held))) return s;
    float* dst = next();
    const int side = TILE + ks - 1;
    const size_t lds = (size_t)(side * side + ks * ks) * 4;
    hipLaunchKernelGGL(k_conv2d, dim3((nx + TILE - 1) / TILE, (ny + TILE - 1) / TILE, count), dim3(CT), lds, st,
                       cur, dst, (const float*)kb.ptr, ks, ny, nx);
    if ((s = launched("conv2d"))) return s;
    cur = dst;
  }
  if (cfg->renormalise) {
    DevBuf& sb = ctx->work(st, 43);
    if ((s = sb.ensure((size_t)count * 8, &ctx->held))) return s;
    hipLaunchKernelGGL(k_image_sum, dim3(count), dim3(CT), 0, st, cur, npix, (double*)sb.ptr);
    float* dst = next();
    hipLaunchKernelGGL(k_div_mean, dim3(blocks_for(npix), count), dim3(CT), 0, st, cur, dst, npix,
                       (const double*)sb.ptr);
    if ((s = launched("renormalise"))) return s;
    cur = dst;
  }
  if (cfg->ref_count > 0) {
    DevBuf& rb = ctx->work(st, 44);   // reference field, then its spectrum
    DevBuf& tb = ctx->work(st, 45);   // transposed row spectra
    DevBuf& cb = ctx->work(st, 46);   // complex images / correlations
    DevBuf& hb = ctx->work(st, 47);   // conj(DFT2(ref)) / ny, [nx][ny]
    DevBuf& ones = ctx->work(st, 48);
    DevBuf& sh = ctx->work(st, 49);
    if ((s = rb.ensure((size_t)npix * 8, &ctx->held)) || (s = tb.ensure((size_t)total * 8, &ctx->held)) ||
        (s = cb.ensure((size_t)total * 8, &ctx->held)) || (s = hb.ensure((size_t)npix * 8, &ctx->held)) ||
        (s = sh.ensure((size_t)count * 8, &ctx->held)))
      return s;
    if (!ones.ptr) {
      std::vector<float2> one(4096, make_float2(1.f, 0.f));
      if ((s = ones.upload(one.data(), one.size() * 8, &ctx->held))) return s;
    }
    const float2* u = (const float2*)ones.ptr;
    const double radius = cfg->mask_radius * std::min(nx, ny) / 2.0;
    hipLaunchKernelGGL(k_ref_mean, dim3(blocks_for(npix)), dim3(CT), 0, st, cur, cfg->ref_count, ny, nx, radius,
                       (float2*)rb.ptr);
    // DFT2(ref): row FFT (transposed out), column FFT with unit chirps
    if ((s = launch_rows_c2c(rb.ptr, HV_C64, tb.ptr, false, nullptr, nullptr, -1, 1, ny, nx, 1.f, st))) return s;
    if ((s = launch_fresnel_cols(tb.ptr, false, rb.ptr, false, u, u, -1, 1, ny, nx, 1.f, st))) return s;
    hipLaunchKernelGGL(k_conj_table, dim3(blocks_for(npix)), dim3(CT), 0, st, (const float2*)rb.ptr,
                       (float2*)hb.ptr, ny, nx);
    // correlations of every image with the reference
    hipLaunchKernelGGL(k_real_to_c64, dim3(blocks_for(total)), dim3(CT), 0, st, cur, (float2*)cb.ptr, total);
    if ((s = launch_rows_c2c(cb.ptr, HV_C64, tb.ptr, false, nullptr, nullptr, -1, count, ny, nx, 1.f, st)))
      return s;
    if ((s = launch_col_full(tb.ptr, cb.ptr, false, (const float2*)hb.ptr, count, ny, nx, st))) return s;
    if ((s = launch_row_inv(cb.ptr, false, cb.ptr, false, count, ny, nx, 1.f / nx, st))) return s;
    hipLaunchKernelGGL(k_argmax, dim3(count), dim3(CT), 0, st, (const float2*)cb.ptr, npix, nx, (int*)sh.ptr);
    float* dst = next();
    hipLaunchKernelGGL(k_shift, dim3(blocks_for(npix), count), dim3(CT), 0, st, cur, dst, ny, nx,
                       (const int*)sh.ptr);
    if ((s = launched("register"))) return s;
    if (shifts && hipMemcpyAsync(shifts, sh.ptr, (size_t)count * 8, hipMemcpyDeviceToDevice, st) != hipSuccess)
      return fail(HV_ERR_DEVICE, "shift copy failed");
    cur = dst;
  }
  if (cfg->accumulate > 1) {
    hipLaunchKernelGGL(k_moving_average, dim3(blocks_for(npix), count), dim3(CT), 0, st, cur, out, npix,
                       cfg->accumulate);
    return launched("accumulate");
  }
  if (hipMemcpyAsync(out, cur, (size_t)total * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return fail(HV_ERR_DEVICE, "output copy failed");
  return HV_OK;
}

extern "C" hv_status hv_bins_image(hv_ctx* ctx, const void* spec, int nwin, int nbins, int ny, int nx, int kind,
                                  float* out, void* hip_stream) {
  using namespace hvi;
  if (!ctx) return fail(HV_ERR_ARG, "NULL context");
  if (kind != HV_IMG_MAGNITUDE && kind != HV_IMG_ARGUMENT) return fail(HV_ERR_ARG, "image kind %d", kind);
  if (nwin < 0 || nwin > 65535 || nbins <= 0 || ny <= 0 || nx <= 0)
    return fail(HV_ERR_SHAPE, "%d windows of %d bins of %dx%d", nwin, nbins, ny, nx);
  if (nwin == 0) return HV_OK;
  if (!spec || !out) return fail(HV_ERR_ARG, "NULL pointer");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(HV_ERR_DEVICE, "hipSetDevice failed");
  const long npix = (long)ny * nx;
  hipStream_t st = (hipStream_t)hip_stream;
  const dim3 grid(blocks_for(npix), (unsigned)nwin);
  if (kind == HV_IMG_ARGUMENT)
    hipLaunchKernelGGL(k_bins_image<true>, grid, dim3(CT), 0, st, (const float2*)spec, nbins, npix, out);
  else
    hipLaunchKernelGGL(k_bins_image<false>, grid, dim3(CT), 0, st, (const float2*)spec, nbins, npix, out);
  return launched("bins_image");
}
