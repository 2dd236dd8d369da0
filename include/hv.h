/* hv.h -- C-ABI of the MI355X (gfx950) hologram-rendering hot path.
 *
 * The operations follow "Holovibes: Real-time Ultrahigh-Speed Digital
 * Hologram Rendering and Short-Time Analysis" (arXiv 2508.03911):
 *   - camera integers converted to complex and spatially transformed frame
 *     by frame, by angular-spectrum propagation or a Fresnel transform
 *     (Abstract; Sec. II-B.3; Sec. III-B.1);
 *   - a temporal transform over a user-sized window of consecutive frames:
 *     a short-time Fourier transform, or PCA via covariance,
 *     eigendecomposition and projection onto a sub-basis (Sec. III-B.1);
 *   - a per-pixel statistical moment over a range of temporal indices
 *     (Sec. III-B.1);
 *   - settings: reconstruction distance, propagation method, temporal
 *     transform, window size and stride (Sec. III-B; Sec. VI-B);
 *   - the back-end exposed as a library (Sec. VII-A, VII-B);
 *   - buffers allocated once, not per frame (Sec. VII-C).
 *
 * Conventions
 *   Arrays are row-major [frames][ny][nx]; x is the fast axis.  Complex
 *   values are interleaved (re, im) float32 ("c64").  z is the signed
 *   propagation distance in metres: a hologram recorded at distance z is
 *   reconstructed with -z.  Supported frame sides: powers of two in
 *   [64, 1024], and 320, 384, 800, 1280 (the mixed-radix sides of the
 *   paper's Table IV frames; non-square allowed).  Windows: 8, 16, 32 or 64
 *   frames (hv_stft_volume: 128, 256, 512).
 *   Exception: hv_stft_moments_host takes pinned HOST frames and images.
 *
 * Ownership and asynchrony
 *   Every data pointer is caller-owned DEVICE memory on the context's
 *   device; the library never frees it.  Input arrays must be 16-byte
 *   aligned (hipMalloc and torch allocations are; HV_ERR_ARG otherwise).  Plans (FP64-built tables,
 *   coefficient fragments) and workspaces belong to the context and are
 *   allocated on first use for a given shape/setting and stream, then
 *   reused; hv_ctx_destroy frees them.  Calls enqueue work on `hip_stream`
 *   (a hipStream_t; NULL = the default stream) and return without waiting.
 *   A context may be used from one host thread at a time; calls on
 *   different streams use different workspaces.
 *
 * Errors
 *   Every call returns HV_OK (0) or a negative hv_status; hv_last_error()
 *   returns a thread-local message for the last failure.  No C++ exception
 *   crosses this boundary.  Invalid shapes return HV_ERR_SHAPE before any
 *   work is enqueued.
 */
#ifndef HV_H
#define HV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HV_OK = 0,
  HV_ERR_ARG = -1,      /* null pointer, bad enum, bad band or range */
  HV_ERR_SHAPE = -2,    /* unsupported frame size, window or frame count */
  HV_ERR_NOMEM = -3,    /* device allocation failed */
  HV_ERR_BUDGET = -4,   /* stream refused: HBM budget exceeded */
  HV_ERR_DEVICE = -5,   /* HIP runtime error */
  HV_ERR_OVERFLOW = -6, /* stream ring full: frames would be lost */
  HV_ERR_STATE = -7     /* nothing to pop / object in the wrong state */
} hv_status;

typedef enum {
  HV_U8 = 0,   /* camera frames, 8 bit */
  HV_U16 = 1,  /* camera frames, up to 16 bit (12-bit data low-bit aligned) */
  HV_C64 = 3,  /* complex field, interleaved float32 */
  HV_C32H = 4  /* complex field, interleaved fp16, holding U * hv_field_scale(...) */
} hv_dtype;

typedef enum { HV_AS = 0, HV_FRESNEL = 1 } hv_method;

/* HV_PREC_FP32: FP32 FFT arithmetic, c64 intermediates, FP32 MFMA GEMMs.
 * HV_PREC_MIXED: FP32 FFT arithmetic, fp16 intermediates in memory with
 * power-of-two scaling, split fp16 (hi + lo) MFMA GEMMs with FP32
 * accumulation; eigensolves stay FP64. */
typedef enum { HV_PREC_FP32 = 0, HV_PREC_MIXED = 1 } hv_precision;

typedef struct hv_ctx hv_ctx;

/* Spatial step (Abstract; Sec. II-B.3; Sec. III-B.1).  highpass_cpp is the
 * spatial high-pass filter of the angular-spectrum benchmark (Sec. VI-B.1):
 * the spectrum keeps the DFT bins with (k_x/nx)^2 + (k_y/ny)^2 >= r^2 (signed
 * indices k, r in cycles per pixel); 0 = no filter.  AS only (HV_ERR_ARG for
 * Fresnel); 0 <= r < 1. */
typedef struct {
  double wavelength_m;
  double pitch_x_m;
  double pitch_y_m;
  double z_m;   /* signed propagation distance, metres; != 0 for Fresnel */
  int method;   /* hv_method */
  double highpass_cpp;
} hv_optics;

/* Temporal step (Sec. III-B.1; Sec. VI-B: window and stride).  The band
 * [f_lo_hz, f_hi_hz] keeps DFT bins ceil(f_lo W/fs) .. floor(f_hi W/fs),
 * limited to 0..W/2 (decided in float64); symmetric_band adds the mirrored
 * bins W-k.  f_k = k fs / W and M_n = sum_k f_k^n |S_k|^2. */
typedef struct {
  int window;
  int stride;
  double fs_hz;
  double f_lo_hz;
  double f_hi_hz;
  int symmetric_band;
} hv_temporal;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the
 * device memory the serving loop may admit (0 = no limit). */
hv_status hv_ctx_create(int device, size_t hbm_budget_bytes, hv_ctx** out);
void hv_ctx_destroy(hv_ctx* ctx);
/* Thread-local text of the last error (never NULL). */
const char* hv_last_error(void);
/* Bytes of device memory held by the context's plans and workspaces. */
size_t hv_ctx_workspace_bytes(const hv_ctx* ctx);
/* Frames per spatial chunk (workspace size knob; 0 = automatic). */
hv_status hv_ctx_set_chunk_frames(hv_ctx* ctx, int frames);

/* Order of the angular-spectrum STFT path of hv_stft_moments and
 * hv_stft_bins.  Both orders compute the same values up to rounding.  The
 * propagation is one linear operator applied to every frame (Sec. II-B.3)
 * and each band bin is a fixed linear combination of a window's frames
 * (Sec. III-B.1), so the bins can be formed from the raw frames and then
 * propagated ("band first"), which transforms nb fields per window instead
 * of W frames.
 *   HV_ORDER_FRAMES_FIRST the paper's order and the default: every frame is
 *                         propagated, then the temporal transform;
 *   HV_ORDER_AUTO         band first where it moves fewer bytes per window
 *                         and the shape is supported (u8/u16 frames, nx a
 *                         power of two in [64, 512], ny 64, 128, 256, 320,
 *                         384 or 512), else frames first;
 *   HV_ORDER_BAND_FIRST   band first wherever the shape is supported.
 * Returns HV_ERR_ARG for another value.  A new context starts from the
 * environment variable HV_STFT_ORDER (0, 1 or 2) when it is set. */
typedef enum { HV_ORDER_AUTO = 0, HV_ORDER_FRAMES_FIRST = 1, HV_ORDER_BAND_FIRST = 2 } hv_stft_order;
hv_status hv_ctx_set_stft_order(hv_ctx* ctx, int order);

/* Per-kernel timing for profiling (Sec. VII-D): when on, every kernel launch
 * is bracketed by HIP events on the stream it is launched on (the caller's,
 * or the second stream of hv_stft_moments); no work is skipped.
 * Turning it on or off clears the totals. */
hv_status hv_ctx_set_timing(hv_ctx* ctx, int on);
/* Waits for the recorded launches and returns the total milliseconds and the
 * launch count of kernel `name` ("row_r2c", "col_as", "rowinv_coef",
 * "row_inv", "field_coef", "rows_c2c", "col_full", "fresnel_rows",
 * "fresnel_cols", "band_rows", "band_cols", "band_power", "gram", "jacobi",
 * "proj_energy"). */
hv_status hv_ctx_kernel_time(hv_ctx* ctx, const char* name, double* total_ms, long* launches);

/* ---------------------------------------------------------------- spatial */

/* Reconstruct n frames (Sec. III-B.1 spatial transformation).
 *   in    [n][ny][nx] of in_t (HV_U8, HV_U16 or HV_C64)
 *   out   [n][ny][nx] of out_t: angular spectrum U = IDFT2(DFT2(x) H_z)
 *         with H_z = exp(2 pi i z sqrt(1/lambda^2 - fx^2 - fy^2)) (0 if
 *         evanescent), or the single-FFT Fresnel transform
 *         U = Q_out DFT_c(x Q_in) / sqrt(nx ny) on the output grid of pitch
 *         lambda|z|/(n pitch) (centred DFT of sign sgn(z)).
 *   out_t HV_C64 (U as float32 pairs) or HV_C32H (U * hv_field_scale(in_t,
 *         ny, nx) as fp16 pairs: half the bytes, about 3 significant
 *         digits; the scale keeps every field of a camera input in range,
 *         a HV_C64 input is taken as |U| < 32768).
 *   prec  selects the intermediate storage (see hv_precision); any prec
 *         goes with either out_t. */
hv_status hv_propagate(hv_ctx* ctx, const void* in, int in_t, int n, int ny, int nx, const hv_optics* optics,
                       int prec, int out_t, void* out, void* hip_stream);

/* The power of two by which an HV_C32H field is multiplied (host call, no
 * device work): 2^-k with k the smallest integer such that
 * sqrt(ny nx) * max input value * 2^-k <= 32768, where the max input value
 * is 255 (HV_U8) or 65535 (HV_U16); a unitary propagation of such frames
 * cannot exceed sqrt(ny nx) times it.  1 for a HV_C64 input. */
hv_status hv_field_scale(int in_t, int ny, int nx, float* scale);

/* ---------------------------------------------------------------- temporal */

/* Doppler moment images (Sec. III-B.1: STFT over the window, then moments
 * over a range of temporal indices).
 *   in        [n][ny][nx] camera frames (HV_U8/HV_U16), or a field (HV_C64)
 *             when optics is NULL.
 *   m0,m1,m2  [J][ny][nx] float32 with J = floor((n - W)/stride) + 1; any of
 *             them may be NULL to skip it (at least one non-NULL).
 * Window j covers frames [j*stride, j*stride + W); S_j[k] =
 * sum_t U[j*stride+t] exp(-2 pi i k t / W) (rectangular, unnormalised).
 * Returns HV_ERR_SHAPE when n < W.
 * Ordering: the frames are processed in chunks; when there is more than one,
 * the chunks alternate between hip_stream and a second stream the context
 * keeps for it, forked from and joined back into hip_stream by events, so
 * the call is ordered on hip_stream like a single launch.  With the angular
 * spectrum, the order of the spatial and temporal steps follows
 * hv_ctx_set_stft_order (per frame unless the caller asks otherwise). */
hv_status hv_stft_moments(hv_ctx* ctx, const void* in, int in_t, int n, int ny, int nx, const hv_optics* optics,
                          const hv_temporal* temporal, int prec, float* m0, float* m1, float* m2,
                          void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * moments as hv_stft_moments, same arguments, layout and results, with
 * every workspace taken from a static device array of the library (256 MiB,
 * one copy per GPU, held until the process ends) instead of allocated.  The
 * call allocates nothing and creates no stream or event:
 *   - the transfer-function or chirp tables and the DFT coefficients must
 *     already be in the context: one call of hv_stft_moments (or
 *     hv_stft_bins) with the same frame shape, optics and temporal settings
 *     builds them; otherwise HV_ERR_STATE;
 *   - it always takes the per-frame order on hip_stream alone, in chunks of
 *     as many windows as the scratch holds;
 *   - a shape whose single window needs more than 256 MiB of workspace
 *     (ny*nx*W*(1.5 or 2)*(8 FP32 or 4 mixed) bytes; 1024 x 1024 FP32 at
 *     W = 32 is one) returns HV_ERR_SHAPE.
 * Every call on one GPU shares that GPU's scratch: calls that overlap on one
 * GPU (two host threads, or two streams whose work overlaps) race and
 * corrupt each other's results; serialise them.  Nothing in the scratch
 * needs clearing: every workspace byte is written before it is read. */
hv_status hv_stft_moments_noalloc(hv_ctx* ctx, const void* in, int in_t, int n, int ny, int nx,
                                  const hv_optics* optics, const hv_temporal* temporal, int prec, float* m0,
                                  float* m1, float* m2, void* hip_stream);

/* hv_stft_moments from host memory (the paper's camera path: frames arrive
 * in host memory and cross PCIe, Sec. II-B.4, VII).  host_in is pinned host
 * memory (hipHostMalloc) [n][ny][nx] HV_U8/HV_U16; host_m0..m2 are pinned
 * host buffers [J][ny][nx] float32 (NULL = skip, at least one non-NULL).
 * Chunks of frames are uploaded, processed and their images downloaded on
 * alternating streams (hip_stream and the context's second stream), so the
 * copies of one chunk overlap the kernels of the other; the call is ordered
 * on hip_stream and the images are complete once hip_stream has drained.
 * Pageable host memory also works but the copies then do not overlap. */
hv_status hv_stft_moments_host(hv_ctx* ctx, const void* host_in, int in_t, int n, int ny, int nx,
                               const hv_optics* optics, const hv_temporal* temporal, int prec, float* host_m0,
                               float* host_m1, float* host_m2, void* hip_stream);

/* The windowed spectrum itself on the band bins, in band order:
 *   spec [J][nbins][ny][nx] c64, nbins as returned by hv_band_bins. */
hv_status hv_stft_bins(hv_ctx* ctx, const void* in, int in_t, int n, int ny, int nx, const hv_optics* optics,
                       const hv_temporal* temporal, int prec, void* spec, void* hip_stream);

/* The full-band STFT volume of the paper's STFT benchmark (Sec. VI-B.1:
 * angular spectrum with the spatial high-pass filter of hv_optics, then the
 * temporal transform over whole windows of W = 128, 256 or 512 frames,
 * every bin rendered): a radix FFT per pixel and window,
 *   power [J][W][ny][nx] float32 = |S_j[k]|^2, k in DFT order,
 * J = floor((n - W)/stride) + 1.  in: camera frames (HV_U8/HV_U16) with
 * optics, or a field (HV_C64) with optics NULL.  Chunks alternate over two
 * streams as in hv_stft_moments.  HV_ERR_SHAPE when n < W or W is not
 * supported. */
hv_status hv_stft_volume(hv_ctx* ctx, const void* in, int in_t, int n, int ny, int nx, const hv_optics* optics,
                         int window, int stride, int prec, float* power, void* hip_stream);

/* The band's bins and frequencies as the library decides them (host call).
 * bins/freqs may be NULL; *nbins receives the count. */
hv_status hv_band_bins(const hv_temporal* temporal, int* nbins, int* bins, double* freqs);

/* ---------------------------------------------------------------- PCA */

/* PCA over each window (Sec. III-B.1: covariance, eigendecomposition,
 * projection onto a sub-basis).  X_j is the window's field as a [P x W]
 * matrix; C_j = X_j^H X_j (no centring, no 1/P); eigenpairs by FP64 Jacobi,
 * eigenvalues descending; m0[p] = sum_{c=comp_lo..comp_hi} |(X_j V)[p,c]|^2.
 *   in       frames (HV_U8/HV_U16 with optics) or field (HV_C64, optics NULL)
 *   m0       [J][ny][nx] float32
 *   eigvals  [J][W] float64, descending (nullable)
 *   cov      [J][W][W] complex float64 interleaved (nullable)
 *   offdiag  [J] float64 (nullable): sqrt(sum of |off-diagonal|^2 / sum of
 *            |all entries|^2) of the rotated matrix when the Jacobi solver
 *            stopped: below 1e-15 when the window converged, larger when it
 *            reached the sweep limit (40) first; the call does not fail then
 * 0 <= comp_lo <= comp_hi < W. */
hv_status hv_pca(hv_ctx* ctx, const void* in, int in_t, int n, int ny, int nx, const hv_optics* optics, int window,
                 int stride, int comp_lo, int comp_hi, int prec, float* m0, double* eigvals, double* cov,
                 double* offdiag, void* hip_stream);

/* SSA + FFT (Sec. III-B.1: the temporal transform "SSA and FFT", its SVD
 * obtained by eigen-decomposition of the data: covariance of the window,
 * eigen-decomposition, projection onto a sub-basis).  Per window X_j
 * ([P x W] as for hv_pca; C_j = X_j^H X_j; FP64 Jacobi; eigenvalues
 * descending), the window is rebuilt from its components
 * comp_lo..comp_hi, X_f = X_j V_S V_S^H, and transformed in time as in
 * hv_stft_moments: S_k = sum_t X_f[:, t] exp(-2 pi i k t / W), with
 * M_n = sum_{k in band} f_k^n |S_k|^2 over the band of `temporal` (window
 * W = temporal->window in {16, 32, 64}, stride temporal->stride).  The
 * projection, the back-projection and the DFT are folded into one set of
 * coefficients per window (FP64-built), so the field is read once by the
 * coefficient GEMM after the Gram GEMM.
 *   in       frames (HV_U8/HV_U16 with optics) or field (HV_C64, optics NULL)
 *   m0..m2   [J][ny][nx] float32 (nullable, not all)
 *   eigvals  [J][W] float64 (nullable), offdiag [J] (nullable) as in hv_pca
 * The default comp_lo = 1, comp_hi = W - 1 removes the dominant (static)
 * component; comp_lo = 0, comp_hi = W - 1 gives hv_stft_moments' moments. */
hv_status hv_ssa_moments(hv_ctx* ctx, const void* in, int in_t, int n, int ny, int nx, const hv_optics* optics,
                         const hv_temporal* temporal, int comp_lo, int comp_hi, int prec, float* m0, float* m1,
                         float* m2, double* eigvals, double* offdiag, void* hip_stream);

/* ---------------------------------------------------------------- serving loop */

/* Camera streams processed as their frames arrive (Sec. II-B.1 and III-A:
 * a GPU-resident input ring fed by frame packets and drained by windows,
 * sized so that it never overflows; Sec. II-B.4: separate streams).  Each
 * stream owns a device ring of ring_frames raw frames (plus W - stride
 * mirrored slots), its own HIP stream, preallocated workspaces and a ring
 * of output images.  Window j covers frames [j*stride, j*stride + W) and
 * is launched as soon as its last frame is pushed; the images are M0/M1/M2
 * exactly as hv_stft_moments computes them on the same frames. */
typedef struct hv_stream hv_stream;

typedef struct {
  int64_t frames_in;          /* frames accepted by pushes */
  int64_t frames_dropped;     /* frames refused with HV_ERR_OVERFLOW */
  int64_t windows_done;       /* windows whose images are complete */
  int64_t streams_admitted;
  int64_t streams_refused;    /* HBM budget (or replay slot limit) */
  int64_t images_overwritten; /* completed images replaced before a pop */
  int64_t latency_samples;
  int64_t lat_p50_ns, lat_p99_ns, lat_max_ns; /* image done - arrival of the window's last frame */
  int64_t admitted_bytes;     /* device bytes charged to open streams */
  int64_t device_errors;      /* completion queries that reported a device error */
} hv_stats;

/* Open a stream of ny x nx frames (HV_U8 or HV_U16).  ring_frames must be a
 * multiple of the stride and >= 2 W (0 = 8 W), and should hold W frames plus
 * the largest packet plus the frames pushed while a window computes;
 * 1 <= stride <= W.  The ring,
 * image slots, workspaces and tables are allocated here (none later) and
 * charged to the context's HBM budget: HV_ERR_BUDGET refuses the stream. */
hv_status hv_stream_open(hv_ctx* ctx, int ny, int nx, int raw_t, const hv_optics* optics,
                         const hv_temporal* temporal, int prec, int ring_frames, hv_stream** out);
/* Copy n_frames consecutive frames into the ring and launch every window
 * they complete.  frames is device memory (copied on the stream's queue,
 * ordered before the windows; the caller's producer work must be complete)
 * or host memory: pinned (hipHostMalloc) at the PCIe rate, pageable at a
 * lower one; host frames are uploaded on a queue of their own and waited
 * for, so the buffer may be reused on return (Sec. II-B.1, the packet
 * path from the camera).  arrival_ns[i] (CLOCK_MONOTONIC ns, nullable =
 * now) is the arrival time of frame i, used for latency.  A packet that
 * would overwrite frames still needed returns HV_ERR_OVERFLOW and is counted
 * as dropped; nothing is overwritten silently.  When a ring copy or a
 * window launch fails, or the device reports an error for a launched
 * window, the stream is
 * marked failed: that push returns the launch error and every later push
 * returns HV_ERR_STATE (not counted as drops) until the stream is closed. */
hv_status hv_stream_push(hv_stream* s, const void* frames, int n_frames, const int64_t* arrival_ns);
/* Oldest completed, unpopped window: copies its M0/M1/M2 (each ny*nx float32,
 * device pointers, nullable) and returns its timestamps.  HV_ERR_STATE when
 * none is ready.  Up to 4 completed images are kept; older ones are counted
 * in images_overwritten. */
hv_status hv_stream_pop(hv_stream* s, float* m0, float* m1, float* m2, int64_t* t_last_arrival_ns,
                        int64_t* t_done_ns);
/* Finish in-flight windows, free the stream and return its bytes to the budget.
 * The stream is released even when the device reports an error while its
 * work drains; that error is returned as HV_ERR_DEVICE. */
hv_status hv_stream_close(hv_stream* s);
/* Per-stream counters (nullable outputs). */
hv_status hv_stream_frames(const hv_stream* s, int64_t* pushed, int64_t* dropped, int64_t* windows_done);
/* Context-wide serving counters and latency percentiles (nearest rank). */
hv_status hv_ctx_stats(hv_ctx* ctx, hv_stats* out);
/* Clear the counters and latency samples. */
hv_status hv_ctx_stats_reset(hv_ctx* ctx);

/* Replay of device-resident synthetic camera blocks as a Poisson stream
 * load (the paper's file mode, where a recording in GPU memory stands in
 * for the camera, Table IV).  Streams arrive at arrival_hz, live
 * Exp(mean_life_s), pick a class uniformly, draw z uniformly in
 * [z_lo_m, z_hi_m] (reconstructed at -z by angular spectrum), and push
 * packet_frames frames at the class frame rate from their block (cyclic).
 * A class admits at most max_active streams; the HBM budget may refuse
 * more.  Latency samples start after warmup_s. */
#define HV_REPLAY_MAX_CLASSES 4
typedef struct {
  int ny, nx, raw_t;
  double fps;               /* camera frame rate = temporal fs */
  int window, stride;
  double f_lo_hz, f_hi_hz;  /* band */
  const void* block;        /* device frames [block_frames][ny][nx] */
  int block_frames;
  int max_active;
  int ring_frames;          /* 0 = 8 W */
} hv_replay_class;

typedef struct {
  int nclass;
  hv_replay_class cls[HV_REPLAY_MAX_CLASSES];
  double wavelength_m, pitch_m, z_lo_m, z_hi_m;
  int prec;
  double arrival_hz, mean_life_s, duration_s, warmup_s;
  int packet_frames;
  uint64_t seed;
} hv_replay_config;

typedef struct {
  int64_t frames_offered, frames_in, frames_dropped, windows_done;
  int64_t streams_admitted, streams_refused;
  int64_t lat_p50_ns, lat_p99_ns, lat_max_ns, latency_samples;
  double seconds, frames_per_s;
  int64_t errors;
} hv_replay_result;

hv_status hv_replay_run(hv_ctx* ctx, const hv_replay_config* cfg, hv_replay_result* res);

/* ---------------------------------------------------------------- post-processing */

/* Post-processing of rendered images (Sec. III-B.2), in the paper's order:
 *   convolution: out = in * kernel (2-D linear convolution, same size,
 *     zero outside the image); kernel_size odd, at most 31 (0 = skip),
 *     kernel: HOST [k][k] row-major float32;
 *   renormalise != 0: each image divided by its own spatial mean;
 *   registration (ref_count > 0): reference = mean of the first ref_count
 *     images times a centred disk of radius mask_radius * min(nx, ny) / 2;
 *     each image is shifted circularly by minus the peak of its circular
 *     cross-correlation c(s) = sum_p img(p + s) ref(p) (ties: lowest flat
 *     index); sides must be supported frame sides;
 *   accumulate > 1: moving average out_j = mean(in_max(0, j-A+1) .. in_j).
 * in, out: device [count][ny][nx] float32 (may not overlap); shifts: device
 * [count][2] int (dy, dx) of the registration, nullable. */
typedef struct {
  int kernel_size;
  const float* kernel;
  int renormalise;
  int ref_count;
  double mask_radius;
  int accumulate;
} hv_post;

hv_status hv_postprocess(hv_ctx* ctx, const float* in, int count, int ny, int nx, const hv_post* cfg, float* out,
                         int* shifts, void* hip_stream);

/* Magnitude or argument image of the windowed spectrum over a range of
 * temporal indices (Sec. III-B.1: besides the moments, the value rendered
 * per pixel may be the magnitude or the argument over a given index range):
 *   HV_IMG_MAGNITUDE  out[j][p] = sum_k |spec[j][k][p]|
 *   HV_IMG_ARGUMENT   out[j][p] = arg(sum_k spec[j][k][p]), in [-pi, pi]
 * (for a one-bin range, |S_k| and arg(S_k)).  spec: device [nwin][nbins]
 * [ny][nx] c64 -- the output of hv_stft_bins, or any range of its bins
 * held contiguously; out: device [nwin][ny][nx] float32.  FP32 arithmetic.
 * HV_ERR_ARG for an unknown kind or NULL pointers, HV_ERR_SHAPE for
 * nwin outside [0, 65535] or non-positive sizes; nwin = 0 does nothing. */
typedef enum { HV_IMG_MAGNITUDE = 0, HV_IMG_ARGUMENT = 1 } hv_image_kind;
hv_status hv_bins_image(hv_ctx* ctx, const void* spec, int nwin, int nbins, int ny, int nx, int kind, float* out,
                        void* hip_stream);

/* ---------------------------------------------------------------- .holo files */

/* The .holo file (Sec. IV, Holofile system) for file-mode replay: a 64-byte
 * header ("HOLO", version, bits per pixel, width, height, image count, data
 * size, endianness, data type; little-endian fields, zero padding), the
 * images as one stream, an optional JSON footer.  Host-side calls on plain
 * host memory; no device work. */
typedef struct {
  uint16_t version;         /* 7; 0 on write means 7 */
  uint16_t bits_per_pixel;  /* 8 or 16 */
  uint32_t width, height, image_count;
  uint64_t data_size;       /* filled on read; computed on write */
  uint8_t endianness;       /* of the pixel data: 0 little, 1 big */
  uint8_t data_type;        /* 0 raw, 1 processed */
} hv_holo_header;

/* Reads and checks the header (HV_ERR_ARG: missing file, bad magic, other bit
 * depths, inconsistent data size); footer_bytes (nullable) receives the
 * footer length. */
hv_status hv_holo_read_header(const char* path, hv_holo_header* out, uint64_t* footer_bytes);
/* Images [first, first + count) into host_dst (count * width * height *
 * bits/8 bytes; pinned memory lets the result go straight to the device),
 * 16-bit pixels in native (little-endian) order. */
hv_status hv_holo_read_frames(const char* path, int64_t first, int64_t count, void* host_dst);
/* The footer text, NUL-terminated, truncated to cap - 1 bytes. */
hv_status hv_holo_read_footer(const char* path, char* dst, uint64_t cap);
/* Writes header, images (host memory, native order; swapped when
 * endianness = 1) and the footer (nullable JSON text). */
hv_status hv_holo_write(const char* path, const hv_holo_header* header, const void* host_frames,
                        const char* footer_json);

/* ---------------------------------------------------------------- autofocus */
/* Learned autofocus with a brute-force scan as fallback and as a check (the
 * paper names machine-learning inference as a plug-in for the pipeline,
 * Sec. VIII).  Holograms are 256 x 256 uint8 off-axis interferograms whose
 * reference carrier is (+1/4, +1/4) cycles/pixel, so the object term sits at
 * (-1/4, -1/4).  All pointers are device memory unless marked host. */
typedef struct hv_af_model hv_af_model;

/* Number of network parameters (30,306): conv3x3 1->32, 3 x conv3x3 32->32
 * (weights [co][ci][3][3] then bias), FC 32->64, FC 64->2 (weights [out][in]
 * then bias), in that order. */
int hv_af_nparams(void);

/* Network inputs: log(1 + |DFT2(h - mean h)|), the 64 x 64 bins centred on DC
 * (fftshift order), standardised per crop to mean 0 and standard deviation 1.
 * out: [n][64][64] fp16 (out_half = 1) or float32. */
hv_status hv_af_crops(hv_ctx* ctx, const uint8_t* holo, int n, int ny, int nx, void* out, int out_half,
                      void* hip_stream);

/* Brute-force scan: n_candidates distances z_c evenly spaced in [z_lo, z_hi];
 * for each, the +1-order sub-band (64 x 64 bins around the object carrier,
 * masked to radius 0.1 cycles/pixel) times exp(-2 pi i z_c sqrt(1/lambda^2 -
 * |f|^2)) at the demodulated frequencies f, inverse DFT at 64 x 64, amplitude
 * A, sharpness = population variance of sqrt(gx^2 + gy^2) with forward
 * differences on the 63 x 63 interior.  z_out[n] = the candidate with the
 * largest sharpness (ties to the lowest z); scores_out [n][n_candidates]
 * nullable. */
hv_status hv_af_scan(hv_ctx* ctx, const uint8_t* holo, int n, int ny, int nx, double wavelength_m, double pitch_m,
                     double z_lo_m, double z_hi_m, int n_candidates, float* z_out, float* scores_out,
                     void* hip_stream);

/* Model with its Adam state and training buffers for up to max_batch crops.
 * init_params: host float32[hv_af_nparams()].  The network predicts the
 * normalised distance (z - z_mean) / z_scale and s = log sigma^2 of it. */
hv_status hv_af_model_create(hv_ctx* ctx, const float* init_params, int max_batch, double z_mean, double z_scale,
                             hv_af_model** out);
void hv_af_model_destroy(hv_af_model* model);
/* Copy parameters, Adam moments (host float32[nparams], nullable) and step out
 * of / into the model (checkpoint and resume). */
hv_status hv_af_model_state(hv_af_model* model, float* params, float* m, float* v, int64_t* step);
hv_status hv_af_model_load(hv_af_model* model, const float* params, const float* m, const float* v, int64_t step);

/* Raw network output [batch][2] = (normalised z, log sigma^2) for fp16 crops
 * (FP32 arithmetic: the forward pass of training). */
hv_status hv_af_forward(hv_af_model* model, const void* crops, int batch, float* out, void* hip_stream);
/* The same output from the inference kernels that hv_af_predict runs: each
 * convolution as an implicit GEMM on the matrix cores with fp16 weights and
 * activations and FP32 accumulation, the first layer evaluated inside the
 * second layer's kernel, the pooling fused into the last convolution.
 * Agrees with hv_af_forward to fp16 rounding.  batch <= max(max_batch,
 * 1024) (HV_ERR_SHAPE otherwise). */
hv_status hv_af_infer(hv_af_model* model, const void* crops, int batch, float* out, void* hip_stream);
/* Mean Gaussian NLL 0.5 (s + (z_n - zhat)^2 e^{-s}) over the batch (loss,
 * device float[1], nullable) and its gradient with respect to every parameter
 * (grad, device float32[nparams]); labels z_m in metres. */
hv_status hv_af_loss_grad(hv_af_model* model, const void* crops, const float* z_m, int batch, float* loss,
                          float* grad, void* hip_stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected) on that gradient. */
hv_status hv_af_train_step(hv_af_model* model, const void* crops, const float* z_m, int batch, float lr,
                           float* loss, void* hip_stream);
/* The same step from 256 x 256 u8 holograms (device [batch][256][256]): their
 * crops (hv_af_crops, fp16) into a workspace of the context, then
 * hv_af_train_step.  batch <= the model's max_batch (HV_ERR_SHAPE). */
hv_status hv_af_train_step_holo(hv_af_model* model, const uint8_t* holo, const float* z_m, int batch, float lr,
                                float* loss, void* hip_stream);
/* The scan of hv_af_scan over per-hologram ranges: n_candidates distances
 * evenly spaced in [z_lo[i], z_hi[i]] (device float32 [n] each) for
 * hologram i; transfer functions from an FP64 table of
 * 2 pi sqrt(1/lambda^2 - |f|^2); the phase is reduced modulo 2 pi in FP64 on
 * the device and its sine and cosine taken in FP32.
 * z_out[n], scores_out [n][n_candidates] (nullable). */
hv_status hv_af_scan_ranges(hv_ctx* ctx, const uint8_t* holo, int n, int ny, int nx, double wavelength_m,
                            double pitch_m, const float* z_lo, const float* z_hi, int n_candidates, float* z_out,
                            float* scores_out, void* hip_stream);
/* Predicted z (metres) and sigma for n holograms (crops, then the inference
 * kernels of hv_af_infer).  With refine_candidates > 0 (>= 4) the network
 * seeds a local scan from the same spectrum: refine_candidates / 2
 * candidates over z +- refine_k sigma (clipped to [0.05, 0.5] m, at least
 * 10 mm wide), then the rest over one coarse step on each side of the best;
 * z_out is that scan's best candidate.  Every hologram with sigma > tau_m is
 * re-estimated by hv_af_scan (128 candidates in [0.05, 0.5] m) and flagged
 * in used_fallback[n] (nullable).  *n_fallback (host, nullable) receives
 * their count.  Synchronises the stream. */
hv_status hv_af_predict(hv_af_model* model, const uint8_t* holo, int n, double wavelength_m, double pitch_m,
                        float tau_m, int refine_candidates, float refine_k, float* z_out, float* sigma_out,
                        int* used_fallback, int* n_fallback, void* hip_stream);
/* Training holograms from the project's own forward model: counter-based
 * complex noise band-limited to a 0.09 cycles/pixel pupil, times 3-8 soft
 * disks (parameters drawn from seed and the hologram index), propagated by
 * +z_m[i] with hv_propagate (runs of equal z share a call), reference of
 * amplitude 3 x rms tilted (+1/4, +1/4) cycles/pixel, mean 64 DN, photon
 * noise (normal approximation), uint8.  z_m: host double[n]. */
hv_status hv_af_synthesize(hv_ctx* ctx, int n, const double* z_m, double wavelength_m, double pitch_m, uint64_t seed,
                           int64_t index_base, uint8_t* out, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* HV_H */
