"""ctypes binding of libhv.so (include/hv.h), same names as the C-ABI.

Argument marshalling only: torch supplies device memory and the HIP stream,
every step of the hot path runs in the library's kernels.  Importing this
module loads the in-tree ``libhv.so`` and raises if it is missing -- there is
no fallback path.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhv.so")

HV_OK, HV_ERR_ARG, HV_ERR_SHAPE, HV_ERR_NOMEM, HV_ERR_BUDGET, HV_ERR_DEVICE, HV_ERR_OVERFLOW, HV_ERR_STATE = (
    0, -1, -2, -3, -4, -5, -6, -7)
HV_U8, HV_U16, HV_C64, HV_C32H = 0, 1, 3, 4
HV_AS, HV_FRESNEL = 0, 1
HV_PREC_FP32, HV_PREC_MIXED = 0, 1
HV_ORDER_AUTO, HV_ORDER_FRAMES_FIRST, HV_ORDER_BAND_FIRST = 0, 1, 2
HV_IMG_MAGNITUDE, HV_IMG_ARGUMENT = 0, 1

_STATUS_NAMES = {0: "HV_OK", -1: "HV_ERR_ARG", -2: "HV_ERR_SHAPE", -3: "HV_ERR_NOMEM", -4: "HV_ERR_BUDGET",
                 -5: "HV_ERR_DEVICE", -6: "HV_ERR_OVERFLOW", -7: "HV_ERR_STATE"}


class HvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(python -m paper_2508_03911_amd.build)")
    return C.CDLL(LIB_PATH)


lib = _load()


class hv_optics(C.Structure):
    _fields_ = [("wavelength_m", C.c_double), ("pitch_x_m", C.c_double), ("pitch_y_m", C.c_double),
                ("z_m", C.c_double), ("method", C.c_int), ("highpass_cpp", C.c_double)]


class hv_holo_header(C.Structure):
    _fields_ = [("version", C.c_uint16), ("bits_per_pixel", C.c_uint16), ("width", C.c_uint32),
                ("height", C.c_uint32), ("image_count", C.c_uint32), ("data_size", C.c_uint64),
                ("endianness", C.c_uint8), ("data_type", C.c_uint8)]


class hv_post(C.Structure):
    _fields_ = [("kernel_size", C.c_int), ("kernel", C.c_void_p), ("renormalise", C.c_int), ("ref_count", C.c_int),
                ("mask_radius", C.c_double), ("accumulate", C.c_int)]


class hv_temporal(C.Structure):
    _fields_ = [("window", C.c_int), ("stride", C.c_int), ("fs_hz", C.c_double), ("f_lo_hz", C.c_double),
                ("f_hi_hz", C.c_double), ("symmetric_band", C.c_int)]


class hv_stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "frames_in", "frames_dropped", "windows_done", "streams_admitted", "streams_refused",
        "images_overwritten", "latency_samples", "lat_p50_ns", "lat_p99_ns", "lat_max_ns", "admitted_bytes",
        "device_errors")]


HV_REPLAY_MAX_CLASSES = 4


class hv_replay_class(C.Structure):
    _fields_ = [("ny", C.c_int), ("nx", C.c_int), ("raw_t", C.c_int), ("fps", C.c_double), ("window", C.c_int),
                ("stride", C.c_int), ("f_lo_hz", C.c_double), ("f_hi_hz", C.c_double), ("block", C.c_void_p),
                ("block_frames", C.c_int), ("max_active", C.c_int), ("ring_frames", C.c_int)]


class hv_replay_config(C.Structure):
    _fields_ = [("nclass", C.c_int), ("cls", hv_replay_class * HV_REPLAY_MAX_CLASSES),
                ("wavelength_m", C.c_double), ("pitch_m", C.c_double), ("z_lo_m", C.c_double),
                ("z_hi_m", C.c_double), ("prec", C.c_int), ("arrival_hz", C.c_double),
                ("mean_life_s", C.c_double), ("duration_s", C.c_double), ("warmup_s", C.c_double),
                ("packet_frames", C.c_int), ("seed", C.c_uint64)]


class hv_replay_result(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "frames_offered", "frames_in", "frames_dropped", "windows_done", "streams_admitted", "streams_refused",
        "lat_p50_ns", "lat_p99_ns", "lat_max_ns", "latency_samples")] + [
        ("seconds", C.c_double), ("frames_per_s", C.c_double), ("errors", C.c_int64)]


_P = C.c_void_p
_I = C.c_int
_sig = {
    "hv_last_error": (C.c_char_p, []),
    "hv_ctx_create": (_I, [_I, C.c_size_t, C.POINTER(_P)]),
    "hv_ctx_destroy": (None, [_P]),
    "hv_ctx_workspace_bytes": (C.c_size_t, [_P]),
    "hv_ctx_set_chunk_frames": (_I, [_P, _I]),
    "hv_ctx_set_stft_order": (_I, [_P, _I]),
    "hv_ctx_set_timing": (_I, [_P, _I]),
    "hv_ctx_kernel_time": (_I, [_P, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_long)]),
    "hv_band_bins": (_I, [C.POINTER(hv_temporal), C.POINTER(_I), C.POINTER(_I), C.POINTER(C.c_double)]),
    "hv_propagate": (_I, [_P, _P, _I, _I, _I, _I, C.POINTER(hv_optics), _I, _I, _P, _P]),
    "hv_field_scale": (_I, [_I, _I, _I, C.POINTER(C.c_float)]),
    "hv_stft_moments": (_I, [_P, _P, _I, _I, _I, _I, C.POINTER(hv_optics), C.POINTER(hv_temporal), _I, _P, _P, _P,
                             _P]),
    "hv_stft_moments_noalloc": (_I, [_P, _P, _I, _I, _I, _I, C.POINTER(hv_optics), C.POINTER(hv_temporal), _I, _P,
                                     _P, _P, _P]),
    "hv_stft_bins": (_I, [_P, _P, _I, _I, _I, _I, C.POINTER(hv_optics), C.POINTER(hv_temporal), _I, _P, _P]),
    "hv_stft_volume": (_I, [_P, _P, _I, _I, _I, _I, C.POINTER(hv_optics), _I, _I, _I, _P, _P]),
    "hv_postprocess": (_I, [_P, _P, _I, _I, _I, C.POINTER(hv_post), _P, _P, _P]),
    "hv_bins_image": (_I, [_P, _P, _I, _I, _I, _I, _I, _P, _P]),
    "hv_holo_read_header": (_I, [C.c_char_p, C.POINTER(hv_holo_header), C.POINTER(C.c_uint64)]),
    "hv_holo_read_frames": (_I, [C.c_char_p, C.c_int64, C.c_int64, _P]),
    "hv_holo_read_footer": (_I, [C.c_char_p, C.c_char_p, C.c_uint64]),
    "hv_holo_write": (_I, [C.c_char_p, C.POINTER(hv_holo_header), _P, C.c_char_p]),
    "hv_stft_moments_host": (_I, [_P, _P, _I, _I, _I, _I, C.POINTER(hv_optics), C.POINTER(hv_temporal), _I, _P,
                                  _P, _P, _P]),
    "hv_stream_open": (_I, [_P, _I, _I, _I, C.POINTER(hv_optics), C.POINTER(hv_temporal), _I, _I, C.POINTER(_P)]),
    "hv_stream_push": (_I, [_P, _P, _I, C.POINTER(C.c_int64)]),
    "hv_stream_pop": (_I, [_P, _P, _P, _P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "hv_stream_close": (_I, [_P]),
    "hv_stream_frames": (_I, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "hv_ctx_stats": (_I, [_P, C.POINTER(hv_stats)]),
    "hv_ctx_stats_reset": (_I, [_P]),
    "hv_replay_run": (_I, [_P, C.POINTER(hv_replay_config), C.POINTER(hv_replay_result)]),
    "hv_af_nparams": (_I, []),
    "hv_af_crops": (_I, [_P, _P, _I, _I, _I, _P, _I, _P]),
    "hv_af_scan": (_I, [_P, _P, _I, _I, _I, C.c_double, C.c_double, C.c_double, C.c_double, _I, _P, _P, _P]),
    "hv_af_model_create": (_I, [_P, C.POINTER(C.c_float), _I, C.c_double, C.c_double, C.POINTER(_P)]),
    "hv_af_model_destroy": (None, [_P]),
    "hv_af_model_state": (_I, [_P, C.POINTER(C.c_float), C.POINTER(C.c_float), C.POINTER(C.c_float),
                               C.POINTER(C.c_int64)]),
    "hv_af_model_load": (_I, [_P, C.POINTER(C.c_float), C.POINTER(C.c_float), C.POINTER(C.c_float), C.c_int64]),
    "hv_af_forward": (_I, [_P, _P, _I, _P, _P]),
    "hv_af_infer": (_I, [_P, _P, _I, _P, _P]),
    "hv_af_loss_grad": (_I, [_P, _P, _P, _I, _P, _P, _P]),
    "hv_af_train_step": (_I, [_P, _P, _P, _I, C.c_float, _P, _P]),
    "hv_af_train_step_holo": (_I, [_P, _P, _P, _I, C.c_float, _P, _P]),
    "hv_af_predict": (_I, [_P, _P, _I, C.c_double, C.c_double, C.c_float, _I, C.c_float, _P, _P, _P, C.POINTER(_I),
                           _P]),
    "hv_af_scan_ranges": (_I, [_P, _P, _I, _I, _I, C.c_double, C.c_double, _P, _P, _I, _P, _P, _P]),
    "hv_af_synthesize": (_I, [_P, _I, C.POINTER(C.c_double), C.c_double, C.c_double, C.c_uint64, C.c_int64, _P,
                              _P]),
    "hv_pca": (_I, [_P, _P, _I, _I, _I, _I, C.POINTER(hv_optics), _I, _I, _I, _I, _I, _P, _P, _P, _P, _P]),
    "hv_ssa_moments": (_I, [_P, _P, _I, _I, _I, _I, C.POINTER(hv_optics), C.POINTER(hv_temporal), _I, _I, _I, _P,
                            _P, _P, _P, _P, _P]),
}
for _name, (_res, _args) in _sig.items():
    _fn = getattr(lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


def last_error() -> str:
    return lib.hv_last_error().decode()


def _check(status: int):
    if status != HV_OK:
        raise HvError(status, last_error())


@dataclass(frozen=True)
class Optics:
    wavelength: float
    pitch_x: float
    pitch_y: float
    z: float
    method: int = HV_AS
    highpass: float = 0.0

    def c(self) -> hv_optics:
        return hv_optics(self.wavelength, self.pitch_x, self.pitch_y, self.z, self.method, self.highpass)


@dataclass(frozen=True)
class Temporal:
    window: int
    stride: int
    fs: float
    f_lo: float
    f_hi: float
    symmetric: bool = False

    def c(self) -> hv_temporal:
        return hv_temporal(self.window, self.stride, self.fs, self.f_lo, self.f_hi, int(self.symmetric))


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.uint8:
        return HV_U8
    if t.dtype in (torch.int16, getattr(torch, "uint16", torch.int16)):
        return HV_U16
    if t.dtype == torch.complex64:
        return HV_C64
    raise TypeError(f"unsupported input dtype {t.dtype}")


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _frames(x: torch.Tensor, host: bool = False):
    if x.dim() != 3:
        raise ValueError("expected a [frames, ny, nx] tensor")
    if host:
        if x.is_cuda or not x.is_pinned() or not x.is_contiguous():
            raise ValueError("input must be a contiguous pinned host tensor")
    elif not x.is_cuda or not x.is_contiguous():
        raise ValueError("input must be a contiguous device tensor")
    return x.shape[0], x.shape[1], x.shape[2]


def holo_read(path, first: int = 0, count: int | None = None, pin: bool = False):
    """(header dict, uint8/uint16 frames [count][height][width] on the host,
    footer text or None) of a .holo file; pin=True reads into pinned memory."""
    h = hv_holo_header()
    fb = C.c_uint64(0)
    p = os.fsencode(path)
    _check(lib.hv_holo_read_header(p, C.byref(h), C.byref(fb)))
    n = h.image_count - first if count is None else count
    dt = torch.uint8 if h.bits_per_pixel == 8 else torch.int16
    frames = torch.empty((n, h.height, h.width), dtype=dt, pin_memory=pin)
    _check(lib.hv_holo_read_frames(p, first, n, C.c_void_p(frames.data_ptr())))
    footer = None
    if fb.value:
        buf = C.create_string_buffer(fb.value + 1)
        _check(lib.hv_holo_read_footer(p, buf, fb.value + 1))
        footer = buf.value.decode()
    head = {f: getattr(h, f) for f, _ in hv_holo_header._fields_}
    return head, frames, footer


def holo_write(path, frames: torch.Tensor, footer: str | None = None, data_type: int = 0, endianness: int = 0):
    """Write host frames [n][height][width] (uint8, or 16-bit) as a .holo file."""
    if frames.is_cuda or frames.dim() != 3 or not frames.is_contiguous():
        raise ValueError("frames must be a contiguous [n, h, w] host tensor")
    bits = 8 * frames.element_size()
    h = hv_holo_header(7, bits, frames.shape[2], frames.shape[1], frames.shape[0], 0, endianness, data_type)
    _check(lib.hv_holo_write(os.fsencode(path), C.byref(h), C.c_void_p(frames.data_ptr()),
                             footer.encode() if footer is not None else None))


def band_bins(temporal: Temporal):
    tp = temporal.c()
    n = C.c_int(0)
    _check(lib.hv_band_bins(C.byref(tp), C.byref(n), None, None))
    bins = (C.c_int * max(1, n.value))()
    freqs = (C.c_double * max(1, n.value))()
    _check(lib.hv_band_bins(C.byref(tp), C.byref(n), bins, freqs))
    return list(bins)[:n.value], list(freqs)[:n.value]


def field_scale(in_t: int, ny: int, nx: int) -> float:
    """The power of two an HV_C32H field holds U multiplied by."""
    v = C.c_float(0)
    _check(lib.hv_field_scale(in_t, ny, nx, C.byref(v)))
    return v.value


class Context:
    """One hv_ctx on a HIP device (plans and workspaces live here)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        self.device = device
        h = C.c_void_p()
        _check(lib.hv_ctx_create(device, hbm_budget, C.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            lib.hv_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self) -> int:
        return lib.hv_ctx_workspace_bytes(self.handle)

    def set_chunk_frames(self, frames: int):
        _check(lib.hv_ctx_set_chunk_frames(self.handle, frames))

    def set_stft_order(self, order: int):
        """HV_ORDER_AUTO, HV_ORDER_FRAMES_FIRST or HV_ORDER_BAND_FIRST."""
        _check(lib.hv_ctx_set_stft_order(self.handle, order))

    def set_timing(self, on: bool):
        """Bracket every kernel launch with HIP events (clears the totals)."""
        _check(lib.hv_ctx_set_timing(self.handle, int(on)))

    def kernel_time(self, name: str):
        """(total milliseconds, launches) of kernel `name` since timing was set."""
        ms = C.c_double(0)
        n = C.c_long(0)
        _check(lib.hv_ctx_kernel_time(self.handle, name.encode(), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def _dev(self):
        return torch.device("cuda", self.device)

    # ---------------------------------------------------------------- spatial
    def hv_propagate(self, x: torch.Tensor, optics: Optics, prec: int = HV_PREC_FP32, out=None,
                     out_dtype: int = HV_C64) -> torch.Tensor:
        """The field as complex64 [n, ny, nx] (HV_C64), or as float16
        [n, ny, nx, 2] (re, im) holding U * field_scale(...) (HV_C32H)."""
        n, ny, nx = _frames(x)
        if out is None:
            if out_dtype == HV_C32H:
                out = torch.empty((n, ny, nx, 2), dtype=torch.float16, device=x.device)
            else:
                out = torch.empty((n, ny, nx), dtype=torch.complex64, device=x.device)
        want = (n, ny, nx, 2) if out_dtype == HV_C32H else (n, ny, nx)
        want_t = torch.float16 if out_dtype == HV_C32H else torch.complex64
        if out_dtype in (HV_C64, HV_C32H) and (tuple(out.shape) != want or out.dtype != want_t
                                               or not out.is_contiguous()):
            raise ValueError(f"out must be a contiguous {want_t} tensor of shape {want}")
        op = optics.c()
        _check(lib.hv_propagate(self.handle, _ptr(x), _dtype_code(x), n, ny, nx, C.byref(op), prec, out_dtype,
                                _ptr(out), _stream(x.device)))
        return out

    # ---------------------------------------------------------------- temporal
    def n_windows(self, n: int, temporal: Temporal) -> int:
        return 0 if n < temporal.window else (n - temporal.window) // temporal.stride + 1

    def hv_stft_moments(self, x: torch.Tensor, optics: Optics | None, temporal: Temporal,
                        prec: int = HV_PREC_FP32, want=(True, True, True), out=None):
        n, ny, nx = _frames(x)
        j = self.n_windows(n, temporal)
        if out is None:
            out = [torch.empty((j, ny, nx), dtype=torch.float32, device=x.device) if w else None for w in want]
        op = optics.c() if optics is not None else None
        tp = temporal.c()
        _check(lib.hv_stft_moments(self.handle, _ptr(x), _dtype_code(x), n, ny, nx,
                                   C.byref(op) if op is not None else None, C.byref(tp), prec,
                                   _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _stream(x.device)))
        return out

    def hv_stft_moments_noalloc(self, x: torch.Tensor, optics: Optics | None, temporal: Temporal,
                                prec: int, out):
        """The moments into caller-allocated out = [m0, m1, m2] (each
        [J][ny][nx] float32 or None) with the library's static scratch as
        workspace: nothing is allocated by this call."""
        n, ny, nx = _frames(x)
        op = optics.c() if optics is not None else None
        tp = temporal.c()
        _check(lib.hv_stft_moments_noalloc(self.handle, _ptr(x), _dtype_code(x), n, ny, nx,
                                           C.byref(op) if op is not None else None, C.byref(tp), prec,
                                           _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _stream(x.device)))
        return out

    def hv_stft_bins(self, x: torch.Tensor, optics: Optics | None, temporal: Temporal,
                     prec: int = HV_PREC_FP32, out=None) -> torch.Tensor:
        n, ny, nx = _frames(x)
        j = self.n_windows(n, temporal)
        nb = len(band_bins(temporal)[0])
        if out is None:
            out = torch.empty((j, nb, ny, nx), dtype=torch.complex64, device=x.device)
        op = optics.c() if optics is not None else None
        tp = temporal.c()
        _check(lib.hv_stft_bins(self.handle, _ptr(x), _dtype_code(x), n, ny, nx,
                                C.byref(op) if op is not None else None, C.byref(tp), prec, _ptr(out),
                                _stream(x.device)))
        return out

    def hv_stft_moments_host(self, x: torch.Tensor, optics: Optics, temporal: Temporal,
                             prec: int = HV_PREC_FP32, out=None, stream=None):
        """x: pinned host frames; out: pinned host tensors [J][ny][nx] float32
        (allocated pinned when None).  Synchronise ``stream`` (default: the
        current device stream) before reading ``out``."""
        n, ny, nx = _frames(x, host=True)
        if out is not None and any(o.is_cuda or not o.is_pinned() or not o.is_contiguous() for o in out):
            raise ValueError("outputs must be contiguous pinned host tensors")
        j = self.n_windows(n, temporal)
        if out is None:
            out = [torch.empty((j, ny, nx), dtype=torch.float32, pin_memory=True) for _ in range(3)]
        op, tp = optics.c(), temporal.c()
        st = stream.cuda_stream if stream is not None else torch.cuda.current_stream().cuda_stream
        _check(lib.hv_stft_moments_host(self.handle, _ptr(x), _dtype_code(x), n, ny, nx, C.byref(op), C.byref(tp),
                                        prec, _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), C.c_void_p(st)))
        return out

    def hv_postprocess(self, images: torch.Tensor, kernel=None, renormalise: bool = False, ref_count: int = 0,
                       mask_radius: float = 1.0, accumulate: int = 1):
        """Convolution (kernel: host [k][k] array), re-normalisation,
        registration and moving average of device images [count][ny][nx]
        float32; returns (images, shifts [count][2] int32 or None)."""
        if not images.is_cuda or images.dim() != 3 or images.dtype != torch.float32 or not images.is_contiguous():
            raise ValueError("images must be a contiguous [count, ny, nx] float32 device tensor")
        count, ny, nx = images.shape
        k = None
        if kernel is not None:
            k = torch.as_tensor(kernel, dtype=torch.float32).contiguous().cpu()
        cfg = hv_post(0 if k is None else k.shape[0], None if k is None else C.c_void_p(k.data_ptr()),
                      int(renormalise), ref_count, mask_radius, accumulate)
        out = torch.empty_like(images)
        shifts = torch.empty((count, 2), dtype=torch.int32, device=images.device) if ref_count > 0 else None
        _check(lib.hv_postprocess(self.handle, _ptr(images), count, ny, nx, C.byref(cfg), _ptr(out), _ptr(shifts),
                                  _stream(images.device)))
        return out, shifts

    def hv_bins_image(self, spec: torch.Tensor, kind: int, out=None) -> torch.Tensor:
        """Magnitude (HV_IMG_MAGNITUDE: sum of moduli) or argument
        (HV_IMG_ARGUMENT: argument of the sum) over the bins of a device
        spectrum [J][nbins][ny][nx] complex64; returns [J][ny][nx] float32."""
        if not spec.is_cuda or spec.dim() != 4 or spec.dtype != torch.complex64 or not spec.is_contiguous():
            raise ValueError("spec must be a contiguous [J, nbins, ny, nx] complex64 device tensor")
        j, nb, ny, nx = spec.shape
        if out is None:
            out = torch.empty((j, ny, nx), dtype=torch.float32, device=spec.device)
        _check(lib.hv_bins_image(self.handle, _ptr(spec), j, nb, ny, nx, kind, _ptr(out), _stream(spec.device)))
        return out

    def hv_stft_volume(self, x: torch.Tensor, optics: Optics | None, window: int, stride: int,
                       prec: int = HV_PREC_FP32, out=None) -> torch.Tensor:
        n, ny, nx = _frames(x)
        j = 0 if n < window else (n - window) // stride + 1
        if out is None:
            out = torch.empty((j, window, ny, nx), dtype=torch.float32, device=x.device)
        op = optics.c() if optics is not None else None
        _check(lib.hv_stft_volume(self.handle, _ptr(x), _dtype_code(x), n, ny, nx,
                                  C.byref(op) if op is not None else None, window, stride, prec, _ptr(out),
                                  _stream(x.device)))
        return out

    # ---------------------------------------------------------------- PCA
    def hv_pca(self, x: torch.Tensor, optics: Optics | None, window: int, stride: int, comp_lo: int = 1,
               comp_hi: int | None = None, prec: int = HV_PREC_FP32, want_eig=True, want_cov=False):
        n, ny, nx = _frames(x)
        if comp_hi is None:
            comp_hi = window - 1
        j = 0 if n < window else (n - window) // stride + 1
        m0 = torch.empty((j, ny, nx), dtype=torch.float32, device=x.device)
        ev = torch.empty((j, window), dtype=torch.float64, device=x.device) if want_eig else None
        cov = torch.empty((j, window, window), dtype=torch.complex128, device=x.device) if want_cov else None
        off = torch.empty((j,), dtype=torch.float64, device=x.device)
        op = optics.c() if optics is not None else None
        _check(lib.hv_pca(self.handle, _ptr(x), _dtype_code(x), n, ny, nx, C.byref(op) if op is not None else None,
                          window, stride, comp_lo, comp_hi, prec, _ptr(m0), _ptr(ev), _ptr(cov), _ptr(off),
                          _stream(x.device)))
        return {"m0": m0, "eigvals": ev, "cov": cov, "offdiag": off}

    def hv_ssa_moments(self, x: torch.Tensor, optics: Optics | None, temporal: Temporal, comp_lo: int = 1,
                       comp_hi: int | None = None, prec: int = HV_PREC_FP32, out=None, want_eig=True):
        """SSA + FFT moments: dict with m0, m1, m2 [J][ny][nx], eigvals [J][W]
        and the Jacobi off-diagonal ratio [J]."""
        n, ny, nx = _frames(x)
        w = temporal.window
        if comp_hi is None:
            comp_hi = w - 1
        j = self.n_windows(n, temporal)
        if out is None:
            out = [torch.empty((j, ny, nx), dtype=torch.float32, device=x.device) for _ in range(3)]
        ev = torch.empty((j, w), dtype=torch.float64, device=x.device) if want_eig else None
        off = torch.empty((j,), dtype=torch.float64, device=x.device)
        op = optics.c() if optics is not None else None
        tp = temporal.c()
        _check(lib.hv_ssa_moments(self.handle, _ptr(x), _dtype_code(x), n, ny, nx,
                                  C.byref(op) if op is not None else None, C.byref(tp), comp_lo, comp_hi, prec,
                                  _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _ptr(ev), _ptr(off),
                                  _stream(x.device)))
        return {"m0": out[0], "m1": out[1], "m2": out[2], "eigvals": ev, "offdiag": off}


    # ---------------------------------------------------------------- serving loop
    def stats(self) -> dict:
        st = hv_stats()
        _check(lib.hv_ctx_stats(self.handle, C.byref(st)))
        return {n: getattr(st, n) for n, _ in hv_stats._fields_}

    def stats_reset(self):
        _check(lib.hv_ctx_stats_reset(self.handle))

    def hv_stream_open(self, ny: int, nx: int, raw_dtype, optics: Optics, temporal: Temporal,
                       prec: int = HV_PREC_FP32, ring_frames: int = 0) -> "Stream":
        code = HV_U8 if raw_dtype == torch.uint8 else HV_U16
        op, tp = optics.c(), temporal.c()
        h = C.c_void_p()
        _check(lib.hv_stream_open(self.handle, ny, nx, code, C.byref(op), C.byref(tp), prec, ring_frames,
                                  C.byref(h)))
        return Stream(self, h, ny, nx)

    def hv_replay_run(self, classes, *, wavelength, pitch, z_lo, z_hi, prec, arrival_hz, mean_life_s,
                      duration_s, warmup_s, packet_frames, seed) -> dict:
        """classes: list of dicts with ny, nx, raw_t, fps, window, stride, f_lo, f_hi, block (device
        tensor [frames, ny, nx]), max_active, ring_frames."""
        cfg = hv_replay_config()
        cfg.nclass = len(classes)
        for i, k in enumerate(classes):
            b = k["block"]
            cfg.cls[i] = hv_replay_class(k["ny"], k["nx"], _dtype_code(b), k["fps"], k["window"], k["stride"],
                                         k["f_lo"], k["f_hi"], C.c_void_p(b.data_ptr()), b.shape[0],
                                         k["max_active"], k.get("ring_frames", 0))
        cfg.wavelength_m, cfg.pitch_m, cfg.z_lo_m, cfg.z_hi_m = wavelength, pitch, z_lo, z_hi
        cfg.prec, cfg.arrival_hz, cfg.mean_life_s = prec, arrival_hz, mean_life_s
        cfg.duration_s, cfg.warmup_s, cfg.packet_frames, cfg.seed = duration_s, warmup_s, packet_frames, seed
        res = hv_replay_result()
        torch.cuda.synchronize()
        st = lib.hv_replay_run(self.handle, C.byref(cfg), C.byref(res))
        out = {n: getattr(res, n) for n, _ in hv_replay_result._fields_}
        _check(st)
        return out


    # ---------------------------------------------------------------- autofocus
    def hv_af_crops(self, holo: torch.Tensor, half: bool = True) -> torch.Tensor:
        n, ny, nx = _frames(holo)
        out = torch.empty((n, 64, 64), dtype=torch.float16 if half else torch.float32, device=holo.device)
        _check(lib.hv_af_crops(self.handle, _ptr(holo), n, ny, nx, _ptr(out), int(half), _stream(holo.device)))
        return out

    def hv_af_scan(self, holo: torch.Tensor, wavelength: float, pitch: float, z_lo: float = 0.05,
                   z_hi: float = 0.5, n_candidates: int = 128, want_scores: bool = False):
        n, ny, nx = _frames(holo)
        z = torch.empty(n, dtype=torch.float32, device=holo.device)
        sc = torch.empty((n, n_candidates), dtype=torch.float32, device=holo.device) if want_scores else None
        _check(lib.hv_af_scan(self.handle, _ptr(holo), n, ny, nx, wavelength, pitch, z_lo, z_hi, n_candidates,
                              _ptr(z), _ptr(sc), _stream(holo.device)))
        return z, sc

    def hv_af_scan_ranges(self, holo: torch.Tensor, wavelength: float, pitch: float, z_lo: torch.Tensor,
                          z_hi: torch.Tensor, n_candidates: int, want_scores: bool = False):
        """The scan over per-hologram ranges [z_lo[i], z_hi[i]] (device float32)."""
        n, ny, nx = _frames(holo)
        z = torch.empty(n, dtype=torch.float32, device=holo.device)
        sc = torch.empty((n, n_candidates), dtype=torch.float32, device=holo.device) if want_scores else None
        _check(lib.hv_af_scan_ranges(self.handle, _ptr(holo), n, ny, nx, wavelength, pitch, _ptr(z_lo), _ptr(z_hi),
                                     n_candidates, _ptr(z), _ptr(sc), _stream(holo.device)))
        return z, sc

    def hv_af_synthesize(self, z_m, wavelength: float, pitch: float, seed: int, index_base: int = 0):
        import numpy as np
        z = np.ascontiguousarray(np.asarray(z_m, dtype=np.float64))
        n = z.shape[0]
        out = torch.empty((n, 256, 256), dtype=torch.uint8, device=self._dev())
        _check(lib.hv_af_synthesize(self.handle, n, z.ctypes.data_as(C.POINTER(C.c_double)), wavelength, pitch,
                                    seed, index_base, _ptr(out), _stream(out.device)))
        return out

    def af_model(self, init_params, max_batch: int, z_mean: float, z_scale: float) -> "AfModel":
        return AfModel(self, init_params, max_batch, z_mean, z_scale)


class Stream:
    """An open serving-loop stream (hv_stream)."""

    def __init__(self, ctx: Context, handle, ny: int, nx: int):
        self.ctx, self.handle, self.ny, self.nx = ctx, handle, ny, nx

    @staticmethod
    def _ready(frames: torch.Tensor):
        if not frames.is_contiguous():
            raise ValueError("frames must be contiguous")
        # a device copy is ordered on the stream's queue: the caller's
        # producer work must be complete; host frames (pinned or pageable)
        # are uploaded and waited for inside the push
        if frames.is_cuda:
            torch.cuda.current_stream(frames.device).synchronize()

    def push(self, frames: torch.Tensor, arrival_ns=None):
        n = frames.shape[0]
        arr = None
        if arrival_ns is not None:
            arr = (C.c_int64 * n)(*[int(a) for a in arrival_ns])
        self._ready(frames)
        _check(lib.hv_stream_push(self.handle, _ptr(frames), n, arr))

    def try_push(self, frames: torch.Tensor) -> int:
        self._ready(frames)
        return lib.hv_stream_push(self.handle, _ptr(frames), frames.shape[0], None)

    def pop(self, m0=None, m1=None, m2=None):
        """Returns (t_last_arrival_ns, t_done_ns) or None when nothing is ready."""
        tl, td = C.c_int64(0), C.c_int64(0)
        st = lib.hv_stream_pop(self.handle, _ptr(m0), _ptr(m1), _ptr(m2), C.byref(tl), C.byref(td))
        if st == HV_ERR_STATE:
            return None
        _check(st)
        return tl.value, td.value

    def counters(self):
        a, b, c = C.c_int64(0), C.c_int64(0), C.c_int64(0)
        _check(lib.hv_stream_frames(self.handle, C.byref(a), C.byref(b), C.byref(c)))
        return {"pushed": a.value, "dropped": b.value, "windows_done": c.value}

    def close(self):
        if self.handle:
            _check(lib.hv_stream_close(self.handle))
            self.handle = None


def af_nparams() -> int:
    return lib.hv_af_nparams()


class AfModel:
    """hv_af_model: the autofocus CNN with its Adam state on the device."""

    def __init__(self, ctx: Context, init_params, max_batch: int, z_mean: float, z_scale: float):
        import numpy as np
        p = np.ascontiguousarray(np.asarray(init_params, dtype=np.float32))
        if p.size != af_nparams():
            raise ValueError(f"expected {af_nparams()} parameters, got {p.size}")
        h = C.c_void_p()
        _check(lib.hv_af_model_create(ctx.handle, p.ctypes.data_as(C.POINTER(C.c_float)), max_batch, z_mean,
                                      z_scale, C.byref(h)))
        self.ctx, self.handle, self.max_batch = ctx, h, max_batch

    def close(self):
        if self.handle:
            lib.hv_af_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, crops: torch.Tensor) -> torch.Tensor:
        out = torch.empty((crops.shape[0], 2), dtype=torch.float32, device=crops.device)
        _check(lib.hv_af_forward(self.handle, _ptr(crops), crops.shape[0], _ptr(out), _stream(crops.device)))
        return out

    def infer(self, crops: torch.Tensor) -> torch.Tensor:
        """hv_af_infer: the prediction kernels (fp16 matrix-core convolutions)."""
        out = torch.empty((crops.shape[0], 2), dtype=torch.float32, device=crops.device)
        _check(lib.hv_af_infer(self.handle, _ptr(crops), crops.shape[0], _ptr(out), _stream(crops.device)))
        return out

    def loss_grad(self, crops: torch.Tensor, z_m: torch.Tensor):
        loss = torch.empty(1, dtype=torch.float32, device=crops.device)
        grad = torch.empty(af_nparams(), dtype=torch.float32, device=crops.device)
        _check(lib.hv_af_loss_grad(self.handle, _ptr(crops), _ptr(z_m), crops.shape[0], _ptr(loss), _ptr(grad),
                                   _stream(crops.device)))
        return loss, grad

    def train_step(self, crops: torch.Tensor, z_m: torch.Tensor, lr: float, loss: torch.Tensor = None):
        _check(lib.hv_af_train_step(self.handle, _ptr(crops), _ptr(z_m), crops.shape[0], lr, _ptr(loss),
                                    _stream(crops.device)))
        return loss

    def train_step_holo(self, holo: torch.Tensor, z_m: torch.Tensor, lr: float, loss: torch.Tensor = None):
        """One Adam step from u8 holograms [batch, 256, 256] (crops taken inside)."""
        _check(lib.hv_af_train_step_holo(self.handle, _ptr(holo), _ptr(z_m), holo.shape[0], lr, _ptr(loss),
                                         _stream(holo.device)))
        return loss

    def state(self):
        import numpy as np
        n = af_nparams()
        p, m, v = (np.empty(n, np.float32) for _ in range(3))
        step = C.c_int64(0)
        f = C.POINTER(C.c_float)
        _check(lib.hv_af_model_state(self.handle, p.ctypes.data_as(f), m.ctypes.data_as(f), v.ctypes.data_as(f),
                                     C.byref(step)))
        return {"params": p, "m": m, "v": v, "step": step.value}

    def load(self, state):
        import numpy as np
        f = C.POINTER(C.c_float)
        arrs = [np.ascontiguousarray(np.asarray(state[k], np.float32)) for k in ("params", "m", "v")]
        _check(lib.hv_af_model_load(self.handle, *[a.ctypes.data_as(f) for a in arrs], int(state["step"])))

    def predict(self, holo: torch.Tensor, wavelength: float, pitch: float, tau: float, refine: int = 0,
                refine_k: float = 2.5):
        """(z, sigma, used_fallback, n_fallback); refine > 0 adds the local
        scan of `refine` candidates seeded by the network (z +- refine_k sigma)."""
        n = holo.shape[0]
        z = torch.empty(n, dtype=torch.float32, device=holo.device)
        sig = torch.empty(n, dtype=torch.float32, device=holo.device)
        used = torch.empty(n, dtype=torch.int32, device=holo.device)
        nf = C.c_int(0)
        _check(lib.hv_af_predict(self.handle, _ptr(holo), n, wavelength, pitch, tau, refine, refine_k, _ptr(z),
                                 _ptr(sig), _ptr(used), C.byref(nf), _stream(holo.device)))
        return z, sig, used, nf.value
