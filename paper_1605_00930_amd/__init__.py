"""Python binding of the MI355X reconstruction library (``libiwpp.so``).

Grayscale morphological reconstruction by dilation as an irregular wavefront
propagation (IWPP), after Gomes & Teodoro.  Every step runs in the HIP
kernels behind the C ABI declared in ``include/iwpp.h``; this module only
marshals torch tensors (device memory) and streams into those calls.  There
is no CPU fallback: if the library is not built, calls raise.

Tensors are 2-D ``torch.uint8`` or ``torch.int32`` on a ROCm device with unit
column stride; the marker is reconstructed in place.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libiwpp.so")

OK = 0
E_ARG = -1
E_MARKER_GT_MASK = -2
E_NOMEM = -3
E_HIP = -4
E_INCOMPLETE = -5
E_BUDGET = -6
E_INTERNAL = -7
E_TIMEOUT = -8
E_UNSUPPORTED = -9
E_SCRATCH = -10
U8, I32 = 0, 1
FLAG_CLAMP_MARKER = 1
FLAG_EROSION = 2


class IwppError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        msg = "%s (%d)" % (strerror(code) if _lib_obj else "error", code)
        if what:
            msg += ": " + what
        if code == E_HIP and _lib_obj:
            msg += ": " + _lib_obj.iwpp_last_error().decode()
        super().__init__(msg)


class Image(ctypes.Structure):
    _fields_ = [("marker", ctypes.c_void_p), ("mask", ctypes.c_void_p),
                ("H", ctypes.c_int64), ("W", ctypes.c_int64), ("ld", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("images", ctypes.c_int32),
                ("tiles", ctypes.c_int64), ("tile_visits", ctypes.c_int64),
                ("sweep_rounds", ctypes.c_int64), ("pixels_queued", ctypes.c_int64),
                ("queue_overflows", ctypes.c_int64), ("reprocessed", ctypes.c_int64),
                ("requeued", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("kernel_ms", ctypes.c_double), ("queue_iterations", ctypes.c_int64),
                ("idle_ms", ctypes.c_double), ("load_ms", ctypes.c_double),
                ("solve_ms", ctypes.c_double), ("store_ms", ctypes.c_double),
                ("sync_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: (float if t is ctypes.c_double else int)(getattr(self, k))
                for k, t in self._fields_}


class Params(ctypes.Structure):
    _fields_ = [("tile_h", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("max_tile_visits", ctypes.c_int64), ("order_seed", ctypes.c_uint32),
                ("spin_limit", ctypes.c_uint32), ("timing", ctypes.c_int32),
                ("seed_queue", ctypes.c_int32), ("queue_waves", ctypes.c_int32),
                ("bands", ctypes.c_int32), ("first_pass", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib_obj = None


def _load():
    """Load libiwpp.so (raises if it has not been built)."""
    global _lib_obj
    if _lib_obj is not None:
        return _lib_obj
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libiwpp.so is not built: run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint32
    P = ctypes.POINTER
    sig = {
        "iwpp_version": ([], i32),
        "iwpp_strerror": ([i32], ctypes.c_char_p),
        "iwpp_last_error": ([], ctypes.c_char_p),
        "iwpp_reconstruct": ([vp, vp, i64, i64, i32, i32], i32),
        "iwpp_reconstruct_async": ([P(Image), i32, i32, u32, P(Params), vp], i32),
        "iwpp_stream_status": ([vp, P(Stats)], i32),
        "iwpp_reconstruct_batched": ([P(Image), ctypes.c_int32, i32, i32, u32, P(Params), vp], i32),
        "iwpp_batch_create": ([P(Image), ctypes.c_int32, i32, i32, u32, P(Params), P(vp)], i32),
        "iwpp_batch_launch": ([vp, vp, i32], i32),
        "iwpp_batch_status": ([vp, P(Stats)], i32),
        "iwpp_batch_destroy": ([vp], i32),
        "iwpp_autotune": ([P(Image), i32, i32, vp, P(Params)], i32),
        "iwpp_server_create": ([ctypes.c_size_t, i32, i32, i32, i32, P(vp)], i32),
        "iwpp_server_submit": ([vp, P(Image), vp, vp, P(ctypes.c_uint64)], i32),
        "iwpp_server_wait": ([vp, ctypes.c_uint64, i64, P(ctypes.c_double)], i32),
        "iwpp_server_destroy": ([vp], i32),
        "iwpp_release_workspace": ([], i32),
        "iwpp_device_copy": ([vp, vp, ctypes.c_size_t, vp], i32),
        "iwpp_reconstruct_noalloc": ([P(Image), i32, i32, u32, P(Params), vp, vp], i32),
        "iwpp_fill_holes_async": ([vp, vp, i64, i64, i64, i32, i32, P(Params), vp], i32),
        "iwpp_edt_async": ([vp, i64, vp, vp, i64, i64, i64, i32, P(Params), vp], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib_obj = lib
    return lib


def strerror(code: int) -> str:
    return _load().iwpp_strerror(code).decode()


def version() -> int:
    return _load().iwpp_version()


# ---------------------------------------------------------------- marshalling


def _dtype_code(t) -> int:
    import torch

    if t.dtype == torch.uint8:
        return U8
    if t.dtype == torch.int32:
        return I32
    raise TypeError("images must be torch.uint8 or torch.int32, got %s" % t.dtype)


def _image(marker, mask) -> tuple[Image, int]:
    if marker.dim() != 2 or mask.dim() != 2 or marker.shape != mask.shape:
        raise ValueError("marker and mask must be 2-D tensors of one shape")
    if marker.dtype != mask.dtype:
        raise TypeError("marker and mask must share a dtype")
    if not (marker.is_cuda and mask.is_cuda) or marker.device != mask.device:
        raise ValueError("marker and mask must live on the same GPU")
    if marker.stride(1) != 1 or mask.stride(1) != 1 or marker.stride(0) != mask.stride(0):
        raise ValueError("rows must be contiguous with one common row pitch")
    H, W = marker.shape
    return Image(marker.data_ptr(), mask.data_ptr(), H, W, marker.stride(0)), _dtype_code(marker)


def _stream_handle(stream) -> int | None:
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, int):
        return stream or None
    return stream.cuda_stream or None


def _params(params) -> Params | None:
    if params is None:
        return None
    if isinstance(params, Params):
        return params
    p = Params()
    for k, v in dict(params).items():
        setattr(p, k, int(v))
    return p


def _ptr(p):
    return ctypes.byref(p) if p is not None else None


# ---------------------------------------------------------------- entry points


def _flags(clamp: bool, erosion: bool) -> int:
    return (FLAG_CLAMP_MARKER if clamp else 0) | (FLAG_EROSION if erosion else 0)


def reconstruct_async(marker, mask, conn: int = 8, *, clamp: bool = False,
                      erosion: bool = False, params=None, stream=None) -> None:
    """Queue R_mask(marker) in place on `stream` (default: torch's current);
    `erosion` selects the reconstruction by erosion (marker >= mask)."""
    im, dt = _image(marker, mask)
    rc = _load().iwpp_reconstruct_async(ctypes.byref(im), dt, conn, _flags(clamp, erosion),
                                        _ptr(_params(params)), _stream_handle(stream))
    if rc != OK:
        raise IwppError(rc, "iwpp_reconstruct_async")


def reconstruct_noalloc(marker, mask, conn: int = 8, *, status=None, clamp: bool = False,
                        erosion: bool = False, params=None, stream=None) -> None:
    """Queue R_mask(marker) in place on `stream` through the entry point that
    allocates nothing (its workspace is a static device array).  `status`, if
    given, is a one-element int32 tensor on the marker's device that receives
    the call's IWPP status when the work has finished on the stream."""
    import torch

    im, dt = _image(marker, mask)
    sp = None
    if status is not None:
        if status.dtype != torch.int32 or status.numel() < 1 or status.device != marker.device:
            raise ValueError("status must be an int32 tensor on the marker's device")
        sp = status.data_ptr()
    rc = _load().iwpp_reconstruct_noalloc(ctypes.byref(im), dt, conn, _flags(clamp, erosion),
                                          _ptr(_params(params)), sp, _stream_handle(stream))
    if rc != OK:
        raise IwppError(rc, "iwpp_reconstruct_noalloc")


def stream_status(stream=None, *, check: bool = True) -> dict:
    """Wait for `stream`; status and counters of its last reconstruction."""
    st = Stats()
    rc = _load().iwpp_stream_status(_stream_handle(stream), ctypes.byref(st))
    if check and rc != OK:
        raise IwppError(rc, "reconstruction")
    d = st.as_dict()
    d["rc"] = rc
    return d


def reconstruct(marker, mask, conn: int = 8, *, clamp: bool = False, erosion: bool = False,
                params=None, stream=None, check: bool = True) -> dict:
    """Synchronous R_mask(marker) in place; returns the work counters."""
    reconstruct_async(marker, mask, conn, clamp=clamp, erosion=erosion, params=params,
                      stream=stream)
    return stream_status(stream, check=check)


def fill_holes(image, out=None, conn: int = 8, *, params=None, stream=None,
               check: bool = True):
    """Fill the holes of `image` into `out` (allocated like `image` if None).
    Returns (out, counters)."""
    import torch

    if out is None:
        out = torch.empty_like(image)
    if image.dim() != 2 or out.shape != image.shape or out.dtype != image.dtype:
        raise ValueError("image and out must be 2-D tensors of one shape and dtype")
    if not (image.is_cuda and out.is_cuda) or image.device != out.device:
        raise ValueError("image and out must live on the same GPU")
    if image.stride(1) != 1 or out.stride(1) != 1 or image.stride(0) != out.stride(0):
        raise ValueError("rows must be contiguous with one common row pitch")
    H, W = image.shape
    rc = _load().iwpp_fill_holes_async(image.data_ptr(), out.data_ptr(), H, W, image.stride(0),
                                       _dtype_code(image), conn, _ptr(_params(params)),
                                       _stream_handle(stream))
    if rc != OK:
        raise IwppError(rc, "iwpp_fill_holes_async")
    return out, stream_status(stream, check=check)


def edt(image, conn: int = 8, *, sites=None, dist2=None, params=None, stream=None,
        check: bool = True):
    """Euclidean distance transform of a uint8 image (0 = background).
    Returns (sites, dist2, counters): int32 tensors of nearest-site positions
    packed (y << 16) | x and squared distances (-1 where there is no site)."""
    sites, dist2 = edt_async(image, conn, sites=sites, dist2=dist2, params=params,
                             stream=stream)
    return sites, dist2, stream_status(stream, check=check)


def edt_async(image, conn: int = 8, *, sites=None, dist2=None, params=None, stream=None):
    """Queue the distance transform on `stream`; returns (sites, dist2)."""
    import torch

    if image.dim() != 2 or image.dtype != torch.uint8 or not image.is_cuda:
        raise ValueError("edt takes a 2-D uint8 tensor on the GPU")
    if image.stride(1) != 1:
        raise ValueError("image rows must be contiguous")
    H, W = image.shape
    if sites is None:
        sites = torch.empty((H, W), dtype=torch.int32, device=image.device)
    if dist2 is None:
        dist2 = torch.empty((H, W), dtype=torch.int32, device=image.device)
    for t in (sites, dist2):
        if t.shape != image.shape or t.dtype != torch.int32 or t.device != image.device:
            raise ValueError("sites and dist2 must be int32 tensors shaped like the image")
    if sites.stride() != dist2.stride() or sites.stride(1) != 1:
        raise ValueError("sites and dist2 must share one contiguous row pitch")
    rc = _load().iwpp_edt_async(image.data_ptr(), image.stride(0), sites.data_ptr(),
                                dist2.data_ptr(), sites.stride(0), H, W, conn,
                                _ptr(_params(params)), _stream_handle(stream))
    if rc != OK:
        raise IwppError(rc, "iwpp_edt_async")
    return sites, dist2


def reconstruct_batched(pairs, conn: int = 8, *, clamp: bool = False, erosion: bool = False,
                        params=None, stream=None, check: bool = True) -> dict:
    """Reconstruct [(marker, mask), ...] in one persistent launch."""
    ims, dts = zip(*(_image(m, k) for m, k in pairs))
    if len(set(dts)) != 1:
        raise TypeError("all images of a batch must share a dtype")
    arr = (Image * len(ims))(*ims)
    rc = _load().iwpp_reconstruct_batched(arr, len(ims), dts[0], conn, _flags(clamp, erosion),
                                          _ptr(_params(params)), _stream_handle(stream))
    if rc != OK:
        raise IwppError(rc, "iwpp_reconstruct_batched")
    return stream_status(stream, check=check)


class Batch:
    """A reusable batch plan (optionally replayed as a HIP graph)."""

    def __init__(self, pairs, conn: int = 8, *, clamp: bool = False, erosion: bool = False,
                 params=None):
        ims, dts = zip(*(_image(m, k) for m, k in pairs))
        if len(set(dts)) != 1:
            raise TypeError("all images of a batch must share a dtype")
        self._keep = list(pairs)
        arr = (Image * len(ims))(*ims)
        h = ctypes.c_void_p()
        rc = _load().iwpp_batch_create(arr, len(ims), dts[0], conn, _flags(clamp, erosion),
                                       _ptr(_params(params)), ctypes.byref(h))
        if rc != OK:
            raise IwppError(rc, "iwpp_batch_create")
        self._h = h

    def launch(self, stream=None, graph: bool = True) -> None:
        rc = _load().iwpp_batch_launch(self._h, _stream_handle(stream), 1 if graph else 0)
        if rc != OK:
            raise IwppError(rc, "iwpp_batch_launch")

    def status(self, check: bool = True) -> dict:
        st = Stats()
        rc = _load().iwpp_batch_status(self._h, ctypes.byref(st))
        if check and rc != OK:
            raise IwppError(rc, "batch")
        d = st.as_dict()
        d["rc"] = rc
        return d

    def close(self) -> None:
        if self._h:
            _load().iwpp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(marker, mask, conn: int = 8, stream=None) -> dict:
    """Time parameter candidates on this image; returns the fastest set."""
    im, dt = _image(marker, mask)
    best = Params()
    rc = _load().iwpp_autotune(ctypes.byref(im), dt, conn, _stream_handle(stream),
                               ctypes.byref(best))
    if rc != OK:
        raise IwppError(rc, "iwpp_autotune")
    return best.as_dict()


class Server:
    """Continuous-batching request server (see iwpp_server_* in iwpp.h)."""

    def __init__(self, budget_bytes: int, dtype: str = "u8", conn: int = 8, streams: int = 2,
                 max_inflight: int = 64):
        h = ctypes.c_void_p()
        rc = _load().iwpp_server_create(budget_bytes, U8 if dtype == "u8" else I32, conn,
                                        streams, max_inflight, ctypes.byref(h))
        if rc != OK:
            raise IwppError(rc, "iwpp_server_create")
        self._h = h
        self._keep = {}

    def submit(self, marker, mask, marker_init=None, stream=None) -> int:
        """Queue R_mask(marker) in place; if `marker_init` is given it is
        copied into `marker` on the device first.  The work starts after what
        was queued on `stream` (default: torch's current stream) before the
        call, so buffers written there just before are ready."""
        im, _ = _image(marker, mask)
        init = None
        if marker_init is not None:
            if marker_init.shape != marker.shape or marker_init.stride() != marker.stride() \
                    or marker_init.dtype != marker.dtype or marker_init.device != marker.device:
                raise ValueError("marker_init must match the marker's shape, pitch and dtype")
            init = marker_init.data_ptr()
        t = ctypes.c_uint64()
        rc = _load().iwpp_server_submit(self._h, ctypes.byref(im), init, _stream_handle(stream),
                                        ctypes.byref(t))
        if rc != OK:
            raise IwppError(rc, "iwpp_server_submit")
        self._keep[t.value] = (marker, mask, marker_init)
        return t.value

    def wait(self, ticket: int, timeout_us: int = -1) -> tuple[int, float]:
        lat = ctypes.c_double()
        rc = _load().iwpp_server_wait(self._h, ticket, timeout_us, ctypes.byref(lat))
        if rc != E_TIMEOUT:
            self._keep.pop(ticket, None)
        return rc, lat.value

    def close(self) -> None:
        if self._h:
            _load().iwpp_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def device_copy(dst, src, stream=None) -> None:
    """The library's plain streaming copy kernel (bandwidth reference)."""
    n = src.numel() * src.element_size()
    rc = _load().iwpp_device_copy(dst.data_ptr(), src.data_ptr(), n, _stream_handle(stream))
    if rc != OK:
        raise IwppError(rc, "iwpp_device_copy")


def release_workspace() -> None:
    rc = _load().iwpp_release_workspace()
    if rc != OK:
        raise IwppError(rc, "iwpp_release_workspace")
