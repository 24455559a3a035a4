"""Sequential CPU oracle for grayscale reconstruction by dilation.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this module.  It shares no
code with the GPU library (``paper_1605_00930_amd``) and never imports it.

The algorithms live in ``oracle.c`` / ``oracle_body.inc`` (plain C, one
thread); this module only builds that file with gcc and marshals numpy
arrays through ctypes.

* :func:`reconstruct` -- the paper's hybrid algorithm: raster scan,
  anti-raster scan with the seed rule, then a FIFO queue (IWPP chapter,
  "Reconstrucao Morfologica", reconstruction algorithm in IWPP form).
* :func:`brute` -- the definition: J <- dilate(J) ^ I on a copy until stable
  (background chapter, reconstruction Equation and its iterative algorithm).
* :func:`widest` -- the same result as a widest-path problem on a max-heap
  (the priority-queue ordering of "Uso de Diferentes Estruturas de Dados").
* :func:`pixels` -- R at chosen pixels only, for sampled checks of images
  too large to reconstruct whole.
* :func:`reconstruct_erode` -- reconstruction by erosion (the "min" choice of
  the IWPP algorithm's max/min update), through the duality of reconstruction
  by erosion and by dilation under an order-reversing complement.
* :func:`fill_holes` -- the "Fill Holes" operation of the IWPP chapter: the
  reconstruction by erosion of the image from its own 1-pixel frame.
* :func:`edt` -- the IWPP chapter's Euclidean distance transform: nearest
  background sites propagated through a FIFO queue (vector propagation).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "oracle.c")]
DEPS = SOURCES + [os.path.join(HERE, "oracle.h"), os.path.join(HERE, "oracle_body.inc")]

OK = 0
E_ARG = -1
E_MARKER_GT_MASK = -2
E_NOMEM = -3
E_INCOMPLETE = -5

FLAG_CLAMP_MARKER = 1
ORDER_FIFO, ORDER_LIFO, ORDER_RANDOM = 0, 1, 2


class Stats(ctypes.Structure):
    _fields_ = [("seeds", ctypes.c_int64), ("pushes", ctypes.c_int64),
                ("pops", ctypes.c_int64), ("iters", ctypes.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (one translation unit)."""
    if not force and os.path.exists(LIB_PATH):
        newest = max(os.path.getmtime(p) for p in DEPS)
        if os.path.getmtime(LIB_PATH) >= newest:
            return LIB_PATH
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", tmp] + SOURCES
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        p = ctypes.c_void_p
        i64 = ctypes.c_int64
        for suf in ("u8", "i32"):
            f = getattr(lib, "oracle_reconstruct_" + suf)
            f.argtypes = [p, p, i64, i64, ctypes.c_int, ctypes.c_uint, ctypes.c_int,
                          ctypes.c_int, ctypes.c_uint64, i64, ctypes.POINTER(Stats)]
            f.restype = ctypes.c_int
            for name in ("oracle_brute_", "oracle_widest_"):
                g = getattr(lib, name + suf)
                g.argtypes = [p, p, i64, i64, ctypes.c_int, ctypes.POINTER(Stats)]
                g.restype = ctypes.c_int
            h = getattr(lib, "oracle_pixels_" + suf)
            h.argtypes = [p, p, i64, i64, ctypes.c_int, p, p, i64, i64, p]
            h.restype = ctypes.c_int
        e = lib.oracle_edt
        e.argtypes = [p, i64, i64, ctypes.c_int, p, p, ctypes.POINTER(Stats)]
        e.restype = ctypes.c_int
        _lib = lib
    return _lib


def _suffix(a: np.ndarray) -> str:
    if a.dtype == np.uint8:
        return "u8"
    if a.dtype == np.int32:
        return "i32"
    raise TypeError("oracle images must be uint8 or int32, got %s" % a.dtype)


def _check_pair(J: np.ndarray, I: np.ndarray):
    if J.ndim != 2 or I.shape != J.shape or I.dtype != J.dtype:
        raise ValueError("marker and mask must be 2-D arrays of one shape and dtype")
    if not (J.flags.c_contiguous and I.flags.c_contiguous):
        raise ValueError("oracle arrays must be C-contiguous")


def reconstruct(J: np.ndarray, I: np.ndarray, conn: int = 8, *, clamp: bool = False,
                nsweeps: int = 1, order: int = ORDER_FIFO, seed: int = 0,
                max_pops: int = -1, stats: bool = False, inplace: bool = False):
    """Hybrid scans + queue.  Returns (status, R[, stats])."""
    _check_pair(J, I)
    R = J if inplace else J.copy()
    st = Stats()
    f = getattr(_load(), "oracle_reconstruct_" + _suffix(R))
    rc = f(R.ctypes.data, I.ctypes.data, R.shape[0], R.shape[1], conn,
           FLAG_CLAMP_MARKER if clamp else 0, nsweeps, order, seed, max_pops,
           ctypes.byref(st))
    return (rc, R, st.as_dict()) if stats else (rc, R)


def brute(J: np.ndarray, I: np.ndarray, conn: int = 8, *, stats: bool = False):
    _check_pair(J, I)
    R = J.copy()
    st = Stats()
    rc = getattr(_load(), "oracle_brute_" + _suffix(R))(
        R.ctypes.data, I.ctypes.data, R.shape[0], R.shape[1], conn, ctypes.byref(st))
    return (rc, R, st.as_dict()) if stats else (rc, R)


def widest(J: np.ndarray, I: np.ndarray, conn: int = 8, *, stats: bool = False):
    _check_pair(J, I)
    R = J.copy()
    st = Stats()
    rc = getattr(_load(), "oracle_widest_" + _suffix(R))(
        R.ctypes.data, I.ctypes.data, R.shape[0], R.shape[1], conn, ctypes.byref(st))
    return (rc, R, st.as_dict()) if stats else (rc, R)


def pixels(J: np.ndarray, I: np.ndarray, rows, cols, conn: int = 8, max_visit: int = 0):
    """R at (rows[k], cols[k]).  Returns (status, int32 values)."""
    _check_pair(J, I)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    if rows.shape != cols.shape or rows.ndim != 1:
        raise ValueError("rows and cols must be 1-D and of equal length")
    out = np.empty(rows.shape[0], dtype=np.int32)
    rc = getattr(_load(), "oracle_pixels_" + _suffix(J))(
        J.ctypes.data, I.ctypes.data, J.shape[0], J.shape[1], conn,
        rows.ctypes.data, cols.ctypes.data, rows.shape[0], max_visit, out.ctypes.data)
    return rc, out


def complement(a: np.ndarray) -> np.ndarray:
    """Order-reversing complement: 255 - x for uint8, -1 - x for int32 (the
    bitwise NOT, an involution on each type's full range)."""
    return np.invert(a)


def reconstruct_erode(J: np.ndarray, I: np.ndarray, conn: int = 8, *, clamp: bool = False):
    """Reconstruction by erosion of mask I from marker J >= I: the limit of
    J <- max(erode(J), I).  Uses the duality R^eps_I(J) = C(R_C(I)(C(J))) for
    any order-reversing bijection C, with the hybrid algorithm above for the
    dilation.  Status E_MARKER_GT_MASK means J < I somewhere (with ``clamp``
    the marker max(J, I) is used instead).  Returns (status, R)."""
    rc, R = reconstruct(complement(J), complement(I), conn, clamp=clamp)
    return rc, complement(R)


def highest(dtype) -> int:
    return int(np.iinfo(dtype).max)


def fill_holes(image: np.ndarray, conn: int = 8):
    """Fill holes: reconstruction by erosion of the image from a marker that
    equals the image on its 1-pixel frame and the type's highest value
    elsewhere.  Regions the frame reaches are lowered back to the image;
    regions it cannot reach (holes) stay raised to the lowest level through
    which they can be left.  Returns (status, filled)."""
    if image.ndim != 2:
        raise ValueError("fill_holes takes a 2-D image")
    F = np.full_like(image, highest(image.dtype))
    F[0, :] = image[0, :]
    F[-1, :] = image[-1, :]
    F[:, 0] = image[:, 0]
    F[:, -1] = image[:, -1]
    return reconstruct_erode(F, np.ascontiguousarray(image), conn)


def edt(image: np.ndarray, conn: int = 8, *, stats: bool = False):
    """Distance transform of a uint8 image whose 0 pixels are background.
    Returns (status, sites int32 packed (y << 16) | x or -1, dist2 int64 or -1
    [, stats])."""
    if image.ndim != 2 or image.dtype != np.uint8:
        raise ValueError("edt takes a 2-D uint8 image")
    img = np.ascontiguousarray(image)
    H, W = img.shape
    sites = np.empty((H, W), np.int32)
    dist2 = np.empty((H, W), np.int64)
    st = Stats()
    rc = _load().oracle_edt(img.ctypes.data, H, W, conn, sites.ctypes.data, dist2.ctypes.data,
                            ctypes.byref(st))
    return (rc, sites, dist2, st.as_dict()) if stats else (rc, sites, dist2)
