"""Seeded synthetic inputs for grayscale reconstruction by dilation.

This module only *draws* masks and markers.  It holds none of the
reconstruction arithmetic, and both the GPU library's tests/benchmark and the
CPU oracle consume exactly the arrays it returns.

The paper measures on brain-tumour tissue images (4K x 4K to 32K x 32K, at
several tissue coverages, results chapter "Configuracao dos Experimentos").
Those images are not available, so these generators stand in for them with
the same shapes and structure: blob-like nuclei for h-dome markers, filled
ellipses on a noisy background for fill-holes markers, smooth int32 fields.

Conventions (fixed here, so every run draws the same bytes):
* ``numpy.random.default_rng(seed)`` (PCG64); parameters are drawn as whole
  vectors in the order the code lists them.
* Real-valued images are computed in float64, rounded with ``np.rint``
  (round half to even), clipped, then cast.
* Pixel (y, x) has its centre at integer coordinates (y, x).
"""
from __future__ import annotations

import hashlib
import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np

# ---------------------------------------------------------------- markers


def hdome_marker(I: np.ndarray, h: int) -> np.ndarray:
    """Marker max(I - h, 0), in the mask's dtype."""
    if I.dtype == np.uint8:
        return np.maximum(I.astype(np.int16) - int(h), 0).astype(np.uint8)
    return np.maximum(I.astype(np.int64) - int(h), 0).astype(I.dtype)


def frame_marker(I: np.ndarray) -> np.ndarray:
    """Marker equal to the mask on the 1-pixel image frame and 0 inside
    (the fill-holes form: what is reachable from the image border)."""
    J = np.zeros_like(I)
    J[0, :] = I[0, :]
    J[-1, :] = I[-1, :]
    J[:, 0] = I[:, 0]
    J[:, -1] = I[:, -1]
    return J


# ---------------------------------------------------------------- masks


def gaussian_blobs(seed: int = 0, H: int = 512, W: int = 512, n: int = 64) -> np.ndarray:
    """uint8 mask: sum of n Gaussian blobs (sigma 4..20 px, amplitude
    40..200) plus integer noise U{0..16}, rounded and clipped to 255."""
    rng = np.random.default_rng(seed)
    cy = rng.uniform(0, H, n)
    cx = rng.uniform(0, W, n)
    sig = rng.uniform(4, 20, n)
    amp = rng.uniform(40, 200, n)
    noise = rng.integers(0, 17, size=(H, W))  # inclusive 0..16
    yy = np.arange(H, dtype=np.float64)[:, None]
    xx = np.arange(W, dtype=np.float64)[None, :]
    f = noise.astype(np.float64)
    for k in range(n):
        f += amp[k] * np.exp(-((yy - cy[k]) ** 2 + (xx - cx[k]) ** 2) / (2.0 * sig[k] ** 2))
    return np.clip(np.rint(f), 0, 255).astype(np.uint8)


def ellipses(rng: np.random.Generator, H: int, W: int, n: int, *, bg_max: int = 40,
             vmin: int = 60, vmax: int = 230, amin: float = 5.0,
             amax: float = 25.0) -> np.ndarray:
    """uint8 tissue-like mask: background U{0..bg_max}, then n filled
    ellipses (centre U[0,H) x U[0,W), semi-axes U[amin, amax], angle
    U[0, pi), value U{vmin..vmax}) painted in draw order."""
    I = rng.integers(0, bg_max + 1, size=(H, W), dtype=np.uint8)
    cy = rng.uniform(0, H, n)
    cx = rng.uniform(0, W, n)
    a = rng.uniform(amin, amax, n)
    b = rng.uniform(amin, amax, n)
    th = rng.uniform(0, math.pi, n)
    v = rng.integers(vmin, vmax + 1, size=n)
    for k in range(n):
        r = max(a[k], b[k])
        y0, y1 = max(0, int(math.floor(cy[k] - r))), min(H, int(math.ceil(cy[k] + r)) + 1)
        x0, x1 = max(0, int(math.floor(cx[k] - r))), min(W, int(math.ceil(cx[k] + r)) + 1)
        if y0 >= y1 or x0 >= x1:
            continue
        dy = np.arange(y0, y1, dtype=np.float64)[:, None] - cy[k]
        dx = np.arange(x0, x1, dtype=np.float64)[None, :] - cx[k]
        c, s = math.cos(th[k]), math.sin(th[k])
        u = (dx * c + dy * s) / a[k]
        w = (-dx * s + dy * c) / b[k]
        inside = u * u + w * w <= 1.0
        I[y0:y1, x0:x1][inside] = v[k]
    return I


def _box9_rows(src: np.ndarray, dst: np.ndarray, r0: int, r1: int) -> None:
    """dst[r0:r1] = 9-wide horizontal box sum of src rows (edge replicate)."""
    W = src.shape[1]
    rows = src[r0:r1]
    acc = np.zeros((r1 - r0, W), dtype=np.int32)
    for d in range(-4, 5):
        if d == 0:
            acc += rows
        elif d < 0:
            acc[:, -d:] += rows[:, : W + d]
            acc[:, :-d] += rows[:, :1]
        else:
            acc[:, : W - d] += rows[:, d:]
            acc[:, W - d:] += rows[:, W - 1:W]
    dst[r0:r1] = acc


def _box9_cols(src: np.ndarray, dst: np.ndarray, r0: int, r1: int) -> None:
    """dst[r0:r1] = floor(9-tall vertical box sum of src / 81)."""
    H = src.shape[0]
    acc = np.zeros((r1 - r0, src.shape[1]), dtype=np.int32)
    for d in range(-4, 5):
        idx = np.clip(np.arange(r0, r1) + d, 0, H - 1)
        acc += src[idx]
    dst[r0:r1] = acc // 81


def smooth_field_i32(seed: int, H: int, W: int, vmax: int = 1 << 20,
                     threads: int = 16) -> np.ndarray:
    """int32 mask: U{0..vmax} smoothed by a 9x9 box filter with edge
    replication, floor-divided by 81."""
    rng = np.random.default_rng(seed)
    U = rng.integers(0, vmax + 1, size=(H, W), dtype=np.int32)
    tmp = np.empty_like(U)
    step = max(1, min(1024, H // max(1, threads)))
    spans = [(r, min(H, r + step)) for r in range(0, H, step)]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda s: _box9_rows(U, tmp, *s), spans))
    del U
    out = np.empty_like(tmp)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda s: _box9_cols(tmp, out, *s), spans))
    return out


# ---------------------------------------------------------------- workloads
# Each returns (mask I, marker J).


def c1(seed: int = 0, H: int = 512, W: int = 512):
    """512x512 uint8 Gaussian-blob mask, h-dome marker I - 40."""
    n = max(1, round(64 * H * W / (512 * 512)))
    I = gaussian_blobs(seed, H, W, n)
    return I, hdome_marker(I, 40)


def c2(seed: int = 1, H: int = 4096, W: int = 4096):
    """4096x4096 uint8 ellipse mask (3000 ellipses, scaled by area for
    other sizes), fill-holes marker (1-px frame of I, 0 inside)."""
    n = max(1, round(3000 * H * W / (4096 * 4096)))
    I = ellipses(np.random.default_rng(seed), H, W, n)
    return I, frame_marker(I)


def c3_i32(seed: int = 2, H: int = 32768, W: int = 32768, h: int = 4096):
    """int32 smooth field (U{0..2^20}, 9x9 box), h-dome marker I - 4096."""
    I = smooth_field_i32(seed, H, W)
    return I, hdome_marker(I, h)


def c3_u8(seed: int = 2, H: int = 32768, W: int = 32768):
    """uint8 ellipse mask at 32K x 32K (192,000 ellipses, the 4K recipe
    scaled by area) with the fill-holes frame marker: the front from the
    frame must cross the whole image."""
    return c2(seed, H, W)


def log_uniform_sides(rng: np.random.Generator, n: int, lo: int, hi: int) -> np.ndarray:
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), n))).astype(np.int64)


def c4(seed: int = 3, n: int = 256, lo: int = 512, hi: int = 4096, only=None):
    """n square uint8 images, sides log-uniform in [lo, hi], ellipse masks
    (3000 ellipses per 4096^2, scaled by area), h-dome markers with
    h ~ U{10..80}.  Returns a list of (I, J); with ``only`` (indices), just
    those images, drawn exactly as in the whole batch."""
    rng = np.random.default_rng(seed)
    sides = log_uniform_sides(rng, n, lo, hi)
    hs = rng.integers(10, 81, size=n)
    out = []
    for i in range(n) if only is None else only:
        s = int(sides[i])
        ne = max(1, round(3000 * s * s / (4096 * 4096)))
        I = ellipses(np.random.default_rng([seed, i]), s, s, ne)
        out.append((I, hdome_marker(I, int(hs[i]))))
    return out


def c5_pool(seed: int = 4, n: int = 256, lo: int = 256, hi: int = 8192, only=None):
    """A pool of n distinct uint8 requests: sides log-uniform in [lo, hi],
    ellipse masks, markers half h-dome (h ~ U{10..80}) and half fill-holes
    frame.  Returns a list of (I, J, kind); with ``only`` (indices), just
    those requests, drawn exactly as in the whole pool."""
    rng = np.random.default_rng(seed)
    sides = log_uniform_sides(rng, n, lo, hi)
    kinds = rng.integers(0, 2, size=n)
    hs = rng.integers(10, 81, size=n)
    out = []
    for i in range(n) if only is None else only:
        s = int(sides[i])
        ne = max(1, round(3000 * s * s / (4096 * 4096)))
        I = ellipses(np.random.default_rng([seed, 1000 + i]), s, s, ne)
        if kinds[i] == 0:
            out.append((I, hdome_marker(I, int(hs[i])), "hdome"))
        else:
            out.append((I, frame_marker(I), "fill"))
    return out


def c5_arrivals(seed: int = 4, rate: float = 2000.0, duration: float = 10.0,
                pool: int = 64):
    """Poisson arrivals: (arrival times in seconds, pool index per request)."""
    rng = np.random.default_rng([seed, 7])
    n_max = int(rate * duration * 1.5) + 64
    gaps = rng.exponential(1.0 / rate, n_max)
    t = np.cumsum(gaps)
    t = t[t < duration]
    idx = rng.integers(0, pool, size=t.shape[0])
    return t, idx


# ---------------------------------------------------------------- fuzz


def random_pair(rng: np.random.Generator, H: int, W: int, dtype, kind: str = "uniform",
                levels: int | None = None):
    """A random (I, J) with J <= I.

    kind: "uniform"  I uniform over the dtype (or ``levels`` values), J = I
                     scaled by U[0,1);
          "sparse"   J zero except a few pixels equal to I;
          "plateau"  few levels, large flat zones (many ties);
          "extreme"  values at the ends of the dtype range.
    """
    dtype = np.dtype(dtype)
    if dtype == np.uint8:
        lo, hi = 0, 255
    else:
        lo, hi = -(2 ** 31), 2 ** 31 - 1
    if levels is not None:
        hi = lo + levels - 1
    if kind == "uniform":
        I = rng.integers(lo, hi, size=(H, W), endpoint=True, dtype=np.int64)
        f = rng.random((H, W))
        J = lo + np.floor((I - lo) * f).astype(np.int64)
    elif kind == "sparse":
        I = rng.integers(lo, hi, size=(H, W), endpoint=True, dtype=np.int64)
        J = np.full((H, W), lo, dtype=np.int64)
        m = rng.random((H, W)) < 0.02
        J[m] = I[m]
    elif kind == "plateau":
        L = rng.integers(2, 5)
        vals = np.sort(rng.integers(lo, hi, size=L, endpoint=True, dtype=np.int64))
        I = vals[rng.integers(0, L, size=(H, W))]
        J = np.where(rng.random((H, W)) < 0.05, I, vals[0])
    elif kind == "extreme":
        I = np.where(rng.random((H, W)) < 0.5, hi, hi - 1).astype(np.int64)
        J = np.where(rng.random((H, W)) < 0.1, I, lo).astype(np.int64)
    else:
        raise ValueError(kind)
    return I.astype(dtype), J.astype(dtype)


def random_pair_above(rng: np.random.Generator, H: int, W: int, dtype,
                      kind: str = "uniform", levels: int | None = None):
    """A random (I, J) with J >= I, for reconstruction by erosion.

    kind: "uniform"  I uniform over the dtype (or ``levels`` values), J
                     between I and the top of the range, scaled by U[0,1);
          "sparse"   J at the top of the range except a few pixels equal to I;
          "plateau"  few levels, large flat zones (many ties);
          "extreme"  values at the ends of the dtype range.
    """
    dtype = np.dtype(dtype)
    if dtype == np.uint8:
        lo, hi = 0, 255
    else:
        lo, hi = -(2 ** 31), 2 ** 31 - 1
    top = hi if levels is None else lo + levels - 1
    if kind == "uniform":
        I = rng.integers(lo, top, size=(H, W), endpoint=True, dtype=np.int64)
        J = I + np.floor((top - I) * rng.random((H, W))).astype(np.int64)
    elif kind == "sparse":
        I = rng.integers(lo, top, size=(H, W), endpoint=True, dtype=np.int64)
        J = np.full((H, W), top, dtype=np.int64)
        m = rng.random((H, W)) < 0.02
        J[m] = I[m]
    elif kind == "plateau":
        L = rng.integers(2, 5)
        vals = np.sort(rng.integers(lo, top, size=L, endpoint=True, dtype=np.int64))
        I = vals[rng.integers(0, L, size=(H, W))]
        J = np.where(rng.random((H, W)) < 0.05, I, vals[-1])
    elif kind == "extreme":
        I = np.where(rng.random((H, W)) < 0.5, lo, lo + 1).astype(np.int64)
        J = np.where(rng.random((H, W)) < 0.1, I, hi).astype(np.int64)
    else:
        raise ValueError(kind)
    return I.astype(dtype), J.astype(dtype)


def diagonal_corridor(H: int, W: int, dtype, direction: int, offset: int,
                      value: int | None = None):
    """A 1-pixel-wide diagonal corridor on a zero background, seeded at one end.

    direction +1: pixels (y, y + offset); direction -1: pixels (y, offset - y).
    The mask holds ``value`` (200 for uint8, 10**6 for int32) on the corridor;
    the marker is zero except at the corridor's first pixel (smallest y), which
    holds ``value``.  Two corridor pixels touch only diagonally, so a front
    along it crosses every tile boundary it meets through a corner or a
    diagonal neighbour.
    """
    dtype = np.dtype(dtype)
    if value is None:
        value = 200 if dtype == np.uint8 else 10 ** 6
    I = np.zeros((H, W), dtype)
    J = np.zeros((H, W), dtype)
    ys = np.arange(H)
    xs = ys + offset if direction > 0 else offset - ys
    ok = (xs >= 0) & (xs < W)
    ys, xs = ys[ok], xs[ok]
    if len(ys):
        I[ys, xs] = value
        J[ys[0], xs[0]] = value
    return I, J


def sha256(*arrays: np.ndarray) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()
