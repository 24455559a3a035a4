"""Independent, definition-level checks used to pin the oracle.

Nothing here shares code with ``oracle/`` (C) or with the GPU library.  Each
function restates a mathematical fact about grayscale reconstruction by
dilation in numpy/scipy:

* :func:`brute_numpy` -- the definition: J <- dilate(J) ^ I until stable
  (the paper's reconstruction Equation and its iterative algorithm).
* :func:`threshold_decomposition` -- the level-set characterisation: R(p) is
  the largest level t such that p lies in a connected component of {I >= t}
  that meets {J >= t}.  Components come from ``scipy.ndimage.label``.
* :func:`line_closed_form` -- the 1-D case: R = max(L, B) with the two
  one-sided running recurrences.
* :func:`dilate` / :func:`is_fixed_point` -- for invariants at any size.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage


def _lowest(dtype) -> int:
    return int(np.iinfo(dtype).min)


def dilate(J: np.ndarray, conn: int) -> np.ndarray:
    """Elementary dilation by the 3x3 (8-conn) or cross (4-conn) element;
    pixels outside the image do not take part."""
    lo = _lowest(J.dtype)
    H, W = J.shape
    P = np.full((H + 2, W + 2), lo, dtype=J.dtype)
    P[1:-1, 1:-1] = J
    out = J.copy()
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy == 0 and dx == 0:
                continue
            if conn == 4 and dy != 0 and dx != 0:
                continue
            np.maximum(out, P[1 + dy:1 + dy + H, 1 + dx:1 + dx + W], out=out)
    return out


def brute_numpy(J: np.ndarray, I: np.ndarray, conn: int) -> np.ndarray:
    R = J.copy()
    while True:
        nxt = np.minimum(dilate(R, conn), I)
        if np.array_equal(nxt, R):
            return R
        R = nxt


def is_fixed_point(R: np.ndarray, I: np.ndarray, conn: int) -> bool:
    return bool(np.array_equal(np.minimum(dilate(R, conn), I), R))


def threshold_decomposition(J: np.ndarray, I: np.ndarray, conn: int) -> np.ndarray:
    structure = np.ones((3, 3), bool) if conn == 8 else ndimage.generate_binary_structure(2, 1)
    levels = np.unique(np.concatenate([np.unique(I), np.unique(J)]))
    R = np.full(I.shape, _lowest(I.dtype), dtype=np.int64)
    for t in levels:  # increasing, so the last level written is the largest
        lab, n = ndimage.label(I >= t, structure=structure)
        if n == 0:
            continue
        hit = np.zeros(n + 1, bool)
        hit[np.unique(lab[(J >= t) & (lab > 0)])] = True
        hit[0] = False
        R[hit[lab]] = t
    return R.astype(I.dtype)


def line_closed_form(J: np.ndarray, I: np.ndarray) -> np.ndarray:
    """1-D reconstruction: L(x) = min(I(x), max(J(x), L(x-1))) from the left,
    B the same from the right, R = max(L, B)."""
    j = J.astype(np.int64).ravel()
    i = I.astype(np.int64).ravel()
    n = j.shape[0]
    L = np.empty(n, np.int64)
    B = np.empty(n, np.int64)
    for x in range(n):
        L[x] = min(i[x], max(j[x], L[x - 1])) if x else j[x]
    for x in range(n - 1, -1, -1):
        B[x] = min(i[x], max(j[x], B[x + 1])) if x < n - 1 else j[x]
    return np.maximum(L, B).astype(I.dtype).reshape(J.shape)


# ------------------------------------------------------------ by erosion


def _footprint(conn: int) -> np.ndarray:
    return np.ones((3, 3), bool) if conn == 8 else ndimage.generate_binary_structure(2, 1)


def brute_erode_scipy(J: np.ndarray, I: np.ndarray, conn: int) -> np.ndarray:
    """Reconstruction by erosion by its definition: J <- max(erode(J), I)
    until stable, with ``scipy.ndimage.grey_erosion`` as the elementary
    erosion (pixels outside the image are the type's highest value, so they
    never win a minimum)."""
    hi = int(np.iinfo(J.dtype).max)
    fp = _footprint(conn)
    R = J.copy()
    while True:
        nxt = np.maximum(ndimage.grey_erosion(R, footprint=fp, mode="constant", cval=hi), I)
        if np.array_equal(nxt, R):
            return R
        R = nxt


def fill_holes_by_levels(image: np.ndarray, conn: int) -> np.ndarray:
    """Grayscale fill-holes by threshold decomposition: for every level t,
    {fill(I) >= t} is ``scipy.ndimage.binary_fill_holes({I >= t})`` with the
    background connectivity `conn` (a flat increasing operator commutes with
    thresholding); the grayscale result is the largest such t."""
    st = _footprint(conn)
    out = np.full(image.shape, np.iinfo(image.dtype).min, dtype=np.int64)
    for t in np.unique(image):
        filled = ndimage.binary_fill_holes(image >= t, structure=st)
        out[filled] = np.maximum(out[filled], int(t))
    return out.astype(image.dtype)


# ------------------------------------------------------------ distance transform


def edt_exact_sq(img: np.ndarray) -> np.ndarray:
    """Exact squared Euclidean distance of every pixel to the nearest
    background (0) pixel, from ``scipy.ndimage.distance_transform_edt``
    (rounded: squared distances between pixel centres are integers); -1
    where the image has no background pixel."""
    if not (img == 0).any():
        return np.full(img.shape, -1, np.int64)
    d = ndimage.distance_transform_edt(img != 0)
    return np.rint(d.astype(np.float64) ** 2).astype(np.int64)


def edt_brute_sq(img: np.ndarray) -> np.ndarray:
    """The same by brute force over all background pixels (tiny images)."""
    ys, xs = np.nonzero(img == 0)
    H, W = img.shape
    if ys.size == 0:
        return np.full((H, W), -1, np.int64)
    yy, xx = np.mgrid[0:H, 0:W]
    d = (yy[..., None] - ys) ** 2 + (xx[..., None] - xs) ** 2
    return d.min(axis=-1).astype(np.int64)


def decode_sites(sites: np.ndarray):
    s = sites.astype(np.int64) & 0xFFFFFFFF
    return s >> 16, s & 0xFFFF


def edt_check_valid(img: np.ndarray, sites: np.ndarray, dist2: np.ndarray, conn: int) -> None:
    """Raise AssertionError unless (sites, dist2) is a valid end state of the
    site propagation: every site is a background pixel, dist2 is the squared
    distance to it, background pixels are their own sites, and no pixel has
    a neighbour holding a strictly closer site (the propagation stopped)."""
    H, W = img.shape
    none = sites == -1
    assert (none == (dist2 == -1)).all(), "sites and distances disagree on 'no site'"
    if (img == 0).any():
        assert not none.any(), "a pixel has no site although the image has background"
    else:
        assert none.all()
        return
    sy, sx = decode_sites(sites)
    assert (sy < H).all() and (sx < W).all(), "site outside the image"
    assert (img[sy, sx] == 0).all(), "a site is not a background pixel"
    yy, xx = np.mgrid[0:H, 0:W]
    np.testing.assert_array_equal(dist2, (yy - sy) ** 2 + (xx - sx) ** 2)
    bg = img == 0
    assert (dist2[bg] == 0).all(), "a background pixel is not its own site"
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if (dy, dx) == (0, 0) or (conn == 4 and dy and dx):
                continue
            # q = (y, x), p = (y + dy, x + dx): d(q, site(p)) >= d(q, site(q))
            y0, y1 = max(0, -dy), H - max(0, dy)
            x0, x1 = max(0, -dx), W - max(0, dx)
            qy, qx = yy[y0:y1, x0:x1], xx[y0:y1, x0:x1]
            psy = sy[y0 + dy:y1 + dy, x0 + dx:x1 + dx]
            psx = sx[y0 + dy:y1 + dy, x0 + dx:x1 + dx]
            offered = (qy - psy) ** 2 + (qx - psx) ** 2
            assert (offered >= dist2[y0:y1, x0:x1]).all(), "propagation had not stopped"
