"""A numpy model of the distance transform's directional passes (CPU, test
infrastructure; it shares no code with the HIP library or the oracle).

The library reaches a fixed point of the site propagation (a pixel takes a
neighbour's site only when that site is strictly closer) by visiting tiles of
32 x 64 pixels: a visit stages the tile with a one-pixel halo and runs rounds
of four passes -- down, up, right, left -- until four passes in a row change
nothing.  In a pass each pixel, in walking order, is offered the site of the
pixel before it on the walking line (and, 8-connected, the sites of the two
diagonal pixels on the incoming side, those of the neighbouring lines just
updated in the same pass), in that order, and keeps the first offer strictly
closer than what it holds.  Pixels outside the image hold no site and never
take one.

This model applies exactly those tile rules in bulk-synchronous rounds: every
tile loads its halo from the image state, solves to its tile-local fixed
point, and writes back; rounds repeat until the image state is stable.  For
images with fewer tiles than the GPU has workers every tile does run at once,
so the model's end state is a fair stand-in for the kind of end state the
GPU reaches.  Which pixels miss the exact transform depends on the order, so
the model does not predict the GPU's output, but how often and by how much the
passes miss does come from the pass rules (4-connected sites travel along
L-shaped column-then-row paths), and that is what the GPU test bounds.
"""
from __future__ import annotations

import numpy as np

TH, TW = 32, 64
_FAR = np.int64(1) << 40  # squared distance of "no site"
_NONE = -(1 << 20)       # site coordinate of "no site"


def _offer(py, px, sy, sx, by, bx, bd):
    """Offer sites (sy, sx) to pixels (py, px) holding (by, bx, bd); returns
    the updated triple (strictly closer wins)."""
    d = (py - sy) ** 2 + (px - sx) ** 2
    d = np.where(sy == _NONE, _FAR, d)
    win = d < bd
    return np.where(win, sy, by), np.where(win, sx, bx), np.where(win, d, bd)


def _pass(SY, SX, D, PY, PX, conn, axis, rev):
    """One directional pass over every tile at once.  Arrays are (N, TH+2,
    TW+2) with the halo at index 0 and -1; D is the squared distance (0 for
    pixels outside the image, which then never change).  Returns whether a
    tile pixel changed, per tile."""
    changed = np.zeros(SY.shape[0], bool)
    if axis == 0:  # vertical: walk rows, one lane per column
        rows = range(TH, 0, -1) if rev else range(1, TH + 1)
        step = 1 if rev else -1
        for r in rows:
            src = r + step
            by, bx, bd = SY[:, r, 1:-1], SX[:, r, 1:-1], D[:, r, 1:-1]
            oy, ox = by.copy(), bx.copy()
            py, px = PY[:, r, 1:-1], PX[:, r, 1:-1]
            offers = [(SY[:, src, 1:-1], SX[:, src, 1:-1])]
            if conn == 8:
                offers.append((SY[:, src, 0:-2], SX[:, src, 0:-2]))
                offers.append((SY[:, src, 2:], SX[:, src, 2:]))
            for sy, sx in offers:
                by, bx, bd = _offer(py, px, sy, sx, by, bx, bd)
            changed |= ((by != oy) | (bx != ox)).any(axis=1)
            SY[:, r, 1:-1], SX[:, r, 1:-1], D[:, r, 1:-1] = by, bx, bd
    else:  # horizontal: walk columns, one lane per row
        cols = range(TW, 0, -1) if rev else range(1, TW + 1)
        step = 1 if rev else -1
        for c in cols:
            src = c + step
            by, bx, bd = SY[:, 1:-1, c], SX[:, 1:-1, c], D[:, 1:-1, c]
            oy, ox = by.copy(), bx.copy()
            py, px = PY[:, 1:-1, c], PX[:, 1:-1, c]
            offers = [(SY[:, 1:-1, src], SX[:, 1:-1, src])]
            if conn == 8:
                offers.append((SY[:, 0:-2, src], SX[:, 0:-2, src]))
                offers.append((SY[:, 2:, src], SX[:, 2:, src]))
            for sy, sx in offers:
                by, bx, bd = _offer(py, px, sy, sx, by, bx, bd)
            changed |= ((by != oy) | (bx != ox)).any(axis=1)
            SY[:, 1:-1, c], SX[:, 1:-1, c], D[:, 1:-1, c] = by, bx, bd
    return changed


def edt_pass_model(img: np.ndarray, conn: int, max_rounds: int = 10000):
    """(sites, dist2) of the end state the tile rules reach from `img`
    (0 = background) in bulk-synchronous rounds, in the library's encoding:
    sites packed (y << 16) | x, squared distances, both -1 everywhere if the
    image has no background."""
    H, W = img.shape
    if not (img == 0).any():
        none = np.full((H, W), -1, np.int64)
        return none, none.copy()
    nty, ntx = -(-H // TH), -(-W // TW)
    GH, GW = nty * TH + 2, ntx * TW + 2
    yy, xx = np.mgrid[0:H, 0:W]
    gsy = np.full((GH, GW), _NONE, np.int64)
    gsx = np.full((GH, GW), _NONE, np.int64)
    bg = img == 0
    gsy[1:H + 1, 1:W + 1] = np.where(bg, yy, _NONE)
    gsx[1:H + 1, 1:W + 1] = np.where(bg, xx, _NONE)
    inside = np.zeros((GH, GW), bool)
    inside[1:H + 1, 1:W + 1] = True
    gy, gx = np.mgrid[0:GH, 0:GW]
    gy, gx = gy - 1, gx - 1

    def tiles(a):
        v = np.lib.stride_tricks.sliding_window_view(a, (TH + 2, TW + 2))[::TH, ::TW]
        return v.reshape(-1, TH + 2, TW + 2).copy()

    PY, PX, IN = tiles(gy), tiles(gx), tiles(inside)
    for _ in range(max_rounds):
        SY, SX = tiles(gsy), tiles(gsx)
        D = (PY - SY) ** 2 + (PX - SX) ** 2
        D = np.where(SY == _NONE, _FAR, D)
        D = np.where(IN, D, 0)  # outside the image: never takes a site
        quiet = np.zeros(SY.shape[0], np.int64)
        k = 0
        while (quiet < 4).any():
            ch = _pass(SY, SX, D, PY, PX, conn, axis=(k & 3) // 2, rev=bool(k & 1))
            quiet = np.where(ch, 0, quiet + 1)
            k += 1
        new_y, new_x = gsy.copy(), gsx.copy()
        for new, S in ((new_y, SY), (new_x, SX)):
            new[1:-1, 1:-1] = (S[:, 1:-1, 1:-1].reshape(nty, ntx, TH, TW)
                               .transpose(0, 2, 1, 3).reshape(nty * TH, ntx * TW))
        new_y = np.where(inside, new_y, _NONE)
        new_x = np.where(inside, new_x, _NONE)
        if (new_y == gsy).all() and (new_x == gsx).all():
            break
        gsy, gsx = new_y, new_x
    else:
        raise RuntimeError("pass model did not settle")
    sy, sx = gsy[1:H + 1, 1:W + 1], gsx[1:H + 1, 1:W + 1]
    return (sy << 16) | sx, (yy - sy) ** 2 + (xx - sx) ** 2
