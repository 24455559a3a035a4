"""A model of a tile visit's directional passes, checked against the fixed
point they must reach.

The GPU tile runs four passes, each a chain of steps over one axis with one
lane per line of the other axis (down/up: a lane per column, stepping over
rows; right/left: a lane per row, stepping over columns).  A step sets a pixel
to min(I, max(J, the incoming-side neighbours)); 8-connected diagonals come
from the neighbouring lanes' chain values.  The halo is shared out between
the passes:
- the vertical passes take the halo row before them (straight and diagonal),
  and their edge lanes take the two halo corners at their first step only;
- the horizontal passes take the halo column before them, straight and, for
  8-connectivity, diagonally through the lanes beside;
- lanes past the last row of a short tile walk the halo row below it without
  writing, and the last row's lane takes diagonals from them.
A pass that changes nothing is quiet; a pass whose direction has seen no
change since it last ran is skipped as quiet (each pass is idempotent); the
tile is at its fixed point when no pass is stale.

The model (numpy, one vector operation per step) runs these rules on random
tiles with random halos (each halo pixel's mask equal to its marker, see
random_tile) and must reach exactly the fixed point of
J <- min(I, max over the 3x3 (or cross) neighbourhood) with the halo held,
computed by brute force.  Two mutants (no corners at the first vertical step,
no halo-column diagonals in the horizontal passes) must fail, so the test can
tell a complete set of relations from an incomplete one.
"""
from __future__ import annotations

import numpy as np
import pytest

TW = 64
LANES = 64


def brute_fixed_point(J, I, conn):
    """Fixed point of J <- min(I, max(J, neighbours)) inside the tile, halo held."""
    J = J.copy()
    TH = J.shape[0] - 2
    offs = [(-1, 0), (1, 0), (0, -1), (0, 1)]
    if conn == 8:
        offs += [(-1, -1), (-1, 1), (1, -1), (1, 1)]
    while True:
        inner = J[1:-1, 1:-1].copy()
        for dy, dx in offs:
            inner = np.maximum(inner, J[1 + dy:TH + 1 + dy, 1 + dx:TW + 1 + dx])
        inner = np.minimum(inner, I[1:-1, 1:-1])
        if np.array_equal(inner, J[1:-1, 1:-1]):
            return J
        J[1:-1, 1:-1] = inner


def shift_lanes(v, d):
    """Lane l receives lane l - d's value (d = +1: from below, -1: from above);
    lanes with no source get -1 (no contribution)."""
    out = np.full_like(v, -1)
    if d > 0:
        out[1:] = v[:-1]
    else:
        out[:-1] = v[1:]
    return out


def pass_vertical(J, I, conn, D, corners=True):
    """Down (D=+1) or up (D=-1); J, I are (TH+2, TW+2) with the halo."""
    TH = J.shape[0] - 2
    rows = range(TH) if D > 0 else range(TH - 1, -1, -1)
    prev = J[(0 if D > 0 else TH + 1), 1:-1].copy()  # halo row before the pass
    changed = False
    for k, y in enumerate(rows):
        row = J[y + 1, 1:-1]
        m = np.maximum(row, prev)
        if conn == 8:
            m = np.maximum(m, shift_lanes(prev, +1))
            m = np.maximum(m, shift_lanes(prev, -1))
            if k == 0 and corners:
                hy = 0 if D > 0 else TH + 1
                m[0] = max(m[0], J[hy, 0])
                m[-1] = max(m[-1], J[hy, TW + 1])
        new = np.minimum(m, I[y + 1, 1:-1])
        changed |= bool((new != row).any())
        J[y + 1, 1:-1] = new
        prev = new
    return changed


def pass_horizontal(J, I, conn, D, halo_diagonals=True):
    """Right (D=+1) or left (D=-1): lane l takes row l; lanes past the last
    row walk the halo row below the tile without writing."""
    TH = J.shape[0] - 2
    assert TH <= LANES
    yl = np.minimum(np.arange(LANES), TH)  # tile row of each lane (TH = halo row)
    live = np.arange(LANES) < TH
    cols = range(TW) if D > 0 else range(TW - 1, -1, -1)
    hx = 0 if D > 0 else TW + 1
    prev = J[yl + 1, hx].copy()
    changed = False
    for k, x in enumerate(cols):
        cur = J[yl + 1, x + 1]
        m = np.maximum(cur, prev)
        if conn == 8 and (k > 0 or halo_diagonals):
            m = np.maximum(m, shift_lanes(prev, +1))
            m = np.maximum(m, shift_lanes(prev, -1))
        new = np.minimum(m, I[yl + 1, x + 1])
        changed |= bool((new[live] != cur[live]).any())
        J[yl[live] + 1, x + 1] = new[live]
        prev = new
    return changed


def solve_tile(J, I, conn, first=0, **mut):
    passes = [lambda: pass_vertical(J, I, conn, +1, mut.get("corners", True)),
              lambda: pass_vertical(J, I, conn, -1, mut.get("corners", True)),
              lambda: pass_horizontal(J, I, conn, +1, mut.get("halo_diagonals", True)),
              lambda: pass_horizontal(J, I, conn, -1, mut.get("halo_diagonals", True))]
    stale, quiet, k = 0xF, 0, 0
    while stale and quiet < 4:
        p = (first + k) & 3
        if (stale >> p) & 1 and passes[p]():
            quiet, stale = 0, 0xF
        else:
            quiet += 1
        stale &= ~(1 << p)
        k += 1
        assert k < 10000
    return J


def random_tile(rng, TH, conn):
    shape = (TH + 2, TW + 2)
    I = rng.integers(0, 60, shape)
    J = np.minimum(I, rng.integers(0, 60, shape) * (rng.random(shape) < 0.04))
    # sparse bright halo pixels, corners included; the halo's mask equals its
    # marker, so lanes that walk the halo row below a short tile reproduce
    # the held values (with a looser halo mask they raise that row towards
    # the neighbour's own result, which the whole-image tests cover)
    for sl in (np.s_[0, :], np.s_[-1, :], np.s_[:, 0], np.s_[:, -1]):
        n = J[sl].shape[0]
        J[sl] = rng.integers(0, 100, n) * (rng.random(n) < 0.15)
        I[sl] = J[sl]
    return J, I


@pytest.mark.parametrize("TH", [32, 64])
@pytest.mark.parametrize("conn", [8, 4])
def test_passes_reach_the_fixed_point(TH, conn):
    rng = np.random.default_rng(TH * 10 + conn)
    for trial in range(25):
        J, I = random_tile(rng, TH, conn)
        want = brute_fixed_point(J, I, conn)
        got = solve_tile(J.copy(), I, conn, first=trial % 4)
        assert np.array_equal(got, want), "trial %d" % trial


@pytest.mark.parametrize("mutant", [{"corners": False}, {"halo_diagonals": False}])
def test_incomplete_relation_sets_are_caught(mutant):
    rng = np.random.default_rng(99)
    misses = 0
    for trial in range(25):
        J, I = random_tile(rng, 64, 8)
        want = brute_fixed_point(J, I, 8)
        got = solve_tile(J.copy(), I, 8, first=trial % 4, **mutant)
        misses += not np.array_equal(got, want)
    assert misses > 0
