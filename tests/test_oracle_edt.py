"""Pins for the oracle's distance transform (the IWPP chapter's Euclidean
distance-transform algorithm: nearest background sites propagated through a
FIFO queue).

The propagation is the vector-propagation approximation of the exact
transform, so the pins are: the exact transform (scipy, and brute force on
tiny images) as a lower bound that is reached on most pixels and wherever
the closed form is known (one background pixel, a background frame around a
rectangle); the end-state conditions (every site is background, distances
match sites, no neighbour offers a strictly closer site); a small bound on
the error where it is not exact.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests import refdefs


def run(img, conn=8):
    rc, sites, d2 = oracle.edt(img, conn)
    assert rc == oracle.OK
    return sites, d2


def test_scipy_exact_matches_brute_force():
    rng = np.random.default_rng(1)
    for (H, W) in [(1, 1), (3, 5), (9, 7), (16, 16), (21, 30)]:
        img = (rng.random((H, W)) < 0.7).astype(np.uint8)
        img[rng.integers(0, H), rng.integers(0, W)] = 0
        np.testing.assert_array_equal(refdefs.edt_exact_sq(img), refdefs.edt_brute_sq(img))


@pytest.mark.parametrize("conn", [8, 4])
def test_single_background_pixel_is_exact(conn):
    for (H, W, y, x) in [(1, 1, 0, 0), (1, 40, 0, 17), (33, 1, 5, 0), (40, 57, 13, 44),
                         (64, 64, 0, 0), (70, 33, 69, 32)]:
        img = np.ones((H, W), np.uint8)
        img[y, x] = 0
        sites, d2 = run(img, conn)
        yy, xx = np.mgrid[0:H, 0:W]
        np.testing.assert_array_equal(d2, (yy - y) ** 2 + (xx - x) ** 2)
        assert (sites == ((y << 16) | x)).all()


@pytest.mark.parametrize("conn", [8, 4])
def test_background_frame_is_exact(conn):
    img = np.ones((45, 61), np.uint8)
    img[0, :] = img[-1, :] = 0
    img[:, 0] = img[:, -1] = 0
    _, d2 = run(img, conn)
    np.testing.assert_array_equal(d2, refdefs.edt_exact_sq(img))


def test_no_background():
    sites, d2 = run(np.full((7, 9), 3, np.uint8))
    assert (sites == -1).all() and (d2 == -1).all()


@pytest.mark.parametrize("conn", [8, 4])
def test_valid_end_state_and_lower_bound(conn):
    rng = np.random.default_rng(7 + conn)
    cases = [(rng.random((60, 80)) < p).astype(np.uint8) for p in (0.3, 0.8, 0.97, 0.999)]
    I = synth.ellipses(np.random.default_rng(2), 256, 256, 60)
    cases.append((I > 50).astype(np.uint8))
    for img in cases:
        sites, d2 = run(img, conn)
        refdefs.edt_check_valid(img, sites, d2, conn)
        ex = refdefs.edt_exact_sq(img)
        assert (d2 >= ex).all()


def test_error_is_small_where_not_exact():
    # large object regions: the propagation misses the exact nearest site on
    # a few pixels, by a fraction of a pixel
    I = synth.ellipses(np.random.default_rng(1), 1024, 1024, 200)
    img = (I > 50).astype(np.uint8)
    _, d2 = run(img, 8)
    ex = refdefs.edt_exact_sq(img)
    assert (d2 >= ex).all()
    wrong = d2 != ex
    assert wrong.mean() < 1e-3
    assert (np.sqrt(d2) - np.sqrt(ex)).max() < 0.5
    # random sparse background: exact everywhere on this case
    img = (np.random.default_rng(3).random((300, 400)) < 0.9).astype(np.uint8)
    _, d2 = run(img, 8)
    np.testing.assert_array_equal(d2, refdefs.edt_exact_sq(img))
