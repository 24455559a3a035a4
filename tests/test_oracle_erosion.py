"""Pins for the oracle's reconstruction by erosion and fill-holes.

The oracle computes both through duality with its reconstruction by
dilation.  These tests hold it against definitions that do not use that
route: iterated ``scipy.ndimage.grey_erosion`` (the definition of the
reconstruction by erosion), ``scipy.ndimage.binary_fill_holes`` on binary
images and, for grayscale images, at every threshold (fill-holes is a flat
increasing operator), plus closed forms for a ring around a hole.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests import refdefs


def _pair_above(rng, H, W, dtype, levels=None):
    """A mask I and a marker J >= I."""
    I, J0 = synth.random_pair(rng, H, W, dtype, "uniform", levels=levels)
    hi = np.iinfo(dtype).max
    bump = rng.integers(0, 4, size=I.shape)
    J = np.minimum(I.astype(np.int64) + bump * (rng.random(I.shape) < 0.3) * 7, hi).astype(dtype)
    return I, J


@pytest.mark.parametrize("conn", [8, 4])
@pytest.mark.parametrize("dtype", [np.uint8, np.int32])
def test_erosion_matches_iterated_grey_erosion(conn, dtype):
    rng = np.random.default_rng(40 + conn + (dtype == np.int32))
    for (H, W) in [(1, 1), (1, 17), (13, 1), (5, 7), (16, 16), (23, 31), (40, 9)]:
        for levels in (3, 8, None):
            I, J = _pair_above(rng, H, W, dtype, levels)
            rc, R = oracle.reconstruct_erode(J, I, conn)
            assert rc == oracle.OK
            np.testing.assert_array_equal(R, refdefs.brute_erode_scipy(J, I, conn))


@pytest.mark.parametrize("conn", [8, 4])
def test_erosion_invariants(conn):
    rng = np.random.default_rng(7)
    I, J = _pair_above(rng, 60, 70, np.uint8, 6)
    rc, R = oracle.reconstruct_erode(J, I, conn)
    assert rc == oracle.OK
    assert (I <= R).all() and (R <= J).all()
    rc, R2 = oracle.reconstruct_erode(R, I, conn)
    np.testing.assert_array_equal(R2, R)  # idempotent
    rc, R3 = oracle.reconstruct_erode(I.copy(), I, conn)
    np.testing.assert_array_equal(R3, I)  # J = I gives I


def test_erosion_precondition_and_clamp():
    I = np.full((6, 6), 50, np.uint8)
    J = np.full((6, 6), 90, np.uint8)
    J[2, 3] = 10  # below the mask
    rc, _ = oracle.reconstruct_erode(J, I, 8)
    assert rc == oracle.E_MARKER_GT_MASK
    rc, R = oracle.reconstruct_erode(J, I, 8, clamp=True)
    assert rc == oracle.OK
    np.testing.assert_array_equal(R, refdefs.brute_erode_scipy(np.maximum(J, I), I, 8))


@pytest.mark.parametrize("conn", [8, 4])
def test_fill_holes_binary_matches_scipy(conn):
    rng = np.random.default_rng(11 + conn)
    st = np.ones((3, 3), bool) if conn == 8 else None
    for (H, W) in [(1, 1), (2, 5), (30, 30), (64, 50), (97, 33)]:
        for density in (0.3, 0.5, 0.6):
            B = rng.random((H, W)) < density
            img = np.where(B, 200, 7).astype(np.uint8)
            rc, F = oracle.fill_holes(img, conn)
            assert rc == oracle.OK
            want = np.where(refdefs.ndimage.binary_fill_holes(B, structure=st), 200, 7)
            np.testing.assert_array_equal(F, want.astype(np.uint8))


@pytest.mark.parametrize("conn", [8, 4])
@pytest.mark.parametrize("dtype", [np.uint8, np.int32])
def test_fill_holes_threshold_decomposition(conn, dtype):
    rng = np.random.default_rng(3 + conn)
    I = synth.ellipses(np.random.default_rng(5), 90, 110, 30)
    if dtype == np.int32:
        I = (I.astype(np.int32) - 100) * 1000  # negative values too
    rc, F = oracle.fill_holes(I, conn)
    assert rc == oracle.OK
    np.testing.assert_array_equal(F, refdefs.fill_holes_by_levels(I, conn))
    # random few-level images
    for _ in range(4):
        R = rng.integers(0, 6, size=(37, 41)).astype(dtype) * 9
        rc, F = oracle.fill_holes(R, conn)
        np.testing.assert_array_equal(F, refdefs.fill_holes_by_levels(R, conn))


@pytest.mark.parametrize("conn", [8, 4])
def test_fill_holes_ring_closed_form(conn):
    # a thick ring of value 100 around a hole of value 20, background 10:
    # the hole fills to 100, everything else is unchanged
    H, W = 41, 47
    yy, xx = np.mgrid[0:H, 0:W]
    r2 = (yy - 20) ** 2 + (xx - 23) ** 2
    img = np.full((H, W), 10, np.uint8)
    img[(r2 <= 14 ** 2) & (r2 >= 8 ** 2)] = 100
    hole = r2 < 8 ** 2
    img[hole] = 20
    img[20, 23] = 5  # a deeper pit inside the hole
    rc, F = oracle.fill_holes(img, conn)
    assert rc == oracle.OK
    want = img.copy()
    want[hole] = 100
    np.testing.assert_array_equal(F, want)


@pytest.mark.parametrize("conn", [8, 4])
def test_fill_holes_properties(conn):
    I = synth.ellipses(np.random.default_rng(9), 128, 160, 60)
    rc, F = oracle.fill_holes(I, conn)
    assert rc == oracle.OK
    assert (F >= I).all()
    np.testing.assert_array_equal(F[0], I[0])
    np.testing.assert_array_equal(F[-1], I[-1])
    np.testing.assert_array_equal(F[:, 0], I[:, 0])
    np.testing.assert_array_equal(F[:, -1], I[:, -1])
    rc, F2 = oracle.fill_holes(F, conn)
    np.testing.assert_array_equal(F2, F)  # idempotent
