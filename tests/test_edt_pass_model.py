"""The CPU model of the distance transform's directional passes
(tests/edt_pass_model.py), which bounds how far the GPU's 4-connected end
state may miss the exact transform, checked against what fixes it: the end
state must be a valid stop of the propagation, never below the exact
transform, and exact wherever the answer is unique."""
from __future__ import annotations

import numpy as np
import pytest

from tests import refdefs
from tests.edt_pass_model import edt_pass_model


@pytest.mark.parametrize("conn", [8, 4])
def test_unique_cases_exact(conn):
    for (H, W, y, x) in [(1, 1, 0, 0), (1, 100, 0, 37), (90, 1, 11, 0), (100, 130, 3, 120),
                         (64, 64, 63, 63), (33, 200, 16, 100)]:
        img = np.ones((H, W), np.uint8)
        img[y, x] = 0
        sites, d2 = edt_pass_model(img, conn)
        np.testing.assert_array_equal(d2, refdefs.edt_exact_sq(img))
        refdefs.edt_check_valid(img, sites, d2, conn)
    frame = np.ones((97, 141), np.uint8)
    frame[0, :] = frame[-1, :] = frame[:, 0] = frame[:, -1] = 0
    sites, d2 = edt_pass_model(frame, conn)
    np.testing.assert_array_equal(d2, refdefs.edt_exact_sq(frame))


@pytest.mark.parametrize("conn", [8, 4])
def test_valid_end_state_never_below_exact(conn):
    rng = np.random.default_rng(7 + conn)
    for (H, W, p) in [(2, 3, 0.5), (65, 63, 0.95), (129, 257, 0.99), (300, 400, 0.9)]:
        img = (rng.random((H, W)) < p).astype(np.uint8)
        sites, d2 = edt_pass_model(img, conn)
        refdefs.edt_check_valid(img, sites, d2, conn)
        assert (d2 >= refdefs.edt_exact_sq(img)).all()


def test_no_background():
    sites, d2 = edt_pass_model(np.ones((5, 7), np.uint8), 4)
    assert (sites == -1).all() and (d2 == -1).all()
