"""Parity at the full 32768 x 32768 sizes, in the configuration bench.py
times (library defaults, 8-connected).

* int32 h-dome: the whole image is compared with the oracle, bit for bit
  (the oracle takes about 35 s of one core).
* uint8 fill-holes: the oracle would take minutes, so the check is
  - properties that hold at any size, computed with plain torch tensor ops:
    J <= R <= I, the fixed-point equation R = min(I, max(R, its 8
    neighbours)) at every pixel, and max R <= max J;
  - R at sampled pixels, computed one by one by the oracle's single-pixel
    search (samples whose search exceeds its visit bound are skipped; most
    samples near the frame complete).
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def iwpp():
    import torch

    import paper_1605_00930_amd as lib

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib._load()
    return lib


def announce(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


def test_c3_i32_full_size_bit_exact(iwpp):
    import torch

    announce("c3 int32 32768x32768: generating")
    I, J = synth.c3_i32()
    dev = torch.device("cuda:0")
    announce("c3 int32 32768x32768: GPU reconstruction")
    Jt = torch.from_numpy(J).to(dev)
    It = torch.from_numpy(I).to(dev)
    st = iwpp.reconstruct(Jt, It, 8)
    assert st["tiles"] == 1024 * 512
    got = Jt.cpu().numpy()
    del Jt, It
    torch.cuda.empty_cache()
    announce("c3 int32 32768x32768: oracle (about 35 s)")
    rc, _ = oracle.reconstruct(J, I, 8, inplace=True)
    assert rc == oracle.OK
    bad = got != J
    if bad.any():
        y, x = np.argwhere(bad)[0]
        raise AssertionError("%d pixels differ, first at (%d, %d): got %d want %d"
                             % (bad.sum(), y, x, got[y, x], J[y, x]))


def test_c3_u8_full_size_properties_and_samples(iwpp):
    import torch

    announce("c3 uint8 32768x32768: generating")
    I, J = synth.c3_u8()
    H, W = I.shape
    dev = torch.device("cuda:0")
    announce("c3 uint8 32768x32768: GPU reconstruction")
    Jt = torch.from_numpy(J).to(dev)
    It = torch.from_numpy(I).to(dev)
    Rt = Jt.clone()
    iwpp.reconstruct(Rt, It, 8)
    announce("c3 uint8: properties")
    assert bool((Jt <= Rt).all()) and bool((Rt <= It).all())
    assert int(Rt.max()) <= int(Jt.max())
    # fixed point: R = min(I, max over the pixel and its 8 neighbours of R);
    # pixels outside the image take no part (padding with 0, the uint8 floor)
    P = torch.zeros((H + 2, W + 2), dtype=torch.uint8, device=dev)
    P[1:-1, 1:-1] = Rt
    m = Rt.clone()
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy or dx:
                torch.maximum(m, P[1 + dy:1 + dy + H, 1 + dx:1 + dx + W], out=m)
    del P
    assert torch.equal(Rt, torch.minimum(It, m))
    del m
    R = Rt.cpu().numpy()
    del Rt, Jt, It
    torch.cuda.empty_cache()
    announce("c3 uint8: sampled pixels")
    rng = np.random.default_rng(77)
    n_edge, n_any = 300, 60
    side = rng.integers(0, 4, n_edge)
    depth = rng.integers(0, 300, n_edge)
    along = rng.integers(0, W, n_edge)
    rows = np.where(side == 0, depth, np.where(side == 1, H - 1 - depth, along % H))
    cols = np.where(side == 2, depth, np.where(side == 3, W - 1 - depth, along))
    rows = np.concatenate([rows, rng.integers(0, H, n_any)])
    cols = np.concatenate([cols, rng.integers(0, W, n_any)])
    rc, vals = oracle.pixels(J, I, rows, cols, 8, max_visit=1_500_000)
    assert rc in (oracle.OK, oracle.E_INCOMPLETE)
    done = vals != np.iinfo(np.int32).min
    announce("c3 uint8: %d of %d samples completed" % (done.sum(), done.size))
    assert done.sum() >= 250
    np.testing.assert_array_equal(R[rows[done], cols[done]].astype(np.int32), vals[done])
