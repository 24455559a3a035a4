"""Parity at the full sizes, in the configurations bench.py times
(8-connected; library defaults for single images, tuned parameters and a
HIP-graph plan for the 256-image batch).

* int32 h-dome: the whole image is compared with the oracle, bit for bit
  (the oracle takes about 35 s of one core).
* uint8 fill-holes: the oracle would take minutes, so the check is
  - properties that hold at any size, computed with plain torch tensor ops:
    J <= R <= I, the fixed-point equation R = min(I, max(R, its 8
    neighbours)) at every pixel, and max R <= max J;
  - R at sampled pixels, computed one by one by the oracle's single-pixel
    search (samples whose search exceeds its visit bound are skipped; most
    samples near the frame complete).
* the 256-image batch (about 1 Gpx): J <= R <= I for every image after each
  graph replay, and 16 sampled images against the oracle, bit for bit.
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


def test_c4_full_batch_sampled(iwpp):
    """The 256-image batch at its full sizes (sides log-uniform 512..4096,
    about 1 Gpx), run as bench.py runs it: parameters tuned on the largest
    image, one plan, launched as a HIP graph and replayed.  Every image is
    checked for J <= R <= I after each replay; 16 images (the smallest, the
    largest and 14 drawn at random) are compared with the oracle bit for bit,
    after the second replay."""
    import torch

    announce("c4 256 images: generating")
    pairs = synth.c4()
    dev = torch.device("cuda:0")
    pristine = [torch.from_numpy(J).to(dev) for I, J in pairs]
    masks = [torch.from_numpy(I).to(dev) for I, J in pairs]
    work = [p.clone() for p in pristine]
    big = max(range(len(masks)), key=lambda k: masks[k].numel())
    announce("c4 256 images: tuning on image %d" % big)
    tuned = {k: v for k, v in iwpp.autotune(pristine[big], masks[big], 8).items() if v}
    plan = iwpp.Batch(list(zip(work, masks)), 8, params=tuned)
    try:
        for replay in range(2):
            for w, p in zip(work, pristine):
                w.copy_(p)
            announce("c4 256 images: graph launch %d, params %s" % (replay, tuned))
            plan.launch(graph=True)
            st = plan.status()
            assert st["rc"] == iwpp.OK and st["images"] == 256
            for k, (w, p, m) in enumerate(zip(work, pristine, masks)):
                assert bool((w >= p).all()) and bool((w <= m).all()), "image %d" % k
    finally:
        plan.close()
    rng = np.random.default_rng(5)
    small = min(range(len(masks)), key=lambda k: masks[k].numel())
    picks = sorted({small, big} | set(int(k) for k in rng.choice(len(pairs), 14, replace=False)))
    for k in picks:
        I, J = pairs[k]
        announce("c4 image %d (%dx%d): oracle" % (k, I.shape[0], I.shape[1]))
        rc, R = oracle.reconstruct(J, I, 8)
        assert rc == oracle.OK
        got = work[k].cpu().numpy()
        bad = got != R
        if bad.any():
            y, x = np.argwhere(bad)[0]
            raise AssertionError("image %d: %d pixels differ, first at (%d, %d): got %d want %d"
                                 % (k, bad.sum(), y, x, got[y, x], R[y, x]))
