"""Randomized GPU parity sweep: seeded random shapes, pixel types,
connectivities, input kinds and launch parameters through the C ABI, each
result compared bit-exactly with the oracle.  The fixed seeds make every case
reproducible; each case prints its description before it runs.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def random_case(rng, max_side):
    dt = np.uint8 if rng.random() < 0.6 else np.int32
    conn = 8 if rng.random() < 0.7 else 4
    H = int(rng.integers(1, max_side))
    W = int(rng.integers(1, max_side))
    kind = ["uniform", "sparse", "plateau", "extreme"][int(rng.integers(0, 4))]
    gen = int(rng.integers(0, 3))
    if gen == 1 and dt == np.uint8 and H >= 16 and W >= 16:
        desc = "ellipses, frame marker"
        I, J = synth.c2(seed=int(rng.integers(0, 1 << 30)), H=H, W=W)
    elif gen == 1 and dt == np.int32 and H >= 16 and W >= 16:
        desc = "smooth field, h-dome marker"
        I, J = synth.c3_i32(seed=int(rng.integers(0, 1 << 30)), H=H, W=W)
    else:
        desc = kind
        levels = int(rng.integers(2, 12)) if (kind == "uniform" and gen == 0) else None
        I, J = synth.random_pair(rng, H, W, dt, kind, levels=levels)
    params = {}
    if rng.random() < 0.5:
        params["sweeps"] = int(rng.choice([-1, 1, 2, 3, 5, 16, 64]))
    if rng.random() < 0.4:
        params["tile_h"] = int(rng.choice([32, 64] if dt == np.int32 else [64, 128]))
    if rng.random() < 0.2:
        params["mode"] = 1
    if rng.random() < 0.2:
        params["seed_queue"] = int(rng.choice([-1, 0, 64, 100000]))
    if rng.random() < 0.2:
        params["order_seed"] = int(rng.integers(1, 1 << 20))
    if rng.random() < 0.15:
        params["grid"] = int(rng.integers(1, 40))
    return I, J, conn, params, "%s %dx%d conn %d %s %s" % (np.dtype(dt).name, H, W, conn, desc,
                                                          params)


@pytest.mark.parametrize("seed,cases,max_side", [(2024, 300, 700), (77, 20, 2000)])
def test_random_cases_bit_exact(seed, cases, max_side):
    import torch

    import paper_1605_00930_amd as iwpp

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(seed)
    for c in range(cases):
        I, J, conn, params, desc = random_case(rng, max_side)
        print("[gpu-case] random %d/%d: %s" % (seed, c, desc), flush=True)
        rc, want = oracle.reconstruct(J, I, conn)
        assert rc == oracle.OK
        Jt = torch.from_numpy(np.ascontiguousarray(J)).to(dev)
        It = torch.from_numpy(np.ascontiguousarray(I)).to(dev)
        iwpp.reconstruct(Jt, It, conn, params=params)
        got = Jt.cpu().numpy()
        if not np.array_equal(got, want):
            y, x = np.argwhere(got != want)[0]
            raise AssertionError("%s: %d pixels differ, first at (%d, %d): got %d want %d"
                                 % (desc, int((got != want).sum()), y, x, got[y, x],
                                    want[y, x]))


def test_random_erosion_and_clamp_bit_exact():
    """Reconstruction by erosion (marker above the mask) and the clamped
    marker, on seeded random cases."""
    import torch

    import paper_1605_00930_amd as iwpp

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(31337)
    for c in range(120):
        dt = np.uint8 if rng.random() < 0.6 else np.int32
        conn = 8 if rng.random() < 0.7 else 4
        H = int(rng.integers(1, 600))
        W = int(rng.integers(1, 600))
        kind = ["uniform", "sparse", "plateau", "extreme"][int(rng.integers(0, 4))]
        erosion = bool(rng.random() < 0.6)
        if erosion:
            I, J = synth.random_pair_above(rng, H, W, dt, kind)
        else:
            I, J = synth.random_pair(rng, H, W, dt, kind)
        clamp = bool(rng.random() < 0.3)
        if clamp:  # move some marker pixels to the wrong side of the mask
            flip = rng.random((H, W)) < 0.05
            other = I[::-1, ::-1]
            moved = np.minimum(J, other) if erosion else np.maximum(J, other)
            J = np.where(flip, moved, J).astype(dt)
        desc = "%s %dx%d conn %d %s erosion=%s clamp=%s" % (np.dtype(dt).name, H, W, conn, kind,
                                                            erosion, clamp)
        print("[gpu-case] random erosion %d: %s" % (c, desc), flush=True)
        if erosion:
            rc, want = oracle.reconstruct_erode(J, I, conn, clamp=clamp)
        else:
            rc, want = oracle.reconstruct(J, I, conn, clamp=clamp)
        Jt = torch.from_numpy(np.ascontiguousarray(J)).to(dev)
        It = torch.from_numpy(np.ascontiguousarray(I)).to(dev)
        st = iwpp.reconstruct(Jt, It, conn, clamp=clamp, erosion=erosion, check=False)
        if rc != oracle.OK:
            # the precondition fails on both sides alike
            assert st["rc"] != iwpp.OK, desc
            continue
        assert st["rc"] == iwpp.OK, desc
        got = Jt.cpu().numpy()
        assert np.array_equal(got, want), desc


def test_random_batches_bit_exact():
    """Seeded random batches of uneven images in one launch, each image
    compared with the oracle on its own."""
    import torch

    import paper_1605_00930_amd as iwpp

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(4711)
    for b in range(12):
        dt = np.uint8 if b % 3 else np.int32
        conn = 8 if b % 4 else 4
        n = int(rng.integers(1, 24))
        pairs, wants = [], []
        for _ in range(n):
            H = int(rng.integers(1, 400))
            W = int(rng.integers(1, 400))
            kind = ["uniform", "sparse", "plateau", "extreme"][int(rng.integers(0, 4))]
            I, J = synth.random_pair(rng, H, W, dt, kind)
            rc, R = oracle.reconstruct(J, I, conn)
            assert rc == oracle.OK
            pairs.append((torch.from_numpy(np.ascontiguousarray(J)).to(dev),
                          torch.from_numpy(np.ascontiguousarray(I)).to(dev)))
            wants.append(R)
        print("[gpu-case] random batch %d: %d %s images conn %d" % (b, n, np.dtype(dt).name,
                                                                     conn), flush=True)
        iwpp.reconstruct_batched(pairs, conn)
        for k, ((Jt, _), R) in enumerate(zip(pairs, wants)):
            assert np.array_equal(Jt.cpu().numpy(), R), "batch %d image %d" % (b, k)
