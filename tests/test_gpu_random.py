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
