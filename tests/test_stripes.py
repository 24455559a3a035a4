"""One image in row stripes, each reconstructed on its own: the seam exchange
that a split of one large image over several devices would run, shown on one.

The stripes overlap by two rows (the last row of one and the first row of
the next are in both).  Each stripe's reconstruction never exceeds the whole
image's (the whole result, restricted to the stripe, satisfies every relation
inside the stripe, and the stripe's result is the least such image above the
marker), so taking the stripes in turn only raises pixels towards the whole
result.  Once a pass over all stripes leaves the shared rows as they were,
every stripe is at its fixed point with the same shared rows, and every
relation across a seam lies inside a stripe that holds both of its rows: the
union is a fixed point above the marker, hence the whole result (the
geodesic reconstruction is the least such fixed point).

The CPU test runs the scheme with the oracle and pins it against the oracle
on the whole image; the GPU test runs the stripes as separate launches on
views of one device image, so the shared rows are exchanged in place.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth


def stripe_bounds(H: int, n: int):
    """Row ranges [a, b) of n stripes over H rows, each overlapping the next
    by two rows."""
    cuts = [round(H * k / n) for k in range(n + 1)]
    return [(max(0, cuts[k] - 1), min(H, cuts[k + 1] + 1)) for k in range(n)]


def shared_rows(bounds):
    rows = set()
    for (a, b), (c, d) in zip(bounds, bounds[1:]):
        rows.update(range(c, b))
    return sorted(rows)


def oracle_by_stripes(I, J, conn, n, max_rounds=200):
    R = J.copy()
    bounds = stripe_bounds(I.shape[0], n)
    rows = shared_rows(bounds)
    for r in range(1, max_rounds + 1):
        before = R[rows].copy()
        for a, b in bounds:
            rc, part = oracle.reconstruct(np.ascontiguousarray(R[a:b]),
                                          np.ascontiguousarray(I[a:b]), conn)
            assert rc == oracle.OK
            R[a:b] = part
        if np.array_equal(before, R[rows]):
            return R, r
    raise AssertionError("stripes did not settle in %d rounds" % max_rounds)


@pytest.mark.parametrize("conn", [8, 4])
@pytest.mark.parametrize("case", ["fill", "hdome_i32"])
def test_oracle_stripes_equal_whole_image(conn, case):
    if case == "fill":
        I, J = synth.c2(seed=5, H=300, W=260)
    else:
        I, J = synth.c3_i32(seed=6, H=240, W=200)
    rc, want = oracle.reconstruct(J, I, conn)
    assert rc == oracle.OK
    for n in (2, 3):
        got, rounds = oracle_by_stripes(I, J, conn, n)
        assert np.array_equal(got, want), "%d stripes" % n
        assert rounds >= 1


def test_stripe_bounds_cover_and_overlap():
    for H, n in [(10, 2), (301, 3), (64, 4), (5, 2)]:
        b = stripe_bounds(H, n)
        assert b[0][0] == 0 and b[-1][1] == H
        for (a, e), (c, d) in zip(b, b[1:]):
            assert e - c == 2 and a < c < e < d


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", [np.uint8, np.int32])
def test_gpu_stripes_exchange_seams(dtype):
    import torch

    import paper_1605_00930_amd as iwpp

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if dtype == np.uint8:
        I, J = synth.c2(seed=7, H=700, W=530)
    else:
        I, J = synth.c3_i32(seed=8, H=520, W=450)
    print("[gpu-case] stripes %s %dx%d" % (np.dtype(dtype).name, *I.shape), flush=True)
    rc, want = oracle.reconstruct(J, I, 8)
    assert rc == oracle.OK
    dev = torch.device("cuda:0")
    Jt = torch.from_numpy(J).to(dev)
    It = torch.from_numpy(I).to(dev)
    bounds = stripe_bounds(I.shape[0], 3)
    rows = torch.tensor(shared_rows(bounds), device=dev)
    settled = False
    for _ in range(200):
        before = Jt[rows].clone()
        for a, b in bounds:
            iwpp.reconstruct(Jt[a:b], It[a:b], 8)
        if torch.equal(before, Jt[rows]):
            settled = True
            break
    assert settled
    got = Jt.cpu().numpy()
    if not np.array_equal(got, want):
        y, x = np.argwhere(got != want)[0]
        raise AssertionError("stripes: first difference at (%d, %d): got %d want %d"
                             % (y, x, got[y, x], want[y, x]))
