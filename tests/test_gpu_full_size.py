"""Parity at the full sizes, in the configurations bench.py times
(8-connected; library defaults for single images, tuned parameters and a
HIP-graph plan for the 256-image batch).

Every image is compared whole: the sha256 of the library's output must equal
the sha256 of the CPU oracle's reconstruction of the same inputs, stored in
tests/golden/full_size_sha256.txt by tests/golden/make_full_size_hashes.py
(which calls only the oracle and the seeded generators).  The inputs' own
digests are checked first, so a drift of the generators cannot pass as a
parity failure or hide one.

The served stream's whole request pool goes through the server the same way.
On a mismatch the tests locate the difference for the report (diagnostics
only, never the pass criterion): the int32 image against the oracle run on
the spot, the uint8 image through properties and sampled single-pixel oracle
searches, a batch image or a request against the oracle.
"""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "full_size_sha256.txt")


def golden():
    """name -> {"I", "J", "R"} sha256 digests (and shape, dtype, conn)."""
    out = {}
    with open(GOLDEN) as f:
        for ln in f:
            if ln.startswith("#") or not ln.strip():
                continue
            name, shape, dt, conn, hI, hJ, hR = ln.split()
            out[name] = {"shape": shape, "dtype": dt, "conn": int(conn),
                         "I": hI, "J": hJ, "R": hR}
    return out


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


def _check_inputs(g, name, I, J):
    assert synth.sha256(I) == g[name]["I"], "%s: mask differs from the stored inputs" % name
    assert synth.sha256(J) == g[name]["J"], "%s: marker differs from the stored inputs" % name


def _first_difference(got, want):
    bad = got != want
    y, x = np.argwhere(bad)[0]
    return "%d pixels differ, first at (%d, %d): got %d want %d" % (
        bad.sum(), y, x, got[y, x], want[y, x])


def test_c3_i32_full_size_bit_exact(iwpp):
    import torch

    g = golden()
    announce("c3 int32 32768x32768: generating")
    I, J = synth.c3_i32()
    _check_inputs(g, "c3i32", I, J)
    dev = torch.device("cuda:0")
    announce("c3 int32 32768x32768: GPU reconstruction")
    Jt = torch.from_numpy(J).to(dev)
    It = torch.from_numpy(I).to(dev)
    st = iwpp.reconstruct(Jt, It, 8)
    assert st["tiles"] == 1024 * 512
    got = Jt.cpu().numpy()
    del Jt, It
    torch.cuda.empty_cache()
    announce("c3 int32: hashing the whole output")
    if synth.sha256(got) == g["c3i32"]["R"]:
        return
    announce("c3 int32: digest differs; oracle for the report (about 35 s)")
    rc, _ = oracle.reconstruct(J, I, 8, inplace=True)
    assert rc == oracle.OK
    raise AssertionError("c3 int32: " + _first_difference(got, J))


def test_c3_u8_full_size_bit_exact(iwpp):
    import torch

    g = golden()
    announce("c3 uint8 32768x32768: generating")
    I, J = synth.c3_u8()
    _check_inputs(g, "c3u8", I, J)
    H, W = I.shape
    dev = torch.device("cuda:0")
    announce("c3 uint8 32768x32768: GPU reconstruction")
    Jt = torch.from_numpy(J).to(dev)
    It = torch.from_numpy(I).to(dev)
    Rt = Jt.clone()
    iwpp.reconstruct(Rt, It, 8)
    R = Rt.cpu().numpy()
    announce("c3 uint8: hashing the whole output")
    if synth.sha256(R) == g["c3u8"]["R"]:
        return
    # diagnostics: which property fails, and sampled pixels against the
    # oracle's single-pixel search
    msgs = []
    if not (bool((Jt <= Rt).all()) and bool((Rt <= It).all())):
        msgs.append("J <= R <= I fails")
    P = torch.zeros((H + 2, W + 2), dtype=torch.uint8, device=dev)
    P[1:-1, 1:-1] = Rt
    m = Rt.clone()
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy or dx:
                torch.maximum(m, P[1 + dy:1 + dy + H, 1 + dx:1 + dx + W], out=m)
    del P
    if not torch.equal(Rt, torch.minimum(It, m)):
        msgs.append("not a fixed point")
    del m, Rt, Jt, It
    torch.cuda.empty_cache()
    rng = np.random.default_rng(77)
    rows = rng.integers(0, H, 200)
    cols = rng.integers(0, W, 200)
    rc, vals = oracle.pixels(J, I, rows, cols, 8, max_visit=1_500_000)
    done = vals != np.iinfo(np.int32).min
    wrong = done & (R[rows, cols].astype(np.int32) != vals)
    msgs.append("%d of %d completed samples differ" % (wrong.sum(), done.sum()))
    raise AssertionError("c3 uint8: digest differs from the oracle's; " + "; ".join(msgs))


def test_c4_full_batch_bit_exact(iwpp):
    """The 256-image batch at its full sizes (sides log-uniform 512..4096,
    about 1 Gpx), run as bench.py runs it: parameters tuned on the largest
    image, one plan, launched as a HIP graph and replayed twice.  After each
    replay every one of the 256 images is compared whole with the oracle's
    result (digests)."""
    import torch

    g = golden()
    announce("c4 256 images: generating")
    pairs = synth.c4()
    for k, (I, J) in enumerate(pairs):
        _check_inputs(g, "c4/%d" % k, I, J)
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
            bad = [k for k, w in enumerate(work)
                   if synth.sha256(w.cpu().numpy()) != g["c4/%d" % k]["R"]]
            if bad:
                I, J = pairs[bad[0]]
                rc, R = oracle.reconstruct(J, I, 8)
                assert rc == oracle.OK
                raise AssertionError("replay %d: %d images differ (%s); image %d: %s" % (
                    replay, len(bad), bad[:8], bad[0],
                    _first_difference(work[bad[0]].cpu().numpy(), R)))
    finally:
        plan.close()


def test_c1_c2_full_size_digests(iwpp):
    """The two small configurations through the plain single-image call, with
    the library defaults, against the stored digests."""
    import torch

    g = golden()
    dev = torch.device("cuda:0")
    for name, (I, J) in (("c1", synth.c1()), ("c2", synth.c2())):
        _check_inputs(g, name, I, J)
        announce("%s %dx%d: GPU reconstruction" % (name, I.shape[0], I.shape[1]))
        Jt = torch.from_numpy(J).to(dev)
        iwpp.reconstruct(Jt, torch.from_numpy(I).to(dev), 8)
        assert synth.sha256(Jt.cpu().numpy()) == g[name]["R"], name


def test_c5_recipe_pool_through_the_server_digests(iwpp):
    """The served stream's full request pool (256 requests, sides log-uniform
    256..8192, h-dome and fill-holes markers), each submitted once in a
    shuffled order to a server set up as bench.py sets it up (64 GB budget,
    two launch slots, up to 64 in flight): every output against the stored
    digest of the oracle's result for its request."""
    import torch

    g = golden()
    announce("c5 pool of 256: generating")
    pool = synth.c5_pool()
    for k, (I, J, _) in enumerate(pool):
        _check_inputs(g, "c5/%d" % k, I, J)
    dev = torch.device("cuda:0")
    masks = [torch.from_numpy(I).to(dev) for I, J, _ in pool]
    markers = [torch.from_numpy(J).to(dev) for I, J, _ in pool]
    order = [int(k) for k in np.random.default_rng(13).permutation(len(pool))]
    announce("c5 pool of 256: submitting")
    srv = iwpp.Server(64 << 30, "u8", 8, streams=2, max_inflight=64)
    try:
        tickets = [(k, srv.submit(markers[k], masks[k])) for k in order]
        for k, t in tickets:
            rc, lat = srv.wait(t)
            assert rc == iwpp.OK and lat > 0, (k, rc)
    finally:
        srv.close()
    announce("c5 pool of 256: comparing digests")
    bad = [k for k in range(len(pool))
           if synth.sha256(markers[k].cpu().numpy()) != g["c5/%d" % k]["R"]]
    if bad:
        I, J, _ = pool[bad[0]]
        rc, R = oracle.reconstruct(J, I, 8)
        assert rc == oracle.OK
        raise AssertionError("%d requests differ (%s); request %d: %s" % (
            len(bad), bad[:8], bad[0], _first_difference(markers[bad[0]].cpu().numpy(), R)))
