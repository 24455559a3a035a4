"""GPU tests of the continuous-batching server: every result equals the CPU
oracle and the same request run alone, whatever else shares the device."""
from __future__ import annotations

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


def _pool(n, lo, hi, seed=4):
    return synth.c5_pool(seed=seed, n=n, lo=lo, hi=hi)


def _expect(I, J):
    rc, R = oracle.reconstruct(J, I, 8)
    assert rc == oracle.OK
    return R


def test_server_mix_equals_alone_equals_oracle(iwpp):
    import torch

    dev = torch.device("cuda:0")
    pool = _pool(24, 40, 600)
    masks = [torch.from_numpy(I).to(dev) for I, J, _ in pool]
    pristine = [torch.from_numpy(J).to(dev) for I, J, _ in pool]
    want = [_expect(I, J) for I, J, _ in pool]
    print("[gpu-case] server mix of 24 requests, 3 copies each", flush=True)
    srv = iwpp.Server(8 << 30, "u8", 8, streams=4, max_inflight=64)
    outs, tickets = [], []
    for rep in range(3):  # many requests in flight at once
        for k in range(len(pool)):
            out = torch.empty_like(pristine[k])
            outs.append((k, out))
            tickets.append(srv.submit(out, masks[k], marker_init=pristine[k]))
    lats = []
    for t in tickets:
        rc, lat = srv.wait(t)
        assert rc == iwpp.OK
        lats.append(lat)
    for k, out in outs:
        np.testing.assert_array_equal(out.cpu().numpy(), want[k])
    # alone: one request at a time through the server and through the plain call
    for k in range(0, len(pool), 5):
        out = pristine[k].clone()
        rc, _ = srv.wait(srv.submit(out, masks[k]))
        assert rc == iwpp.OK
        np.testing.assert_array_equal(out.cpu().numpy(), want[k])
        out = pristine[k].clone()
        iwpp.reconstruct(out, masks[k], 8)
        np.testing.assert_array_equal(out.cpu().numpy(), want[k])
    srv.close()
    assert all(l > 0 for l in lats)


def test_server_budget_admission(iwpp):
    import torch

    dev = torch.device("cuda:0")
    pool = _pool(6, 200, 300, seed=9)
    masks = [torch.from_numpy(I).to(dev) for I, J, _ in pool]
    pristine = [torch.from_numpy(J).to(dev) for I, J, _ in pool]
    biggest = max(2 * I.size for I, J, _ in pool)
    print("[gpu-case] server with a budget for about one request", flush=True)
    # room for about one request at a time: admission has to wait
    srv = iwpp.Server(int(biggest * 1.5) + (1 << 16), "u8", 8, streams=2, max_inflight=8)
    outs = [p.clone() for p in pristine]
    tickets = [srv.submit(o, m) for o, m in zip(outs, masks)]
    for t in tickets:
        rc, _ = srv.wait(t)
        assert rc == iwpp.OK
    for (I, J, _), o in zip(pool, outs):
        np.testing.assert_array_equal(o.cpu().numpy(), _expect(I, J))
    # a request that can never fit is refused at submit time
    big = torch.zeros((2000, 2000), dtype=torch.uint8, device=dev)
    with pytest.raises(iwpp.IwppError) as e:
        srv.submit(big, big.clone())
    assert e.value.code == iwpp.E_BUDGET
    srv.close()


def test_server_wait_timeout_and_unknown_ticket(iwpp):
    import torch

    dev = torch.device("cuda:0")
    I, J = synth.c2(H=256, W=256)
    srv = iwpp.Server(1 << 30, "u8", 8, streams=1, max_inflight=4)
    m = torch.from_numpy(I).to(dev)
    o = torch.from_numpy(J).to(dev)
    t = srv.submit(o, m)
    rc, _ = srv.wait(t, timeout_us=10_000_000)
    assert rc == iwpp.OK
    rc, _ = srv.wait(t)  # already collected
    assert rc == iwpp.E_ARG
    srv.close()
    np.testing.assert_array_equal(o.cpu().numpy(), _expect(I, J))


def test_server_full_size_stream(iwpp):
    """Requests at the served stream's full sizes (sides log-uniform
    256..8192, h-dome and fill-holes markers), three copies of each in a
    shuffled order, through a server set up as the benchmark sets it up
    (64 GB budget, two launch slots, up to 64 in flight): every result equals
    the oracle's for its request."""
    import torch

    dev = torch.device("cuda:0")
    pool = synth.c5_pool(seed=11, n=12, lo=256, hi=8192)
    print("[gpu-case] server full-size stream: %s"
          % [(I.shape[0], kind) for I, _, kind in pool], flush=True)
    masks = [torch.from_numpy(I).to(dev) for I, J, _ in pool]
    pristine = [torch.from_numpy(J).to(dev) for I, J, _ in pool]
    order = np.random.default_rng(12).permutation(np.repeat(np.arange(len(pool)), 3))
    srv = iwpp.Server(64 << 30, "u8", 8, streams=2, max_inflight=64)
    try:
        outs = []
        for k in order:
            out = torch.empty_like(pristine[k])
            outs.append((int(k), out, srv.submit(out, masks[k], marker_init=pristine[k])))
        for k, _, t in outs:
            rc, lat = srv.wait(t)
            assert rc == iwpp.OK and lat > 0
    finally:
        srv.close()
    for k, (I, J, _) in enumerate(pool):
        want = _expect(I, J)
        for kk, out, _ in outs:
            if kk == k:
                np.testing.assert_array_equal(out.cpu().numpy(), want)


def test_server_waits_for_the_callers_stream(iwpp):
    """A marker and mask written on a stream just before submit (here behind
    a long dummy computation on that stream) are what the request reads: the
    request's work starts after the work queued on the submitting stream."""
    import torch

    dev = torch.device("cuda:0")
    pool = _pool(4, 700, 900, seed=21)
    srv = iwpp.Server(8 << 30, "u8", 8, streams=2, max_inflight=16)
    side = torch.cuda.Stream()
    try:
        outs = []
        for I, J, _ in pool:
            with torch.cuda.stream(side):
                a = torch.randn(4096, 4096, device=dev)
                for _ in range(8):  # keeps the stream busy for a while
                    a = a @ a
                    a = a / a.abs().max()
                mask = torch.from_numpy(I).to(dev, non_blocking=True)
                marker = torch.from_numpy(J).to(dev, non_blocking=True)
                marker.add_(0)
                t = srv.submit(marker, mask, stream=side)
            outs.append((marker, mask, t))
        for marker, mask, t in outs:
            rc, _ = srv.wait(t)
            assert rc == iwpp.OK
        torch.cuda.synchronize()
        for (I, J, _), (marker, _, _) in zip(pool, outs):
            np.testing.assert_array_equal(marker.cpu().numpy(), _expect(I, J))
    finally:
        srv.close()
