"""The entry point that allocates nothing (iwpp_reconstruct_noalloc, for
callers that cannot allocate) gives the same result as the existing
single-image entry point, iwpp_reconstruct_async, bit for bit; both are
called through the C ABI.  Two calls in a row share the static workspace, the
second with a smaller image, so what the first left there must not leak into
the second."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

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


def _abi_existing(iwpp, J, I, flags, stream):
    """iwpp_reconstruct_async on a copy of J; returns (status, result)."""
    out = J.clone()
    im, dt = iwpp._image(out, I)
    rc = iwpp._load().iwpp_reconstruct_async(ctypes.byref(im), dt, 8, flags, None,
                                             stream.cuda_stream)
    assert rc == iwpp.OK
    st = iwpp.Stats()
    rc = iwpp._load().iwpp_stream_status(stream.cuda_stream, ctypes.byref(st))
    return rc, out


def _abi_noalloc(iwpp, J, I, flags, stream):
    """iwpp_reconstruct_noalloc on a copy of J; returns (status, result)."""
    import torch

    out = J.clone()
    status = torch.full((1,), 12345, dtype=torch.int32, device=J.device)
    im, dt = iwpp._image(out, I)
    torch.cuda.synchronize()
    rc = iwpp._load().iwpp_reconstruct_noalloc(ctypes.byref(im), dt, 8, flags, None,
                                               status.data_ptr(), stream.cuda_stream)
    assert rc == iwpp.OK
    stream.synchronize()
    return int(status.item()), out


@pytest.mark.parametrize("dtype", ["u8", "i32"])
def test_noalloc_matches_existing_entry_point(iwpp, dtype):
    import torch

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    if dtype == "u8":
        first = synth.c2(H=1500, W=1700)     # fill-holes form: long fronts
        second = synth.c1(H=300, W=200)      # smaller, ragged
    else:
        first = synth.c3_i32(H=1200, W=1300)
        second = synth.c3_i32(seed=5, H=200, W=333)
    for call, (I, J) in enumerate((first, second)):
        print("[gpu-case] noalloc %s call %d: %dx%d" % (dtype, call, I.shape[0], I.shape[1]),
              flush=True)
        It = torch.from_numpy(I).to(dev)
        Jt = torch.from_numpy(J).to(dev)
        rc_a, want = _abi_existing(iwpp, Jt, It, 0, stream)
        rc_b, got = _abi_noalloc(iwpp, Jt, It, 0, stream)
        assert rc_a == iwpp.OK and rc_b == iwpp.OK
        assert torch.equal(got, want), "call %d: %d pixels differ" % (
            call, int((got != want).sum()))


def test_noalloc_reports_marker_above_mask(iwpp):
    import torch

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    I, J = synth.c1(H=260, W=130)
    J = J.copy()
    J[100, 70] = min(255, int(I[100, 70]) + 5)
    It = torch.from_numpy(I).to(dev)
    Jt = torch.from_numpy(J).to(dev)
    for flags, want_rc in ((0, iwpp.E_MARKER_GT_MASK), (iwpp.FLAG_CLAMP_MARKER, iwpp.OK)):
        rc_a, want = _abi_existing(iwpp, Jt, It, flags, stream)
        rc_b, got = _abi_noalloc(iwpp, Jt, It, flags, stream)
        assert rc_a == want_rc and rc_b == want_rc
        assert torch.equal(got, want)
