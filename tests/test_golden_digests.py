"""The stored full-size digests (tests/golden/full_size_sha256.txt, written by
tests/golden/make_full_size_hashes.py from the oracle and the generators)
agree with the oracle and the generators as they stand: the cheap entries are
recomputed here, the large ones are checked for form."""
from __future__ import annotations

import os

import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size_sha256.txt")


def entries():
    out = {}
    for ln in open(GOLDEN):
        if ln.startswith("#") or not ln.strip():
            continue
        f = ln.split()
        assert len(f) == 7, ln
        out[f[0]] = f[1:]
    return out


def test_form():
    e = entries()
    assert len(e) == 4 + 256 + 256
    for name, (shape, dt, conn, hI, hJ, hR) in e.items():
        H, W = (int(v) for v in shape.split("x"))
        assert H >= 1 and W >= 1 and dt in ("u8", "i32") and conn == "8"
        assert all(len(h) == 64 and int(h, 16) >= 0 for h in (hI, hJ, hR))
    assert e["c3i32"][:2] == ["32768x32768", "i32"]
    assert e["c3u8"][:2] == ["32768x32768", "u8"]


@pytest.mark.parametrize("name", ["c1", "c2", "c4/0", "c4/255", "c5/1"])
def test_recomputed(name):
    base, _, k = name.partition("/")
    if base == "c1":
        I, J = synth.c1()
    elif base == "c2":
        I, J = synth.c2()
    elif base == "c4":
        (I, J), = synth.c4(only=[int(k)])
    else:
        (I, J, _), = synth.c5_pool(n=256, only=[int(k)])
    shape, dt, conn, hI, hJ, hR = entries()[name]
    assert shape == "%dx%d" % I.shape
    assert synth.sha256(I) == hI and synth.sha256(J) == hJ
    rc, R = oracle.reconstruct(J, I, 8)
    assert rc == oracle.OK
    assert synth.sha256(R) == hR
