"""The pins must be strong enough to catch plausible mistakes in the oracle.

Each case copies the oracle's C sources to a temporary directory, plants one
mistake (a dropped term, a wrong sign or index, a transposed operand), builds
that copy with gcc and checks that the definition-level pin (brute-force
iteration, tests/refdefs.py) rejects it on a modest fuzz set.  The real
oracle is never modified.
"""
from __future__ import annotations

import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth
from tests import refdefs

SRC = os.path.dirname(oracle.__file__)

# (file, original text, planted mistake, entry point exercised)
MUTANTS = {
    # (The raster half N+ is not listed: the anti-raster scan alone sets up
    # the seed invariant, so a wrong N+ only costs work, not correctness.)
    "anti_raster_wrong_column_order": (
        "oracle_body.inc", "for (int64_t c = W - 1; c >= 0; --c) {",
        "for (int64_t c = 0; c < W; ++c) {", "reconstruct"),
    "anti_raster_half_dropped_term": (
        "oracle.c", "NMINUS8[4] = {{0, 1}, {1, -1}, {1, 0}, {1, 1}}",
        "NMINUS8[4] = {{0, 1}, {1, 1}, {1, 0}, {1, 1}}", "reconstruct"),
    "full_neighbourhood_dropped_corner": (
        "oracle.c", "{0, 1},   {1, -1}, {1, 0},  {1, 1}}",
        "{0, 1},   {1, -1}, {1, 0},  {1, 0}}", "reconstruct"),
    "propagation_drops_mask": (
        "oracle_body.inc", "J[qq] = J[p] < I[qq] ? J[p] : I[qq];", "J[qq] = J[p];",
        "reconstruct"),
    "seed_rule_reversed": (
        "oracle_body.inc",
        "          if (J[qq] < J[p] && J[qq] < I[qq]) {\n            if (queue_push(&q, p)) goto nomem;\n            if (st) st->seeds++;\n            break;\n          }\n        }\n      }\n    }\n  }\n  if (nsweeps == 0)",
        "          if (J[qq] > J[p] && J[qq] < I[qq]) {\n            if (queue_push(&q, p)) goto nomem;\n            if (st) st->seeds++;\n            break;\n          }\n        }\n      }\n    }\n  }\n  if (nsweeps == 0)",
        "reconstruct"),
    "scan_mask_on_wrong_pixel": (
        "oracle_body.inc",
        "        J[p] = m < I[p] ? m : I[p];\n        if (!last) continue;",
        "        J[p] = m < I[p] ? m : I[p];\n        if (p + 1 < H * W && J[p] > I[p + 1]) J[p] = I[p + 1];\n        if (!last) continue;",
        "reconstruct"),
    "heap_drops_mask": (
        "oracle_body.inc",
        "const int64_t cand = e.key < (int64_t)I[qq] ? e.key : (int64_t)I[qq];",
        "const int64_t cand = e.key;", "widest"),
    "brute_stops_after_one_pass": (
        "oracle_body.inc", "if (nv != J[p]) changed = 1;", "(void)0;", "brute"),
}


def _build_mutant(tmp_path, fname, old, new):
    d = tmp_path / "src"
    d.mkdir()
    for f in ("oracle.c", "oracle.h", "oracle_body.inc"):
        shutil.copy(os.path.join(SRC, f), d / f)
    text = (d / fname).read_text()
    assert text.count(old) >= 1, "mutation anchor not found: %r" % old
    (d / fname).write_text(text.replace(old, new, 1))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", str(lib),
                    str(d / "oracle.c")], check=True)
    return ctypes.CDLL(str(lib))


def _run(lib, entry, J, I, conn):
    suf = "u8" if J.dtype == np.uint8 else "i32"
    R = J.copy()
    st = oracle.Stats()
    if entry == "reconstruct":
        f = getattr(lib, "oracle_reconstruct_" + suf)
        f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                      ctypes.c_int, ctypes.c_uint, ctypes.c_int, ctypes.c_int,
                      ctypes.c_uint64, ctypes.c_int64, ctypes.POINTER(oracle.Stats)]
        rc = f(R.ctypes.data, I.ctypes.data, R.shape[0], R.shape[1], conn, 0, 1, 0, 0, -1,
               ctypes.byref(st))
    else:
        f = getattr(lib, "oracle_%s_%s" % (entry, suf))
        f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                      ctypes.c_int, ctypes.POINTER(oracle.Stats)]
        rc = f(R.ctypes.data, I.ctypes.data, R.shape[0], R.shape[1], conn, ctypes.byref(st))
    return rc, R


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name, tmp_path):
    fname, old, new, entry = MUTANTS[name]
    lib = _build_mutant(tmp_path, fname, old, new)
    rng = np.random.default_rng(1234)
    caught = 0
    for t in range(400):
        H, W = (int(v) for v in rng.integers(1, 17, 2))
        dtype = np.uint8 if t % 2 else np.int32
        I, J = synth.random_pair(rng, H, W, dtype, "uniform", levels=int(rng.integers(2, 9)))
        rc, R = _run(lib, entry, J, I, 8)
        if rc != 0 or not np.array_equal(R, refdefs.brute_numpy(J, I, 8)):
            caught += 1
    assert caught > 0, "planted mistake %s went unnoticed" % name
