"""Writes tests/golden/full_size_sha256.txt: sha256 digests of the inputs and of
the CPU oracle's reconstruction for every synthetic workload at its full size.

It calls only ``synth`` (the seeded input generators) and ``oracle`` (the
sequential hybrid algorithm: raster scan, anti-raster scan with the seed rule,
FIFO queue; IWPP chapter, reconstruction algorithm in IWPP form).  Nothing
here touches the GPU library.  The GPU parity tests and bench.py hash the
library's whole output and compare it with these digests.

One line per image:
    name  HxW  dtype  conn  sha256(I)  sha256(J)  sha256(R)
Names: c1, c2, c3i32, c3u8, c4/<k> for the 256 images of the batch, c5/<k> for
the 256 requests of the served stream's pool.

Run from the repository root (about 5 minutes on 8 cores; the 32768^2 uint8
fill-holes image alone takes the oracle about 4 minutes of one core):
    python tests/golden/make_full_size_hashes.py [--jobs N]
"""
from __future__ import annotations

import argparse
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "full_size_sha256.txt")
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _line(name, I, J, conn=8):
    import oracle
    import synth

    rc, R = oracle.reconstruct(J, I, conn)
    if rc != oracle.OK:
        raise RuntimeError("%s: oracle status %d" % (name, rc))
    return "%s %dx%d %s %d %s %s %s" % (name, I.shape[0], I.shape[1],
                                         "u8" if I.dtype.name == "uint8" else "i32", conn,
                                         synth.sha256(I), synth.sha256(J), synth.sha256(R))


def job(spec):
    """One work item: a single image, or a range of batch / pool images."""
    import synth

    kind = spec[0]
    t0 = time.perf_counter()
    if kind == "c1":
        out = [_line("c1", *synth.c1())]
    elif kind == "c2":
        out = [_line("c2", *synth.c2())]
    elif kind == "c3i32":
        out = [_line("c3i32", *synth.c3_i32())]
    elif kind == "c3u8":
        out = [_line("c3u8", *synth.c3_u8())]
    elif kind == "c4":
        lo, hi = spec[1], spec[2]
        pairs = synth.c4(only=range(lo, hi))
        out = [_line("c4/%d" % k, *p) for k, p in zip(range(lo, hi), pairs)]
    elif kind == "c5":
        lo, hi = spec[1], spec[2]
        pool = synth.c5_pool(n=256, only=range(lo, hi))
        out = [_line("c5/%d" % k, I, J) for k, (I, J, _) in zip(range(lo, hi), pool)]
    else:
        raise ValueError(kind)
    print("[golden] %s done in %.1f s" % (spec, time.perf_counter() - t0), flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    args = ap.parse_args()
    specs = [("c3u8",), ("c3i32",), ("c1",), ("c2",)]
    specs += [("c4", k, min(256, k + 32)) for k in range(0, 256, 32)]
    specs += [("c5", k, min(256, k + 32)) for k in range(0, 256, 32)]
    with ProcessPoolExecutor(max_workers=args.jobs) as ex:
        results = list(ex.map(job, specs))
    lines = [ln for r in results for ln in r]
    order = {"c1": 0, "c2": 1, "c3i32": 2, "c3u8": 3, "c4": 4, "c5": 5}

    def key(ln):
        name = ln.split()[0]
        base, _, k = name.partition("/")
        return (order[base], int(k) if k else 0)

    lines.sort(key=key)
    with open(OUT + ".tmp", "w") as f:
        f.write("# name HxW dtype conn sha256(I) sha256(J) sha256(R); written by "
                "tests/golden/make_full_size_hashes.py from synth/ and oracle/ only\n")
        for ln in lines:
            f.write(ln + "\n")
    os.replace(OUT + ".tmp", OUT)
    print("[golden] wrote %d lines to %s" % (len(lines), OUT))


if __name__ == "__main__":
    main()
