"""Register and scratch budget of the persistent tile workers (CPU only).

The persistent kernels are sized for two wavefronts per SIMD (eight tiles per
CU), which holds only while one wavefront needs at most 256 registers (VGPRs
plus AGPRs) and no scratch.  The inliner may stop inlining a helper when a
kernel grows; the helper then becomes a call with a stack frame and the
kernel's register count is reported as a max() over its callees.  This test
compiles the device code to gfx950 assembly and checks every persistent
kernel for all three.
"""
from __future__ import annotations

import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1605_00930_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _asm(src, out):
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", out]
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)


@pytest.fixture(scope="module")
def resources(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    d = tmp_path_factory.mktemp("asm")
    jobs = []
    for src in ("iwpp_kernels.hip", "iwpp_edt.hip"):
        out = str(d / (src + ".s"))
        jobs.append((out, _asm(src, out)))
    res = {}
    pat = re.compile(r"^\s*\.set\s+(\S*k_persistent\S*)\.(num_vgpr|num_agpr|private_seg_size),\s*(.+)$")
    for out, p in jobs:
        log = p.communicate()[0].decode(errors="replace")
        assert p.returncode == 0, log
        for line in open(out):
            m = pat.match(line)
            if m:
                res.setdefault(m.group(1), {})[m.group(2)] = m.group(3).strip()
    assert res, "no persistent kernels found in the assembly"
    return res


def test_persistent_kernels_fit_two_waves_per_simd(resources):
    bad = []
    for name, r in sorted(resources.items()):
        vals = {k: r.get(k, "") for k in ("num_vgpr", "num_agpr", "private_seg_size")}
        if not all(v.isdigit() for v in vals.values()):
            bad.append("%s calls out-of-line helpers: %s" % (name, vals))
            continue
        v, a, p = (int(vals[k]) for k in ("num_vgpr", "num_agpr", "private_seg_size"))
        if p != 0 or v + a > 256:
            bad.append("%s: %d VGPR + %d AGPR, %d B scratch" % (name, v, a, p))
    assert not bad, "\n".join(bad)
