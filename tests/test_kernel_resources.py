"""Register budget, scratch use and memory coherence of the persistent tile
workers (CPU only).

The persistent kernels are sized for two wavefronts per SIMD (eight tiles per
CU), which holds only while one wavefront needs at most 256 registers (VGPRs
plus AGPRs) and no scratch.  The inliner may stop inlining a helper when a
kernel grows; the helper then becomes a call with a stack frame and the
kernel's register count is reported as a max() over its callees.  This test
compiles the device code to gfx950 assembly and checks every persistent
kernel for all three.

Tiles are handed from a workgroup on one XCD to a workgroup on another, each
with its own L2, without any L2 write-back or invalidate: every access to
memory that other workgroups write during a launch (the marker J, the packed
side columns of J and I, tile states, flags, queues) is an agent-scope
relaxed atomic, served coherently device-wide (`sc1` on gfx950), and only the
mask I, which nothing writes, is read with plain loads.  Two checks hold the
sources to that: a lint of the device sources (every subscript of a pointer
into the marker or the packed columns sits inside `ld_coherent` /
`st_coherent`, and a buffer resource built over the marker is read only with
`ld_coherent_b128`, the 16-byte load with the same cache policy; four planted
plain accesses must be caught), and the compiled persistent kernels (every
global store carries `sc1`, and no `buffer_wbl2` or `buffer_inv` appears).
"""
from __future__ import annotations

import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1605_00930_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
DEVICE_SOURCES = ("iwpp_device.h", "iwpp_kernels.hip", "iwpp_edt.hip")


def _asm(src, out):
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", out]
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)


@pytest.fixture(scope="module")
def persistent_asm(tmp_path_factory):
    """{kernel symbol: (resource fields, body lines)} of every persistent kernel."""
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    d = tmp_path_factory.mktemp("asm")
    jobs = []
    for src in ("iwpp_kernels.hip", "iwpp_edt.hip"):
        out = str(d / (src + ".s"))
        jobs.append((out, _asm(src, out)))
    res = {}
    pat = re.compile(r"^\s*\.set\s+(\S*k_persistent\S*)\.(num_vgpr|num_agpr|private_seg_size),\s*(.+)$")
    label = re.compile(r"^(_Z\S+):")
    for out, p in jobs:
        log = p.communicate()[0].decode(errors="replace")
        assert p.returncode == 0, log
        cur = None
        for line in open(out):
            m = pat.match(line)
            if m:
                res.setdefault(m.group(1), ({}, []))[0][m.group(2)] = m.group(3).strip()
                continue
            m = label.match(line)
            if m:
                cur = m.group(1) if "k_persistent" in m.group(1) else None
                continue
            if line.startswith("\t.end_amdgpu") or line.startswith(".Lfunc_end"):
                cur = None
            if cur:
                res.setdefault(cur, ({}, []))[1].append(line.strip())
    assert res, "no persistent kernels found in the assembly"
    return res


def test_persistent_kernels_fit_two_waves_per_simd(persistent_asm):
    bad = []
    for name, (r, _) in sorted(persistent_asm.items()):
        vals = {k: r.get(k, "") for k in ("num_vgpr", "num_agpr", "private_seg_size")}
        if not all(v.isdigit() for v in vals.values()):
            bad.append("%s calls out-of-line helpers: %s" % (name, vals))
            continue
        v, a, p = (int(vals[k]) for k in ("num_vgpr", "num_agpr", "private_seg_size"))
        if p != 0 or v + a > 256:
            bad.append("%s: %d VGPR + %d AGPR, %d B scratch" % (name, v, a, p))
    assert not bad, "\n".join(bad)


def test_persistent_kernels_store_coherently_without_l2_maintenance(persistent_asm):
    bad = []
    checked = 0
    for name, (_, body) in sorted(persistent_asm.items()):
        stores = [l for l in body if l.startswith("global_store")]
        if not stores:
            continue
        checked += 1
        plain = [l for l in stores if not re.search(r"\bsc1\b", l)]
        if plain:
            bad.append("%s: %d of %d global stores without sc1, e.g. %s"
                       % (name, len(plain), len(stores), plain[0]))
        maint = [l for l in body if l.startswith(("buffer_wbl2", "buffer_inv"))]
        if maint:
            bad.append("%s: L2 maintenance %s" % (name, maint[0]))
        # the marker rows go out as stores, never through the scalar cache
        if any(l.startswith(("s_store", "s_buffer_store")) for l in body):
            bad.append("%s: scalar store" % name)
    assert checked >= 10, "expected the u8, i32 and distance-transform workers"
    assert not bad, "\n".join(bad)


# ----------------------------------------------------------------- source lint

_SHARED_BASES = r"(?:im\.J|kp\.colJ|kp\.colI)\b"


def _strip_comments(text):
    text = re.sub(r"/\*.*?\*/", lambda m: " " * len(m.group(0)), text, flags=re.S)
    return re.sub(r"//[^\n]*", "", text)


def _shared_pointer_names(code):
    """Local pointers initialised from the marker or a packed column, or
    from another such pointer."""
    names = set()
    decl = re.compile(r"\b(?:const\s+)?gptr<[^;=]*?>\s+(\w+)\s*=\s*([^;]*);")
    decls = [(m.group(1), m.group(2)) for m in decl.finditer(code)]
    while True:
        known = [_SHARED_BASES] + [r"\b%s\b" % re.escape(n) for n in names]
        pat = re.compile("|".join(known))
        new = {n for n, init in decls if pat.search(init)} - names
        if not new:
            return names
        names |= new


def _inside_coherent_call(prefix):
    """True if `prefix` (the text before an access) ends inside the pointer
    argument of ld_coherent / st_coherent: only '&', '(' and pointer casts
    may stand between the call and the access."""
    p = prefix.rstrip()
    while True:
        q = re.sub(r"\(\s*(?:const\s+)?gptr<[^()]*?>\s*\)\s*$", "", p).rstrip()
        q = re.sub(r"[&(]\s*$", "", q).rstrip()
        if q == p:
            break
        p = q
    return re.search(r"\b(?:ld|st)_coherent\s*$", p) is not None


def lint_coherent_access(sources):
    """Accesses to the marker or the packed side columns that are not
    agent-scope atomics: a list of 'file:line: text' findings."""
    found = []
    for fname, text in sources.items():
        code = _strip_comments(text)
        names = _shared_pointer_names(code)
        pats = [re.compile(r"\b%s\s*\[" % re.escape(n)) for n in names]
        pats.append(re.compile(_SHARED_BASES + r"\s*\)\s*\["))  # ((gptr<T>)kp.colJ)[k]
        pats.append(re.compile(_SHARED_BASES + r"\s*\["))       # kp.colJ[k]
        # a pointer is never multiplied, so '*' before one is a dereference
        derefs = [re.compile(r"\*\s*%s\b" % re.escape(n)) for n in names]
        lines = code.split("\n")
        for i, line in enumerate(lines, 1):
            for pat in pats:
                for m in pat.finditer(line):
                    if not _inside_coherent_call(line[:m.start()]):
                        found.append("%s:%d: %s" % (fname, i, line.strip()))
            for pat in derefs:
                if pat.search(line):
                    found.append("%s:%d: %s" % (fname, i, line.strip()))
            if names and re.search(r"\b(?:%s)\s*->" % "|".join(map(re.escape, names)), line):
                found.append("%s:%d: %s" % (fname, i, line.strip()))
        # buffer resources over the marker: every use is a coherent 16-byte load
        shared = re.compile("|".join([_SHARED_BASES] + [r"\b%s\b" % re.escape(n) for n in names]))
        for m in re.finditer(r"(\w+)\s*=\s*rows_rsrc\(([^;]*)\);", code):
            if not shared.search(m.group(2)):
                continue
            for u in re.finditer(r"\b%s\b" % re.escape(m.group(1)), code[m.end():]):
                at = m.end() + u.start()
                if not re.search(r"\bld_coherent_b128\s*\(\s*$", code[:at]):
                    i = code.count("\n", 0, at) + 1
                    found.append("%s:%d: %s" % (fname, i, lines[i - 1].strip()))
    return sorted(set(found))


def _read_sources():
    return {f: open(os.path.join(CSRC, f)).read() for f in DEVICE_SOURCES}


def test_marker_and_side_columns_are_accessed_coherently():
    src = _read_sources()
    code = _strip_comments(src["iwpp_kernels.hip"])
    # the lint sees the pointers it has to police
    assert {"gJ", "row"} <= _shared_pointer_names(code)
    assert "gI" not in _shared_pointer_names(code)  # the mask is read-only
    assert "gS" in _shared_pointer_names(_strip_comments(src["iwpp_edt.hip"]))
    # the int32 tiles' 16-byte marker loads go through a buffer resource
    assert re.search(r"\brj\s*=\s*rows_rsrc\(\(const void\*\)\(gJ\b", code)
    assert lint_coherent_access(src) == []


@pytest.mark.parametrize("old,new", [
    ("(int)ld_coherent(&gJ[gy * im.ld + gx])", "(int)gJ[gy * im.ld + gx]"),
    ("st_coherent(row, w[q]);", "*row = w[q];"),
    ("ld_coherent(&((gptr<const T>)kp.colI)[k])", "((gptr<const T>)kp.colI)[k]"),
    ("p.r.jq[q] = ld_coherent_b128(rj,", "p.r.jq[q] = ld_plain_b128(rj,"),
])
def test_lint_catches_a_plain_access(old, new):
    src = _read_sources()
    assert old in src["iwpp_kernels.hip"], old
    src["iwpp_kernels.hip"] = src["iwpp_kernels.hip"].replace(old, new, 1)
    found = lint_coherent_access(src)
    assert len(found) == 1 and new in found[0], found


def test_lint_follows_derived_pointers():
    src = {"probe.hip": """
      const gptr<const T> gJ = (gptr<const T>)im.J;
      const gptr<const uint64_t> pj = (gptr<const uint64_t>)(gJ + gy * im.ld + gx);
      const gptr<const T> gI = (gptr<const T>)im.I;
      a = ld_coherent(&pj[0]);
      b = gI[k];
      c = pj[1];
    """}
    found = lint_coherent_access(src)
    assert len(found) == 1 and "c = pj[1]" in found[0], found
