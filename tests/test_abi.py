"""The C-ABI library loads, exports every function include/iwpp.h declares,
and rejects bad arguments on the host before any GPU work (these tests make
no GPU call and run on a CPU-only host)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "iwpp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(iwpp_[a-z_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    import paper_1605_00930_amd as iwpp

    if not os.path.exists(iwpp.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()
    return iwpp._load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("iwpp_reconstruct", "iwpp_reconstruct_async", "iwpp_stream_status",
                 "iwpp_reconstruct_batched", "iwpp_batch_create", "iwpp_batch_launch",
                 "iwpp_autotune", "iwpp_server_create", "iwpp_server_submit",
                 "iwpp_server_wait", "iwpp_strerror"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(lib):
    assert lib.iwpp_version() >= 10000
    for code in range(0, -11, -1):
        assert lib.iwpp_strerror(code)
    assert lib.iwpp_strerror(-2) == b"marker exceeds mask at some pixel"


def test_argument_errors_before_gpu_work(lib):
    import paper_1605_00930_amd as iwpp

    E = iwpp.E_ARG
    buf = ctypes.create_string_buffer(64)
    other = ctypes.create_string_buffer(64)
    a, b = ctypes.addressof(buf), ctypes.addressof(other)
    # sizes, dtype, connectivity, null pointers
    assert lib.iwpp_reconstruct(a, b, 0, 4, 0, 8) == E
    assert lib.iwpp_reconstruct(a, b, 4, -1, 0, 8) == E
    assert lib.iwpp_reconstruct(a, b, 4, 4, 2, 8) == E
    assert lib.iwpp_reconstruct(a, b, 4, 4, 0, 6) == E
    assert lib.iwpp_reconstruct(None, b, 4, 4, 0, 8) == E
    assert lib.iwpp_reconstruct(a, a, 4, 4, 0, 8) == E  # marker and mask overlap
    im = iwpp.Image(a, b, 4, 4, 3)  # pitch < width
    assert lib.iwpp_reconstruct_async(ctypes.byref(im), 0, 8, 0, None, None) == E
    im = iwpp.Image(a, b, 4, 4, 0)
    assert lib.iwpp_reconstruct_async(ctypes.byref(im), 0, 8, 4, None, None) == E  # flags
    assert lib.iwpp_reconstruct_async(ctypes.byref(im), 0, 8, 8, None, None) == E
    p = iwpp.Params()
    p.tile_h = 48
    assert lib.iwpp_reconstruct_async(ctypes.byref(im), 0, 8, 0, ctypes.byref(p), None) == E
    p = iwpp.Params()
    p.mode = 3
    assert lib.iwpp_reconstruct_async(ctypes.byref(im), 0, 8, 0, ctypes.byref(p), None) == E
    p = iwpp.Params()
    p.first_pass = 3
    assert lib.iwpp_reconstruct_async(ctypes.byref(im), 0, 8, 0, ctypes.byref(p), None) == E
    im32 = iwpp.Image(a + 1, b, 4, 4, 0)  # misaligned int32
    assert lib.iwpp_reconstruct_async(ctypes.byref(im32), 1, 8, 0, None, None) == E
    arr = (iwpp.Image * 1)(iwpp.Image(a, b, 0, 4, 0))
    assert lib.iwpp_reconstruct_batched(arr, 1, 0, 8, 0, None, None) == E
    assert lib.iwpp_reconstruct_batched(arr, 0, 0, 8, 0, None, None) == E
    h = ctypes.c_void_p()
    assert lib.iwpp_batch_create(arr, 1, 0, 8, 0, None, ctypes.byref(h)) == E
    assert lib.iwpp_device_copy(a, b, 15, None) == E
    # fill holes: overlap, sizes, pitch, dtype, connectivity
    assert lib.iwpp_fill_holes_async(a, a, 4, 4, 0, 0, 8, None, None) == E
    assert lib.iwpp_fill_holes_async(a, b, 0, 4, 0, 0, 8, None, None) == E
    assert lib.iwpp_fill_holes_async(a, b, 4, 4, 3, 0, 8, None, None) == E
    assert lib.iwpp_fill_holes_async(a, b, 4, 4, 0, 7, 8, None, None) == E
    assert lib.iwpp_fill_holes_async(a, b, 4, 4, 0, 0, 5, None, None) == E
    assert lib.iwpp_fill_holes_async(None, b, 4, 4, 0, 0, 8, None, None) == E


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_1605_00930_amd as iwpp

    monkeypatch.setattr(iwpp, "_lib_obj", None)
    monkeypatch.setattr(iwpp, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        iwpp._load()


def test_noalloc_host_checks_before_gpu_work(lib):
    """iwpp_reconstruct_noalloc (the entry point for callers that cannot
    allocate) rejects bad arguments and images whose workspace exceeds its
    static array on the host, before any device call."""
    import paper_1605_00930_amd as iwpp

    buf = ctypes.create_string_buffer(64)
    other = ctypes.create_string_buffer(64)
    a, b = ctypes.addressof(buf), ctypes.addressof(other)
    f = lib.iwpp_reconstruct_noalloc

    def call(H, W, dtype=iwpp.U8, conn=8, mask=None, mode=0):
        im = iwpp.Image(a, b if mask is None else mask, H, W, 0)
        p = iwpp.Params()
        p.mode = mode
        return f(ctypes.byref(im), dtype, conn, 0, ctypes.byref(p), None, None)

    assert call(0, 5) == iwpp.E_ARG
    assert call(5, 5, conn=6) == iwpp.E_ARG
    assert call(5, 5, dtype=7) == iwpp.E_ARG
    assert call(5, 5, mode=1) == iwpp.E_UNSUPPORTED
    assert call(5, 5, mode=2) == iwpp.E_UNSUPPORTED
    far = b + (1 << 40)  # never dereferenced: the size check comes first
    assert call(40000, 40000, dtype=iwpp.I32, mask=far) == iwpp.E_SCRATCH
    assert call(16384, 32768, dtype=iwpp.I32, mask=far) == iwpp.E_SCRATCH
    assert call(65536, 65536, mask=far) == iwpp.E_SCRATCH
