"""GPU distance transform through the C ABI against the CPU oracle.

The site propagation stops at a state that depends on the order in which
pixels were processed only through ties and the rare pixels where the
propagation misses the exact nearest site.  The unique parts are compared
exactly: wherever the answer is unique (one background pixel, a background
frame around a rectangle) the distances must equal the oracle's bit for
bit.  Elsewhere the GPU result must be a valid end state (every site is
background, distances match sites, no neighbour offers a strictly closer
site) and never below the exact transform.  With 8-connectivity it must be
no farther from the exact transform than the oracle is: at most twice the
oracle's rate of pixels that miss the exact distance (plus 1e-4 of the
image), by at most twice its largest miss.  With 4-connectivity the passes
carry a site along a column, then along a row, where the oracle's FIFO queue
moves it in staircases, and they miss more often than the oracle; there the
same bound is taken against a CPU model of the library's passes
(tests/edt_pass_model.py: the tile rules in bulk-synchronous rounds), which
misses as the passes do.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth
from tests import refdefs
from tests.edt_pass_model import edt_pass_model

pytestmark = pytest.mark.gpu


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


def gpu_edt(iwpp, img, conn, **kw):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(img)).to(torch.device("cuda:0"))
    sites, d2, st = iwpp.edt(t, conn, **kw)
    return sites.cpu().numpy(), d2.cpu().numpy().astype(np.int64), st


def oracle_edt(img, conn):
    rc, sites, d2 = oracle.edt(img, conn)
    assert rc == oracle.OK
    return sites, d2


@pytest.mark.parametrize("conn", [8, 4])
def test_unique_cases_bit_exact(iwpp, conn):
    cases = []
    for (H, W, y, x) in [(1, 1, 0, 0), (1, 100, 0, 37), (90, 1, 11, 0), (100, 130, 3, 120),
                         (64, 64, 63, 63), (33, 200, 16, 100)]:
        img = np.ones((H, W), np.uint8)
        img[y, x] = 0
        cases.append(img)
    frame = np.ones((97, 141), np.uint8)
    frame[0, :] = frame[-1, :] = frame[:, 0] = frame[:, -1] = 0
    cases.append(frame)
    for img in cases:
        announce("edt unique %dx%d conn %d" % (img.shape[0], img.shape[1], conn))
        sites, d2, _ = gpu_edt(iwpp, img, conn)
        _, want = oracle_edt(img, conn)
        np.testing.assert_array_equal(d2, want)
        refdefs.edt_check_valid(img, sites, d2, conn)


@pytest.mark.parametrize("conn", [8, 4])
def test_valid_and_close_to_oracle(iwpp, conn):
    rng = np.random.default_rng(20 + conn)
    cases = [(rng.random((H, W)) < p).astype(np.uint8)
             for (H, W, p) in [(2, 3, 0.5), (31, 65, 0.6), (65, 63, 0.95), (129, 257, 0.99),
                               (200, 199, 0.999), (300, 400, 0.9)]]
    I = synth.ellipses(np.random.default_rng(1), 700, 900, 80)
    cases.append((I > 50).astype(np.uint8))
    cases.append((I <= 50).astype(np.uint8))
    for img in cases:
        announce("edt %dx%d conn %d" % (img.shape[0], img.shape[1], conn))
        sites, d2, st = gpu_edt(iwpp, img, conn)
        refdefs.edt_check_valid(img, sites, d2, conn)
        ex = refdefs.edt_exact_sq(img)
        assert (d2 >= ex).all()
        # both sides miss the exact transform on a few pixels, not always the
        # same ones: the GPU may miss at most twice as often as the oracle
        # (plus 1e-4 of the pixels) and by at most twice its largest miss
        _, want = oracle_edt(img, conn)
        o_rate = (want != ex).mean()
        o_err = (np.sqrt(want) - np.sqrt(ex)).max()
        g_rate = (d2 != ex).mean()
        g_err = (np.sqrt(d2) - np.sqrt(ex)).max()
        announce("  misses exact: gpu %.5f (max %.3f px), oracle %.5f (max %.3f px)"
                 % (g_rate, g_err, o_rate, o_err))
        if conn == 8:
            assert g_rate <= 2 * o_rate + 1e-4
            assert g_err <= max(2 * o_err, 0.1)
        else:
            # 4-connected sites travel along a column in one pass and along a
            # row in the next (L-shaped paths) where the FIFO queue moves them
            # in staircases; more of them are blocked by competing sites, as
            # in the model of the passes
            _, model = edt_pass_model(img, conn)
            m_rate = (model != ex).mean()
            m_err = (np.sqrt(model) - np.sqrt(ex)).max()
            announce("  pass model %.5f (max %.3f px)" % (m_rate, m_err))
            assert g_rate <= 2 * m_rate + 1e-4
            assert g_err <= max(2 * m_err, 0.1)
        assert st["tile_visits"] >= st["tiles"]


def test_no_background_and_pitch(iwpp):
    import torch

    img = np.full((70, 90), 9, np.uint8)
    announce("edt no background")
    sites, d2, _ = gpu_edt(iwpp, img, 8)
    assert (sites == -1).all() and (d2 == -1).all()
    # pitched input and outputs
    dev = torch.device("cuda:0")
    img = (np.random.default_rng(5).random((150, 170)) < 0.97).astype(np.uint8)
    big = torch.ones((150, 170 + 13), dtype=torch.uint8, device=dev)
    big[:, :170] = torch.from_numpy(img).to(dev)
    s_big = torch.zeros((150, 170 + 5), dtype=torch.int32, device=dev)
    d_big = torch.zeros_like(s_big)
    announce("edt pitched")
    iwpp.edt(big[:, :170], 8, sites=s_big[:, :170], dist2=d_big[:, :170])
    d2 = d_big[:, :170].cpu().numpy().astype(np.int64)
    refdefs.edt_check_valid(img, s_big[:, :170].cpu().numpy(), d2, 8)
    _, want = oracle_edt(img, 8)
    np.testing.assert_array_equal(d2, want)


def test_full_size_ellipses_sampled(iwpp):
    # 4096 x 4096 objects of the fill-holes workload: the whole map is checked
    # against the exact transform (valid lower bound, rare small misses)
    I, _ = synth.c2()
    img = (I > 50).astype(np.uint8)
    announce("edt 4096x4096 ellipses")
    sites, d2, _ = gpu_edt(iwpp, img, 8)
    ex = refdefs.edt_exact_sq(img)
    assert (d2 >= ex).all()
    assert (d2 != ex).mean() <= 1e-3
    assert (np.sqrt(d2) - np.sqrt(ex)).max() < 0.5
    sy, sx = refdefs.decode_sites(sites)
    assert (img[sy, sx] == 0).all()
