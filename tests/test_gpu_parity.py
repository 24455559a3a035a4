"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Integer work, so the bar is bit-exact equality.  Inputs come from the seeded
generators in ``synth``; expected values only ever come from ``oracle``.
"""
from __future__ import annotations

import sys

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


def run(iwpp, I, J, conn=8, ld_pad=0, check=True, col0=0, **kw):
    """Reconstruct on the device; with ld_pad the images sit in wider
    buffers (row pitch W + ld_pad) starting at column col0 of each row."""
    import torch

    dev = torch.device("cuda:0")
    H, W = I.shape
    if ld_pad:
        assert 0 <= col0 <= ld_pad
        bigJ = torch.zeros((H, W + ld_pad), dtype=torch.from_numpy(J).dtype, device=dev)
        bigI = torch.zeros_like(bigJ)
        bigJ[:, col0:col0 + W] = torch.from_numpy(J).to(dev)
        bigI[:, col0:col0 + W] = torch.from_numpy(I).to(dev)
        Jt, It = bigJ[:, col0:col0 + W], bigI[:, col0:col0 + W]
    else:
        Jt = torch.from_numpy(np.ascontiguousarray(J)).to(dev)
        It = torch.from_numpy(np.ascontiguousarray(I)).to(dev)
    st = iwpp.reconstruct(Jt, It, conn, check=check, **kw)
    return Jt.cpu().numpy(), st


def expect(I, J, conn, clamp=False):
    rc, R = oracle.reconstruct(J, I, conn, clamp=clamp)
    assert rc == oracle.OK
    return R


def same(got, want, label=""):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        y, x = bad[0]
        raise AssertionError("%s: %d pixels differ, first at (%d, %d): got %d want %d"
                             % (label, len(bad), y, x, got[y, x], want[y, x]))


def announce(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


# ------------------------------------------------------------------ small


@pytest.mark.parametrize("conn", [8, 4])
def test_c1_full_size(iwpp, conn):
    I, J = synth.c1()
    announce("c1 512x512 u8 conn %d" % conn)
    got, st = run(iwpp, I, J, conn)
    same(got, expect(I, J, conn), "c1")
    assert st["tile_visits"] >= st["tiles"]


@pytest.mark.parametrize("conn", [8, 4])
def test_fill_holes_scaled(iwpp, conn):
    I, J = synth.c2(H=1000, W=777)
    announce("c2-scaled 1000x777 u8 conn %d" % conn)
    got, _ = run(iwpp, I, J, conn)
    same(got, expect(I, J, conn), "c2-scaled")


@pytest.mark.parametrize("conn", [8, 4])
def test_smooth_i32_scaled(iwpp, conn):
    I, J = synth.c3_i32(H=700, W=900)
    announce("c3-i32-scaled 700x900 conn %d" % conn)
    got, _ = run(iwpp, I, J, conn)
    same(got, expect(I, J, conn), "c3-i32-scaled")


SIZES = [(1, 1), (1, 200), (200, 1), (2, 3), (63, 63), (64, 64), (65, 65), (127, 129),
         (128, 128), (129, 127), (97, 211), (257, 61), (13, 640)]


@pytest.mark.parametrize("dtype", [np.uint8, np.int32])
@pytest.mark.parametrize("conn", [8, 4])
def test_fuzz_shapes(iwpp, dtype, conn):
    rng = np.random.default_rng(100 + conn + (dtype == np.int32))
    for (H, W) in SIZES:
        for kind in ("uniform", "sparse", "plateau", "extreme"):
            I, J = synth.random_pair(rng, H, W, dtype, kind,
                                     levels=8 if kind == "uniform" else None)
            announce("fuzz %dx%d %s %s conn %d" % (H, W, np.dtype(dtype).name, kind, conn))
            got, _ = run(iwpp, I, J, conn)
            same(got, expect(I, J, conn), "fuzz %dx%d %s" % (H, W, kind))


def test_row_pitch(iwpp):
    I, J = synth.c2(H=300, W=250)
    announce("pitch 300x250 ld=250+37")
    got, _ = run(iwpp, I, J, 8, ld_pad=37)
    same(got, expect(I, J, 8), "pitched")


@pytest.mark.parametrize("ld_pad,col0", [(4, 0), (4, 1), (8, 3), (37, 0)])
@pytest.mark.parametrize("conn", [8, 4])
def test_int32_row_alignment(iwpp, ld_pad, col0, conn):
    """int32 tiles inside the image load their rows sixteen bytes to a lane
    when every row starts 16-byte aligned (pitch a multiple of four pixels,
    aligned base); other images take the pixel-at-a-time path for every
    tile.  Both, against the oracle: a pitch of W + 4 with the image at
    column 0 (sixteen-byte loads, pitch != width) and at column 1 (rows
    4-byte aligned only), W + 8 at column 3, W + 37."""
    I, J = synth.c3_i32(H=330, W=452)
    announce("int32 pitch 330x452 ld=452+%d col0=%d conn %d" % (ld_pad, col0, conn))
    got, _ = run(iwpp, I, J, conn, ld_pad=ld_pad, col0=col0)
    same(got, expect(I, J, conn), "int32 ld=W+%d col0=%d" % (ld_pad, col0))


# ------------------------------------------------------------------ parameters


@pytest.mark.parametrize("params", [
    {"mode": 1}, {"sweeps": -1}, {"sweeps": 1}, {"sweeps": 4}, {"tile_h": 128},
    {"tile_h": 32}, {"order_seed": 7}, {"order_seed": 12345, "sweeps": -1}, {"grid": 3},
    {"grid": 1}, {"mode": 1, "sweeps": -1}, {"mode": 1, "tile_h": 128}, {"seed_queue": -1},
    {"seed_queue": 100000}, {"seed_queue": 100000, "sweeps": -1}, {"queue_waves": 1},
    {"queue_waves": -1}, {"queue_waves": 2, "seed_queue": 100000, "sweeps": -1},
    {"mode": 2}, {"mode": 2, "bands": 3}, {"mode": 2, "bands": 300, "sweeps": 1},
    {"mode": 2, "bands": 64, "seed_queue": 100000, "queue_waves": 2},
    {"first_pass": 1}, {"first_pass": 2}, {"first_pass": 2, "grid": 5},
])
def test_parameters_do_not_change_the_result(iwpp, params):
    th = params.get("tile_h")
    u8_ok = th in (None, 64, 128)
    i32_ok = th in (None, 32, 64)
    cases = []
    if u8_ok:
        cases += [(*synth.c2(H=600, W=520), 8), (*synth.c1(H=400, W=333), 4)]
    if i32_ok:
        cases += [(*synth.c3_i32(H=300, W=450), 8), (*synth.c3_i32(H=131, W=77), 4)]
    for (I, J, conn) in cases:
        announce("params %s %s %dx%d conn %d" % (params, I.dtype, I.shape[0], I.shape[1], conn))
        got, _ = run(iwpp, I, J, conn, params=params)
        same(got, expect(I, J, conn), "params %s" % params)


# ------------------------------------------------------------------ errors / restart


def test_marker_above_mask(iwpp):
    I, J = synth.c1(H=200, W=150)
    J = J.copy()
    J[50, 60] = 255
    J[199, 149] = 255
    I[199, 149] = 3
    announce("marker>mask error path")
    got, st = run(iwpp, I, J, 8, check=False)
    assert st["rc"] == iwpp.E_MARKER_GT_MASK
    got, st = run(iwpp, I, J, 8, clamp=True)
    assert st["rc"] == iwpp.OK
    same(got, expect(I, J, 8, clamp=True), "clamped")


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_restart_from_partial_result(iwpp, mode):
    import torch

    I, J = synth.c2(H=700, W=640)
    R = expect(I, J, 8)
    dev = torch.device("cuda:0")
    Jt = torch.from_numpy(J).to(dev)
    It = torch.from_numpy(I).to(dev)
    announce("restart mode %d" % mode)
    st = iwpp.reconstruct(Jt, It, 8, params={"max_tile_visits": 20, "mode": mode}, check=False)
    assert st["rc"] == iwpp.E_INCOMPLETE
    part = Jt.cpu().numpy()
    assert (J <= part).all() and (part <= R).all()
    st = iwpp.reconstruct(Jt, It, 8, params={"mode": mode})
    same(Jt.cpu().numpy(), R, "restarted")


def test_stats_report_work(iwpp):
    I, J = synth.c2(H=512, W=512)
    announce("stats")
    _, st = run(iwpp, I, J, 8)
    assert st["tiles"] == 8 * 8
    assert st["tile_visits"] >= st["tiles"]
    assert st["pixels_queued"] >= 0 and st["sweep_rounds"] > 0
    assert st["launches"] >= 2


def maze(seed, cells=31, reps=2):
    """A perfect maze (depth-first search on a cells x cells grid: 1-pixel
    corridors at odd coordinates, 1-pixel walls), tiled reps x reps, as a
    uint8 mask (corridors 200, walls 0) with the marker lit at one corner: a
    front that must wind through every corridor."""
    rng = np.random.default_rng(seed)
    n = 2 * cells + 2
    T = np.zeros((n, n), np.uint8)
    seen = np.zeros((cells, cells), bool)
    stack = [(0, 0)]
    seen[0, 0] = True
    T[1, 1] = 200
    while stack:
        cy, cx = stack[-1]
        nb = [(cy + dy, cx + dx) for dy, dx in ((0, 1), (1, 0), (0, -1), (-1, 0))
              if 0 <= cy + dy < cells and 0 <= cx + dx < cells and not seen[cy + dy, cx + dx]]
        if not nb:
            stack.pop()
            continue
        ny, nx = nb[rng.integers(len(nb))]
        T[2 * cy + 1 + (ny - cy), 2 * cx + 1 + (nx - cx)] = 200
        T[2 * ny + 1, 2 * nx + 1] = 200
        seen[ny, nx] = True
        stack.append((ny, nx))
    I = np.tile(T, (reps, reps))
    # open the tiles' shared borders here and there so the front crosses them
    for k in range(1, reps):
        I[k * n - 1: k * n + 1, 1::8] = 200
        I[1::8, k * n - 1: k * n + 1] = 200
    J = np.zeros_like(I)
    J[1, 1] = 200
    return np.ascontiguousarray(I), J


@pytest.mark.parametrize("conn", [8, 4])
def test_queue_carries_winding_fronts_with_uint8_defaults(iwpp, conn):
    """A maze defeats the rounds of directional passes (each round follows a
    front through a few turns only), so under the uint8 defaults (16 rounds,
    then the seed scan and the tile queue) the queue carries what the rounds
    leave; the result is exact."""
    I, J = maze(5)
    announce("maze %dx%d u8 defaults, %d-conn" % (I.shape + (conn,)))
    got, st = run(iwpp, I, J, conn)
    same(got, expect(I, J, conn), "maze")
    announce("maze: %d pixels queued in %d waves, %d rounds"
             % (st["pixels_queued"], st["queue_iterations"], st["sweep_rounds"]))
    assert st["pixels_queued"] > 0 and st["queue_iterations"] > 0, st


def test_queue_overflow_falls_back_to_passes(iwpp):
    """Without scan rounds before the queue (sweeps -1), an int32 h-dome tile
    queues more receivers than its LDS queue holds (an eighth of the tile):
    every first visit overflows, falls back to rounds of passes, and the
    result is exact."""
    I, J = synth.c3_i32(H=300, W=330)
    announce("queue overflow int32")
    got, st = run(iwpp, I, J, 8, params={"sweeps": -1})
    same(got, expect(I, J, 8), "overflow")
    assert st["queue_overflows"] > 0, st


def test_queue_wave_bound_hands_over_to_passes(iwpp):
    """With queue_waves 1 a tile queue that still holds receivers after one
    wave hands the tile to rounds of passes (and a new scan); without a bound
    the queue alone carries the maze front.  Both are exact."""
    I, J = maze(9)
    announce("queue wave bound")
    base = {"sweeps": -1, "seed_queue": 100000}
    got_a, st_a = run(iwpp, I, J, 8, params=dict(base, queue_waves=-1))
    got_b, st_b = run(iwpp, I, J, 8, params=dict(base, queue_waves=1))
    want = expect(I, J, 8)
    same(got_a, want, "unbounded waves")
    same(got_b, want, "one wave")
    assert st_a["queue_overflows"] == 0 and st_a["sweep_rounds"] == 0, st_a
    assert st_b["sweep_rounds"] > 0, st_b
    assert st_a["queue_iterations"] > st_b["queue_iterations"], (st_a, st_b)


# ------------------------------------------------------------------ batched


def test_batched_uneven_sizes(iwpp):
    import torch

    dev = torch.device("cuda:0")
    batch = synth.c4(n=12, lo=40, hi=700)
    pairs = [(torch.from_numpy(J).to(dev), torch.from_numpy(I).to(dev)) for I, J in batch]
    announce("batched 12 images")
    st = iwpp.reconstruct_batched(pairs, 8)
    assert st["images"] == 12
    for k, (I, J) in enumerate(batch):
        same(pairs[k][0].cpu().numpy(), expect(I, J, 8), "batched image %d" % k)


@pytest.mark.parametrize("first_pass", [1, 2])
def test_batched_first_pass_orders(iwpp, first_pass):
    """Each image of a batch runs its own four groups of first visits; both
    group orders, uint8 and int32 images of uneven sizes, against the
    oracle."""
    import torch

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(41 + first_pass)
    batch = synth.c4(n=6, lo=40, hi=500)
    pairs = [(torch.from_numpy(J).to(dev), torch.from_numpy(I).to(dev)) for I, J in batch]
    announce("batched u8, first_pass %d" % first_pass)
    iwpp.reconstruct_batched(pairs, 8, params={"first_pass": first_pass})
    for k, (I, J) in enumerate(batch):
        same(pairs[k][0].cpu().numpy(), expect(I, J, 8), "u8 image %d" % k)
    b32 = [synth.c3_i32(H=int(h), W=int(w)) for h, w in rng.integers(33, 400, size=(5, 2))]
    p32 = [(torch.from_numpy(J).to(dev), torch.from_numpy(I).to(dev)) for I, J in b32]
    announce("batched int32, first_pass %d" % first_pass)
    iwpp.reconstruct_batched(p32, 8, params={"first_pass": first_pass})
    for k, (I, J) in enumerate(b32):
        same(p32[k][0].cpu().numpy(), expect(I, J, 8), "int32 image %d" % k)


def test_batch_plan_graph_replays(iwpp):
    import torch

    dev = torch.device("cuda:0")
    batch = synth.c4(n=9, lo=64, hi=500)
    batch.append(synth.c2(H=300, W=301))
    pristine = [torch.from_numpy(J).to(dev) for I, J in batch]
    pairs = [(p.clone(), torch.from_numpy(I).to(dev)) for p, (I, J) in zip(pristine, batch)]
    want = [expect(I, J, 8) for I, J in batch]
    plan = iwpp.Batch(pairs, 8)
    stream = torch.cuda.Stream()
    for rep in range(4):
        announce("graph replay %d" % rep)
        with torch.cuda.stream(stream):
            for (m, _), p in zip(pairs, pristine):
                m.copy_(p)
        plan.launch(stream=stream, graph=rep % 2 == 0 or rep == 3)
        st = plan.status()
        torch.cuda.synchronize()
        for k in range(len(batch)):
            same(pairs[k][0].cpu().numpy(), want[k], "replay %d image %d" % (rep, k))
        assert st["images"] == len(batch)
    plan.close()


# ------------------------------------------------------------------ by erosion / fill holes


def expect_erode(I, J, conn, clamp=False):
    rc, R = oracle.reconstruct_erode(J, I, conn, clamp=clamp)
    assert rc == oracle.OK
    return R


@pytest.mark.parametrize("dtype", [np.uint8, np.int32])
@pytest.mark.parametrize("conn", [8, 4])
def test_erosion_fuzz_shapes(iwpp, dtype, conn):
    rng = np.random.default_rng(300 + conn + (dtype == np.int32))
    for (H, W) in SIZES + [(300, 257)]:
        for kind in ("uniform", "sparse", "plateau", "extreme"):
            I, J = synth.random_pair_above(rng, H, W, dtype, kind,
                                           levels=8 if kind == "uniform" else None)
            announce("erosion %dx%d %s %s conn %d" % (H, W, np.dtype(dtype).name, kind, conn))
            got, _ = run(iwpp, I, J, conn, erosion=True)
            same(got, expect_erode(I, J, conn), "erosion %dx%d %s" % (H, W, kind))


def test_erosion_marker_below_mask(iwpp):
    rng = np.random.default_rng(5)
    I, J = synth.random_pair_above(rng, 150, 170, np.uint8, "uniform", levels=20)
    J = J.copy()
    J[40, 41] = 0
    I[40, 41] = 9
    announce("erosion marker<mask error path")
    _, st = run(iwpp, I, J, 8, check=False, erosion=True)
    assert st["rc"] == iwpp.E_MARKER_GT_MASK
    got, st = run(iwpp, I, J, 8, clamp=True, erosion=True)
    assert st["rc"] == iwpp.OK
    same(got, expect_erode(I, J, 8, clamp=True), "erosion clamped")


def test_erosion_bands(iwpp):
    rng = np.random.default_rng(9)
    for dtype in (np.uint8, np.int32):
        I, J = synth.random_pair_above(rng, 230, 310, dtype, "uniform", levels=40)
        announce("erosion gray-level bands %s" % np.dtype(dtype).name)
        got, _ = run(iwpp, I, J, 8, erosion=True, params={"mode": 2, "bands": 8})
        same(got, expect_erode(I, J, 8), "erosion bands")


def test_bands_rejects_batches(iwpp):
    import torch

    dev = torch.device("cuda:0")
    I, J = synth.c1(H=100, W=90)
    pairs = [(torch.from_numpy(J).to(dev), torch.from_numpy(I).to(dev))]
    with pytest.raises(iwpp.IwppError):
        iwpp.reconstruct_batched(pairs, 8, params={"mode": 2})


def test_erosion_batched(iwpp):
    import torch

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(8)
    batch = [synth.random_pair_above(rng, h, w, np.int32, "uniform", levels=30)
             for h, w in [(70, 300), (257, 64), (5, 5), (190, 211)]]
    pairs = [(torch.from_numpy(J).to(dev), torch.from_numpy(I).to(dev)) for I, J in batch]
    announce("erosion batched 4 images")
    iwpp.reconstruct_batched(pairs, 8, erosion=True)
    for k, (I, J) in enumerate(batch):
        same(pairs[k][0].cpu().numpy(), expect_erode(I, J, 8), "erosion batched %d" % k)


def fill(iwpp, img, conn, **kw):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(img)).to(torch.device("cuda:0"))
    out, st = iwpp.fill_holes(t, None, conn, **kw)
    return out.cpu().numpy(), st


@pytest.mark.parametrize("conn", [8, 4])
def test_fill_holes_ellipses(iwpp, conn):
    I, _ = synth.c2(H=777, W=1000)
    announce("fill holes 777x1000 u8 conn %d" % conn)
    got, _ = fill(iwpp, I, conn)
    rc, want = oracle.fill_holes(I, conn)
    assert rc == oracle.OK
    same(got, want, "fill holes")


@pytest.mark.parametrize("conn", [8, 4])
def test_fill_holes_i32_and_small(iwpp, conn):
    rng = np.random.default_rng(21 + conn)
    cases = [synth.smooth_field_i32(3, 200, 333) - (1 << 19)]
    for (H, W) in [(1, 1), (1, 50), (50, 1), (2, 2), (3, 3), (65, 63), (130, 70)]:
        cases.append(rng.integers(-5, 5, size=(H, W)).astype(np.int32) * 1000)
        cases.append(rng.integers(0, 4, size=(H, W)).astype(np.uint8) * 60)
    for img in cases:
        announce("fill holes %dx%d %s conn %d" % (img.shape[0], img.shape[1], img.dtype, conn))
        got, _ = fill(iwpp, img, conn)
        rc, want = oracle.fill_holes(img, conn)
        assert rc == oracle.OK
        same(got, want, "fill holes %s" % (img.shape,))


# ------------------------------------------------------------------ full sizes


def test_c2_full_size_bit_exact(iwpp):
    I, J = synth.c2()
    announce("c2 full 4096x4096 u8 conn 8")
    got, st = run(iwpp, I, J, 8)
    same(got, expect(I, J, 8), "c2 full")


# ------------------------------------------------------------------ diagonal seams


@pytest.mark.parametrize("dtype,tile_h", [(np.uint8, None), (np.uint8, 128), (np.int32, None),
                                          (np.int32, 64)])
def test_diagonal_corridors_cross_tile_corners(iwpp, dtype, tile_h):
    """A front that can only step diagonally from tile to tile: through tile
    corners (offset 0 on a square grid of tiles), next to them, and across
    the row groups of 128-row tiles.  Each corridor is one case."""
    H, W = 300, 330
    params = {} if tile_h is None else {"tile_h": tile_h}
    for direction, offset in [(1, 0), (1, 1), (1, -1), (1, 64), (1, -64), (1, 63),
                              (-1, 127), (-1, 128), (-1, 191), (-1, 255), (-1, 256)]:
        I, J = synth.diagonal_corridor(H, W, dtype, direction, offset)
        announce("diagonal %s tile_h %s dir %d offset %d" % (np.dtype(dtype), tile_h,
                                                             direction, offset))
        want = expect(I, J, 8)
        assert int(want.astype(np.int64).sum()) > int(J.astype(np.int64).sum())
        got, _ = run(iwpp, I, J, 8, params=params)
        same(got, want, "diagonal dir %d offset %d" % (direction, offset))
