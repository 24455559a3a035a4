"""Pins for the CPU oracle: it must agree with facts fixed by the paper and by
the mathematics of reconstruction, through code paths it does not share.

P1  the definition (brute-force iteration of J <- dilate(J) ^ I), fuzzed and
    exhaustive on tiny grids;
P2  threshold decomposition through scipy's connected-component labelling;
P3  the widest-path (max-heap) formulation;
P4  closed forms for special inputs;
P5  invariants (bounds, fixed point, idempotence, monotonicity);
P6  dihedral symmetry of the square grid;
P7  independence of sweep count, queue order and restarts;
plus the one numeric fragment the paper prints (tests/golden).
"""
from __future__ import annotations

import itertools
import os

import numpy as np
import pytest

import oracle
import synth
from tests import refdefs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
DTYPES = [np.uint8, np.int32]
CONNS = [4, 8]


def recon(J, I, conn, **kw):
    rc, R = oracle.reconstruct(J, I, conn, **kw)
    assert rc == oracle.OK
    return R


# ------------------------------------------------------------------- P1


@pytest.mark.parametrize("conn", CONNS)
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("kind", ["uniform", "sparse", "plateau", "extreme"])
def test_p1_fuzz_vs_definition(conn, dtype, kind):
    rng = np.random.default_rng(hash((conn, np.dtype(dtype).name, kind)) & 0xFFFF)
    for _ in range(120):
        H, W = (int(v) for v in rng.integers(1, 25, 2))
        levels = None if kind != "uniform" or rng.random() < 0.5 else int(rng.integers(2, 8))
        I, J = synth.random_pair(rng, H, W, dtype, kind, levels=levels)
        np.testing.assert_array_equal(recon(J, I, conn), refdefs.brute_numpy(J, I, conn))


@pytest.mark.parametrize("conn", CONNS)
def test_p1_exhaustive_2x2_three_levels(conn):
    pairs = [(j, i) for i in range(3) for j in range(i + 1)]  # J <= I
    for combo in itertools.product(pairs, repeat=4):
        J = np.array([c[0] for c in combo], np.uint8).reshape(2, 2)
        I = np.array([c[1] for c in combo], np.uint8).reshape(2, 2)
        np.testing.assert_array_equal(recon(J, I, conn), refdefs.brute_numpy(J, I, conn))


@pytest.mark.parametrize("conn", CONNS)
def test_p1_exhaustive_3x3_two_levels(conn):
    pairs = [(0, 0), (0, 1), (1, 1)]
    combos = np.array(list(itertools.product(range(3), repeat=9)))
    rng = np.random.default_rng(conn)
    # all 3^9 cases for the 8-connected grid; a quarter of them for 4-conn
    if conn == 4:
        combos = combos[rng.random(combos.shape[0]) < 0.25]
    lut = np.array(pairs, np.int32)
    for row in combos:
        JI = lut[row]
        J = JI[:, 0].reshape(3, 3).astype(np.int32)
        I = JI[:, 1].reshape(3, 3).astype(np.int32)
        np.testing.assert_array_equal(recon(J, I, conn), refdefs.brute_numpy(J, I, conn))


def test_p1_c_brute_matches_numpy_definition():
    rng = np.random.default_rng(11)
    for _ in range(200):
        H, W = (int(v) for v in rng.integers(1, 20, 2))
        conn = int(rng.choice(CONNS))
        I, J = synth.random_pair(rng, H, W, np.int32, "uniform", levels=6)
        rc, B = oracle.brute(J, I, conn)
        assert rc == oracle.OK
        np.testing.assert_array_equal(B, refdefs.brute_numpy(J, I, conn))


# ------------------------------------------------------------------- P2


@pytest.mark.parametrize("conn", CONNS)
def test_p2_threshold_decomposition_c1_full_size(conn):
    I, J = synth.c1()
    np.testing.assert_array_equal(recon(J, I, conn), refdefs.threshold_decomposition(J, I, conn))


@pytest.mark.parametrize("conn", CONNS)
def test_p2_threshold_decomposition_fill_holes(conn):
    I, J = synth.c2(H=384, W=320)
    np.testing.assert_array_equal(recon(J, I, conn), refdefs.threshold_decomposition(J, I, conn))


@pytest.mark.parametrize("conn", CONNS)
def test_p2_threshold_decomposition_i32_small(conn):
    rng = np.random.default_rng(5)
    for _ in range(30):
        H, W = (int(v) for v in rng.integers(1, 40, 2))
        I, J = synth.random_pair(rng, H, W, np.int32, "uniform", levels=None)
        np.testing.assert_array_equal(recon(J, I, conn),
                                      refdefs.threshold_decomposition(J, I, conn))


# ------------------------------------------------------------------- P3


@pytest.mark.parametrize("conn", CONNS)
def test_p3_widest_path(conn):
    cases = [synth.c1(), synth.c2(H=512, W=640)]
    I = synth.smooth_field_i32(2, 300, 257, threads=2)
    cases.append((I, synth.hdome_marker(I, 4096)))
    for I, J in cases:
        rc, Wd = oracle.widest(J, I, conn)
        assert rc == oracle.OK
        np.testing.assert_array_equal(recon(J, I, conn), Wd)


@pytest.mark.parametrize("conn", CONNS)
def test_p3_single_pixel_queries(conn):
    I, J = synth.c2(H=300, W=280)
    R = recon(J, I, conn)
    rng = np.random.default_rng(3)
    rows = rng.integers(0, 300, 500)
    cols = rng.integers(0, 280, 500)
    rc, vals = oracle.pixels(J, I, rows, cols, conn)
    assert rc == oracle.OK
    np.testing.assert_array_equal(vals, R[rows, cols].astype(np.int32))
    # a visit cap marks the queries it cut short and reports them
    rc, vals = oracle.pixels(J, I, rows, cols, conn, max_visit=3)
    assert rc == oracle.E_INCOMPLETE
    ok = vals != np.iinfo(np.int32).min
    np.testing.assert_array_equal(vals[ok], R[rows, cols][ok].astype(np.int32))


# ------------------------------------------------------------------- P4


@pytest.mark.parametrize("conn", CONNS)
@pytest.mark.parametrize("dtype", DTYPES)
def test_p4_closed_forms(conn, dtype):
    rng = np.random.default_rng(7)
    lo = np.iinfo(dtype).min
    for _ in range(20):
        H, W = (int(v) for v in rng.integers(1, 30, 2))
        I, J = synth.random_pair(rng, H, W, dtype, "uniform")
        # (i) marker equal to the mask
        np.testing.assert_array_equal(recon(I.copy(), I, conn), I)
        # (ii) marker at the lowest level stays there
        Z = np.full_like(I, lo)
        np.testing.assert_array_equal(recon(Z, I, conn), Z)
        # (iii) flat mask: the largest marker value floods everything
        c = I.max()
        C = np.full_like(I, c)
        np.testing.assert_array_equal(recon(J, C, conn), np.full_like(I, J.max()))
        # (iv) one row or one column: the two running recurrences
        row_I, row_J = I[:1, :], J[:1, :]
        np.testing.assert_array_equal(recon(row_J.copy(), row_I.copy(), conn),
                                      refdefs.line_closed_form(row_J, row_I))
        col_I, col_J = np.ascontiguousarray(I[:, :1]), np.ascontiguousarray(J[:, :1])
        np.testing.assert_array_equal(recon(col_J, col_I, conn),
                                      refdefs.line_closed_form(col_J, col_I))


@pytest.mark.parametrize("conn", CONNS)
def test_p4_diagonal_step_needs_8_connectivity(conn):
    I = np.array([[5, 0], [0, 5]], np.uint8)
    J = np.array([[5, 0], [0, 0]], np.uint8)
    expect = I if conn == 8 else J
    np.testing.assert_array_equal(recon(J, I, conn), expect)


@pytest.mark.parametrize("conn", CONNS)
def test_p4_flat_background_frame_marker(conn):
    """Ellipses brighter than a flat background b, frame marker: every path
    from the frame starts on the background, so R == b everywhere."""
    rng = np.random.default_rng(9)
    b = 17
    I = synth.ellipses(rng, 200, 180, 60, bg_max=0, vmin=60, vmax=230)
    I = np.where(I == 0, b, I).astype(np.uint8)
    I[0, :] = I[-1, :] = b
    I[:, 0] = I[:, -1] = b
    R = recon(synth.frame_marker(I), I, conn)
    np.testing.assert_array_equal(R, np.full_like(I, b))


@pytest.mark.parametrize("conn", CONNS)
def test_p4_fill_holes_ring(conn):
    """fill(I) = C(R_{C(I)}(F)), C(x) = 255 - x, F = C(I) on the frame and 0
    inside (the fill-holes construction through the complement): a hole of
    value h inside a closed ring of value v > h is raised to v."""
    n, v, h = 41, 150, 30
    yy, xx = np.mgrid[0:n, 0:n]
    d = np.maximum(abs(yy - n // 2), abs(xx - n // 2))
    I = np.zeros((n, n), np.uint8)
    I[(d >= 8) & (d <= 10)] = v
    I[d < 8] = h
    C = (255 - I).astype(np.uint8)
    F = np.zeros_like(C)
    F[0, :], F[-1, :], F[:, 0], F[:, -1] = C[0, :], C[-1, :], C[:, 0], C[:, -1]
    filled = (255 - recon(F, C, conn)).astype(np.uint8)
    expect = I.copy()
    expect[d < 8] = v
    np.testing.assert_array_equal(filled, expect)


def test_p4_isolated_blob_hdome():
    """A noiseless radially decreasing blob of peak A on a 0 background with
    marker I - h: the reconstruction is min(I, A - h)."""
    n, A, h = 61, 200, 40
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    I = np.rint(A * np.exp(-((yy - 30) ** 2 + (xx - 30) ** 2) / (2 * 9.0 ** 2))).astype(np.uint8)
    J = synth.hdome_marker(I, h)
    for conn in CONNS:
        np.testing.assert_array_equal(recon(J, I, conn), np.minimum(I, A - h))


# ------------------------------------------------------------------- P5


@pytest.mark.parametrize("conn", CONNS)
def test_p5_invariants(conn):
    rng = np.random.default_rng(13)
    cases = [synth.c1(), synth.c2(H=700, W=600)]
    for _ in range(6):
        H, W = (int(v) for v in rng.integers(20, 120, 2))
        cases.append(synth.random_pair(rng, H, W, np.int32, "uniform", levels=50))
    for I, J in cases:
        R = recon(J, I, conn)
        assert (J <= R).all() and (R <= I).all()
        assert refdefs.is_fixed_point(R, I, conn)
        np.testing.assert_array_equal(recon(R.copy(), I, conn), R)  # idempotent
        # monotone in the marker and in the mask
        J2 = np.minimum(np.maximum(J, rng.permutation(J.ravel()).reshape(J.shape)), I)
        assert (recon(J2, I, conn) >= R).all()
        I2 = np.maximum(I, rng.permutation(I.ravel()).reshape(I.shape)).astype(I.dtype)
        assert (recon(J, I2, conn) >= R).all()


# ------------------------------------------------------------------- P6


@pytest.mark.parametrize("conn", CONNS)
def test_p6_dihedral_symmetry(conn):
    I, J = synth.c2(H=257, W=193)
    R = recon(J, I, conn)
    for f in (np.flipud, np.fliplr, np.transpose, lambda a: np.rot90(a, 1)):
        Rf = recon(np.ascontiguousarray(f(J)), np.ascontiguousarray(f(I)), conn)
        np.testing.assert_array_equal(Rf, f(R))


# ------------------------------------------------------------------- P7


@pytest.mark.parametrize("conn", CONNS)
def test_p7_sweeps_order_restart(conn):
    I, J = synth.c2(H=300, W=310)
    R = recon(J, I, conn)
    for k in range(5):
        np.testing.assert_array_equal(recon(J, I, conn, nsweeps=k), R)
    for order in (oracle.ORDER_LIFO, oracle.ORDER_RANDOM):
        for seed in (1, 2):
            np.testing.assert_array_equal(recon(J, I, conn, order=order, seed=seed), R)
    for cut in (0, 10, 1000, 20000):
        rc, P = oracle.reconstruct(J, I, conn, max_pops=cut)
        assert rc in (oracle.OK, oracle.E_INCOMPLETE)
        assert (J <= P).all() and (P <= R).all()
        np.testing.assert_array_equal(recon(P, I, conn), R)


def test_p7_heap_does_less_work_than_fifo():
    """The paper's priority-queue observation: processing the highest values
    first touches fewer elements than FIFO order on the same input."""
    I, J = synth.c2(H=512, W=512)
    _, _, st_fifo = oracle.reconstruct(J, I, 8, nsweeps=0, stats=True)
    _, _, st_heap = oracle.widest(J, I, 8, stats=True)
    assert st_heap["pushes"] < st_fifo["pushes"]


# ------------------------------------------------------------------- errors


def test_marker_above_mask_error_and_clamp():
    I = np.array([[3, 3, 3], [3, 9, 3]], np.uint8)
    J = np.array([[0, 5, 0], [0, 1, 0]], np.uint8)  # J > I at (0, 1)
    rc, R = oracle.reconstruct(J, I, 8)
    assert rc == oracle.E_MARKER_GT_MASK
    np.testing.assert_array_equal(R, J)  # untouched
    rc, R = oracle.reconstruct(J, I, 8, clamp=True)
    assert rc == oracle.OK
    np.testing.assert_array_equal(R, refdefs.brute_numpy(np.minimum(J, I), I, 8))


def test_argument_errors():
    I = np.zeros((2, 2), np.uint8)
    assert oracle.reconstruct(I, I, 6)[0] == oracle.E_ARG
    assert oracle.reconstruct(I, I, 8, nsweeps=-1)[0] == oracle.E_ARG
    with pytest.raises(TypeError):
        oracle.reconstruct(I.astype(np.int16), I.astype(np.int16), 8)


# ------------------------------------------------------------------- golden


def _load_golden(path):
    sections, cur, meta = {}, None, {}
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        if line.split()[0] in ("conn", "dtype"):
            k, v = line.split()
            meta[k] = v
        elif line.isalpha():
            cur = line
            sections[cur] = []
        else:
            sections[cur].append([int(t) for t in line.split()])
    dt = np.uint8 if meta["dtype"] == "u8" else np.int32
    return int(meta["conn"]), {k: np.array(v, dt) for k, v in sections.items()}


# worked-example fixtures (full_size_sha256.txt holds digests, checked in
# test_golden_digests.py)
@pytest.mark.parametrize("name", sorted(f for f in os.listdir(GOLDEN)
                                        if f.endswith(".txt") and not f.startswith("full_size")))
def test_golden(name):
    conn, arr = _load_golden(os.path.join(GOLDEN, name))
    np.testing.assert_array_equal(recon(arr["J"], arr["I"], conn), arr["R"])
