"""The input generators are deterministic and draw what their recipes say."""
import numpy as np

import synth


def test_generators_are_deterministic():
    a = synth.c1()
    b = synth.c1()
    assert synth.sha256(*a) == synth.sha256(*b)
    c = synth.c2(H=300, W=200)
    d = synth.c2(H=300, W=200)
    assert synth.sha256(*c) == synth.sha256(*d)
    assert synth.sha256(*synth.c2(seed=5, H=300, W=200)) != synth.sha256(*c)


def test_recipes():
    I, J = synth.c1()
    assert I.shape == (512, 512) and I.dtype == np.uint8
    np.testing.assert_array_equal(J, np.maximum(I.astype(int) - 40, 0))
    I, J = synth.c2(H=256, W=256)
    assert (J[1:-1, 1:-1] == 0).all() and (J[0] == I[0]).all() and (J[:, -1] == I[:, -1]).all()
    assert I.min() >= 0 and I.max() <= 230
    I, J = synth.c3_i32(H=64, W=80)
    assert I.dtype == np.int32 and I.min() >= 0 and I.max() <= 2 ** 20
    np.testing.assert_array_equal(J, np.maximum(I.astype(np.int64) - 4096, 0))
    batch = synth.c4(n=4, lo=64, hi=128)
    assert len(batch) == 4 and all(64 <= I.shape[0] <= 128 for I, _ in batch)
    pool = synth.c5_pool(n=6, lo=32, hi=64)
    assert {k for _, _, k in pool} <= {"hdome", "fill"}
    t, idx = synth.c5_arrivals(rate=1000, duration=0.5, pool=6)
    assert (np.diff(t) > 0).all() and t.max() < 0.5 and idx.max() < 6


def test_random_pairs_respect_precondition():
    rng = np.random.default_rng(0)
    for kind in ("uniform", "sparse", "plateau", "extreme"):
        for dt in (np.uint8, np.int32):
            I, J = synth.random_pair(rng, 17, 9, dt, kind)
            assert I.dtype == dt and J.dtype == dt and (J <= I).all()
