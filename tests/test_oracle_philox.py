"""Pins of the oracle's Philox4x32-10 and Gaussian sketch."""
import os

import numpy as np

from oracle.philox import philox4x32_10, box_muller, sketch_omega

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        rows.append([int(t, 16) for t in line.split()])
    return rows


def test_philox_known_answers():
    rows = _kat()
    assert len(rows) == 3
    for r in rows:
        out = philox4x32_10(np.uint32(r[0]), np.uint32(r[1]), np.uint32(r[2]), np.uint32(r[3]), r[4], r[5])
        assert [int(o) for o in out] == r[6:10]


def test_box_muller_moments():
    n = 200000
    x0, x1, _, _ = philox4x32_10(np.arange(n, dtype=np.uint32), 7, 0, 0, 12345, 678)
    z = box_muller(x0, x1)
    assert abs(z.mean()) < 5.0 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 10.0 / np.sqrt(n)
    assert abs(np.mean(z ** 3)) < 10.0 / np.sqrt(n)
    assert abs(np.mean(z ** 4) - 3.0) < 50.0 / np.sqrt(n)


def test_sketch_is_a_function_of_the_multi_index():
    a = sketch_omega(99, 3, 0, 4, (3, 5, 2), 6)
    b = sketch_omega(99, 3, 0, 7, (4, 6, 3), 9)
    assert a.shape == (4, 3, 5, 2, 6)
    assert np.array_equal(a, b[:4, :3, :5, :2, :6])
    c = sketch_omega(99, 4, 0, 4, (3, 5, 2), 6)
    assert not np.allclose(a, c)
    d = sketch_omega(100, 3, 0, 4, (3, 5, 2), 6)
    assert not np.allclose(a, d)
