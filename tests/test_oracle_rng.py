"""Pins of the oracle's counter-based generator.

* Philox4x32-10 reproduces the published known-answer vectors (tests/golden).
* Normals: the even/odd pair of an index shares one counter; moments of a
  large sample match N(0, 1) within sampling error.
"""
import os

import numpy as np

from oracle import rng

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox_kat.txt")


def test_philox_known_answers():
    n = 0
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        out = rng.philox4x32_10(*[np.uint64(x) for x in v[:6]])
        assert [int(o) for o in out] == v[6:]
        n += 1
    assert n == 3


def test_normals_pairing_and_moments():
    z = rng.normals(12345, 1, 7, np.arange(400000))
    assert abs(z.mean()) < 5 * (1 / np.sqrt(4e5))
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / 4e5)
    assert abs(np.mean(z ** 4) - 3) < 5 * np.sqrt(96 / 4e5)
    # Box-Muller pair from one counter: z0^2 + z1^2 = -2 log u1 > 0 and independent of the angle
    a = rng.normals(1, 0, 0, np.array([10, 11]))
    b = rng.normals(1, 0, 0, np.array([11, 10]))
    assert a[0] == b[1] and a[1] == b[0]
    # different streams / steps / seeds decorrelate
    z2 = rng.normals(12345, 0, 7, np.arange(400000))
    assert abs(np.corrcoef(z, z2)[0, 1]) < 0.01
