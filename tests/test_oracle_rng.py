"""Pins of the oracle's noise generator (spontaneous-emission source of the
Simulations section, drawn from a counter-based Philox4x32-10 stream).

* bit-exact known-answer vectors published with Philox (golden file);
* Box-Muller statistics: mean, variance and a Kolmogorov-Smirnov test of the
  normals, pair independence of the three components.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v = [int(t, 16) for t in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(ctr, key, expect):
    got = O.philox4x32_10(ctr, key)
    assert [int(x) for x in got] == expect


def test_philox_is_a_bijection_on_a_sample():
    # distinct counters give distinct outputs (a dropped round or a fixed
    # output word would collide immediately)
    outs = {tuple(O.philox4x32_10([c, 7, 3, 0], [11, 13])) for c in range(4096)}
    assert len(outs) == 4096


def test_normals_statistics():
    n = 40000
    xs = np.array([O.normals3(12345, cell, 17, 2) for cell in range(n)])
    for c in range(3):
        x = xs[:, c]
        assert abs(x.mean()) < 5.0 / math.sqrt(n)
        assert abs(x.var() - 1.0) < 5.0 * math.sqrt(2.0 / n)
        assert stats.kstest(x, "norm").pvalue > 1e-4
    corr = np.corrcoef(xs.T)
    assert np.all(np.abs(corr - np.eye(3)) < 5.0 / math.sqrt(n))


def test_normals_depend_on_every_key_part():
    base = O.normals3(5, 10, 20, 30)
    for args in [(6, 10, 20, 30), (5, 11, 20, 30), (5, 10, 21, 30), (5, 10, 20, 31),
                 (5 + (1 << 32), 10, 20, 30)]:
        assert not np.allclose(O.normals3(*args), base)


def test_normals_uniform_mapping_matches_definition():
    # 24-bit uniforms from the Philox words, then Box-Muller (cos, sin) pairs
    w = O.philox4x32_10([3, 4, 5, 0], [9, 0])
    u = ((w >> 8).astype(np.float64) + 0.5) / 2.0 ** 24
    r0 = math.sqrt(-2 * math.log(u[0]))
    r1 = math.sqrt(-2 * math.log(u[2]))
    expect = [r0 * math.cos(2 * math.pi * u[1]), r0 * math.sin(2 * math.pi * u[1]),
              r1 * math.cos(2 * math.pi * u[3])]
    assert np.allclose(O.normals3(9, 3, 4, 5), expect, rtol=0, atol=1e-15)
