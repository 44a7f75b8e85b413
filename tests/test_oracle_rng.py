"""Oracle pins: the Philox4x32-10 stream and the derived uniforms / normals.

Pinned against the published Philox known-answer vectors and against the
distributions the paper asks for (xi ~ N(0, I) in Eq. aboba, u ~ U[0, 1] in
Eq. reflectionVerify).
"""
import os

import numpy as np
import pytest
from scipy import stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(ora, ctr, key, expect):
    assert ora.philox4x32_10(ctr, key) == expect


def test_uniform_range_and_law(ora):
    u = np.array([ora.uniform(7, 0, s) for s in range(1, 20001)])
    assert np.all(u > 0.0) and np.all(u <= 1.0)
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_uniform_keys_are_distinct(ora):
    # different replica, step or seed must give different numbers
    a = ora.uniform(1, 0, 5)
    assert a != ora.uniform(1, 1, 5)
    assert a != ora.uniform(1, 0, 6)
    assert a != ora.uniform(2, 0, 5)
    assert a == ora.uniform(1, 0, 5)


def test_normals_law_and_independence(ora):
    xi = np.concatenate([ora.normals(11, 3, s, 500) for s in range(1, 41)])  # 20000 x 3
    for d in range(3):
        assert stats.kstest(xi[:, d], "norm").pvalue > 1e-3
    c = np.corrcoef(xi.T)
    assert np.max(np.abs(c - np.eye(3))) < 0.03
    # steps are independent draws
    a, b = ora.normals(11, 3, 1, 4000), ora.normals(11, 3, 2, 4000)
    assert abs(np.corrcoef(a.ravel(), b.ravel())[0, 1]) < 0.03


def test_normals_use_box_muller_on_stream_words(ora):
    # component (i, d) takes Box-Muller output d&1 of block d>>1 at counter i:
    # the radius of block 0 comes from the first two words of that block.
    seed, rep, step, i = 99, 2, 12345, 7
    w = ora.philox4x32_10([i, step & 0xFFFFFFFF, step >> 32, (rep << 8) | (1 << 4) | 0],
                          [seed & 0xFFFFFFFF, seed >> 32])
    u1 = (((w[1] << 32) | w[0]) >> 11) + 1
    u1 = u1 / 2.0 ** 53
    xi = ora.normals(seed, rep, step, 8)
    r2 = xi[i, 0] ** 2 + xi[i, 1] ** 2
    assert r2 == pytest.approx(-2.0 * np.log(u1), rel=1e-12)
