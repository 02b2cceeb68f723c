"""Pins of the oracle's Gaussian generator (CPU only).

The paper only requires a standard Gaussian test matrix (Algorithm 1 and
Theorem "projector"); the generator's own published definition pins the bits.
"""
import os

import numpy as np
import pytest
from scipy import stats

from oracle.philox import philox4x32_10, raw_bits, gaussian_matrix

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([int(x, 16) for x in line.split()])
    return rows


def test_philox_known_answers():
    rows = _kat()
    assert len(rows) == 3
    for r in rows:
        out = philox4x32_10(r[0], r[1], r[2], r[3], r[4], r[5])
        assert [int(x) for x in out] == r[6:10]


def test_counter_layout_and_pairing():
    seed = (7 << 32) | 12345
    bits = raw_bits(seed, 2, 5, 0, 8)
    for row in range(5):
        for j in range(2):
            x = philox4x32_10(row, j, 2, 0, 12345, 7)
            assert [int(v) for v in x] == [int(b) for b in bits[row, 4 * j:4 * j + 4]]
    # Box-Muller pairing (x0,x1) -> cols 4j,4j+1 and (x2,x3) -> 4j+2,4j+3
    Om = gaussian_matrix(seed, 2, 5, 0, 8)
    xa, xb = bits[3, 6].astype(np.float64), bits[3, 7].astype(np.float64)
    u1 = (xa + 1.0) * 2.0 ** -32
    u2 = xb * 2.0 ** -32
    assert Om[3, 6] == np.sqrt(-2 * np.log(u1)) * np.cos(2 * np.pi * u2)
    assert Om[3, 7] == np.sqrt(-2 * np.log(u1)) * np.sin(2 * np.pi * u2)


@pytest.mark.parametrize("col0,ncols", [(0, 1), (3, 5), (5, 17), (16, 16), (30, 3)])
def test_global_columns_are_a_prefix_stream(col0, ncols):
    full = gaussian_matrix(99, 1, 7, 0, 64)
    part = gaussian_matrix(99, 1, 7, col0, ncols)
    assert np.array_equal(part, full[:, col0:col0 + ncols])


def test_streams_and_seeds_differ():
    a = gaussian_matrix(1, 1, 50, 0, 8)
    b = gaussian_matrix(1, 2, 50, 0, 8)
    c = gaussian_matrix(2, 1, 50, 0, 8)
    assert not np.allclose(a, b) and not np.allclose(a, c)


def test_uniforms_in_range():
    bits = raw_bits(3, 1, 200, 0, 64).astype(np.float64)
    u1 = (bits + 1.0) * 2.0 ** -32
    assert np.all(u1 > 0) and np.all(u1 <= 1)


def test_gaussian_statistics():
    Om = gaussian_matrix(2024, 1, 4000, 0, 64)      # 256k draws
    x = Om.ravel()
    assert abs(x.mean()) < 5 * 1 / np.sqrt(x.size)
    assert abs(x.var() - 1.0) < 5 * np.sqrt(2.0 / x.size)
    assert stats.kstest(x, "norm").pvalue > 1e-4
    # column independence (the Gaussian matrix of Proposition 10.1/10.2)
    C = np.corrcoef(Om.T)
    off = C[~np.eye(64, dtype=bool)]
    assert np.max(np.abs(off)) < 6 / np.sqrt(4000)
    # even/odd members of a Box-Muller pair are uncorrelated too
    assert abs(np.corrcoef(Om[:, 0], Om[:, 1])[0, 1]) < 6 / np.sqrt(4000)
