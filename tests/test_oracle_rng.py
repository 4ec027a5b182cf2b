"""Pins of the oracle's counter-based random streams (Philox4x32-10)."""
import os

import numpy as np

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    for line in open(GOLD):
        line = line.strip()
        if line and not line.startswith("#"):
            w = [int(x, 16) for x in line.split()]
            yield w[0:4], w[4:6], w[6:10]


def test_philox_known_answers(orc):
    rows = list(_kat_rows())
    assert len(rows) == 3
    for ctr, key, expect in rows:
        assert list(orc.philox4x32_10(ctr, key)) == expect


def test_uniform_is_top_53_bits(orc):
    # u = (x >> 11) * 2^-53 with x = out0 | out1 << 32 of the Philox block of
    # counter (electron, sweep, walker, purpose << 16 | sub) and key = seed.
    seed, purpose, sub, w, s, e = 0x1234567890ABCDEF, 2, 1, 7, 3, 5
    o = orc.philox4x32_10([e, s, w, (purpose << 16) | sub], [seed & 0xFFFFFFFF, seed >> 32])
    x0 = int(o[0]) | (int(o[1]) << 32)
    x1 = int(o[2]) | (int(o[3]) << 32)
    u = orc.uniform2(seed, purpose, sub, w, s, e)
    assert u[0] == (x0 >> 11) * 2.0 ** -53
    assert u[1] == (x1 >> 11) * 2.0 ** -53


def test_streams_differ_by_purpose_and_index(orc):
    a = orc.uniform2(0, 2, 0, 0, 0, 0)
    assert not np.array_equal(a, orc.uniform2(0, 3, 0, 0, 0, 0))
    assert not np.array_equal(a, orc.uniform2(0, 2, 1, 0, 0, 0))
    assert not np.array_equal(a, orc.uniform2(0, 2, 0, 1, 0, 0))
    assert not np.array_equal(a, orc.uniform2(0, 2, 0, 0, 1, 0))
    assert not np.array_equal(a, orc.uniform2(0, 2, 0, 0, 0, 1))
    assert not np.array_equal(a, orc.uniform2(1, 2, 0, 0, 0, 0))


def test_gaussian_moments_and_uniform_range(orc):
    n = 20000
    xi = np.array([orc.gauss3(0, w % 64, w // 64, 3) for w in range(n)])
    assert abs(xi.mean()) < 4.0 / np.sqrt(3 * n)
    assert abs(xi.var() - 1.0) < 6.0 * np.sqrt(2.0 / (3 * n))
    # fourth moment of a normal is 3
    assert abs((xi ** 4).mean() - 3.0) < 0.15
    u = np.array([orc.accept_uniform(0, w, 0, 0) for w in range(n)])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 4.0 / np.sqrt(12 * n)


def test_box_muller_from_uniforms(orc):
    # xi_x, xi_y from sub-block 0 and xi_z from sub-block 1 (Box-Muller).
    seed, w, s, e = 9, 4, 11, 2
    a = orc.uniform2(seed, 2, 0, w, s, e)
    b = orc.uniform2(seed, 2, 1, w, s, e)
    ra = np.sqrt(-2 * np.log(1 - a[0]))
    rb = np.sqrt(-2 * np.log(1 - b[0]))
    expect = [ra * np.cos(2 * np.pi * a[1]), ra * np.sin(2 * np.pi * a[1]), rb * np.cos(2 * np.pi * b[1])]
    np.testing.assert_allclose(orc.gauss3(seed, w, s, e), expect, rtol=1e-14, atol=1e-15)
