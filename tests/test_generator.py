"""Pins of the seeded input generator: Philox4x32-10 known answers, the normal
transform, the bf16 split, and the statistics of the drawn matrices."""
import os

import numpy as np
import pytest

from paper_2311_03824_amd import instances as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        ctr, key, out = w[:4], w[4:6], w[6:]
        got = I.philox4x32_10(*[np.array([c], np.uint32) for c in ctr], key[0], key[1])
        assert [int(g[0]) for g in got] == out


def test_normal_transform_quantiles():
    T = I.normal_table()
    assert T.shape == (32 * 64 + 2,) and T[-1] == 0 and T[-2] == 0
    # v = (2w + 1) 2^-33 with w = 2^30 - 1 is 1/4 - 2^-33: z = Phi^{-1}(3/4) = 0.6744897...
    z = I.words_to_normal(np.array([2**30 - 1, 0x80000000 | (2**30 - 1)], np.uint32), T)
    assert abs(z[0] - 0.6744897501960817) < 1e-6 and z[1] == -z[0]
    # the largest |z| is -Phi^{-1}(2^-33), the smallest 0
    z = I.words_to_normal(np.array([0, 0x7FFFFFFF], np.uint32), T)
    assert abs(z[0] - 6.3379575) < 1e-5 and z[1] == 0.0
    # monotone in v: larger low word, smaller |z|
    x = np.sort(np.random.default_rng(0).integers(0, 2**31, 10000, dtype=np.uint64)).astype(np.uint32)
    zz = I.words_to_normal(x, T)
    assert np.all(np.diff(zz) <= 0)


def test_philox_matrix_is_standard_normal():
    inst = I.make_instance(300, 40, 120, 2, 3, 11, a_form="philox")
    a = inst.At[:, :, :120].ravel().astype(np.float64)
    assert abs(a.mean()) < 0.01 and abs(a.std() - 1.0) < 0.01
    from scipy import stats
    assert stats.kstest(a, "norm").pvalue > 1e-3
    assert abs(stats.kurtosis(a, fisher=False) - 3.0) < 0.05


def test_bf16_split_is_exact():
    a = np.random.default_rng(1).standard_normal(100000).astype(np.float32)
    hb, lb, canon = I.split_bf16(a)
    hi = (hb.astype(np.uint32) << 16).view(np.float32)
    lo = (lb.astype(np.uint32) << 16).view(np.float32)
    assert np.array_equal(hi.astype(np.float64) + lo.astype(np.float64), canon.astype(np.float64))
    assert np.all(np.abs(canon - a) <= np.abs(a) * 2.0 ** -15)
    assert np.all(np.abs(hi - a) <= np.abs(a) * 2.0 ** -8)


def test_instance_measurements_are_exact():
    inst = I.make_instance(50, 7, 20, 2, 3, 3)
    A = inst.A64()
    y = np.matmul(A, inst.X_star.T[:, :, None])[:, :, 0]
    assert np.allclose(y, inst.Y64, rtol=1e-12, atol=1e-12)
    assert np.all((inst.S_star != 0).sum(axis=0) == 3)
    assert np.allclose(inst.U_star.T @ inst.U_star, np.eye(2), atol=1e-12)
