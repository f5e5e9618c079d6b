"""Pins for the oracle's Philox4x32-10, normal draws and Euler-Maruyama (CPU).

The paper names no generator (section 6.8.1 only says the kernel PRNG is less
optimised); the oracle uses Philox4x32-10 (Salmon et al., SC'11), pinned to
that generator's published known-answer vectors.  Euler-Maruyama (section
5.2.2; SDE of section 3.3, eq. 11) is pinned by its exact discrete moments for
GBM and by the sigma = 0 case, which reduces it to a closed form.
"""
import os

import numpy as np
import pytest
from scipy import stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def kat_rows():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                v = [int(x, 16) for x in line.split()]
                rows.append((v[:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(orc):
    rows = kat_rows()
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert list(orc.philox4x32_10(ctr, key)) == want


def test_uniform_map_is_exact_and_open(orc):
    assert orc.uniform(0) == 2.0 ** -24
    assert orc.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    rng = np.random.default_rng(0)
    for x in rng.integers(0, 2**32, 1000, dtype=np.uint64):
        u = orc.uniform(int(x))
        assert 0.0 < u < 1.0
        assert np.float32(u) == u          # exactly representable in FP32
        assert u == (2 * (int(x) >> 9) + 1) / 2.0**24


def _normals(orc, count):
    z = []
    key = [0x1234, 0x5678]
    for s in range(count // 4):
        r = orc.philox4x32_10([s, 7, 0, 0], key)
        z.extend(orc.box_muller(int(r[0]), int(r[1])))
        z.extend(orc.box_muller(int(r[2]), int(r[3])))
    return np.array(z)


def test_box_muller_normals_distribution(orc):
    z = _normals(orc, 40000)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 5 / np.sqrt(len(z))
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / len(z))
    assert abs(stats.kurtosis(z)) < 5 * np.sqrt(24 / len(z))
    assert abs(np.corrcoef(z[:-1], z[1:])[0, 1]) < 5 / np.sqrt(len(z))


def test_em_sigma_zero_is_explicit_euler(orc):
    """sigma = 0: EM is explicit Euler, X_N = (1 + mu h)^N X_0 exactly."""
    N = 16
    mu = np.linspace(-0.5, 0.5, N)
    params = np.stack([mu, np.zeros(N)])
    out = orc.em(params, np.ones((4, N)), 1 / 256, 256, seed=9)
    ex = (1 + mu / 256) ** 256
    assert np.abs(out / ex - 1).max() < 1e-13


def test_em_one_step_is_textbook_update(orc):
    """One step: X_1 = X_0 (1 + mu h + sigma sqrt(h) Z) with Z from Philox
    counter (0, i, 0, 0) through Box-Muller."""
    N = 3
    params = np.array([[0.3, -0.2, 0.0], [0.4, 0.1, 0.25]])
    u0 = np.array([[1.0, 2.0, 0.5]] * 4)
    h = 0.01
    seed = (7 << 32) | 5
    out = orc.em(params, u0, h, 1, seed=seed)
    for i in range(N):
        r = orc.philox4x32_10([0, i, 0, 0], [5, 7])
        z = list(orc.box_muller(int(r[0]), int(r[1]))) + list(orc.box_muller(int(r[2]), int(r[3])))
        for c in range(4):
            ex = u0[c, i] * (1 + params[0, i] * h + params[1, i] * np.sqrt(h) * z[c])
            assert abs(out[c, i] - ex) < 1e-15


def em_moment_z(X, mu, sigma, h, n):
    """z-scores of the first two standardised moments of EM for GBM.

    With a = mu h, b = sigma sqrt(h) and Y = X_N / (1 + a)^N (X_0 = 1):
    E[Y] = 1, E[Y^2] = (1 + b^2/(1+a)^2)^N, E[Y^4] = ((1+a)^4 + 6(1+a)^2 b^2
    + 3 b^4)^N / (1+a)^{4N}  (moments of 1 + a + b Z, Z ~ N(0,1)).
    """
    a = mu * h
    b2 = sigma**2 * h
    Y = X / (1 + a) ** n
    m2 = (1 + b2 / (1 + a) ** 2) ** n
    m4 = (((1 + a) ** 4 + 6 * (1 + a) ** 2 * b2 + 3 * b2**2) / (1 + a) ** 4) ** n
    z1 = (Y - 1).sum() / np.sqrt((m2 - 1).sum())
    z2 = (Y**2 - m2).sum() / np.sqrt((m4 - m2**2).sum())
    return z1, z2


def test_em_gbm_discrete_moments(orc):
    N = 1 << 14
    rng = np.random.default_rng(4)
    mu = rng.uniform(-0.5, 0.5, N)
    sigma = rng.uniform(0.05, 0.5, N)
    out = orc.em(np.stack([mu, sigma]), np.ones((4, N)), 1 / 256, 256, seed=4)
    X = out.reshape(-1)
    z1, z2 = em_moment_z(X, np.tile(mu, 4), np.tile(sigma, 4), 1 / 256, 256)
    assert abs(z1) < 5 and abs(z2) < 5, (z1, z2)
    # a planted mistake of the classic kind (variance h instead of sqrt(h)
    # scaling of the increment) would be far outside these bounds
    bad = orc.em(np.stack([mu, sigma * np.sqrt(1 / 256)]), np.ones((4, N)), 1 / 256, 256, seed=4)
    bz1, bz2 = em_moment_z(bad.reshape(-1), np.tile(mu, 4), np.tile(sigma, 4), 1 / 256, 256)
    assert abs(bz2) > 20
