"""Pins for the oracle's Gaussian generator (Alg. 1 step 4)."""
import os

import numpy as np
import scipy.stats

from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox.philox4x32_10(v[0:4], v[4:6])
        assert [int(o) for o in out] == v[6:10]


def test_stream_slices_agree():
    z = philox.normals(7, philox.stream_word(1, 2), 3, 0, 1003)
    for s, c in [(0, 1), (1, 7), (2, 2), (3, 5), (5, 100), (998, 5)]:
        np.testing.assert_array_equal(philox.normals(7, philox.stream_word(1, 2), 3, s, c), z[s:s + c])


def test_streams_differ():
    a = philox.normals(1, philox.stream_word(1, 0), 0, 0, 64)
    b = philox.normals(1, philox.stream_word(1, 1), 0, 0, 64)
    c = philox.normals(1, philox.stream_word(1, 0), 1, 0, 64)
    d = philox.normals(2, philox.stream_word(1, 0), 0, 0, 64)
    for x in (b, c, d):
        assert not np.any(a == x)


def test_box_muller_radius_identity():
    # z0^2 + z1^2 = -2 ln u(w0) for each pair
    n = 4000
    c = np.arange(n, dtype=np.uint64)
    w = philox.philox4x32_10((c, 0, 5, 0), (9, 0))
    z = philox.normals(9, 5, 0, 0, 4 * n).reshape(n, 4)
    np.testing.assert_allclose(z[:, 0] ** 2 + z[:, 1] ** 2, -2 * np.log(philox.uniform(w[0])), rtol=1e-13)
    np.testing.assert_allclose(z[:, 2] ** 2 + z[:, 3] ** 2, -2 * np.log(philox.uniform(w[2])), rtol=1e-13)


def test_normal_distribution():
    z = philox.normals(20190105, philox.stream_word(1, 0), 0, 0, 400000)
    assert abs(z.mean()) < 0.01
    assert abs(z.var() - 1) < 0.01
    assert abs(scipy.stats.kurtosis(z)) < 0.05
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3
    # lanes are not correlated with each other
    q = z.reshape(-1, 4)
    cc = np.corrcoef(q.T)
    assert np.max(np.abs(cc - np.eye(4))) < 0.01


def test_uniform_words_chi2():
    c = np.arange(100000, dtype=np.uint64)
    w = philox.philox4x32_10((c, 0, 0, 0), (1, 2))
    for lane in w:
        counts = np.bincount((lane >> np.uint64(24)).astype(np.int64), minlength=256)
        assert scipy.stats.chisquare(counts).pvalue > 1e-4
