"""The replica statistics of a result (Sec. III.1 averaging; the SAR of Sec. III.2.a
scales both): the oracle's mean and standard error against scipy's standard error of
the mean, and the invariants any correct estimator keeps."""
import numpy as np
from scipy import stats

from oracle import kmc


def test_replica_stats_matches_scipy_sem():
    rng = np.random.default_rng(5)
    for R in (2, 3, 17, 64, 1000):
        a = rng.normal(1234.0, 50.0, size=R)
        mean, se = kmc.replica_stats(a)
        assert abs(mean - np.mean(a)) <= 1e-12 * abs(mean)
        assert abs(se - stats.sem(a, ddof=1)) <= 1e-12 * se


def test_replica_stats_invariants():
    a = np.array([1.0, 2.0, 4.0, 8.0])
    m, s = kmc.replica_stats(a)
    # a shift moves the mean only; a scale scales both; one replica has no error
    m2, s2 = kmc.replica_stats(a + 1e3)
    assert abs(m2 - (m + 1e3)) < 1e-12 and abs(s2 - s) < 1e-12
    m3, s3 = kmc.replica_stats(-3.0 * a)
    assert abs(m3 + 3.0 * m) < 1e-12 and abs(s3 - 3.0 * s) < 1e-12
    assert kmc.replica_stats([7.5]) == (7.5, 0.0)
    assert kmc.replica_stats([2.0, 2.0, 2.0])[1] == 0.0
    # the same sample repeated k times: the sample variance tends to (n-1)/n of the
    # original's, and the error of the mean falls as 1/sqrt(k n)
    k, n = 50, a.size
    _, sk = kmc.replica_stats(np.tile(a, k))
    var = np.var(a)  # population variance of the four values
    assert abs(sk - np.sqrt(var * k * n / (k * n - 1) / (k * n))) < 1e-12
