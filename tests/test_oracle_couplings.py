"""The oracle's seeded instance generator (mc3o_couplings) pinned to what its
definition fixes: symmetric, zero diagonal, +-1 values with fair signs, and Gaussian
values of variance 1/N, which a Kolmogorov-Smirnov test checks against the normal law.
A dropped factor in sqrt(-2 ln u1), an angle of pi u2 instead of 2 pi u2 or one
uniform used twice fails the moment or distribution checks."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle


@pytest.mark.parametrize("kind", [oracle.COUPLINGS_PM1, oracle.COUPLINGS_GAUSS])
def test_symmetric_zero_diagonal_reproducible(kind):
    J, _ = oracle.couplings(96, kind, 11)
    assert np.array_equal(J, J.T)
    assert not np.diag(J).any()
    J2, _ = oracle.couplings(96, kind, 11)
    assert np.array_equal(J, J2)
    J3, _ = oracle.couplings(96, kind, 12)
    assert not np.array_equal(J, J3)
    # growing N keeps the draws of the first rows (pair (a, b) has its own counter);
    # Gaussian couplings carry the factor 1/sqrt(N)
    Jb, _ = oracle.couplings(128, kind, 11)
    if kind == oracle.COUPLINGS_PM1:
        assert np.array_equal(Jb[:96, :96], J)
    else:
        np.testing.assert_allclose(Jb[:96, :96] * math.sqrt(128), J * math.sqrt(96), rtol=1e-14, atol=0)


def test_pm1_values_and_fair_signs():
    N = 512
    J, scale = oracle.couplings(N, oracle.COUPLINGS_PM1, 3)
    assert scale == 1.0 / math.sqrt(N)
    u = J[np.triu_indices(N, 1)]
    assert set(np.unique(u)) == {-1.0, 1.0}
    n = u.size
    plus = int(np.sum(u > 0))
    assert abs(plus - n / 2) < 5 * math.sqrt(n / 4)
    # neighbouring pairs are not correlated
    assert abs(np.mean(u[1:] * u[:-1])) < 5 / math.sqrt(n)


def test_gauss_moments_and_law():
    N = 512
    J, scale = oracle.couplings(N, oracle.COUPLINGS_GAUSS, 5)
    assert scale == 1.0
    z = J[np.triu_indices(N, 1)] * math.sqrt(N)
    n = z.size
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    assert abs(stats.skew(z)) < 5 * math.sqrt(6.0 / n)
    assert abs(stats.kurtosis(z)) < 5 * math.sqrt(24.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    assert abs(np.mean(z[1:] * z[:-1])) < 5 / math.sqrt(n)


def test_unknown_kind_is_refused():
    with pytest.raises(ValueError):
        oracle.couplings(8, 2, 0)
