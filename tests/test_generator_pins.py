"""Pins for the reference flood-field generator: Philox4x32-10 against the
published known-answer vectors, and the Poisson sampler against the Poisson
distribution (mean, variance, goodness of fit)."""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        w = [int(v, 16) for v in r]
        assert oracle.philox4x32_10(w[:4], w[4:6]) == w[6:10]


@pytest.mark.parametrize("mu", [0.3, 3.0, 9.9, 10.0, 47.5, 420.0])
def test_poisson_mean_and_variance(mu):
    n = 20000
    x = np.array([oracle.poisson(mu, e, 7, 12345) for e in range(n)])
    assert np.all(x == np.floor(x)) and x.min() >= 0
    se = math.sqrt(mu / n)
    assert abs(x.mean() - mu) < 5 * se
    # variance of the sample variance ~ (2 mu^2 + mu) / n
    assert abs(x.var() - mu) < 5 * math.sqrt((2 * mu * mu + mu) / n)


@pytest.mark.parametrize("mu", [4.0, 35.0])
def test_poisson_goodness_of_fit(mu):
    from scipy import stats
    n = 40000
    x = np.array([oracle.poisson(mu, e, 3, 99) for e in range(n)]).astype(int)
    lo, hi = int(max(0, mu - 4 * math.sqrt(mu))), int(mu + 4 * math.sqrt(mu))
    ks = np.arange(lo, hi + 1)
    obs = np.array([(x == k).sum() for k in ks] + [(x < lo).sum() + (x > hi).sum()])
    pmf = stats.poisson.pmf(ks, mu)
    exp = np.concatenate([pmf, [1 - pmf.sum()]]) * n
    keep = exp > 5
    chi2 = ((obs[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-3


def test_generated_positions_fill_the_region_uniformly():
    wl = W.workload(2)
    sig, truth = oracle.generate(wl.lrf, 0, 90.0, 0.0, 50.0, 500.0, 2000.0, 20000, seed=5)
    r = np.hypot(truth[:, 0], truth[:, 1])
    assert r.max() <= 90.0
    # uniform over the disc: r^2 uniform in [0, 90^2]
    from scipy import stats
    assert stats.kstest(r ** 2 / 8100.0, "uniform").pvalue > 1e-3
    assert stats.kstest(truth[:, 2] / 50.0, "uniform").pvalue > 1e-3
    # noiseless means add up to E_tot
    sig0, truth0 = oracle.generate(wl.lrf, 0, 90.0, 0.0, 50.0, 500.0, 2000.0, 200, seed=5,
                                   noiseless=True)
    np.testing.assert_allclose(sig0.sum(1), truth0[:, 3], rtol=1e-12)
    np.testing.assert_array_equal(truth0, truth[:200])
