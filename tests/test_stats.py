"""Pins of the Gamma-method error analysis (paper_0903_3053_amd/stats.py)
against processes whose autocorrelation is known in closed form."""
import numpy as np

from paper_0903_3053_amd.stats import autocovariance, gamma_method


def ar1(n, rho, rng, chains=1):
    """x_t = rho x_{t-1} + sqrt(1 - rho^2) e_t, started in equilibrium; its
    integrated autocorrelation time is (1 + rho) / (2 (1 - rho))."""
    e = rng.standard_normal((chains, n))
    x = np.empty((chains, n))
    x[:, 0] = e[:, 0]
    s = np.sqrt(1.0 - rho * rho)
    for t in range(1, n):
        x[:, t] = rho * x[:, t - 1] + s * e[:, t]
    return x


def test_autocovariance_matches_direct_sum():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(300)
    d = x - x.mean()
    g = autocovariance(x)
    for t in (0, 1, 7, 150, 299):
        assert abs(g[t] - np.dot(d[: 300 - t], d[t:]) / (300 - t)) < 1e-12


def test_uncorrelated_series():
    rng = np.random.default_rng(2)
    x = rng.standard_normal(100_000)
    m, err, tau, dtau, w = gamma_method(x)
    assert abs(tau - 0.5) < 0.05
    assert abs(err / (x.std() / np.sqrt(len(x))) - 1.0) < 0.05


def test_ar1_tau_int():
    rng = np.random.default_rng(3)
    for rho in (0.5, 0.8, 0.95):
        x = ar1(200_000, rho, rng)[0]
        _, _, tau, dtau, _ = gamma_method(x)
        exact = (1 + rho) / (2 * (1 - rho))
        assert abs(tau - exact) < max(3 * dtau, 0.02 * exact), (rho, tau, exact, dtau)


def test_error_covers_the_true_mean():
    """300 AR(1) chains of 2000 samples at tau_int = 9.5: the z-scores of their
    means (true mean 0) have unit spread, and about 95 % lie within 2."""
    rng = np.random.default_rng(4)
    xs = ar1(2000, 0.9, rng, chains=300)
    z = np.array([m / e for m, e, *_ in map(gamma_method, xs)])
    assert 0.85 < z.std() < 1.2
    assert np.mean(np.abs(z) < 2.0) > 0.9
