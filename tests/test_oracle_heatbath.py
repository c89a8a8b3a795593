"""Pins the oracle's heat-bath update (Sec. 2.4, Eqs. (5)-(7)) against exact
distributions, closed forms and equilibrium identities."""
import numpy as np
import pytest
from scipy import stats

import oracle
import su2_inputs
import su2_np
from exact_density import X0Cdf, haar_cdf, kp_accept_probability, mean_x0

SEED = 1


def _kp_samples(alpha, n, seed=SEED, prec32=True):
    xs, tries = [], []
    for site in range(n):
        t, a0, amag, _ = oracle.kp_draw(alpha, seed, site, 1, 17, prec32)
        tries.append(t)
        if t >= 0:
            xs.append(a0)
            assert abs(a0 * a0 + amag * amag - 1.0) < 1e-6
    return np.array(xs), np.array(tries)


@pytest.mark.parametrize("alpha", [0.5, 1.0, 2.3, 5.0, 13.8, 40.0])
def test_kp_draw_follows_exact_density(alpha):
    x, tries = _kp_samples(alpha, 20000)
    cdf = X0Cdf(alpha)
    p = stats.kstest(x, cdf).pvalue
    assert p > 1e-3, (alpha, p)
    # mean against I2/I1
    m, se = x.mean(), x.std(ddof=1) / np.sqrt(len(x))
    assert abs(m - mean_x0(alpha)) < 4 * se, (alpha, m, mean_x0(alpha), se)


@pytest.mark.parametrize("alpha", [0.24, 1.0, 5.0])
def test_kp_acceptance_and_cap(alpha):
    """Per-attempt acceptance is E[sqrt(1-lambda^2)] under the Gamma(3/2)
    proposal; the cap fails with probability (1-p)^8."""
    n = 20000
    _, tries = _kp_samples(alpha, n)
    p = kp_accept_probability(alpha)
    attempts = np.where(tries >= 0, tries + 1, 8)
    # attempts per update, truncated geometric
    a = np.arange(1, 9)
    pa = np.where(a < 8, p * (1 - p) ** (a - 1), (1 - p) ** 7)
    expect = np.sum(a * pa)
    sd = np.sqrt(np.sum(a * a * pa) - expect ** 2)
    assert abs(attempts.mean() - expect) < 4 * sd / np.sqrt(n)
    fail = np.mean(tries < 0)
    pf = (1 - p) ** 8
    assert abs(fail - pf) < 4 * np.sqrt(pf * (1 - pf) / n) + 1e-4


def test_kp_fp64_mode_same_distribution():
    x, _ = _kp_samples(2.3, 20000, prec32=False)
    assert stats.kstest(x, X0Cdf(2.3)).pvalue > 1e-3


def test_hot_start_is_haar():
    dims = (8, 8, 8, 8)
    U = oracle.init(dims, 3, oracle.HOT)
    q = U.reshape(-1, 4)
    np.testing.assert_allclose(np.linalg.norm(q, axis=1), 1.0, atol=2e-7)
    for c in range(4):
        assert stats.kstest(q[:, c], haar_cdf).pvalue > 1e-3
    C = q.T @ q / len(q)
    np.testing.assert_allclose(C, np.eye(4) / 4, atol=4 * 0.25 / np.sqrt(len(q)) * 2)
    P = oracle.plaquette(dims, U)[0]
    assert abs(P) < 4 * 0.5 / np.sqrt(6 * su2_inputs.volume(dims))


def test_cold_single_pass_draws_at_six_beta():
    """Cold start, one pass (odd, mu=0): every staple is 6*(1,0,0,0), so the new
    links are i.i.d. X with x0 at alpha = 6 beta and a uniform direction."""
    dims = (8, 8, 8, 8)
    beta = 2.3
    U = oracle.init(dims, SEED, oracle.COLD)
    res = oracle.heatbath_pass(dims, U, beta, SEED, 0, 1, 0)
    odd = res.tries >= 0
    q = U[odd, 0]
    assert stats.kstest(q[:, 0], X0Cdf(6 * beta)).pvalue > 1e-3
    n = q[:, 1:] / np.linalg.norm(q[:, 1:], axis=1, keepdims=True)
    for c in range(3):
        assert stats.kstest(n[:, c], stats.uniform(-1, 2).cdf).pvalue > 1e-3
    # other links untouched
    assert np.all(U[~odd, 0] == np.array([1.0, 0, 0, 0]))
    assert np.all(U[:, 1:] == np.array([1.0, 0, 0, 0]))


def test_rotation_about_staple_direction():
    """All links equal to one SU(2) element g: every staple is 6 g, so U' = X g
    with dot(U', g) = x0 ~ exact density at 6 beta and U' g^dag isotropic."""
    dims = (4, 4, 4, 4)
    beta = 1.1
    g = np.array([0.3, -0.5, 0.7, 0.2])
    g /= np.linalg.norm(g)
    g = g.astype(np.float32).astype(np.float64)
    x0s, dirs = [], []
    for s in range(60):
        U = np.tile(g, (256, 4, 1)).copy()
        oracle.heatbath_pass(dims, U, beta, SEED, s, 0, 2)
        even = np.array([sum(np.unravel_index(i, (4, 4, 4, 4))) % 2 == 0 for i in range(256)])
        for q in U[even, 2]:
            X = su2_np.from_matrix(su2_np.to_matrix(q) @ su2_np.dag(su2_np.to_matrix(g)))
            x0s.append(X[0])
            dirs.append(X[1:] / np.linalg.norm(X[1:]))
    x0s, dirs = np.array(x0s), np.array(dirs)
    assert stats.kstest(x0s, X0Cdf(6 * beta)).pvalue > 1e-3
    for c in range(3):
        assert stats.kstest(dirs[:, c], stats.uniform(-1, 2).cdf).pvalue > 1e-3


def test_pass_touches_only_its_links_and_staples_do_not_depend_on_them():
    dims = (4, 4, 2, 6)
    U = su2_inputs.random_links(dims, 11).astype(np.float64)
    for parity in (1, 0):
        for mu in range(4):
            before = U.copy()
            W0 = su2_np.staples(before, dims)[:, mu]
            oracle.heatbath_pass(dims, U, 2.0, SEED, 3, parity, mu)
            lex = np.arange(U.shape[0])
            x = np.array(np.unravel_index(lex, dims[::-1]))  # (x3,x2,x1,x0)
            par = x.sum(axis=0) % 2
            changed = np.any(U != before, axis=2)
            mask = np.zeros_like(changed)
            mask[par == parity, mu] = True
            assert not np.any(changed & ~mask)
            # staples of the updated links are the same before and after, so
            # the update order inside a pass cannot matter
            W1 = su2_np.staples(U, dims)[:, mu]
            np.testing.assert_allclose(W1[par == parity], W0[par == parity], atol=1e-12)


def test_beta_zero_gives_haar():
    dims = (8, 8, 8, 8)
    c = oracle.Chain(dims, 0.0, 5, oracle.COLD)
    c.sweep(1)
    q = c.U.reshape(-1, 4)
    assert stats.kstest(q[:, 0], haar_cdf).pvalue > 1e-3
    ps = []
    for _ in range(10):
        ps.append(c.plaquette()[0])
        c.sweep(1)
    # each sweep redraws every link independently: configurations are independent
    sigma = 0.5 / np.sqrt(6 * su2_inputs.volume(dims) * len(ps))
    assert abs(np.mean(ps)) < 4 * sigma


def _binned_mean(x, nbins=10):
    x = np.asarray(x)
    b = len(x) // nbins
    means = x[: b * nbins].reshape(nbins, b).mean(axis=1)
    return means.mean(), means.std(ddof=1) / np.sqrt(nbins)


def test_strong_coupling():
    """<P> = I2(beta)/I1(beta) + O(beta^5) at small beta."""
    dims = (8, 8, 8, 8)
    beta = 0.1
    c = oracle.Chain(dims, beta, 21, oracle.HOT)
    c.sweep(20)
    ps = []
    for _ in range(100):
        c.sweep(1)
        ps.append(c.plaquette()[0])
    m, se = _binned_mean(ps)
    assert abs(m - mean_x0(beta)) < 4 * se, (m, mean_x0(beta), se)


def test_equilibrium_identity():
    """In equilibrium <dot(U, W)> = <k I2(beta k)/I1(beta k)> link by link;
    summed, 6 <P> = <mean over links of k I2(beta k)/I1(beta k)>."""
    dims = (4, 4, 4, 4)
    beta = 2.3
    c = oracle.Chain(dims, beta, 31, oracle.HOT)
    c.sweep(50)
    D = []
    for _ in range(200):
        c.sweep(1)
        W = su2_np.staples(c.U, dims)
        k = np.linalg.norm(W, axis=2)
        rhs = np.mean(k * mean_x0(beta * k))
        D.append(6 * c.plaquette()[0] - rhs)
    m, se = _binned_mean(D)
    assert abs(m) < 4 * se, (m, se)
    assert se < 0.01


def test_update_sites_equals_pass():
    dims = (4, 6, 4, 2)
    U = su2_inputs.random_links(dims, 12).astype(np.float64)
    x = np.array(np.unravel_index(np.arange(U.shape[0]), dims[::-1]))
    par = x.sum(axis=0) % 2
    sites = np.flatnonzero(par == 1)[::3]
    out, tries, _ = oracle.update_sites(dims, U, 2.2, SEED, 4, 3, sites)
    U2 = U.copy()
    res = oracle.heatbath_pass(dims, U2, 2.2, SEED, 4, 1, 3)
    np.testing.assert_array_equal(out, U2[sites, 3])
    np.testing.assert_array_equal(tries, res.tries[sites])


def test_init_sites_equals_init():
    dims = (4, 6, 4, 2)
    sites = np.array([0, 1, 5, 77, 190, 191])
    for start in (0, 1):
        for prec32 in (True, False):
            U = oracle.init(dims, SEED, start, prec32)
            np.testing.assert_array_equal(oracle.init_sites(dims, SEED, start, sites, prec32), U[sites])
    with pytest.raises(ValueError):
        oracle.init_sites(dims, SEED, 1, [192])


@pytest.mark.parametrize("draw", [oracle.kp_draw, oracle.creutz_draw])
def test_fp32_mode_changes_only_the_decision(draw):
    """With FP32 link storage (the paper's, Sec. 2.4) only the accept test is
    taken in FP32: whenever both precisions accept the same attempt, the drawn
    x0 and |a| are the same FP64 numbers, not FP32 roundings of them."""
    same = not_f32 = 0
    for alpha in (0.3, 1.7, 2.3, 9.0, 40.0):
        for site in range(400):
            t32, a32, m32, _ = draw(alpha, 5, site, 2, 3, True)
            t64, a64, m64, _ = draw(alpha, 5, site, 2, 3, False)
            if t32 >= 0 and t32 == t64:
                same += 1
                assert a32 == a64 and m32 == m64, (alpha, site)
                not_f32 += int(np.float64(np.float32(a32)) != a32)
    assert same >= 1800
    assert not_f32 >= 0.9 * same
