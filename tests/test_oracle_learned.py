"""Pins the learned-proposal pieces of the oracle: the CDF/quantile integrator,
the network's analytic gradient, BF16 rounding, and the exactness of the
independence-Metropolis step."""
import numpy as np
import pytest
from scipy import optimize, special, stats

import oracle
import su2_inputs
from exact_density import X0Cdf, haar_cdf
from oracle import cdf, mlp


@pytest.mark.parametrize("alpha", [0.5, 2.3, 13.8, 40.0])
def test_normaliser_closed_form(alpha):
    # int sqrt(1-t^2) e^{alpha (t-1)} dt = pi I1(alpha) e^{-alpha} / alpha
    ref = np.pi * special.ive(1, alpha) / alpha
    assert abs(cdf.normaliser(alpha) / ref - 1) < 1e-12


def test_alpha_zero_closed_form():
    assert abs(cdf.normaliser(0.0) - np.pi / 2) < 1e-13
    for x in np.linspace(-0.99, 0.99, 13):
        assert abs(cdf.cdf(x, 0.0) - haar_cdf(x)) < 1e-12
    y = cdf.knots(0.0)
    for j in range(1, 32):
        xj = optimize.brentq(lambda x: haar_cdf(x) - j / 32, -1, 1, xtol=1e-15)
        assert abs(y[j] - xj) < 1e-11


@pytest.mark.parametrize("alpha", [0.7, 8.0, 31.0])
def test_knots_consistent_and_match_tabulation(alpha):
    y = cdf.knots(alpha)
    assert y[0] == -1 and y[32] == 1 and np.all(np.diff(y) > 0)
    for j in range(1, 32):
        assert abs(cdf.cdf(y[j], alpha) - j / 32) < 1e-11
    tab = X0Cdf(alpha)
    np.testing.assert_allclose(y[1:-1], tab.inverse(np.arange(1, 32) / 32), atol=2e-6)


def test_bf16_rounding_matches_library():
    import torch
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.standard_normal(5000).astype(np.float32) * 10,
                        np.float32([0.0, -0.0, 1.0, 1.00390625, 1.005859375, 3.0e-39])])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    np.testing.assert_array_equal(mlp.bf16_round(x), ref)


def test_forward_gives_monotone_knots():
    th = mlp.bf16_round(su2_inputs.mlp_init(1))
    y, logw, _ = mlp.forward(th, su2_inputs.alpha_grid(50))
    assert y.shape == (50, 33)
    assert np.all(y[:, 0] == -1) and np.all(y[:, -1] == 1)
    assert np.all(np.diff(y, axis=1) > 0)
    np.testing.assert_allclose(np.exp(logw).sum(axis=1), 2.0, rtol=1e-13)


@pytest.mark.parametrize("rounded", [False, True])
def test_gradient_matches_finite_differences(rounded):
    rng = np.random.default_rng(9)
    th = su2_inputs.mlp_init(2).astype(np.float64) + 0.1 * rng.standard_normal(mlp.NPARAM)
    if rounded:
        th = mlp.bf16_round(th)
    alphas = su2_inputs.random_alphas(7, 3)
    target = np.log(np.full((7, 32), 2.0 / 32)) + 0.3 * rng.standard_normal((7, 32))
    L, g = mlp.loss_and_grad(th, alphas, target)
    idx = np.concatenate([rng.choice(mlp.NPARAM, 60, replace=False),
                          [0, 64, 128, 4160, 4224, mlp.NPARAM - 34, mlp.NPARAM - 1]])
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.NPARAM)
        e[i] = h
        fd = (mlp.loss_and_grad(th + e, alphas, target)[0]
              - mlp.loss_and_grad(th - e, alphas, target)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-6 * abs(g[i]), (i, fd, g[i])
    # the reserved output 32 never receives gradient
    W3 = mlp.unpack(g)["W3"]
    assert np.all(W3[32] == 0) and mlp.unpack(g)["b3"][32] == 0


def _imh_chain_samples(table, beta, passes, thin=10, burn=40):
    """All links equal to g: every (parity 0, mu 1) link has staple 6 g and keeps
    it while that pass is repeated, so each link runs its own chain at alpha = 6
    beta.  Returns thinned x0 = dot(U, g) samples and the acceptance rate
    after the burn-in."""
    dims = (4, 4, 4, 4)
    g = np.array([0.5, 0.5, -0.5, 0.5])
    U = np.tile(g, (256, 4, 1)).copy()
    par = np.array([sum(np.unravel_index(i, dims)) % 2 for i in range(256)])
    xs, prop, acc = [], 0, 0
    for s in range(passes):
        _, _, p, a = oracle.imh_pass(dims, U, beta, 7, s, 0, 1, table)
        if s >= burn:  # the start (x0 = 1, where pi vanishes) accepts every proposal
            prop += p
            acc += a
        if s >= burn and s % thin == 0:
            xs.append(U[par == 0, 1] @ g)
    return np.concatenate(xs), acc / prop


def _table_with_row(alpha_exact_row, knots_row):
    t = np.tile(np.linspace(-1, 1, 33), (41, 1))
    t[alpha_exact_row] = knots_row
    return t


def _expected_acceptance(alpha, knots, per_segment=4000):
    """Stationary acceptance of the independence sampler, E min(1, W(x')/W(x))
    for x ~ pi, x' ~ q, W = pi / q, by midpoint quadrature: pi(x) ~
    sqrt(1 - x^2) e^{alpha x} and q = 1/32 per segment, ~ e^{alpha x} inside.
    Written from those two densities alone (no part of the oracle's draw)."""
    xs, pis, qs = [], [], []
    for j in range(32):
        a, b = knots[j], knots[j + 1]
        h = (b - a) / per_segment
        x = a + h * (np.arange(per_segment) + 0.5)
        t = np.exp(alpha * (x - b))                     # e^{alpha (x - b)} <= 1
        qx = t / np.sum(t) / 32.0                       # segment mass 1/32
        xs.append(x)
        qs.append(qx)
        pis.append(np.sqrt(1.0 - x * x) * np.exp(alpha * (x - 1.0)) * h)
    x, q, pi = np.concatenate(xs), np.concatenate(qs), np.concatenate(pis)
    pi /= pi.sum()
    W = pi / q
    order = np.argsort(W)
    W, q, pi = W[order], q[order], pi[order]
    # for x at rank i: proposals with W' >= W_i accept surely, the others with W'/W_i
    q_above = np.cumsum(q[::-1])[::-1]
    qw_below = np.concatenate([[0.0], np.cumsum(q * W)[:-1]])
    # a current value where W = 0 (a zero-width segment: pi puts no mass there) adds nothing
    safe = np.where(W > 0, W, 1.0)
    return float(np.sum(np.where(W > 0, pi * (q_above + qw_below / safe), 0.0)))


def test_imh_step_leaves_the_conditional_invariant():
    """At alpha = 6 every link runs its own chain: its x0 samples follow the
    conditional (KS), and the acceptance rate equals the quadrature value for
    the tilted proposal (it would be 0.935 for one flat inside each segment)."""
    beta = 1.0  # alpha = 6: row 6 of a 41-row table on [0, 40]
    exact = cdf.knots(6.0)
    x, rate = _imh_chain_samples(_table_with_row(6, exact), beta, 400)
    want = _expected_acceptance(6.0, exact)
    print(f"alpha 6, exact knots: acceptance {rate:.4f}, quadrature {want:.4f}")
    assert want > 0.97 and abs(rate - want) < 3e-3
    assert stats.kstest(x, X0Cdf(6.0)).pvalue > 1e-3
    # a poor proposal (uniform knots) is slower but still exact
    uniform = np.linspace(-1, 1, 33)
    x2, rate2 = _imh_chain_samples(np.tile(uniform, (41, 1)), beta, 1200, thin=30, burn=120)
    want2 = _expected_acceptance(6.0, uniform)
    print(f"alpha 6, uniform knots: acceptance {rate2:.4f}, quadrature {want2:.4f}")
    assert rate2 < rate and abs(rate2 - want2) < 6e-3
    assert stats.kstest(x2, X0Cdf(6.0)).pvalue > 1e-3


def test_imh_knots_between_table_rows():
    """alpha = 6.5 lies halfway between rows 6 and 7 of a 41-row table on
    [0, 40]: row 6 holds the exact knots at alpha 6, row 7 uniform knots, so
    the proposal uses their even mix.  The chain stays exact (KS against the
    exact CDF at 6.5) and its acceptance equals the quadrature value for the
    mixed knots -- far from that of either row alone."""
    t = np.tile(np.linspace(-1, 1, 33), (41, 1))
    t[6] = cdf.knots(6.0)
    beta = 6.5 / 6.0
    x, rate = _imh_chain_samples(t, beta, 800, thin=20, burn=80)
    mixed = 0.5 * (t[6] + t[7])
    want = _expected_acceptance(6.5, mixed)
    only6, only7 = _expected_acceptance(6.5, t[6]), _expected_acceptance(6.5, t[7])
    print(f"alpha 6.5 between rows: acceptance {rate:.4f}, quadrature {want:.4f} "
          f"(row 6 alone {only6:.4f}, row 7 alone {only7:.4f})")
    # at 36 % acceptance the accept indicator is correlated over many passes:
    # about 0.004 of statistical spread, far below the rows' own values
    assert abs(rate - want) < 1e-2
    assert min(abs(want - only6), abs(want - only7)) > 0.1
    assert stats.kstest(x, X0Cdf(6.5)).pvalue > 1e-3


def test_imh_zero_width_segment():
    """A table whose segment 10 has zero width (an atom of the proposal):
    proposals drawn there are rejected and the chain stays exact; the
    acceptance equals the quadrature value, in which that atom contributes
    nothing (0.92, against 0.98 with the exact knots: the neighbouring segment
    also carries two quantiles' mass at one quantile's probability)."""
    k = cdf.knots(6.0).copy()
    k[11] = k[10]
    t = np.tile(np.linspace(-1, 1, 33), (41, 1))
    t[6] = k
    x, rate = _imh_chain_samples(t, 1.0, 400)
    want = _expected_acceptance(6.0, k)
    print(f"alpha 6, zero-width segment: acceptance {rate:.4f}, quadrature {want:.4f}")
    assert abs(rate - want) < 5e-3 and want < 0.97
    assert stats.kstest(x, X0Cdf(6.0)).pvalue > 1e-3


def test_imh_rejection_redraws_the_direction():
    """A rejected proposal keeps x0 = dot(U, V) and draws the direction about V
    afresh: after a pass with a poor (uniform) table on Haar links (FP64
    links), every rejected link has the same x0 to 1e-12, the direction n of
    U' V^dag is uniform on the sphere (KS of n_z on [-1, 1] and of its
    azimuth) and uncorrelated with the old one."""
    import su2_np
    dims = (8, 8, 8, 8)
    U0 = su2_inputs.random_links(dims, 17).astype(np.float64)
    mu, parity = 2, 0
    W = su2_np.staples(U0, dims)[:, mu]
    V = W / np.linalg.norm(W, axis=1)[:, None]
    U = U0.copy()
    res, _, p, a = oracle.imh_pass(dims, U, 1.0, 3, 0, parity, mu, np.tile(np.linspace(-1, 1, 33), (5, 1)),
                                   prec32=False)
    rej = res == 11
    assert rej.sum() > 500 and p - a == rej.sum()

    def x_of(Q):  # Q V^dag as quaternions
        return su2_np.from_matrix(su2_np.to_matrix(Q) @ su2_np.dag(su2_np.to_matrix(V[rej])))
    xn, xo = x_of(U[rej, mu]), x_of(U0[rej, mu])
    assert np.max(np.abs(xn[:, 0] - xo[:, 0])) < 1e-12
    n_new = xn[:, 1:] / np.linalg.norm(xn[:, 1:], axis=1)[:, None]
    n_old = xo[:, 1:] / np.linalg.norm(xo[:, 1:], axis=1)[:, None]
    assert stats.kstest(n_new[:, 2], stats.uniform(-1, 2).cdf).pvalue > 1e-3
    assert stats.kstest(np.arctan2(n_new[:, 1], n_new[:, 0]), stats.uniform(-np.pi, 2 * np.pi).cdf).pvalue > 1e-3
    assert abs(np.mean(np.sum(n_new * n_old, axis=1))) < 4.0 / np.sqrt(rej.sum())


def test_imh_fallbacks_by_alpha():
    """Updates whose alpha lies above the table's range use the plain heat-bath
    (identical links and codes); those inside use the proposal; alpha = 0 takes
    the Haar branch."""
    import su2_np
    dims = (4, 4, 4, 4)
    beta, amax, mu, parity = 1.2, 3.0, 2, 1
    U0 = su2_inputs.random_links(dims, 5).astype(np.float64)
    alpha = beta * np.linalg.norm(su2_np.staples(U0, dims)[:, mu], axis=1)
    par = np.array([sum(np.unravel_index(i, dims)) % 2 for i in range(256)])
    sel = par == parity
    assert np.any(alpha[sel] > amax) and np.any(alpha[sel] <= amax)
    tab = np.tile(np.linspace(-1, 1, 33), (5, 1))
    U = U0.copy()
    res, _, p, a = oracle.imh_pass(dims, U, beta, 1, 0, parity, mu, tab, alpha_max=amax)
    U2 = U0.copy()
    plain = oracle.heatbath_pass(dims, U2, beta, 1, 0, parity, mu)
    hi = sel & (alpha > amax)
    lo = sel & (alpha <= amax)
    assert np.all(res[hi] <= 9) and np.all(res[lo] >= 10)
    np.testing.assert_array_equal(res[hi], plain.tries[hi])
    np.testing.assert_array_equal(U[hi], U2[hi])
    assert p == int(lo.sum())
    U3 = U0.copy()
    res, _, p, a = oracle.imh_pass(dims, U3, 0.0, 1, 0, parity, mu, tab)
    assert np.all(res[sel] == 9) and p == 0
