"""Pins of the oracle's small-alpha heat-bath switch: Creutz's draw of x0
(Phys. Rev. D 21 (1980) 2308) in place of Kennedy-Pendleton's below a switch
in alpha, for the same local conditional of Sec. 2.4 (Eqs. (5)-(7)).

What fixes the answers: the exact density of x0 (quadrature CDF, and the
semicircle law in closed form as alpha -> 0); the per-attempt acceptance of
both methods in closed form (Bessel functions), which also fixes the switch
where the two are equal; and, for whole chains at strong coupling, the
expansion <P> = u + 4 u^5 + O(u^9) with u = I2(beta) / I1(beta) (Drouffe and
Zuber, Phys. Rep. 102 (1983) 1; the u^5 term is the cube around a plaquette,
four cubes per plaquette in four dimensions)."""
import numpy as np
import pytest
from scipy import optimize, special, stats

import oracle
import su2_inputs
from exact_density import (X0Cdf, creutz_accept_probability, haar_cdf, kp_accept_closed_form,
                           kp_accept_probability, mean_x0)
from paper_0903_3053_amd.stats import gamma_method

SWITCH = 1.6847376  # the binding's suggested switch, pinned below


def _samples(draw, alpha, n, prec32=True):
    xs, tries = [], []
    for site in range(n):
        t, a0, amag, _ = draw(alpha, 3, site, 2, 9, prec32)
        tries.append(t)
        if t >= 0:
            xs.append(a0)
            assert abs(a0 * a0 + amag * amag - 1.0) < 1e-6
    return np.array(xs), np.array(tries)


@pytest.mark.parametrize("alpha", [0.05, 0.3, 1.0, SWITCH, 3.0])
def test_creutz_draw_follows_exact_density(alpha):
    x, tries = _samples(oracle.creutz_draw, alpha, 20000)
    assert stats.kstest(x, X0Cdf(alpha)).pvalue > 1e-3
    m, se = x.mean(), x.std(ddof=1) / np.sqrt(len(x))
    assert abs(m - mean_x0(alpha)) < 4 * se


def test_creutz_draw_semicircle_limit():
    """alpha -> 0: the proposal is uniform on [-1, 1] and the accepted x0
    follow the semicircle law F(x) = 1/2 + (x sqrt(1-x^2) + arcsin x) / pi;
    the FP64 form (expm1, log1p) stays exact there."""
    for prec32 in (True, False):
        x, tries = _samples(oracle.creutz_draw, 1e-7, 20000, prec32)
        assert stats.kstest(x, haar_cdf).pvalue > 1e-3
        p = np.mean(tries >= 0)
        assert p > 1 - (1 - np.pi / 4) ** 8 - 1e-3


@pytest.mark.parametrize("alpha", [0.1, 0.5, SWITCH, 4.0])
def test_creutz_acceptance_closed_form(alpha):
    """Attempts per update follow the truncated geometric law of the closed-form
    per-attempt acceptance pi I1(alpha) / (2 sinh alpha)."""
    n = 20000
    _, tries = _samples(oracle.creutz_draw, alpha, n)
    p = float(creutz_accept_probability(alpha))
    a = np.arange(1, 9)
    pa = np.where(a < 8, p * (1 - p) ** (a - 1), (1 - p) ** 7)
    expect = np.sum(a * pa)
    sd = np.sqrt(np.sum(a * a * pa) - expect ** 2)
    attempts = np.where(tries >= 0, tries + 1, 8)
    assert abs(attempts.mean() - expect) < 4 * sd / np.sqrt(n)


def test_acceptance_closed_forms_and_switch():
    """Kennedy-Pendleton's closed form agrees with its quadrature; the two
    acceptance curves cross once, at the suggested switch; below it Creutz's
    is the higher one (towards pi/4 and 0 as alpha -> 0), above it KP's."""
    for a in (0.24, 1.0, 5.0):
        assert abs(float(kp_accept_closed_form(a)) - kp_accept_probability(a)) < 1e-7
    cross = optimize.brentq(lambda a: float(kp_accept_closed_form(a) - creutz_accept_probability(a)), 0.5, 3.0)
    assert abs(cross - SWITCH) < 1e-6
    assert abs(float(creutz_accept_probability(cross)) - 0.71138) < 1e-5
    assert abs(float(creutz_accept_probability(1e-9)) - np.pi / 4) < 1e-8
    for a in (0.05, 0.5, 1.5):
        assert creutz_accept_probability(a) > kp_accept_closed_form(a)
    for a in (1.8, 3.0, 10.0):
        assert creutz_accept_probability(a) < kp_accept_closed_form(a)


def test_switch_selects_the_draw():
    """A switch below every alpha leaves the chain bit-identical to plain KP;
    a switch above every alpha makes every update a Creutz update (its
    attempt counts match the per-link Creutz draws)."""
    dims = (4, 2, 4, 2)
    U0 = su2_inputs.random_links(dims, 41).astype(np.float64)
    Ua, Ub = U0.copy(), U0.copy()
    ra = oracle.heatbath_pass(dims, Ua, 0.4, 7, 3, 1, 2)
    rb = oracle.heatbath_pass(dims, Ub, 0.4, 7, 3, 1, 2, creutz_below=1e-30)
    assert np.array_equal(Ua, Ub) and np.array_equal(ra.tries, rb.tries)
    Uc = U0.copy()
    rc = oracle.heatbath_pass(dims, Uc, 0.4, 7, 3, 1, 2, creutz_below=4.0)  # alpha <= 0.4 * 6
    sites = np.nonzero(rc.tries >= 0)[0]
    for lex in sites:
        w = oracle.staple(dims, U0, int(lex), 2)
        t, a0, _, _ = oracle.creutz_draw(0.4 * np.linalg.norm(w), 7, int(lex), 2, 3)
        assert t == rc.tries[lex]


@pytest.mark.parametrize("beta", [0.25, 0.5])
def test_strong_coupling_plaquette_with_switch(beta):
    """Whole chains with the switch: <P> against the strong-coupling series,
    cap failures within their bound, and far fewer attempts than plain KP
    (which at beta = 0.25 leaves several per cent of the links unchanged at
    the cap)."""
    dims = (6, 6, 6, 6)
    c = oracle.Chain(dims, beta, 5, oracle.HOT, creutz_below=SWITCH)
    c.sweep(100)
    a0, f0 = c.attempts, c.failures
    P = []
    for _ in range(1500):
        c.sweep(1)
        P.append(c.plaquette()[0])
    m, se, _, _, _ = gamma_method(np.array(P))
    u = special.iv(2, beta) / special.iv(1, beta)
    ex = u + 4 * u ** 5
    print(f"beta {beta}: <P> {m:.6f}+-{se:.6f}, series {ex:.6f}")
    assert abs(m - ex) < 4 * se
    n_upd = 1500 * 4 * int(np.prod(dims))
    # with the switch every update's per-attempt acceptance is at least the
    # 71% at the switch, so the cap fails at most (1 - 0.71138)^8 = 4.8e-5 of the time
    assert (c.failures - f0) / n_upd < (1 - 0.71138) ** 8
    att_creutz = (c.attempts - a0) / n_upd
    k = oracle.Chain(dims, beta, 5, oracle.HOT)
    k.sweep(100)
    a1, f1 = k.attempts, k.failures
    k.sweep(200)
    att_kp = (k.attempts - a1) / (200 * 4 * int(np.prod(dims)))
    fail_kp = (k.failures - f1) / (200 * 4 * int(np.prod(dims)))
    print(f"beta {beta}: attempts per update Creutz {att_creutz:.3f}, KP {att_kp:.3f} (cap failures {fail_kp:.4f})")
    assert att_creutz < 0.75 * att_kp
    if beta == 0.25:
        assert fail_kp > 0.05
