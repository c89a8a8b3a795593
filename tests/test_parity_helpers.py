"""Host checks of the parity helpers (tests/parity.py) and of the oracle's
per-link diagnostics they use (no GPU)."""
import numpy as np

import oracle
import su2_inputs
from parity import (LINK_TOL, compare_links_conditioned, conditioning, link_tolerance, parity_of,
                    pass_index, staple_inputs)


def test_staple_inputs_are_exactly_the_links_the_staple_reads():
    """Changing any of the 18 listed links changes the oracle's staple sum;
    changing any other link leaves it unchanged (brute force on 4x6x4x6)."""
    dims = (4, 6, 4, 6)
    U = su2_inputs.random_links(dims, 3).astype(np.float64)
    rng = np.random.default_rng(4)
    V = U.shape[0]
    for lex, mu in [(0, 0), (37, 1), (V - 1, 3), (200, 2)]:
        w0 = oracle.staple(dims, U, lex, mu)
        s, d = staple_inputs(dims, [lex], mu)
        listed = set(zip(s[0].tolist(), d[0].tolist()))
        assert len(listed) == 18
        for (y, nu) in list(listed) + [(int(rng.integers(V)), int(rng.integers(4))) for _ in range(40)]:
            W = U.copy()
            W[y, nu] = [0.6, 0.0, 0.8, 0.0]
            changed = np.max(np.abs(oracle.staple(dims, W, lex, mu) - w0)) > 1e-12
            assert changed == ((y, nu) in listed), (lex, mu, y, nu)


def test_pass_diagnostics_match_the_staple_and_the_new_link():
    """diag=True returns, per updated site, k = |w| of the oracle's staple and
    the accepted x0 = dot(U_new, w) / k (FP32 storage of U_new aside)."""
    dims, beta = (4, 4, 6, 4), 2.3
    U = su2_inputs.random_links(dims, 8).astype(np.float64)
    U0 = U.copy()
    res = oracle.heatbath_pass(dims, U, beta, 5, 2, 1, 2, diag=True)
    sel = np.flatnonzero(parity_of(dims) == 1)
    assert np.all(np.isnan(res.knorm[parity_of(dims) == 0]))
    for lex in sel[:40]:
        w = oracle.staple(dims, U0, int(lex), 2)
        k = np.linalg.norm(w)
        assert abs(res.knorm[lex] - k) <= 1e-12 * k
        if res.tries[lex] <= 7:
            assert abs(res.x0[lex] - np.dot(U[lex, 2], w) / k) <= 1e-6
        else:
            assert np.isnan(res.x0[lex])
    kn = oracle.or_pass(dims, U.copy(), 0, 3, diag=True)
    lex = int(np.flatnonzero(parity_of(dims) == 0)[5])
    assert abs(kn[lex] - np.linalg.norm(oracle.staple(dims, U, lex, 3))) <= 1e-12


def test_conditioned_comparison_flags_a_wrong_link():
    n = 1000
    rng = np.random.default_rng(1)
    ora = rng.standard_normal((n, 4))
    k = rng.uniform(1.0, 6.0, n)
    x0 = rng.uniform(-0.5, 0.9, n)
    margin = np.full(n, 1.0)
    gpu = ora + 1e-7
    st = compare_links_conditioned(gpu, ora, margin, k, x0)
    assert st["unexplained"] == 0 and st["over"] == 0
    gpu[7] += 3e-4  # well-conditioned link off by far more than rounding
    st = compare_links_conditioned(gpu, ora, margin, k, x0)
    assert st["unexplained"] == 1
    # the same error at a link with k = 1e-3 is within its bar
    k[7] = 1e-3
    assert compare_links_conditioned(gpu, ora, margin, k, x0)["unexplained"] == 0
    # ... and near x0 = -1
    k[7], x0[7] = 3.0, -1.0 + 1e-9
    assert compare_links_conditioned(gpu, ora, margin, k, x0)["unexplained"] == 0
    # a flip (small oracle margin) is counted, not failed
    k[7], x0[7], margin[7] = 3.0, 0.5, 1e-7
    st = compare_links_conditioned(gpu, ora, margin, k, x0)
    assert st["unexplained"] == 0 and st["flips"] == 1


def test_tolerance_is_the_plain_bar_for_well_conditioned_links():
    cond, _ = conditioning([6.0, 3.0], [0.9, 0.0])
    assert np.all(cond < 10.0)
    np.testing.assert_array_equal(link_tolerance([6.0, 3.0], [0.9, 0.0]), [LINK_TOL, LINK_TOL])
    assert pass_index(1, 0) == 0 and pass_index(1, 3) == 3 and pass_index(0, 0) == 4 and pass_index(0, 3) == 7
