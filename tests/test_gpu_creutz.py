"""The heat-bath's small-alpha switch (Creutz's draw below alpha_below, the
same cap and Philox slots) through the C ABI against the oracle: single
passes element by element (<= 1e-5 per component, flips only where the oracle
reports a decision margin below 1e-5, which includes alpha within 1e-5 of the
switch), counters exact without flips; sweeps from the oracle's state; the
fused-pair kernels' Creutz variants, bit-identical to the single passes; and a
strong-coupling chain on the GPU against <P> = u + 4 u^5, u = I2/I1."""
import numpy as np
import pytest
from scipy import special

import oracle
import su2_inputs
from parity import UNIT_TOL, compare_links, parity_of, unitarity_error
from paper_0903_3053_amd.stats import gamma_method

pytestmark = pytest.mark.gpu

SHAPES = [(8, 6, 10, 4), (2, 4, 2, 6), (12, 12, 12, 12), (2, 2, 2, 2)]


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_0903_3053_amd import su2
    su2.load()
    yield su2
    su2.su2_finalize()


def _pass_case(lib, dims, U0, beta, seed, s, parity, mu, switch):
    V = int(np.prod(dims))
    lib.su2_init(dims, beta, seed, lib.COLD)
    lib.su2_set_creutz(switch)
    lib.su2_set_links(U0, s)
    lib.su2_pass(parity, mu)
    gpu = lib.su2_links()
    att, fail = lib.su2_counters()[:2]
    U = U0.astype(np.float64)
    res = oracle.heatbath_pass(dims, U, beta, seed, s, parity, mu, creutz_below=switch)
    nflip, err = compare_links(gpu[:, mu], U[:, mu], res.margin)
    other = np.ones((V, 4), dtype=bool)
    other[parity_of(dims) == parity, mu] = False
    assert np.array_equal(gpu[other], U0[other])
    assert unitarity_error(gpu[parity_of(dims) == parity, mu]) <= UNIT_TOL
    if nflip == 0:
        assert (att, fail) == (res.attempts, res.failures)
    return nflip, err


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("beta,switch", [(0.25, 1.6847376), (0.9, 1.6847376), (0.6, 4.0), (2.3, 1.6847376)])
def test_pass_parity_with_switch(lib, dims, beta, switch):
    U0 = su2_inputs.random_links(dims, 201)
    flips, worst, n = 0, 0.0, 0
    for parity in (1, 0):
        for mu in range(4):
            f, e = _pass_case(lib, dims, U0, beta, 31, 3 + mu, parity, mu, switch)
            flips += f
            worst = max(worst, e)
            n += int(np.prod(dims)) // 2
    print(f"Creutz pass parity {dims} beta {beta} switch {switch}: {n} updates, {flips} flips, max err {worst:.2e}")
    assert flips <= max(2, n * 1e-4)


def test_sweeps_from_oracle_state(lib):
    """8x6x10x4 at beta 0.7 from a hot start, 20 sweeps each started from the
    oracle's state (a flip stays inside its sweep); attempts and cap failures
    summed over the sweeps."""
    dims, beta, seed, sw = (8, 6, 10, 4), 0.7, 4, 1.6847376
    U = oracle.init(dims, seed, oracle.HOT)
    lib.su2_init(dims, beta, seed, lib.HOT)
    lib.su2_set_creutz(sw)
    off, att_o, att_g = 0, 0, 0
    for s in range(20):
        lib.su2_set_links(U.astype(np.float32), s)
        c0 = lib.su2_counters()
        lib.su2_sweep(1)
        c1 = lib.su2_counters()
        gpu = lib.su2_links()
        a, _ = oracle.sweep(dims, U, beta, seed, s, creutz_below=sw)
        att_o += a
        att_g += c1[0] - c0[0]
        off += int(np.sum(np.max(np.abs(gpu - U), axis=2) > 1e-5))
        assert unitarity_error(gpu) <= UNIT_TOL
    print(f"Creutz sweeps {dims}: {20 * 4 * 1920} updates, {off} links off by > 1e-5, attempts gpu {att_g} oracle {att_o}")
    assert off <= 5
    assert abs(att_g - att_o) <= 8 * off


@pytest.mark.parametrize("dims", [(8, 6, 10, 4), (2, 4, 2, 6), (16, 16, 16, 16), (32, 8, 6, 10)])
def test_fused_plan_with_switch(lib, dims):
    """The fused-pair kernels' Creutz variants against the single passes with
    the switch: links and counters bit-identical after three sweeps (the last
    measured), the in-sweep plaquette to 1e-13 and to the plaquette kernel;
    with the switch off again the fused heat-bath kernels are back
    (bit-identical to the single passes)."""
    beta, seed, sw = 0.8, 12, 1.6847376
    lib.su2_init(dims, beta, seed, lib.HOT)
    lib.su2_set_creutz(sw)
    lib.su2_sweep(2)
    m_ref = lib.su2_sweep_measure(1, 1)
    ref, c_ref = lib.su2_links(), lib.su2_counters()
    lib.su2_init(dims, beta, seed, lib.HOT)
    lib.su2_set_plan(lib.FUSED_PAIRS, 0)
    lib.su2_set_creutz(sw)
    lib.su2_sweep(2)
    m = lib.su2_sweep_measure(1, 1)
    assert np.array_equal(lib.su2_links(), ref)
    assert lib.su2_counters() == c_ref
    np.testing.assert_allclose(m, m_ref, rtol=0, atol=1e-13)
    np.testing.assert_allclose(lib.su2_plaquette_st(), m[0], rtol=0, atol=2e-6)
    lib.su2_set_creutz(0.0)
    lib.su2_sweep(1)
    after_fused = lib.su2_links()
    lib.su2_set_plan(0, 0)
    lib.su2_set_links(ref, 3)
    lib.su2_sweep(1)
    assert np.array_equal(lib.su2_links(), after_fused)


def test_switch_errors_and_proposal_reset(lib):
    """The switch is refused outside [0, 4] and survives su2_set_proposal(0)."""
    dims, beta, seed, sw = (4, 4, 4, 4), 0.5, 2, 1.6847376
    lib.su2_init(dims, beta, seed, lib.HOT)
    for bad in (-0.1, 4.5, float("nan"), float("inf")):
        with pytest.raises(lib.Su2Error):
            lib.su2_set_creutz(bad)
    lib.su2_set_creutz(sw)
    lib.su2_set_proposal(0)  # the heat-bath again: the switch stays on
    lib.su2_sweep(1)
    U = oracle.init(dims, seed, oracle.HOT)
    oracle.sweep(dims, U, beta, seed, 0, creutz_below=sw)
    assert np.sum(np.max(np.abs(lib.su2_links() - U), axis=2) > 1e-5) <= 10


def test_strong_coupling_chain_on_gpu(lib):
    """16^4 at beta 0.25 with the switch, 600 measured sweeps after 100:
    <P> against the strong-coupling series within 4 sigma, cap failures
    within (1 - 0.71138)^8 per update, about 1.29 attempts per update (plain
    KP needs about 3.2 and leaves 8.5% of the links at the cap)."""
    dims, beta, seed = (16, 16, 16, 16), 0.25, 7
    lib.su2_init(dims, beta, seed, lib.HOT)
    lib.su2_set_creutz(1.6847376)
    lib.su2_sweep(100)
    c0 = lib.su2_counters()
    hist = lib.su2_sweep_measure(600, 1)
    c1 = lib.su2_counters()
    m, se, tau, _, _ = gamma_method(hist[:, 0])
    u = special.iv(2, beta) / special.iv(1, beta)
    ex = u + 4 * u ** 5
    n_upd = 600 * 4 * 16 ** 4
    att = (c1[0] - c0[0]) / n_upd
    fail = (c1[1] - c0[1]) / n_upd
    print(f"16^4 beta 0.25 with the switch: <P> {m:.6f}+-{se:.6f} series {ex:.6f}; "
          f"attempts/update {att:.3f}, cap failures/update {fail:.2e}")
    assert abs(m - ex) < 4 * se
    assert fail < (1 - 0.71138) ** 8
    assert 1.2 < att < 1.4
