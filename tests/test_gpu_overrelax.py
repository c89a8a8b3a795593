"""Overrelaxation on the GPU (U -> V U^dag V about the staple direction) against
the oracle and against what the move must conserve: links of one sweep within
the per-sweep bar of the oracle's sweep from the same state, the (total)
plaquette unchanged up to FP32 rounding, a pass applied twice giving the links back, the
same links for every launch plan, and a chain of 1 heat-bath : 3
overrelaxation sweeps with the heat-bath chain's <P>."""
import numpy as np
import pytest

import oracle
from paper_0903_3053_amd.stats import gamma_method
from parity import UNIT_TOL, unitarity_error

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_0903_3053_amd import su2
    su2.load()
    yield su2
    su2.su2_finalize()


@pytest.mark.parametrize("dims", [(8, 6, 10, 4), (4, 4, 4, 4), (2, 4, 2, 6)])
def test_overrelax_sweep_against_oracle(lib, dims):
    lib.su2_init(dims, 2.3, 5, lib.HOT)
    lib.su2_sweep(2)
    U = lib.su2_links().astype(np.float64)
    s0, c0 = lib.su2_sweep_index(), lib.su2_counters()
    oracle.or_sweep(dims, U, prec32=True)
    lib.su2_overrelax(1)
    gpu = lib.su2_links()
    err = float(np.max(np.abs(gpu - U)))
    print(f"overrelaxation sweep {dims} vs oracle: max |dU| {err:.1e}")
    assert err <= 1e-5
    assert unitarity_error(gpu) <= UNIT_TOL
    assert lib.su2_sweep_index() == s0 and lib.su2_counters() == c0


def test_overrelax_conserves_plaquette_and_undoes_itself(lib):
    dims = (16, 16, 16, 16)
    lib.su2_init(dims, 2.3, 8, lib.HOT)
    lib.su2_sweep(5)
    P0 = lib.su2_plaquette_st()
    U0 = lib.su2_links()
    lib.su2_overrelax(3)
    P1 = lib.su2_plaquette_st()
    moved = float(np.max(np.abs(lib.su2_links() - U0)))
    print(f"16^4: P before {P0[0]:.9f} after 3 overrelaxation sweeps {P1[0]:.9f} (P_s {P0[1]:.6f} -> "
          f"{P1[1]:.6f}, P_t {P0[2]:.6f} -> {P1[2]:.6f}); max link change {moved:.2f}")
    # each link keeps dot(U, w) for its whole staple sum, so the total plaquette
    # is conserved; the spatial/temporal split is not
    assert abs(P1[0] - P0[0]) <= 2e-6
    assert moved > 0.1
    lib.su2_init(dims, 2.3, 8, lib.HOT)
    lib.su2_sweep(5)
    for p in (1, 0):
        for mu in range(4):
            lib.su2_overrelax_pass(p, mu)
            lib.su2_overrelax_pass(p, mu)
    assert float(np.max(np.abs(lib.su2_links() - U0))) <= 1e-6


def test_overrelax_graphs_equal_single_sweeps(lib):
    """Runs of overrelaxation sweeps replay graphs of up to 16 sweeps; the
    links equal those of one-sweep calls, bit for bit."""
    dims = (8, 6, 10, 4)
    lib.su2_init(dims, 2.3, 9, lib.HOT)
    lib.su2_sweep(2)
    for _ in range(22):
        lib.su2_overrelax(1)
    ref = lib.su2_links()
    lib.su2_init(dims, 2.3, 9, lib.HOT)
    lib.su2_sweep(2)
    lib.su2_overrelax(3)
    lib.su2_overrelax(19)
    assert np.array_equal(lib.su2_links(), ref)


def test_overrelax_same_for_every_plan(lib):
    dims = (64, 64, 8, 8)
    ref = None
    for plan in [(0, 0), (108, 32768), (1108, 32768), (lib.FUSED_PAIRS, 0)]:
        lib.su2_init(dims, 2.3, 6, lib.HOT)
        lib.su2_set_plan(*plan)
        lib.su2_sweep(1)
        lib.su2_overrelax(2)
        U = lib.su2_links()
        if ref is None:
            ref = U
        assert np.array_equal(U, ref), plan


def test_overrelax_errors(lib):
    lib.su2_init((4, 4, 4, 4), 2.3, 1, lib.COLD)
    with pytest.raises(lib.Su2Error):
        lib.su2_overrelax(-1)
    with pytest.raises(lib.Su2Error):
        lib.su2_overrelax_pass(2, 0)
    with pytest.raises(lib.Su2Error):
        lib.su2_overrelax_pass(0, 4)
    lib.su2_overrelax(0)
    lib.su2_overrelax(2)  # every staple of the cold lattice is 6 (1, 0, 0, 0): a fixed point
    U = lib.su2_links()
    assert np.all(U[..., 0] == 1.0) and np.all(U[..., 1:] == 0.0)


def test_overrelaxed_chain_matches_heat_bath(lib):
    """16^4 beta 2.3, same hot start: <P> of 1 heat-bath + 3 overrelaxation
    sweeps per step agrees with the plain heat-bath chain within 3 sigma
    (Gamma-method errors, 400 steps after 50)."""
    dims, beta = (16, 16, 16, 16), 2.3
    lib.su2_init(dims, beta, 4, lib.HOT)
    lib.su2_sweep(50)
    hb = lib.su2_sweep_measure(400, 1)[:, 0]
    lib.su2_init(dims, beta, 4, lib.HOT)
    for _ in range(50):
        lib.su2_sweep(1)
        lib.su2_overrelax(3)
    orx = []
    for _ in range(400):
        lib.su2_sweep(1)
        lib.su2_overrelax(3)
        orx.append(lib.su2_plaquette())
    m1, s1, t1, _, _ = gamma_method(hb)
    m2, s2, t2, _, _ = gamma_method(np.asarray(orx))
    z = (m2 - m1) / np.hypot(s1, s2)
    print(f"16^4 beta 2.3: <P> heat-bath {m1:.6f}+-{s1:.6f} (tau_int {t1:.2f} steps), 1 HB + 3 OR "
          f"{m2:.6f}+-{s2:.6f} (tau_int {t2:.2f} steps), z = {z:+.2f}")
    assert abs(z) < 3.0
