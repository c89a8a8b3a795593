"""Batched replicas through the C ABI: every replica must evolve bit for bit
as the same lattice run alone (whose parity with the oracle is tested in
test_gpu_parity.py), in every launch mode; one small replica is also checked
against the oracle directly."""
import numpy as np
import pytest

import oracle
import su2_inputs
from parity import UNIT_TOL, unitarity_error

pytestmark = pytest.mark.gpu

REPLICAS = [((8, 8, 8, 8), 2.2, 11), ((12, 12, 12, 12), 1.9, 12), ((6, 4, 10, 8), 2.6, 13),
            ((4, 4, 4, 4), 2.3, 1), ((16, 16, 16, 16), 2.4, 15), ((2, 2, 2, 2), 0.5, 16)]
MODES = [(0, 1, 0), (0, 2, 24576), (1, 1, 0), (1, 4, 24576), (1, 2, 0)]
NSWEEPS = 3


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_0903_3053_amd import su2
    su2.load()
    yield su2
    su2.su2_batch_finalize()
    su2.su2_finalize()


@pytest.fixture(scope="module")
def singles(lib):
    """Each replica run alone: links, counters and plaquette after NSWEEPS."""
    out = []
    for dims, beta, seed in REPLICAS:
        lib.su2_init(dims, beta, seed, lib.HOT)
        lib.su2_sweep(NSWEEPS)
        out.append((lib.su2_links(), lib.su2_counters()[:2], lib.su2_plaquette_st()))
    return out


def _batch(lib, mode):
    dims = [r[0] for r in REPLICAS]
    lib.su2_batch_init(dims, [r[1] for r in REPLICAS], [r[2] for r in REPLICAS], lib.HOT)
    lib.su2_batch_set_mode(*mode)


@pytest.mark.parametrize("mode", MODES)
def test_batch_bit_identical_to_single_runs(lib, singles, mode):
    _batch(lib, mode)
    lib.su2_batch_sweep(1)
    lib.su2_batch_sweep(NSWEEPS - 1)
    assert lib.su2_batch_sweep_index() == NSWEEPS
    P = lib.su2_batch_plaquette()
    for r, (U, ctr, Ps) in enumerate(singles):
        assert np.array_equal(lib.su2_batch_links(r), U), (mode, r)
        assert lib.su2_batch_counters(r) == ctr, (mode, r)
        np.testing.assert_allclose(P[r], Ps, rtol=0, atol=1e-12)


def test_batch_replica_against_oracle(lib):
    """One sweep of the persistent launch against the oracle from the same hot
    start.  Link-level agreement is a one-sweep statement: rounding
    differences grow by about x1.3 per further sweep (chaotic map, common
    random numbers), so later sweeps are tied to the oracle through the
    bit-identity with single-lattice runs (test_batch_tune_keeps_state and the
    single-lattice parity tests)."""
    _batch(lib, (1, 1, 0))
    lib.su2_batch_sweep(1)
    r = 3  # the 4^4 beta = 2.3 seed 1 replica
    dims, beta, seed = REPLICAS[r]
    ch = oracle.Chain(dims, beta, seed, oracle.HOT)
    ch.sweep(1)
    U = lib.su2_batch_links(r)
    err = float(np.max(np.abs(U - ch.U)))
    print(f"batch replica {dims} beta {beta}: one sweep, max |dU| vs oracle {err:.1e}")
    assert err <= 1e-5
    assert unitarity_error(U) <= UNIT_TOL


def test_batch_tune_keeps_state(lib, singles):
    _batch(lib, (0, 1, 0))
    lib.su2_batch_sweep(1)
    before = [lib.su2_batch_links(r) for r in range(len(REPLICAS))]
    choice = lib.su2_batch_tune(1)
    assert choice[0] in (0, 1) and choice[1] in (1, 2, 4, 8, 16)
    assert lib.su2_batch_sweep_index() == 1
    for r in range(len(REPLICAS)):
        assert np.array_equal(lib.su2_batch_links(r), before[r])
    lib.su2_batch_sweep(NSWEEPS - 1)
    for r, (U, ctr, _) in enumerate(singles):
        assert np.array_equal(lib.su2_batch_links(r), U)
        assert lib.su2_batch_counters(r) == ctr


def test_persistent_wait_limit_reports_and_recovers(lib, singles):
    """A one-tick bound on the persistent kernel's dependency waits: the launch
    must end (every workgroup leaves) and report the timeout as an error if
    any wait was needed; a fresh batch afterwards is exact again."""
    _batch(lib, (1, 1, 0))
    lib.su2_batch_set_spin_limit(1)
    try:
        lib.su2_batch_sweep(4)
        timed_out = False
    except lib.Su2Error as e:
        timed_out = True
        assert "time limit" in str(e)
    print(f"one-tick wait bound: timed out = {timed_out}")
    _batch(lib, (1, 1, 0))
    lib.su2_batch_sweep(NSWEEPS)
    for r, (U, _, _) in enumerate(singles):
        assert np.array_equal(lib.su2_batch_links(r), U)


def test_persistent_equals_grouped_on_64_replicas(lib):
    """The 64-replica workload (L in {8, ..., 24}, beta in [1.8, 2.8]): three
    sweeps in the persistent mode (replicas pinned to XCDs, several tile
    counts per item) leave every link of every replica bit-identical to the
    grouped mode."""
    table = su2_inputs.replica_table(64, 1)
    args = ([t["dims"] for t in table], [t["beta"] for t in table], [t["seed"] for t in table], lib.HOT)
    lib.su2_batch_init(*args)
    lib.su2_batch_set_mode(0, 1, 0)
    lib.su2_batch_sweep(3)
    ref = [lib.su2_batch_links(r) for r in range(len(table))]
    for mode in [(1, 1, 0), (1, 8, 24576)]:
        lib.su2_batch_init(*args)
        lib.su2_batch_set_mode(*mode)
        lib.su2_batch_sweep(1)
        lib.su2_batch_sweep(2)
        for r in range(len(table)):
            assert np.array_equal(lib.su2_batch_links(r), ref[r]), (mode, r)


def test_batch_errors(lib):
    with pytest.raises(lib.Su2Error):
        lib.su2_batch_init([(3, 4, 4, 4)], [2.0], [1], lib.HOT)
    with pytest.raises(lib.Su2Error):
        lib.su2_batch_init([(4, 4, 4, 4)], [-1.0], [1], lib.HOT)
    _batch(lib, (0, 1, 0))
    with pytest.raises(lib.Su2Error):
        lib.su2_batch_set_mode(2, 1, 0)
    with pytest.raises(lib.Su2Error):
        lib.su2_batch_links(len(REPLICAS))


def test_batch_64_replica_workload(lib):
    """The 64-replica workload (L uniform on {8, 12, 16, 20, 24}, beta uniform
    on [1.8, 2.8], hot starts, replica seed = 1 + 1 + r): two sweeps in the
    tuned mode; four replicas (including the largest) equal their single runs,
    every link stays unit."""
    table = su2_inputs.replica_table(64, 1)
    dims = [t["dims"] for t in table]
    lib.su2_batch_init(dims, [t["beta"] for t in table], [t["seed"] for t in table], lib.HOT)
    mode = lib.su2_batch_tune(1)
    lib.su2_batch_sweep(2)
    P = lib.su2_batch_plaquette()
    assert np.all(np.isfinite(P)) and np.all(np.abs(P) < 1)
    sizes = [int(np.prod(d)) for d in dims]
    check = sorted({int(np.argmax(sizes)), 0, 17, 63})
    for r in check:
        t = table[r]
        Ub = lib.su2_batch_links(r)
        assert unitarity_error(Ub) <= UNIT_TOL
        lib.su2_init(t["dims"], t["beta"], t["seed"], lib.HOT)
        lib.su2_sweep(2)
        assert np.array_equal(Ub, lib.su2_links()), r
    print(f"64 replicas, {sum(sizes)} sites, tuned mode {mode}")
