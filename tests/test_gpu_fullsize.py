"""Parity at the benchmark's full size, in the benchmark's launch plan:
64^4, beta 2.4, hot start (Philox seed 1), tile order 1108 (order 108, every
second pass walked backwards) with 32 KiB of LDS reserved per workgroup.

Each updated link is held to LINK_TOL = 1e-5, except where FP32 rounding can
move it further: tests/parity.py derives the per-link bar from the oracle's
own numbers for that update -- the staple norm k = |w| (V = w/k and
alpha = beta k carry the staple's rounding divided by k) and the accepted x0
(|a| = 2 sqrt(lambda^2 (1 - lambda^2)) carries lambda^2's rounding times
sqrt(lambda^2 / (1 - lambda^2)), large as x0 -> -1) -- and, in a free-running
sweep, from the errors of the input links an earlier pass of the same sweep
wrote.  A mismatch at an oracle decision margin below 1e-5 is a flipped
accept decision and is counted.  Every link over 1e-5 is printed with its
error, k, x0 and error / bar.
"""
import numpy as np
import pytest

import oracle
from parity import (KAPPA_OVERRELAX, LINK_TOL, UNIT_TOL, compare_links_conditioned,
                    link_tolerance, parity_of, pass_index, staple_inputs, unitarity_error)

pytestmark = pytest.mark.gpu

DIMS, BETA, SEED = (64, 64, 64, 64), 2.4, 1
PLAN = (1108, 32768)
V = 64 ** 4


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_0903_3053_amd import su2
    su2.load()
    yield su2
    su2.su2_finalize()


@pytest.fixture(scope="module")
def par():
    return parity_of(DIMS)


def _report(tag, st, extra=""):
    print(f"{tag}: {st['n']} updates, {st['flips']} flipped decisions, {st['over']} links over "
          f"{LINK_TOL:g} (all within their bar: {st['unexplained'] == 0}), max err of the rest "
          f"{st['max_err_rest']:.2e}, max err / bar {st['max_ratio']:.3f}{extra}")
    order = np.argsort(-st["over_err"])[:12]
    for i in order:
        x0 = st["over_x0"][i] if st["over_x0"] is not None else float("nan")
        print(f"    err {st['over_err'][i]:.2e}  k {st['over_k'][i]:.4f}  x0 {x0:+.6f}  "
              f"err/bar {st['over_ratio'][i]:.3f}")
    if st["over"]:
        print(f"    over-1e-5 links: k in [{st['over_k'].min():.3g}, {st['over_k'].max():.3g}]")


def _inherited(err, par, over_lex, over_mu):
    """Largest error among the input links of each listed update that an
    earlier pass of the same sweep wrote (0 where none did)."""
    d_in = np.zeros(len(over_lex))
    for mu in range(4):
        sel = np.flatnonzero(over_mu == mu)
        if not len(sel):
            continue
        lexs = over_lex[sel]
        s, d = staple_inputs(DIMS, lexs, mu)
        earlier = (1 - par[s]) * 4 + d < np.array([pass_index(p, mu) for p in par[lexs]])[:, None]
        d_in[sel] = np.max(np.where(earlier, err[s, d], 0.0), axis=1)
    return d_in


def test_pass_level_64x64x64x64(lib, par):
    """Each of the eight passes of sweep 0, started from the oracle's state
    after the previous pass (so nothing carries over between passes)."""
    U = oracle.init(DIMS, SEED, oracle.HOT)
    lib.su2_init(DIMS, BETA, SEED, lib.HOT)
    lib.su2_set_plan(*PLAN)
    tot = dict(n=0, flips=0, over=0, rest=0.0, ratio=0.0)
    for p in (1, 0):
        sel = par == p
        for mu in range(4):
            prev = U.astype(np.float32)
            lib.su2_set_links(prev, 0)
            c0 = lib.su2_counters()
            lib.su2_pass(p, mu)
            c1 = lib.su2_counters()
            gpu = lib.su2_links()
            res = oracle.heatbath_pass(DIMS, U, BETA, SEED, 0, p, mu, diag=True)
            st = compare_links_conditioned(gpu[sel, mu], U[sel, mu], res.margin[sel], res.knorm[sel],
                                           res.x0[sel])
            _report(f"64^4 pass (parity {p}, mu {mu})", st)
            assert st["unexplained"] == 0
            assert st["flips"] <= 1e-5 * st["n"]
            # links outside the pass are untouched, bit for bit
            for nu in range(4):
                if nu != mu:
                    assert np.array_equal(gpu[:, nu], prev[:, nu])
            assert np.array_equal(gpu[~sel, mu], prev[~sel, mu])
            assert unitarity_error(gpu[sel, mu]) <= UNIT_TOL
            if st["flips"] == 0:
                assert (c1[0] - c0[0], c1[1] - c0[1]) == (res.attempts, res.failures)
            tot["n"] += st["n"]
            tot["flips"] += st["flips"]
            tot["over"] += st["over"]
            tot["rest"] = max(tot["rest"], st["max_err_rest"])
            tot["ratio"] = max(tot["ratio"], st["max_ratio"])
    print(f"64^4 pass level, one sweep: {tot['n']} updates, {tot['flips']} flips, {tot['over']} links "
          f"over 1e-5 (each within its conditioning bar), max err of the rest {tot['rest']:.2e}, "
          f"max err / bar {tot['ratio']:.3f}")
    assert tot["over"] <= 1e-5 * tot["n"]


def test_free_running_sweep_64x64x64x64(lib, par):
    """One measured sweep of the benchmark workload against the oracle's sweep
    of the whole lattice: the hot start to 1e-6, every link to its bar (with
    the errors it inherits from earlier passes of the sweep), the fused
    plaquette to 2e-6, and equal attempt counts where no decision moved."""
    U = oracle.init(DIMS, SEED, oracle.HOT)
    lib.su2_init(DIMS, BETA, SEED, lib.HOT)
    lib.su2_set_plan(*PLAN)
    assert np.max(np.abs(lib.su2_links() - U)) <= 1e-6
    hist = lib.su2_sweep_measure(1, 1)
    gpu = lib.su2_links()
    att_g, fail_g = lib.su2_counters()[:2]
    knorm = np.full((V, 4), np.nan)
    x0 = np.full((V, 4), np.nan)
    margin = np.full((V, 4), np.inf)
    att_o = fail_o = 0
    for p in (1, 0):
        sel = par == p
        for mu in range(4):
            res = oracle.heatbath_pass(DIMS, U, BETA, SEED, 0, p, mu, diag=True)
            knorm[sel, mu] = res.knorm[sel]
            x0[sel, mu] = res.x0[sel]
            margin[sel, mu] = res.margin[sel]
            att_o += res.attempts
            fail_o += res.failures
    err = np.max(np.abs(gpu.astype(np.float64) - U), axis=2)
    over = np.argwhere(err > LINK_TOL)
    d_in = _inherited(err, par, over[:, 0], over[:, 1])
    st = compare_links_conditioned(gpu[over[:, 0], over[:, 1]], U[over[:, 0], over[:, 1]],
                                   margin[over[:, 0], over[:, 1]], knorm[over[:, 0], over[:, 1]],
                                   x0[over[:, 0], over[:, 1]], d_in)
    tol = link_tolerance(knorm[over[:, 0], over[:, 1]], x0[over[:, 0], over[:, 1]], d_in)
    rest = float(np.max(err[err <= LINK_TOL]))
    P = oracle.plaquette(DIMS, U)
    print(f"64^4 one free-running sweep: {4 * V} updates, {len(over)} links over 1e-5 "
          f"({st['flips']} at a flipped decision, {st['unexplained']} beyond their bar), max err of "
          f"the rest {rest:.2e}; inherited input error of those links up to "
          f"{d_in.max() if len(d_in) else 0.0:.2e}; P gpu {hist[0, 0]:.8f} oracle {P[0]:.8f}; attempts "
          f"gpu {att_g} oracle {att_o}, cap failures {fail_g} / {fail_o}")
    for i in np.argsort(-err[over[:, 0], over[:, 1]])[:12]:
        lx, m = over[i]
        print(f"    link ({lx}, {m}) parity {par[lx]}: err {err[lx, m]:.2e}  k {knorm[lx, m]:.4f}  "
              f"x0 {x0[lx, m]:+.6f}  inherited {d_in[i]:.2e}  err/bar {err[lx, m] / tol[i]:.3f}  "
              f"margin {margin[lx, m]:.1e}")
    assert st["unexplained"] == 0
    assert len(over) <= 1e-5 * 4 * V
    assert np.all(np.abs(hist[0, :3] - P) <= 2e-6)
    assert abs(att_g - att_o) <= 8 * len(over)
    assert unitarity_error(gpu) <= UNIT_TOL


def test_overrelaxation_sweep_64x64x64x64(lib, par):
    """One overrelaxation sweep (the benchmark plan's tile order) from the
    oracle's state after one heat-bath sweep, against the oracle's
    overrelaxation sweep: links to their bar (the move carries the staple
    direction twice), the total plaquette conserved."""
    U = oracle.init(DIMS, SEED, oracle.HOT)
    oracle.sweep(DIMS, U, BETA, SEED, 0)
    U1 = U.astype(np.float32)
    lib.su2_init(DIMS, BETA, SEED, lib.COLD)
    lib.su2_set_plan(*PLAN)
    lib.su2_set_links(U1, 1)
    P0 = lib.su2_plaquette_st()
    lib.su2_overrelax(1)
    gpu = lib.su2_links()
    P1 = lib.su2_plaquette_st()
    knorm = np.full((V, 4), np.nan)
    for p in (1, 0):
        sel = par == p
        for mu in range(4):
            kn = oracle.or_pass(DIMS, U, p, mu, diag=True)
            knorm[sel, mu] = kn[sel]
    err = np.max(np.abs(gpu.astype(np.float64) - U), axis=2)
    over = np.argwhere(err > LINK_TOL)
    d_in = _inherited(err, par, over[:, 0], over[:, 1])
    tol = link_tolerance(knorm[over[:, 0], over[:, 1]], None, d_in, kappa_x=KAPPA_OVERRELAX)
    bad = err[over[:, 0], over[:, 1]] > tol
    rest = float(np.max(err[err <= LINK_TOL]))
    print(f"64^4 overrelaxation sweep: {4 * V} updates, {len(over)} links over 1e-5 "
          f"({int(bad.sum())} beyond their bar), max err of the rest {rest:.2e}; "
          f"P before {P0[0]:.8f} after {P1[0]:.8f}")
    for i in np.argsort(-err[over[:, 0], over[:, 1]])[:8]:
        lx, m = over[i]
        print(f"    link ({lx}, {m}): err {err[lx, m]:.2e}  k {knorm[lx, m]:.4f}  inherited {d_in[i]:.2e}  "
              f"err/bar {err[lx, m] / tol[i]:.3f}")
    assert not np.any(bad)
    assert len(over) <= 1e-5 * 4 * V
    assert abs(P1[0] - P0[0]) <= 2e-6
    assert unitarity_error(gpu) <= UNIT_TOL


def test_polyakov_64x64x64x64(lib):
    """The Polyakov loop (64 ordered FP32 products per site, FP64 mean) on the
    hot start and after one sweep, against the oracle on the same links."""
    U = oracle.init(DIMS, SEED, oracle.HOT)
    lib.su2_init(DIMS, BETA, SEED, lib.HOT)
    lib.su2_set_plan(*PLAN)
    got0 = lib.su2_polyakov()
    ref0 = oracle.polyakov(DIMS, U)
    lib.su2_sweep(1)
    got1 = lib.su2_polyakov()
    ref1 = oracle.polyakov(DIMS, lib.su2_links().astype(np.float64))
    print(f"64^4 Polyakov loop: hot start gpu {got0:+.3e} oracle {ref0:+.3e}; after one sweep gpu "
          f"{got1:+.3e} oracle {ref1:+.3e}")
    assert abs(got0 - ref0) <= 1e-5 and abs(got1 - ref1) <= 1e-5
