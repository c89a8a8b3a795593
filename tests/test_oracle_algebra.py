"""Pins the oracle's quaternion algebra, staple, plaquette and Polyakov loop
against independent 2x2 complex-matrix arithmetic (tests/su2_np.py) and exact
identities (Eqs. (2)-(4), (6))."""
import numpy as np
import pytest

import oracle
import su2_inputs
import su2_np

DIMS_ASYM = (4, 2, 6, 4)


def test_qmul_matches_matrix_product():
    rng = np.random.default_rng(1)
    for _ in range(50):
        a, b = rng.standard_normal(4), rng.standard_normal(4)
        c = oracle.qmul(a, b)
        m = su2_np.to_matrix(a) @ su2_np.to_matrix(b)
        np.testing.assert_allclose(su2_np.to_matrix(c), m, atol=1e-14)


def test_half_trace_is_dot_product():
    rng = np.random.default_rng(2)
    for _ in range(20):
        a, b = rng.standard_normal(4), rng.standard_normal(4)
        bd = np.array([b[0], -b[1], -b[2], -b[3]])
        ab = oracle.qmul(a, bd)
        m = su2_np.to_matrix(a) @ su2_np.dag(su2_np.to_matrix(b))
        assert abs(ab[0] - np.dot(a, b)) < 1e-14
        assert abs(0.5 * np.trace(m).real - np.dot(a, b)) < 1e-14


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), DIMS_ASYM, (2, 2, 2, 2)])
def test_plaquette_matches_matrices(dims):
    U = su2_inputs.random_links(dims, 3).astype(np.float64)
    got = oracle.plaquette(dims, U)
    ref = su2_np.plaquette(U, dims)
    np.testing.assert_allclose(got, ref, atol=1e-13)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), DIMS_ASYM])
def test_staple_matches_matrices(dims):
    U = su2_inputs.random_links(dims, 4).astype(np.float64)
    ref = su2_np.staples(U, dims)
    V = su2_inputs.volume(dims)
    for lex in range(0, V, 7):
        for mu in range(4):
            np.testing.assert_allclose(oracle.staple(dims, U, lex, mu), ref[lex, mu], atol=1e-13)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), DIMS_ASYM])
def test_staple_gives_local_action(dims):
    """Changing one link U -> U' changes S_W by -beta (dot(U', W) - dot(U, W)):
    W is exactly the local part of the Wilson action, Eq. (2)."""
    beta = 1.7
    U = su2_inputs.random_links(dims, 5).astype(np.float64)
    rng = np.random.default_rng(6)
    S0 = su2_np.wilson_action(U, dims, beta)
    V = su2_inputs.volume(dims)
    for lex in rng.choice(V, size=6, replace=False):
        for mu in range(4):
            w = oracle.staple(dims, U, lex, mu)
            new = rng.standard_normal(4)
            new /= np.linalg.norm(new)
            U2 = U.copy()
            U2[lex, mu] = new
            dS = su2_np.wilson_action(U2, dims, beta) - S0
            pred = -beta * (np.dot(new, w) - np.dot(U[lex, mu], w))
            assert abs(dS - pred) < 1e-10, (lex, mu)


def test_staple_sum_identity():
    """sum over links of dot(U, W) = 24 V P on any configuration."""
    dims = DIMS_ASYM
    U = su2_inputs.random_links(dims, 7).astype(np.float64)
    V = su2_inputs.volume(dims)
    lhs = oracle.staple_action(dims, U)
    P = oracle.plaquette(dims, U)[0]
    assert abs(lhs - 24 * V * P) < 1e-10 * V


def test_polyakov_matches_matrices():
    for dims in [(4, 4, 4, 4), (2, 4, 2, 6)]:
        U = su2_inputs.random_links(dims, 8).astype(np.float64)
        assert abs(oracle.polyakov(dims, U) - su2_np.polyakov(U, dims)) < 1e-13


def test_gauge_invariance():
    dims = (4, 4, 2, 4)
    U = su2_inputs.random_links(dims, 9, dtype=np.float64)
    G = su2_inputs.random_links(dims, 10, dtype=np.float64)[:, 0]
    Ug = su2_np.gauge_transform(U, dims, G)
    np.testing.assert_allclose(oracle.plaquette(dims, Ug), oracle.plaquette(dims, U), atol=1e-13)
    assert abs(oracle.polyakov(dims, Ug) - oracle.polyakov(dims, U)) < 1e-13


def test_cold_start_special_case():
    dims = (4, 4, 4, 4)
    U = oracle.init(dims, 1, oracle.COLD)
    np.testing.assert_array_equal(oracle.plaquette(dims, U), [1.0, 1.0, 1.0])
    assert oracle.polyakov(dims, U) == 1.0
    w = oracle.staple(dims, U, 5, 2)
    np.testing.assert_array_equal(w, [6.0, 0.0, 0.0, 0.0])


def test_invalid_dims_rejected():
    with pytest.raises(ValueError):
        oracle.init((3, 4, 4, 4), 1, 0)
    with pytest.raises(ValueError):
        oracle.init((4, 4, 0, 4), 1, 0)
