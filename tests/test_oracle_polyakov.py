"""Pins of the oracle's Polyakov-loop field and correlator (observables of
the paper's finite-temperature L_t x L_s^3 lattices, Sec. 2.4, Table 1): the
field against the same ordered product taken with 2x2 complex matrices, its
mean against the oracle's Polyakov average, invariance under a random gauge
transformation (only a correctly ordered, closed product is invariant), and
the cold lattice (every loop 1)."""
import numpy as np

import oracle
import su2_np


def hot(dims, seed, sweeps=2):
    U = oracle.init(dims, seed, oracle.HOT, prec32=False)
    for s in range(sweeps):
        oracle.sweep(dims, U, 2.3, seed, s, prec32=False)
    return U


def matrix_field(U, dims):
    F = su2_np.field(U, dims)[3]
    P = np.broadcast_to(su2_np.ID2, F.shape[1:]).copy()
    for t in range(dims[3]):
        P = P @ F[t]
    return 0.5 * np.real(np.trace(P, axis1=-2, axis2=-1)).ravel()


def test_field_matches_matrices_and_mean():
    dims = (4, 6, 2, 8)
    U = hot(dims, 5)
    f = oracle.polyakov_field(dims, U)
    np.testing.assert_allclose(f, matrix_field(U, dims), rtol=0, atol=1e-13)
    assert abs(f.mean() - oracle.polyakov(dims, U)) <= 1e-15


def test_field_gauge_invariant():
    dims = (4, 4, 6, 4)
    U = hot(dims, 7)
    rng = np.random.default_rng(1)
    G = rng.standard_normal((int(np.prod(dims)), 4))
    G /= np.linalg.norm(G, axis=1, keepdims=True)
    Ug = np.ascontiguousarray(su2_np.gauge_transform(U, dims, G))
    np.testing.assert_allclose(oracle.polyakov_field(dims, Ug), oracle.polyakov_field(dims, U), rtol=0, atol=1e-12)
    np.testing.assert_allclose(oracle.polyakov_correlator(dims, Ug, 2), oracle.polyakov_correlator(dims, U, 2),
                               rtol=0, atol=1e-12)


def test_cold_lattice_correlator_is_one():
    dims = (4, 4, 4, 6)
    U = oracle.init(dims, 1, oracle.COLD, prec32=False)
    np.testing.assert_array_equal(oracle.polyakov_correlator(dims, U, 2), np.ones(3))


def test_correlator_zero_distance_is_mean_square():
    dims = (6, 4, 4, 4)
    U = hot(dims, 9)
    f = oracle.polyakov_field(dims, U)
    assert abs(oracle.polyakov_correlator(dims, U, 0)[0] - np.mean(f * f)) <= 1e-15
