"""Pins of the oracle's overrelaxation step U -> V U^dag V, V = w/|w| (the
standard SU(2) reflection; the paper names overrelaxation in Sec. 2.4 without
a formula), against what the mathematics fixes: the same move computed with
2x2 complex matrices, conservation of each link's local action dot(U, w) and
of the plaquette (no plaquette holds two links of one pass), and the move
undoing itself.  All in FP64 (prec32 off) on small hot lattices."""
import numpy as np
import pytest

import oracle

SIGMA = [np.array([[0, 1], [1, 0]], dtype=complex), np.array([[0, -1j], [1j, 0]], dtype=complex),
         np.array([[1, 0], [0, -1]], dtype=complex)]


def to_matrix(q):
    """U = u0 I + i sigma.u (Eq. (4))."""
    return q[0] * np.eye(2) + 1j * sum(q[k + 1] * SIGMA[k] for k in range(3))


def from_matrix(M):
    return np.array([np.trace(M).real / 2] + [np.trace(SIGMA[k] @ M).imag / 2 for k in range(3)])


def hot(dims, seed, sweeps=2, beta=2.3):
    U = oracle.init(dims, seed, oracle.HOT, prec32=False)
    for s in range(sweeps):
        oracle.sweep(dims, U, beta, seed, s, prec32=False)
    return U


def parity_sites(dims, p):
    L0, L1, L2, L3 = dims
    out = []
    for lex in range(L0 * L1 * L2 * L3):
        x0 = lex % L0
        x1 = (lex // L0) % L1
        x2 = (lex // (L0 * L1)) % L2
        x3 = lex // (L0 * L1 * L2)
        if (x0 + x1 + x2 + x3) % 2 == p:
            out.append(lex)
    return out


@pytest.mark.parametrize("dims,p,mu", [((4, 4, 4, 4), 1, 2), ((2, 4, 2, 6), 0, 0), ((6, 4, 4, 2), 1, 3)])
def test_or_pass_matches_matrix_reflection_and_keeps_local_action(dims, p, mu):
    U0 = hot(dims, 7)
    U1 = U0.copy()
    oracle.or_pass(dims, U1, p, mu, prec32=False)
    for lex in parity_sites(dims, p):
        # the staple of a link does not involve links of its own pass
        w = oracle.staple(dims, U0, lex, mu)
        k = np.linalg.norm(w)
        Vm = to_matrix(w / k)
        want = from_matrix(Vm @ to_matrix(U0[lex, mu]).conj().T @ Vm)
        np.testing.assert_allclose(U1[lex, mu], want, rtol=0, atol=1e-13)
        assert abs(np.dot(U1[lex, mu], w) - np.dot(U0[lex, mu], w)) <= 1e-12
    # links of the other parity and other directions untouched
    others = np.ones(U0.shape[:2], dtype=bool)
    others[parity_sites(dims, p), mu] = False
    assert np.array_equal(U1[others], U0[others])


def test_or_pass_undoes_itself():
    dims = (4, 6, 2, 4)
    U0 = hot(dims, 3)
    U = U0.copy()
    for p in (1, 0):
        for mu in range(4):
            oracle.or_pass(dims, U, p, mu, prec32=False)
            oracle.or_pass(dims, U, p, mu, prec32=False)
    np.testing.assert_allclose(U, U0, rtol=0, atol=1e-13)


def test_or_sweep_conserves_plaquette():
    dims = (6, 4, 4, 6)
    U = hot(dims, 11, sweeps=3)
    P0 = oracle.plaquette(dims, U)
    oracle.or_sweep(dims, U, prec32=False)
    P1 = oracle.plaquette(dims, U)
    np.testing.assert_allclose(P1[0], P0[0], rtol=0, atol=1e-13)
    # the configuration did move
    U2 = hot(dims, 11, sweeps=3)
    assert np.max(np.abs(U - U2)) > 0.1


def test_or_cold_start_is_fixed_point():
    """Every staple of the cold lattice is 6 (1, 0, 0, 0): V = 1 and V U^dag V = 1."""
    dims = (4, 4, 4, 4)
    U = oracle.init(dims, 1, oracle.COLD, prec32=False)
    oracle.or_sweep(dims, U, prec32=False)
    assert np.array_equal(U, oracle.init(dims, 1, oracle.COLD, prec32=False))
