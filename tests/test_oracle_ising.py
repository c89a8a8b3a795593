"""Pins of the 2-D Ising oracle (Metropolis, red-black partition, Sec. 2.3,
Eq. (1)) against what the mathematics fixes: the exact Boltzmann averages of
the 4x4 lattice by enumeration of its 2^16 states, Onsager's infinite-lattice
energy above the critical point and Yang's spontaneous magnetisation below
it (a 32x32 lattice far from criticality differs from them by much less than
the statistical error), and the integer observables of simple states."""
import itertools

import numpy as np
import pytest
from scipy import special

import oracle.ising as ising
from paper_0903_3053_amd.stats import gamma_method

BETA_C = 0.5 * np.log(1.0 + np.sqrt(2.0))


def exact_4x4(beta):
    """<E>/N and <|m|> of the periodic 4x4 lattice by enumeration."""
    L = 4
    states = np.array(list(itertools.product([-1, 1], repeat=L * L)), dtype=np.int8).reshape(-1, L, L)
    bonds = (states * np.roll(states, 1, axis=1)).sum(axis=(1, 2)) + (states * np.roll(states, 1, axis=2)).sum(axis=(1, 2))
    H = -bonds.astype(np.float64)
    m = np.abs(states.sum(axis=(1, 2))) / (L * L)
    w = np.exp(-beta * (H - H.min()))
    return float((w * H).sum() / w.sum() / (L * L)), float((w * m).sum() / w.sum())


def onsager_energy(beta):
    k = 2.0 * np.sinh(2 * beta) / np.cosh(2 * beta) ** 2
    return float(-1.0 / np.tanh(2 * beta) * (1 + 2 / np.pi * (2 * np.tanh(2 * beta) ** 2 - 1) * special.ellipk(k * k)))


def chain(dims, beta, seed, start, therm, n):
    s = ising.init(dims, seed, start)
    ising.sweep(dims, s, beta, seed, 0, therm)
    E, M = np.empty(n), np.empty(n)
    for i in range(n):
        ising.sweep(dims, s, beta, seed, therm + i, 1)
        E[i], M[i] = ising.observables(dims, s)
    return E, np.abs(M)


def test_observables_of_simple_states():
    dims = (6, 4)
    s = np.ones(24, dtype=np.int8)
    assert ising.observables(dims, s) == (-2.0, 1.0)
    x, y = np.meshgrid(np.arange(6), np.arange(4))
    s = np.where((x + y) % 2 == 0, 1, -1).astype(np.int8).ravel()  # Neel state: every bond unsatisfied
    assert ising.observables(dims, s) == (2.0, 0.0)
    assert np.all(ising.init(dims, 1, 0) == 1)


@pytest.mark.parametrize("beta", [0.2, 0.44, 0.7])
def test_4x4_against_enumeration(beta):
    e_ex, m_ex = exact_4x4(beta)
    E, M = chain((4, 4), beta, 3, 1, 500, 30000)
    me, se, te, _, _ = gamma_method(E)
    mm, sm, tm, _, _ = gamma_method(M)
    print(f"4x4 beta {beta}: E {me:.5f}+-{se:.5f} exact {e_ex:.5f}; |m| {mm:.5f}+-{sm:.5f} exact {m_ex:.5f}")
    assert abs(me - e_ex) < 4 * se
    assert abs(mm - m_ex) < 4 * sm


def test_onsager_energy_above_critical_point():
    beta = 0.3
    E, _ = chain((32, 32), beta, 5, 1, 200, 3000)
    m, s, t, _, _ = gamma_method(E)
    ex = onsager_energy(beta)
    print(f"32x32 beta {beta}: E {m:.5f}+-{s:.5f}, Onsager {ex:.5f}")
    assert abs(m - ex) < 4 * s


def test_spontaneous_magnetisation_below_critical_point():
    beta = 0.6
    _, M = chain((32, 32), beta, 6, 0, 200, 3000)
    m, s, t, _, _ = gamma_method(M)
    ex = (1.0 - np.sinh(2 * beta) ** -4) ** 0.125
    print(f"32x32 beta {beta}: |m| {m:.5f}+-{s:.5f}, Yang {ex:.5f}")
    assert beta > BETA_C
    assert abs(m - ex) < 4 * s + 1e-3
