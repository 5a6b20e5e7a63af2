"""Pins of the oracle's Trotterised time evolution (Sec. 3: Hamiltonians
evolved with the Trotter decomposition) against the exact propagator
exp(-i t H) of the dense Hamiltonian (scipy's matrix exponential of the
Kronecker-product construction in oracle/brute.py): exact for commuting
terms, first-order error falling as 1/steps and second-order as 1/steps^2
for non-commuting ones, and unitarity."""
import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle import brute


def rand_state(n, seed):
    r = np.random.default_rng(seed)
    v = r.standard_normal(1 << n) + 1j * r.standard_normal(1 << n)
    return v / np.linalg.norm(v)


def exact(psi, H, t):
    return scipy.linalg.expm(-1j * t * brute.hamiltonian_dense(H)) @ psi


@pytest.mark.parametrize("order", [1, 2])
def test_commuting_terms_are_exact(orc, order):
    n = 6
    H = W.maxcut(n, [(0, 1), (1, 2), (2, 5), (3, 4), (0, 5)])
    Hz = W.pauli_sum(n, [("Z", [1], 0.7), ("ZZ", [2, 4], -1.3), ("", [], 0.25)])
    psi = rand_state(n, 1)
    for h in (H, Hz):
        got = orc.trotter(psi, h, 0.37, 3, order)
        assert np.max(np.abs(got - exact(psi, h, 3 * 0.37))) <= 1e-12


@pytest.mark.parametrize("order,ratio", [(1, 2.0), (2, 4.0)])
def test_error_order(orc, order, ratio):
    n, t = 5, 0.8
    for H in (W.tfim_chain(n, 0.9), W.xxz_chain(n, 0.5)):
        psi = rand_state(n, 2)
        ref = exact(psi, H, t)
        e = [np.linalg.norm(orc.trotter(psi, H, t / s, s, order) - ref) for s in (16, 32, 64)]
        assert e[0] > 1e-6
        for a, b in zip(e, e[1:]):
            assert 0.8 * ratio <= a / b <= 1.2 * ratio, e


def test_single_term_and_unitarity(orc):
    n = 4
    H = W.pauli_sum(n, [("XYZ", [0, 2, 3], 0.9)])
    psi = rand_state(n, 3)
    got = orc.trotter(psi, H, 0.3, 1, 1)
    assert np.max(np.abs(got - exact(psi, H, 0.3))) <= 1e-13
    H = W.tfim_chain(n, 1.1)
    out = orc.trotter(psi, H, 0.05, 10, 2)
    assert abs(np.linalg.norm(out) - 1) <= 1e-13
    back = orc.trotter(out, H, -0.05, 10, 2)       # symmetric steps: U(-tau) = U(tau)^dagger
    assert np.max(np.abs(back - psi)) <= 1e-13
