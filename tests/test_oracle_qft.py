"""Pins of the QFT workload (the quantum Fourier transform circuit among the
paper's built-in models, Sec. 3) run through the oracle: the circuit must equal
the unitary discrete Fourier transform |x> -> 2^(-n/2) sum_y exp(2 pi i x y /
2^n) |y>, which numpy's inverse FFT with orthonormal scaling computes; basis
inputs have closed-form outputs; without the final swaps the output comes in
bit-reversed order."""
import numpy as np
import pytest

import workloads as W


def rand_state(n, seed):
    r = np.random.default_rng(seed)
    v = r.standard_normal(1 << n) + 1j * r.standard_normal(1 << n)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 10])
def test_qft_is_unitary_dft(orc, n):
    psi = rand_state(n, 60 + n)
    got = orc.run(W.qft(n), psi0=psi)
    assert np.max(np.abs(got - np.fft.ifft(psi, norm="ortho"))) <= 1e-13


def test_qft_basis_closed_form(orc):
    n = 6
    N = 1 << n
    for x in (0, 1, 5, 32, 63):
        psi = np.zeros(N, dtype=np.complex128)
        psi[x] = 1.0
        got = orc.run(W.qft(n), psi0=psi)
        y = np.arange(N)
        want = np.exp(2j * np.pi * ((x * y) % N) / N) / np.sqrt(N)
        assert np.max(np.abs(got - want)) <= 1e-14


def test_qft_without_swaps_is_bit_reversed(orc):
    n = 7
    psi = rand_state(n, 5)
    got = orc.run(W.qft(n, swaps=False), psi0=psi)
    rev = np.array([int("{:07b}".format(i)[::-1], 2) for i in range(1 << n)])
    assert np.max(np.abs(got[rev] - np.fft.ifft(psi, norm="ortho"))) <= 1e-13
