"""Brute-force dense constructions used to pin the C oracle -- TEST INFRASTRUCTURE ONLY.

Everything here builds full 2**n x 2**n matrices with ``numpy.kron`` (n <= 10)
and shares nothing with ``oracle.c``: a gate becomes U = P^T (Gc (x) I) P with
Gc = blockdiag(I, ..., I, G) for the controls, the gate's qubits moved to the
most significant Kronecker slots by an explicit permutation matrix P; an
observable becomes the dense sum of Kronecker products of 2x2 Pauli matrices.
"""
from __future__ import annotations

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def slot_permutation(n, order):
    """Permutation matrix P with (P psi)[kron index] = psi[computational index],
    where Kronecker slot s (s = 0 most significant) holds qubit order[s] and
    the computational index has qubit j at bit j."""
    N = 1 << n
    P = np.zeros((N, N))
    for comp in range(N):
        kron = 0
        for s, q in enumerate(order):
            kron |= ((comp >> q) & 1) << (n - 1 - s)
        P[kron, comp] = 1.0
    return P


def controlled(G, c):
    """blockdiag(I, ..., I, G): G acts only when all c leading qubits are 1."""
    d = G.shape[0]
    M = np.eye(d << c, dtype=np.complex128)
    M[-d:, -d:] = G
    return M


def gate_unitary(n, targets, controls, G):
    targets, controls = list(targets), list(controls)
    rest = [q for q in range(n) if q not in targets and q not in controls]
    order = controls + targets + rest
    M = np.kron(controlled(np.asarray(G, np.complex128), len(controls)),
                np.eye(1 << len(rest), dtype=np.complex128))
    P = slot_permutation(n, order)
    return P.T @ M @ P


def pauli_dense(n, x, z):
    """Dense matrix of the Pauli string with masks (x, z); qubit n-1 is the
    leftmost Kronecker factor so that qubit j is bit j."""
    M = np.ones((1, 1), dtype=np.complex128)
    for q in reversed(range(n)):
        xb, zb = (x >> q) & 1, (z >> q) & 1
        s = Y if (xb and zb) else (X if xb else (Z if zb else I2))
        M = np.kron(M, s)
    return M


def hamiltonian_dense(H):
    N = 1 << H.n
    M = np.zeros((N, N), dtype=np.complex128)
    for x, z, c in zip(H.x_mask, H.z_mask, H.coeff):
        M += c * pauli_dense(H.n, int(x), int(z))
    return M
