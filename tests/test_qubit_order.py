"""Qubit order in the Python layer.  The C ABI numbers qubit j as index bit j
(little-endian); order="big" takes qubit 0 as the most significant bit (the
convention of Qibo's own software) by passing qubit q on as n - 1 - q and
bit-reversing masks and basis indices.  CPU tests pin the marshalling and,
with the oracle, that the mapped circuit is the big-endian Kronecker-product
operator; the GPU test runs the library with order="big" against it."""
import numpy as np
import pytest

import workloads as W
from paper_2202_07017_amd import qsv


def big_endian_operator(n, targets, controls, G):
    """Dense operator of G on `targets` (first listed = most significant bit of
    G's index) controlled on `controls`, qubit 0 = leftmost Kronecker factor."""
    dim = 1 << n
    U = np.zeros((dim, dim), dtype=complex)
    k = len(targets)
    for col in range(dim):
        bits = [(col >> (n - 1 - q)) & 1 for q in range(n)]
        if not all(bits[c] for c in controls):
            U[col, col] = 1.0
            continue
        tau_in = sum(bits[t] << (k - 1 - j) for j, t in enumerate(targets))
        for tau_out in range(1 << k):
            b = list(bits)
            for j, t in enumerate(targets):
                b[t] = (tau_out >> (k - 1 - j)) & 1
            row = sum(b[q] << (n - 1 - q) for q in range(n))
            U[row, col] += G[tau_out, tau_in]
    return U


def test_marshalling():
    assert qsv.map_qubits([0, 3], 5, "big") == [4, 1]
    assert qsv.map_qubits([0, 3], 5) == [0, 3]
    assert qsv.reverse_bits(0b00011, 5) == 0b11000
    with pytest.raises(ValueError):
        qsv.map_qubits([0], 3, "middle")
    circ = W.Circuit(5, [W.Op("x", (1,), controls=(0, 4)), W.Op("ry", (2,), param=0)], 1)
    c = qsv.CircuitC(circ, "big")
    assert list(c.ops[0].targets[:1]) == [3] and list(c.ops[0].controls[:2]) == [4, 0]
    assert list(c.ops[1].targets[:1]) == [2]
    H = W.pauli_sum(5, [("XZ", (0, 3), 0.5)])
    P = qsv.PauliSum(H, "big")
    assert int(P.x[0]) == 1 << 4 and int(P.z[0]) == 1 << 1


def test_mapped_circuit_is_big_endian_operator(orc):
    """The oracle applying the mapped circuit (little-endian indexing) equals
    the big-endian Kronecker-product operators applied in order."""
    n = 5
    rng = np.random.default_rng(21)
    ops = [((0,), (), W.haar_unitary(rng, 2)), ((1, 3), (), W.haar_unitary(rng, 4)),
           ((4,), (0,), W.haar_unitary(rng, 2)), ((2, 0, 4), (), W.haar_unitary(rng, 8)),
           ((3,), (1, 2), W.haar_unitary(rng, 2))]
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi /= np.linalg.norm(psi)
    ref = psi.copy()
    for t, c, G in ops:
        ref = big_endian_operator(n, t, c, G) @ ref
    mapped = W.Circuit(n, [W.Op("matrix", tuple(qsv.map_qubits(t, n, "big")),
                                controls=tuple(qsv.map_qubits(c, n, "big")), matrix=G)
                           for t, c, G in ops])
    assert np.max(np.abs(orc.run(mapped, psi0=psi) - ref)) < 1e-13


@pytest.mark.gpu
def test_big_order_on_gpu(orc):
    import torch
    qsv.lib()
    n = 6
    d = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    qsv.qsv_init_basis(d, 0, order="big")
    qsv.qsv_apply_gate(d, (0,), (), np.array([[0, 1], [1, 0]], dtype=complex), order="big")
    got = d.cpu().numpy()
    assert got[1 << (n - 1)] == 1.0 and np.count_nonzero(got) == 1
    qsv.qsv_init_basis(d, 0b000011, order="big")  # qubits 4 and 5 set: little index 0b110000
    assert d.cpu().numpy()[0b110000] == 1.0
    rng = np.random.default_rng(22)
    ops = [W.Op("matrix", (0,), matrix=W.haar_unitary(rng, 2)),
           W.Op("matrix", (1, 4), matrix=W.haar_unitary(rng, 4)),
           W.Op("matrix", (5,), controls=(0, 2), matrix=W.haar_unitary(rng, 2)),
           W.Op("matrix", (3, 2, 0), matrix=W.haar_unitary(rng, 8))]
    ref = np.zeros(1 << n, dtype=complex)
    ref[0] = 1.0
    for op in ops:
        ref = big_endian_operator(n, op.targets, op.controls, op.matrix) @ ref
    plan = qsv.Plan(W.Circuit(n, ops), 2, 5, order="big")
    qsv.qsv_init_basis(d, 0)
    plan.run(d)
    torch.cuda.synchronize()
    assert np.max(np.abs(d.cpu().numpy() - ref)) < 1e-12
