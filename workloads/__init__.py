"""Seeded synthetic inputs for the state-vector path.

This module only draws random numbers and lays out gate lists and Pauli-sum
observables as plain data.  It contains none of the simulation arithmetic
(no gate application, no expectation values, no gradients): both the CPU
oracle and the GPU library receive these objects as inputs and implement the
method on their own.

Qubit j is bit j of an amplitude index (weight 2**j).  For a dense gate on
targets (t_0, ..., t_{k-1}) the first-listed target is the most significant
bit of the gate matrix's row/column index (numpy ``kron`` order).

Workload families (each seeded; the default seed of family c is 1000 + c):

* ``random_u2_cz``   - layers of Haar U(2) on every qubit followed by CZ on
  even pairs (0,1),(2,3),... on even layers and odd pairs on odd layers.
* ``random_u2_pairs`` - layers of Haar U(2) on every qubit, then a random
  perfect matching whose pairs each get CNOT, CZ or CRZ(theta), theta~U[0,2pi).
* ``random_dense_123`` - layers that partition the qubits at random into
  groups of 1, 2 or 3 and put a Haar U(2**size) on each group.
* ``hea``            - hardware-efficient ansatz: per layer RY(theta) then
  RZ(phi) on every qubit, then the CNOT ladder 0->1->...->n-1.
* ``tfim_chain``     - open-chain H = sum_i Z_i Z_{i+1} + h * sum_i X_i.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

TWO_PI = 2.0 * np.pi


@dataclass
class Op:
    """One gate.  ``kind`` is one of
    matrix, h, x, y, z, rx, ry, rz, swap.
    ``controls`` turns any kind into its controlled version (all control bits
    must be 1).  Rotations read their angle from ``params[param]``.
    ``matrix`` (complex128, 2**k x 2**k) is only set for kind == "matrix"."""
    kind: str
    targets: Tuple[int, ...]
    controls: Tuple[int, ...] = ()
    param: int = -1
    matrix: Optional[np.ndarray] = None


@dataclass
class Circuit:
    n: int
    ops: List[Op] = field(default_factory=list)
    nparams: int = 0


@dataclass
class PauliSum:
    """sum_j coeff[j] * P_j with P_j given by bit masks: qubit q carries
    X if only x_mask bit q is set, Z if only z_mask bit q is set, Y if both."""
    n: int
    x_mask: np.ndarray  # uint64
    z_mask: np.ndarray  # uint64
    coeff: np.ndarray   # float64


ROT_KINDS = ("rx", "ry", "rz")


def haar_unitary(rng: np.random.Generator, dim: int) -> np.ndarray:
    """Haar-random U(dim) by Mezzadri's recipe (Notices AMS 54, 2007):
    QR of a complex Ginibre matrix, columns re-phased by R's diagonal."""
    z = (rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    return (q * (d / np.abs(d))[None, :]).astype(np.complex128)


def random_u2_cz(n: int = 20, depth: int = 10, seed: int = 1000) -> Circuit:
    """Haar U(2) on every qubit, then CZ on (0,1),(2,3).. (even layers) or
    (1,2),(3,4).. (odd layers); layers are 0-based."""
    rng = np.random.default_rng(seed)
    c = Circuit(n)
    for layer in range(depth):
        for q in range(n):
            c.ops.append(Op("matrix", (q,), matrix=haar_unitary(rng, 2)))
        start = 0 if layer % 2 == 0 else 1
        for a in range(start, n - 1, 2):
            c.ops.append(Op("z", (a + 1,), controls=(a,)))
    return c


def random_u2_pairs(n: int = 28, depth: int = 20, seed: int = 1001):
    """Haar U(2) on every qubit, then a seeded random perfect matching; each
    pair independently gets CNOT, CZ or CRZ(theta ~ U[0, 2pi)) with equal
    probability; the first element of a shuffled pair is the control.
    Returns (circuit, params) where params holds the CRZ angles."""
    rng = np.random.default_rng(seed)
    c = Circuit(n)
    params: List[float] = []
    for _ in range(depth):
        for q in range(n):
            c.ops.append(Op("matrix", (q,), matrix=haar_unitary(rng, 2)))
        perm = rng.permutation(n)
        for p in range(0, n - 1, 2):
            a, b = int(perm[p]), int(perm[p + 1])
            choice = int(rng.integers(3))
            if choice == 0:
                c.ops.append(Op("x", (b,), controls=(a,)))
            elif choice == 1:
                c.ops.append(Op("z", (b,), controls=(a,)))
            else:
                params.append(float(rng.uniform(0.0, TWO_PI)))
                c.ops.append(Op("rz", (b,), controls=(a,), param=len(params) - 1))
    c.nparams = len(params)
    return c, np.asarray(params, dtype=np.float64)


def random_dense_123(n: int = 32, depth: int = 12, seed: int = 1002) -> Circuit:
    """Each layer: a random permutation of the qubits cut into consecutive
    groups of size drawn uniformly from {1,2,3} (the last group truncated);
    each group gets a Haar U(2**size) with its targets in the permuted order."""
    rng = np.random.default_rng(seed)
    c = Circuit(n)
    for _ in range(depth):
        perm = [int(v) for v in rng.permutation(n)]
        pos = 0
        while pos < n:
            size = int(rng.integers(1, 4))
            group = tuple(perm[pos:pos + size])
            pos += size
            c.ops.append(Op("matrix", group, matrix=haar_unitary(rng, 2 ** len(group))))
    return c


def hea(n: int, layers: int = 8) -> Circuit:
    """Hardware-efficient ansatz: per layer l and qubit q, RY(params[(l*n+q)*2])
    then RZ(params[(l*n+q)*2+1]); then CNOT(0->1), CNOT(1->2), ..., CNOT(n-2->n-1)."""
    c = Circuit(n)
    for l in range(layers):
        for q in range(n):
            base = (l * n + q) * 2
            c.ops.append(Op("ry", (q,), param=base))
            c.ops.append(Op("rz", (q,), param=base + 1))
        for q in range(n - 1):
            c.ops.append(Op("x", (q + 1,), controls=(q,)))
    c.nparams = 2 * n * layers
    return c


def random_params(count: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(0.0, TWO_PI, size=count)


def pauli_sum(n: int, terms: Sequence[Tuple[str, Sequence[int], float]]) -> PauliSum:
    """Build a PauliSum from (letters, qubits, coeff) triples, e.g.
    ("ZZ", (0, 1), 1.0).  An empty letter string is the identity."""
    xs, zs, cs = [], [], []
    for letters, qubits, coeff in terms:
        x = z = 0
        for ch, q in zip(letters, qubits):
            if ch in "XY":
                x |= 1 << q
            if ch in "ZY":
                z |= 1 << q
        xs.append(x)
        zs.append(z)
        cs.append(coeff)
    return PauliSum(n, np.asarray(xs, dtype=np.uint64), np.asarray(zs, dtype=np.uint64),
                    np.asarray(cs, dtype=np.float64))


def tfim_chain(n: int, h: float = 1.0) -> PauliSum:
    terms = [("ZZ", (i, i + 1), 1.0) for i in range(n - 1)]
    terms += [("X", (i,), h) for i in range(n)]
    return pauli_sum(n, terms)


def xxz_chain(n: int, delta: float) -> PauliSum:
    terms = []
    for i in range(n - 1):
        terms += [("XX", (i, i + 1), 1.0), ("YY", (i, i + 1), 1.0), ("ZZ", (i, i + 1), delta)]
    return pauli_sum(n, terms)


def maxcut(n: int, edges: Sequence[Tuple[int, int]]) -> PauliSum:
    """sum over edges of (1 - Z_i Z_j)/2: identity terms plus ZZ terms."""
    terms = []
    for i, j in edges:
        terms += [("", (), 0.5), ("ZZ", (i, j), -0.5)]
    return pauli_sum(n, terms)


def random_pauli_sum(n: int, nterms: int, seed: int) -> PauliSum:
    rng = np.random.default_rng(seed)
    terms = []
    for _ in range(nterms):
        letters = rng.choice(list("IXYZ"), size=n)
        qs = [q for q in range(n) if letters[q] != "I"]
        terms.append(("".join(letters[q] for q in qs), qs, float(rng.normal())))
    return pauli_sum(n, terms)


@dataclass
class BatchInstance:
    circuit: Circuit
    params: np.ndarray
    hamiltonian: PauliSum


def batched_hea(count: int = 1024, nmin: int = 12, nmax: int = 22, lmin: int = 2,
                lmax: int = 10, seed: int = 1004) -> List[BatchInstance]:
    """Uneven batch: n ~ U{nmin..nmax}, L ~ U{lmin..lmax}, params ~ U[0, 2pi),
    observable = open-chain TFIM with h = 1."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        layers = int(rng.integers(lmin, lmax + 1))
        circ = hea(n, layers)
        params = rng.uniform(0.0, TWO_PI, size=circ.nparams)
        out.append(BatchInstance(circ, params, tfim_chain(n)))
    return out


def random_gate(rng: np.random.Generator, n: int, k: int, c: int = 0):
    """A random placement of k targets and c controls with a Haar U(2**k)."""
    qs = [int(v) for v in rng.choice(n, size=k + c, replace=False)]
    return tuple(qs[:k]), tuple(qs[k:]), haar_unitary(rng, 2 ** k)


def random_state_seed_list(count: int, seed: int) -> List[int]:
    rng = np.random.default_rng(seed)
    return [int(v) for v in rng.integers(1, 2 ** 62, size=count)]


def uniforms(count: int, seed: int) -> np.ndarray:
    """Seeded uniforms in [0, 1) (float64) that drive measurement sampling."""
    return np.random.default_rng(seed).random(count)


def qft(n: int, swaps: bool = True) -> Circuit:
    """Quantum Fourier transform (the QFT circuit of the paper's built-in
    models, Sec. 3) as a gate list: taking bit n-1 as the most significant,
    for each bit b from n-1 down to 0 a Hadamard on b, then for each lower bit
    c < b a phase diag(1, exp(2 pi i / 2^(b-c+1))) on b controlled by c; then
    swaps (b, n-1-b) that reverse the bit order.  The map is
    |x> -> 2^(-n/2) sum_y exp(+2 pi i x y / 2^n) |y>."""
    c = Circuit(n)
    for b in range(n - 1, -1, -1):
        c.ops.append(Op("h", (b,)))
        for ctl in range(b - 1, -1, -1):
            phi = TWO_PI / float(1 << (b - ctl + 1))
            c.ops.append(Op("matrix", (b,), controls=(ctl,),
                            matrix=np.diag([1.0, np.exp(1j * phi)]).astype(np.complex128)))
    if swaps:
        for b in range(n // 2):
            c.ops.append(Op("swap", (b, n - 1 - b)))
    return c
