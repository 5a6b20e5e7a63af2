"""CPU oracle for the state-vector path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports, links
or calls it.  ``oracle.c`` holds the arithmetic (complex128, out of place,
the plain definition of eq. (1) of the paper, Sec. 2); this module only
marshals numpy arrays into it.  ``brute.py`` holds an independent numpy
Kronecker-product construction used to pin the C code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

KIND = {"matrix": 0, "h": 1, "x": 2, "y": 3, "z": 4, "rx": 5, "ry": 6, "rz": 7, "swap": 8}

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_U = ctypes.POINTER(ctypes.c_uint64)
_L = ctypes.POINTER(ctypes.c_longlong)


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
                               "-fopenmp", "-ffp-contract=off", "-fno-fast-math", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            L.orc_apply.argtypes = [ctypes.c_int, _D, _D, _I, ctypes.c_int, _I, ctypes.c_int, _D]
            L.orc_inner.argtypes = [ctypes.c_int, _D, _D, _D]
            L.orc_expect.argtypes = [ctypes.c_int, _D, ctypes.c_int, _U, _U, _D, _D, _D]
            L.orc_apply_hamiltonian.argtypes = [ctypes.c_int, _D, _D, ctypes.c_int, _U, _U, _D]
            L.orc_norm2.argtypes = [ctypes.c_int, _D, _D]
            L.orc_random_norm2.argtypes = [ctypes.c_int, ctypes.c_uint64, _D]
            L.orc_random_state.argtypes = [ctypes.c_int, ctypes.c_uint64, _D]
            L.orc_random_amps.argtypes = [ctypes.c_uint64, ctypes.c_double, _U, ctypes.c_int, _D]
            L.orc_apply_sampled_random.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_double,
                                                   _I, ctypes.c_int, _I, ctypes.c_int, _D, _U,
                                                   ctypes.c_int, _D]
            circ = [ctypes.c_int, ctypes.c_int, _I, _I, _I, _I, _I, _I, _L, _D]
            L.orc_run.argtypes = circ + [_D, _D, _D]
            L.orc_energy.argtypes = circ + [_D, ctypes.c_int, _U, _U, _D, _D]
            L.orc_grad.argtypes = circ + [_D, ctypes.c_int, ctypes.c_int, _U, _U, _D, _I,
                                          ctypes.c_int, ctypes.c_int, ctypes.c_double, _D]
            L.orc_adjoint.argtypes = circ + [_D, ctypes.c_int, ctypes.c_int, _U, _U, _D, _D, _D]
            L.orc_probabilities.argtypes = [ctypes.c_int, _D, _I, ctypes.c_int, _D]
            L.orc_sample.argtypes = [ctypes.c_int, _D, _D, ctypes.c_longlong, _L]
            L.orc_frequencies.argtypes = [ctypes.c_int, _L, ctypes.c_longlong, _I, ctypes.c_int, _L]
            L.orc_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_longlong, _D]
            L.orc_collapse.argtypes = [ctypes.c_int, _D, _D, _I, ctypes.c_int, ctypes.c_uint64,
                                       ctypes.c_double]
            _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _as_c128(psi) -> np.ndarray:
    return np.ascontiguousarray(psi, dtype=np.complex128)


def _ints(seq, size=None):
    a = np.zeros(size if size is not None else max(len(seq), 1), dtype=np.int32)
    a[:len(seq)] = seq
    return a


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle %s failed with code %d" % (what, rc))


def apply(psi, targets, controls, G) -> np.ndarray:
    """psi' = eq. (1) applied to psi (complex128 array of length 2**n)."""
    psi = _as_c128(psi)
    n = int(psi.size).bit_length() - 1
    G = np.ascontiguousarray(G, dtype=np.complex128)
    out = np.empty_like(psi)
    t = _ints(list(targets))
    c = _ints(list(controls))
    _check(lib().orc_apply(n, _p(psi, _D), _p(out, _D), _p(t, _I), len(targets), _p(c, _I),
                           len(controls), _p(G, _D)), "apply")
    return out


def inner(a, b) -> complex:
    a, b = _as_c128(a), _as_c128(b)
    n = int(a.size).bit_length() - 1
    out = np.zeros(2)
    lib().orc_inner(n, _p(a, _D), _p(b, _D), _p(out, _D))
    return complex(out[0], out[1])


def norm2(psi) -> float:
    psi = _as_c128(psi)
    out = np.zeros(1)
    lib().orc_norm2(int(psi.size).bit_length() - 1, _p(psi, _D), _p(out, _D))
    return float(out[0])


def probabilities(psi, qubits) -> np.ndarray:
    """Marginal Born probabilities of `qubits` (first listed = most significant
    bit of the outcome index), length 2**len(qubits), FP64."""
    psi = _as_c128(psi)
    n = int(psi.size).bit_length() - 1
    q = _ints(list(qubits))
    out = np.zeros(1 << len(qubits))
    _check(lib().orc_probabilities(n, _p(psi, _D), _p(q, _I), len(qubits), _p(out, _D)),
           "probabilities")
    return out


def sample(psi, u) -> np.ndarray:
    """Whole-register outcomes for the uniforms `u` by inverse-transform
    sampling of the Born probabilities (int64, one per uniform)."""
    psi = _as_c128(psi)
    n = int(psi.size).bit_length() - 1
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(max(u.size, 1), dtype=np.int64)
    _check(lib().orc_sample(n, _p(psi, _D), _p(u, _D), u.size, _p(out, _L)), "sample")
    return out[:u.size]


_PAULI2 = {(0, 0): np.eye(2, dtype=np.complex128),
           (1, 0): np.array([[0, 1], [1, 0]], dtype=np.complex128),
           (1, 1): np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
           (0, 1): np.array([[1, 0], [0, -1]], dtype=np.complex128)}


def pauli_factor(x: int, z: int, theta: float):
    """exp(-i theta P) for the Pauli string (x, z) on its support (targets in
    descending qubit order, first target = most significant), by the matrix
    exponential of the Kronecker product of its 2x2 factors.  The identity
    string gives exp(-i theta) I on qubit 0."""
    import scipy.linalg
    supp = [q for q in range(63, -1, -1) if ((x | z) >> q) & 1]
    if not supp:
        return [0], scipy.linalg.expm(-1j * theta * _PAULI2[(0, 0)])
    P = np.ones((1, 1), dtype=np.complex128)
    for q in supp:
        P = np.kron(P, _PAULI2[((x >> q) & 1, (z >> q) & 1)])
    return supp, scipy.linalg.expm(-1j * theta * P)


def trotter(psi, H, tau: float, steps: int, order: int = 1) -> np.ndarray:
    """Trotterised exp(-i steps tau H) psi (Sec. 3, time evolution with the
    Trotter decomposition): per step, order 1 applies exp(-i tau c_j P_j) for
    j = 0..T-1; order 2 applies exp(-i tau c_j P_j / 2) for j = 0..T-1 and
    then for j = T-1..0.  Each factor goes through eq. (1) (`apply`)."""
    if order not in (1, 2):
        raise ValueError("order must be 1 or 2")
    terms = list(zip(H.x_mask, H.z_mask, H.coeff))
    w = tau if order == 1 else tau / 2
    seq = [pauli_factor(int(x), int(z), w * float(c)) for x, z, c in terms]
    if order == 2:
        seq = seq + seq[::-1]
    out = _as_c128(psi).copy()
    for _ in range(steps):
        for t, G in seq:
            out = apply(out, t, [], G)
    return out


def frequencies(n: int, samples, qubits) -> np.ndarray:
    """Counts of the outcomes of `qubits` (first listed = most significant)
    over whole-register samples of an n-qubit state (int64, 2**len(qubits))."""
    smp = np.ascontiguousarray(samples, dtype=np.int64)
    q = _ints(list(qubits))
    out = np.zeros(1 << len(qubits), dtype=np.int64)
    _check(lib().orc_frequencies(n, _p(smp, _L), smp.size, _p(q, _I), len(qubits), _p(out, _L)),
           "frequencies")
    return out


def seeded_uniforms(seed: int, count: int) -> np.ndarray:
    """u[s] = top 53 bits of draw s of the seed's counter-based stream / 2^53
    (key = SplitMix64's first output from the seed, draw s = the output of the
    generator started at the key after s + 1 steps); seeded sampling draws
    these."""
    out = np.zeros(max(count, 1))
    _check(lib().orc_uniforms(seed, count, _p(out, _D)), "uniforms")
    return out[:count]


def collapse(psi, qubits, outcome: int, p: float) -> np.ndarray:
    """State after measuring `qubits` (first listed = most significant) with
    result `outcome` of probability p: projected and divided by sqrt(p)."""
    psi = _as_c128(psi)
    n = int(psi.size).bit_length() - 1
    q = _ints(list(qubits))
    out = np.empty_like(psi)
    _check(lib().orc_collapse(n, _p(psi, _D), _p(out, _D), _p(q, _I), len(qubits), int(outcome),
                              float(p)), "collapse")
    return out


def expect(psi, H, per_term: bool = False):
    """sum_j c_j <psi|P_j|psi> as a complex number (imaginary part ~ 0)."""
    psi = _as_c128(psi)
    n = int(psi.size).bit_length() - 1
    x = np.ascontiguousarray(H.x_mask, dtype=np.uint64)
    z = np.ascontiguousarray(H.z_mask, dtype=np.uint64)
    cf = np.ascontiguousarray(H.coeff, dtype=np.float64)
    out = np.zeros(2)
    terms = np.zeros(2 * max(len(cf), 1))
    _check(lib().orc_expect(n, _p(psi, _D), len(cf), _p(x, _U), _p(z, _U), _p(cf, _D),
                            _p(out, _D), _p(terms, _D)), "expect")
    e = complex(out[0], out[1])
    if per_term:
        return e, terms[0::2][:len(cf)] + 1j * terms[1::2][:len(cf)]
    return e


def apply_hamiltonian(psi, H) -> np.ndarray:
    """H psi for a Pauli sum H."""
    psi = _as_c128(psi)
    n = int(psi.size).bit_length() - 1
    x, z, cf = _ham(H)
    out = np.empty_like(psi)
    _check(lib().orc_apply_hamiltonian(n, _p(psi, _D), _p(out, _D), len(cf), _p(x, _U), _p(z, _U),
                                       _p(cf, _D)), "apply_hamiltonian")
    return out


def random_norm2(n: int, seed: int) -> float:
    out = np.zeros(1)
    lib().orc_random_norm2(n, seed, _p(out, _D))
    return float(out[0])


def random_state(n: int, seed: int) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    lib().orc_random_state(n, seed, _p(psi, _D))
    return psi


def random_amps(seed: int, scale: float, idx) -> np.ndarray:
    idx = np.ascontiguousarray(idx, dtype=np.uint64)
    out = np.empty(idx.size, dtype=np.complex128)
    lib().orc_random_amps(seed, scale, _p(idx, _U), idx.size, _p(out, _D))
    return out


def apply_sampled_random(n, seed, scale, targets, controls, G, idx) -> np.ndarray:
    """eq. (1) on the normalised random state (seed), evaluated at idx only."""
    idx = np.ascontiguousarray(idx, dtype=np.uint64)
    G = np.ascontiguousarray(G, dtype=np.complex128)
    out = np.empty(idx.size, dtype=np.complex128)
    t = _ints(list(targets))
    c = _ints(list(controls))
    _check(lib().orc_apply_sampled_random(n, seed, scale, _p(t, _I), len(targets), _p(c, _I),
                                          len(controls), _p(G, _D), _p(idx, _U), idx.size,
                                          _p(out, _D)), "apply_sampled_random")
    return out


class _Flat:
    """A workloads.Circuit laid out as the oracle's flat arrays."""

    def __init__(self, circ):
        ops = circ.ops
        m = max(len(ops), 1)
        self.n = circ.n
        self.nops = len(ops)
        self.kind = np.zeros(m, np.int32)
        self.k = np.zeros(m, np.int32)
        self.tgt = np.zeros(5 * m, np.int32)
        self.c = np.zeros(m, np.int32)
        self.ctl = np.zeros(4 * m, np.int32)
        self.param = np.full(m, -1, np.int32)
        self.moff = np.full(m, -1, np.int64)
        mats = []
        off = 0
        for i, op in enumerate(ops):
            self.kind[i] = KIND[op.kind]
            self.k[i] = len(op.targets)
            self.tgt[5 * i:5 * i + len(op.targets)] = op.targets
            self.c[i] = len(op.controls)
            self.ctl[4 * i:4 * i + len(op.controls)] = op.controls
            self.param[i] = op.param
            if op.kind == "matrix":
                flat = np.ascontiguousarray(op.matrix, dtype=np.complex128).view(np.float64).ravel()
                self.moff[i] = off
                mats.append(flat)
                off += flat.size
        self.mats = np.concatenate(mats) if mats else np.zeros(1)

    def args(self):
        return (self.n, self.nops, _p(self.kind, _I), _p(self.k, _I), _p(self.tgt, _I),
                _p(self.c, _I), _p(self.ctl, _I), _p(self.param, _I), _p(self.moff, _L),
                _p(self.mats, _D))


def _params(p, circ):
    p = np.ascontiguousarray(p if p is not None else np.zeros(max(circ.nparams, 1)), np.float64)
    if p.size == 0:
        p = np.zeros(1)
    return p


def _ham(H):
    x = np.ascontiguousarray(H.x_mask, dtype=np.uint64)
    z = np.ascontiguousarray(H.z_mask, dtype=np.uint64)
    cf = np.ascontiguousarray(H.coeff, dtype=np.float64)
    return x, z, cf


def run(circ, params=None, psi0=None) -> np.ndarray:
    """Final state of the circuit applied to |0...0> (or to psi0)."""
    F = _Flat(circ)
    p = _params(params, circ)
    out = np.empty(1 << circ.n, dtype=np.complex128)
    p0 = _as_c128(psi0) if psi0 is not None else None
    _check(lib().orc_run(*F.args(), _p(p, _D), _p(p0, _D) if p0 is not None else None,
                         _p(out, _D)), "run")
    return out


def energy(circ, params, H) -> float:
    F = _Flat(circ)
    p = _params(params, circ)
    x, z, cf = _ham(H)
    E = np.zeros(1)
    _check(lib().orc_energy(*F.args(), _p(p, _D), len(cf), _p(x, _U), _p(z, _U), _p(cf, _D),
                            _p(E, _D)), "energy")
    return float(E[0])


def _grad(circ, params, H, which, mode, h):
    F = _Flat(circ)
    p = _params(params, circ)
    x, z, cf = _ham(H)
    which = np.ascontiguousarray(which if which is not None else np.arange(circ.nparams), np.int32)
    out = np.zeros(max(which.size, 1))
    _check(lib().orc_grad(*F.args(), _p(p, _D), circ.nparams, len(cf), _p(x, _U), _p(z, _U),
                          _p(cf, _D), _p(which, _I), which.size, mode, h, _p(out, _D)), "grad")
    return out[:which.size]


def grad_param_shift(circ, params, H, which=None) -> np.ndarray:
    return _grad(circ, params, H, which, 0, 0.0)


def grad_finite_diff(circ, params, H, which=None, h: float = 1e-6) -> np.ndarray:
    return _grad(circ, params, H, which, 1, h)


def adjoint(circ, params, H):
    """(E, grad) by the oracle's own adjoint sweep."""
    F = _Flat(circ)
    p = _params(params, circ)
    x, z, cf = _ham(H)
    E = np.zeros(1)
    g = np.zeros(max(circ.nparams, 1))
    _check(lib().orc_adjoint(*F.args(), _p(p, _D), circ.nparams, len(cf), _p(x, _U), _p(z, _U),
                             _p(cf, _D), _p(E, _D), _p(g, _D)), "adjoint")
    return float(E[0]), g[:circ.nparams]
