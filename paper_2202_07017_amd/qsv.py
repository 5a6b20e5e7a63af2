"""ctypes binding of libqsv.so (include/qsv.h): argument marshalling only.

Every computation runs in the HIP kernels of libqsv.so.  PyTorch supplies
device memory (tensors) and streams (torch.cuda.current_stream()).  There is
no CPU fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqsv.so")

C64, C128 = 1, 2
OK, ERR_ARG, ERR_QUBIT, ERR_UNSUPPORTED, ERR_HIP, ERR_NOMEM = range(6)
MAX_TARGETS, MAX_CONTROLS, MAX_QUBITS = 5, 4, 40
KIND = {"matrix": 0, "h": 1, "x": 2, "y": 3, "z": 4, "rx": 5, "ry": 6, "rz": 7, "swap": 8}

_D = ctypes.POINTER(ctypes.c_double)
_U = ctypes.POINTER(ctypes.c_uint64)
_I = ctypes.POINTER(ctypes.c_int)
_vp = ctypes.c_void_p


class QsvError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("qsv status %d: %s" % (status, message))
        self.status = status


class qsv_block(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("targets", ctypes.c_int * MAX_TARGETS), ("M", _D)]


class qsv_pauli_sum(ctypes.Structure):
    _fields_ = [("nterms", ctypes.c_int), ("x_mask", _U), ("z_mask", _U), ("coeff", _D)]


class qsv_op(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("k", ctypes.c_int),
                ("targets", ctypes.c_int * MAX_TARGETS), ("c", ctypes.c_int),
                ("controls", ctypes.c_int * MAX_CONTROLS), ("param", ctypes.c_int), ("M", _D)]


class qsv_circuit(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("nops", ctypes.c_int), ("ops", ctypes.POINTER(qsv_op)),
                ("nparams", ctypes.c_int)]


_lib = None
_lock = threading.Lock()

_SIGS = {
    "qsv_last_error": ([], ctypes.c_char_p),
    "qsv_version": ([], ctypes.c_char_p),
    "qsv_state_bytes": ([ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "qsv_state_alloc": ([ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp)], ctypes.c_int),
    "qsv_state_free": ([_vp], ctypes.c_int),
    "qsv_init_basis": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, _vp], ctypes.c_int),
    "qsv_init_random": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, _vp, _vp], ctypes.c_int),
    "qsv_apply_gate": ([_vp, ctypes.c_int, ctypes.c_int, _I, ctypes.c_int, _I, ctypes.c_int, _D,
                        _vp], ctypes.c_int),
    "qsv_apply_fused": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(qsv_block), ctypes.c_int,
                         _vp], ctypes.c_int),
    "qsv_reduce_workspace_bytes": ([ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "qsv_norm2": ([_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp], ctypes.c_int),
    "qsv_expectation": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(qsv_pauli_sum), _vp, _vp,
                         _vp], ctypes.c_int),
    "qsv_expectation_launches": ([ctypes.POINTER(qsv_pauli_sum), ctypes.c_int, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "qsv_expectation_noalloc": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(qsv_pauli_sum),
                                 _vp, _vp], ctypes.c_int),
    "qsv_inner": ([_vp, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp], ctypes.c_int),
    "qsv_apply_pauli_sum": ([_vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(qsv_pauli_sum),
                             _vp], ctypes.c_int),
    "qsv_measure_workspace_bytes": ([ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
                                    ctypes.c_int),
    "qsv_probabilities": ([_vp, ctypes.c_int, ctypes.c_int, _I, ctypes.c_int, _vp, _vp, _vp],
                          ctypes.c_int),
    "qsv_sample": ([_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int64, _vp, _vp, _vp],
                   ctypes.c_int),
    "qsv_sample_seeded": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_int64, _vp, _vp,
                           _vp], ctypes.c_int),
    "qsv_collapse": ([_vp, ctypes.c_int, ctypes.c_int, _I, ctypes.c_int, ctypes.c_uint64, _vp, _vp],
                     ctypes.c_int),
    "qsv_frequencies": ([_vp, ctypes.c_int64, ctypes.c_int, _I, ctypes.c_int, _vp, _vp],
                        ctypes.c_int),
    "qsv_plan_create": ([ctypes.POINTER(qsv_circuit), ctypes.c_int, ctypes.c_int, _D,
                         ctypes.POINTER(_vp)], ctypes.c_int),
    "qsv_trotter_plan_create": ([ctypes.POINTER(qsv_pauli_sum), ctypes.c_int, ctypes.c_double,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.POINTER(_vp)], ctypes.c_int),
    "qsv_plan_run": ([_vp, _vp, _vp, _vp], ctypes.c_int),
    "qsv_plan_info": ([_vp, _I, _D, _D], ctypes.c_int),
    "qsv_plan_destroy": ([_vp], ctypes.c_int),
    "qsv_adjoint_plan_create": ([ctypes.POINTER(qsv_circuit), ctypes.POINTER(qsv_pauli_sum),
                                 ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp),
                                 ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "qsv_adjoint_run": ([_vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "qsv_adjoint_energy": ([_vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "qsv_adjoint_state": ([_vp, _vp, ctypes.c_int, ctypes.POINTER(_vp)], ctypes.c_int),
    "qsv_adjoint_plan_destroy": ([_vp], ctypes.c_int),
    "qsv_adjoint_gradient": ([ctypes.POINTER(qsv_circuit), _vp, ctypes.POINTER(qsv_pauli_sum),
                              ctypes.c_int, ctypes.c_int, _vp, ctypes.c_size_t, _vp, _vp, _vp],
                             ctypes.c_int),
    "qsv_batch_plan_create": ([ctypes.POINTER(qsv_circuit), ctypes.POINTER(qsv_pauli_sum),
                               ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp),
                               ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "qsv_batch_offsets": ([_vp, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "qsv_batch_run": ([_vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "qsv_batch_tune": ([_vp, _vp, _vp, _vp, _vp, _vp, _I], ctypes.c_int),
    "qsv_batch_plan_destroy": ([_vp], ctypes.c_int),
}

EXPORTED = tuple(_SIGS)


def lib():
    """Load libqsv.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("libqsv.so is missing at %s: run __graft_entry__.build() "
                                   "(the HIP library is required; there is no fallback)" % LIB_PATH)
            L = ctypes.CDLL(LIB_PATH)
            for name, (args, res) in _SIGS.items():
                f = getattr(L, name)
                f.argtypes = args
                f.restype = res
            _lib = L
    return _lib


def _check(status):
    if status != OK:
        raise QsvError(status, lib().qsv_last_error().decode())


def dtype_code(t) -> int:
    import torch
    if t.dtype == torch.complex64:
        return C64
    if t.dtype == torch.complex128:
        return C128
    raise TypeError("state tensors must be complex64 or complex128, got %s" % t.dtype)


def _nqubits(t) -> int:
    n = int(t.numel()).bit_length() - 1
    if t.numel() != (1 << n):
        raise ValueError("state length %d is not a power of two" % t.numel())
    return n


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return _vp(s.cuda_stream)


def _ptr(t):
    return _vp(t.data_ptr()) if t is not None else None


def _ints(seq):
    seq = list(seq)
    arr = (ctypes.c_int * max(len(seq), 1))(*seq)
    return arr


def _mat(G):
    G = np.ascontiguousarray(G, dtype=np.complex128)
    return G, G.view(np.float64).ctypes.data_as(_D)


# ------------------------------------------------------------ qubit order
#
# The C ABI numbers qubit j as index bit j (weight 2^j).  order="big" accepts
# the opposite convention (qubit 0 = most significant bit, as in Qibo's own
# software): qubit q of an n-qubit state is passed on as n - 1 - q, masks and
# basis indices are bit-reversed over n bits.  Marshalling only.

def _order_ok(order):
    if order not in ("little", "big"):
        raise ValueError("order must be 'little' or 'big', not %r" % (order,))


def map_qubits(qubits, n: int, order: str = "little"):
    _order_ok(order)
    return [int(q) for q in qubits] if order == "little" else [n - 1 - int(q) for q in qubits]


def reverse_bits(v: int, n: int) -> int:
    return int("{:0{w}b}".format(int(v), w=n)[::-1], 2) if n > 0 else 0


# ---------------------------------------------------------------- states

def state_empty(n: int, dtype, device="cuda"):
    import torch
    return torch.empty(1 << n, dtype=dtype, device=device)


_work_cache = {}


def reduce_workspace(device):
    """A cached device buffer of qsv_reduce_workspace_bytes() bytes."""
    import torch
    key = (str(device), torch.cuda.current_stream(device).cuda_stream)
    w = _work_cache.get(key)
    if w is None:
        size = ctypes.c_size_t()
        _check(lib().qsv_reduce_workspace_bytes(ctypes.byref(size)))
        w = torch.empty(size.value // 8, dtype=torch.float64, device=device)
        _work_cache[key] = w
    return w


def qsv_init_basis(psi, index: int = 0, stream=None, order="little"):
    _order_ok(order)
    n = _nqubits(psi)
    idx = index if order == "little" else reverse_bits(index, n)
    _check(lib().qsv_init_basis(_ptr(psi), n, dtype_code(psi), idx, _stream(stream)))


def qsv_init_random(psi, seed: int, stream=None):
    work = reduce_workspace(psi.device)
    _check(lib().qsv_init_random(_ptr(psi), _nqubits(psi), dtype_code(psi), seed, _ptr(work),
                                 _stream(stream)))


def qsv_apply_gate(psi, targets: Sequence[int], controls: Sequence[int], G, stream=None,
                   order="little"):
    n = _nqubits(psi)
    t, c = _ints(map_qubits(targets, n, order)), _ints(map_qubits(controls, n, order))
    _G, gp = _mat(G)
    _check(lib().qsv_apply_gate(_ptr(psi), _nqubits(psi), dtype_code(psi), t, len(targets), c,
                                len(controls), gp, _stream(stream)))


def qsv_apply_fused(psi, blocks, stream=None, order="little"):
    """blocks: sequence of (targets, matrix)."""
    n = _nqubits(psi)
    arr = (qsv_block * max(len(blocks), 1))()
    keep = []
    for j, (targets, M) in enumerate(blocks):
        Mc, mp = _mat(M)
        keep.append(Mc)
        arr[j].k = len(targets)
        for i, q in enumerate(map_qubits(targets, n, order)):
            arr[j].targets[i] = q
        arr[j].M = mp
    _check(lib().qsv_apply_fused(_ptr(psi), _nqubits(psi), dtype_code(psi), arr, len(blocks),
                                 _stream(stream)))


class PauliSum:
    """ctypes view of a Pauli sum (x_mask, z_mask, coeff arrays kept alive)."""

    def __init__(self, H, order="little"):
        _order_ok(order)
        x, z = H.x_mask, H.z_mask
        if order == "big":
            x = [reverse_bits(v, H.n) for v in x]
            z = [reverse_bits(v, H.n) for v in z]
        self.x = np.ascontiguousarray(x, dtype=np.uint64)
        self.z = np.ascontiguousarray(z, dtype=np.uint64)
        self.c = np.ascontiguousarray(H.coeff, dtype=np.float64)
        self.n = H.n
        self.s = qsv_pauli_sum(len(self.c), self.x.ctypes.data_as(_U), self.z.ctypes.data_as(_U),
                               self.c.ctypes.data_as(_D))


def qsv_norm2(psi, out=None, stream=None):
    import torch
    out = out if out is not None else torch.empty(1, dtype=torch.float64, device=psi.device)
    _check(lib().qsv_norm2(_ptr(psi), _nqubits(psi), dtype_code(psi), _ptr(out),
                           _ptr(reduce_workspace(psi.device)), _stream(stream)))
    return out


def qsv_expectation(psi, H, out=None, stream=None):
    import torch
    P = H if isinstance(H, PauliSum) else PauliSum(H)
    out = out if out is not None else torch.empty(2, dtype=torch.float64, device=psi.device)
    _check(lib().qsv_expectation(_ptr(psi), _nqubits(psi), dtype_code(psi), ctypes.byref(P.s),
                                 _ptr(out), _ptr(reduce_workspace(psi.device)), _stream(stream)))
    return out


def expectation_launches(H, n: int, dtype_code_: int) -> int:
    """Kernel launches one qsv_expectation of H on an n-qubit state enqueues."""
    P = H if isinstance(H, PauliSum) else PauliSum(H)
    c = ctypes.c_int()
    _check(lib().qsv_expectation_launches(ctypes.byref(P.s), n, dtype_code_, ctypes.byref(c)))
    return c.value


def qsv_expectation_noalloc(psi, H, out=None, stream=None):
    """qsv_expectation with the library's static per-GPU scratch (no
    workspace; calls overlapping on one GPU race)."""
    import torch
    P = H if isinstance(H, PauliSum) else PauliSum(H)
    out = out if out is not None else torch.empty(2, dtype=torch.float64, device=psi.device)
    _check(lib().qsv_expectation_noalloc(_ptr(psi), _nqubits(psi), dtype_code(psi), ctypes.byref(P.s),
                                         _ptr(out), _stream(stream)))
    return out


def qsv_inner(a, b, out=None, stream=None):
    import torch
    out = out if out is not None else torch.empty(2, dtype=torch.float64, device=a.device)
    _check(lib().qsv_inner(_ptr(a), _ptr(b), _nqubits(a), dtype_code(a), _ptr(out),
                           _ptr(reduce_workspace(a.device)), _stream(stream)))
    return out


def qsv_apply_pauli_sum(psi, out, H, stream=None):
    P = H if isinstance(H, PauliSum) else PauliSum(H)
    _check(lib().qsv_apply_pauli_sum(_ptr(psi), _ptr(out), _nqubits(psi), dtype_code(psi),
                                     ctypes.byref(P.s), _stream(stream)))


# ----------------------------------------------------------- measurement

_measure_cache = {}


def measure_workspace(n: int, dtype_code_: int, device):
    """A cached device buffer of at least qsv_measure_workspace_bytes(n) bytes
    (grown on demand, one per device and stream)."""
    import torch
    size = ctypes.c_size_t()
    _check(lib().qsv_measure_workspace_bytes(n, dtype_code_, ctypes.byref(size)))
    key = (str(device), torch.cuda.current_stream(device).cuda_stream)
    w = _measure_cache.get(key)
    if w is None or w.numel() * 8 < size.value:
        w = torch.empty((size.value + 7) // 8, dtype=torch.float64, device=device)
        _measure_cache[key] = w
    return w


def qsv_probabilities(psi, qubits: Sequence[int], out=None, stream=None, order="little"):
    """Marginal Born probabilities of `qubits` (first listed = most significant
    outcome bit): a float64 device tensor of 2**len(qubits) entries."""
    import torch
    n = _nqubits(psi)
    q = _ints(map_qubits(qubits, n, order))
    out = out if out is not None else torch.empty(1 << len(qubits), dtype=torch.float64,
                                                  device=psi.device)
    work = measure_workspace(n, dtype_code(psi), psi.device)
    _check(lib().qsv_probabilities(_ptr(psi), n, dtype_code(psi), q, len(qubits), _ptr(out),
                                   _ptr(work), _stream(stream)))
    return out


def qsv_sample(psi, u, out=None, stream=None):
    """Whole-register outcomes (int64 device tensor, amplitude indices with
    qubit j at bit j) for the float64 device uniforms `u`, by inverse-transform
    sampling of the Born probabilities."""
    import torch
    n = _nqubits(psi)
    if u.dtype != torch.float64 or not u.is_contiguous():
        raise ValueError("u must be a contiguous float64 device tensor")
    out = out if out is not None else torch.empty(u.numel(), dtype=torch.int64, device=psi.device)
    work = measure_workspace(n, dtype_code(psi), psi.device)
    _check(lib().qsv_sample(_ptr(psi), n, dtype_code(psi), _ptr(u), u.numel(), _ptr(out),
                            _ptr(work), _stream(stream)))
    return out


def qsv_sample_seeded(psi, seed: int, nshots: int, out=None, stream=None):
    """qsv_sample with device-drawn uniforms: u[s] = top 53 bits of draw s of
    the seed's counter-based SplitMix64 stream / 2^53 (see qsv.h)."""
    import torch
    n = _nqubits(psi)
    out = out if out is not None else torch.empty(nshots, dtype=torch.int64, device=psi.device)
    work = measure_workspace(n, dtype_code(psi), psi.device)
    _check(lib().qsv_sample_seeded(_ptr(psi), n, dtype_code(psi), int(seed), int(nshots), _ptr(out),
                                   _ptr(work), _stream(stream)))
    return out


def qsv_collapse(psi, qubits: Sequence[int], outcome: int, prob, stream=None, order="little"):
    """Project psi onto `outcome` of `qubits` (first listed = most significant)
    and divide by sqrt(prob[0]) (prob: float64 device tensor, e.g. a slice of
    qsv_probabilities' result), in place."""
    import torch
    if prob.dtype != torch.float64:
        raise ValueError("prob must be a float64 device tensor")
    n = _nqubits(psi)
    q = _ints(map_qubits(qubits, n, order))
    _check(lib().qsv_collapse(_ptr(psi), n, dtype_code(psi), q, len(qubits), int(outcome), _ptr(prob),
                              _stream(stream)))


def qsv_frequencies(samples, n: int, qubits: Sequence[int], out=None, stream=None, order="little"):
    """Counts (int64 device tensor of 2**len(qubits)) of the outcomes of
    `qubits` (first listed = most significant) over whole-register samples."""
    import torch
    if samples.dtype != torch.int64 or not samples.is_contiguous():
        raise ValueError("samples must be a contiguous int64 device tensor")
    q = _ints(map_qubits(qubits, n, order))
    out = out if out is not None else torch.empty(1 << len(qubits), dtype=torch.int64,
                                                  device=samples.device)
    _check(lib().qsv_frequencies(_ptr(samples), samples.numel(), n, q, len(qubits), _ptr(out),
                                 _stream(stream)))
    return out


# -------------------------------------------------------------- circuits

class CircuitC:
    """ctypes form of a circuit (any object with n, ops, nparams whose ops
    have kind, targets, controls, param, matrix)."""

    def __init__(self, circ, order="little"):
        self.mats = []
        ops = (qsv_op * max(len(circ.ops), 1))()
        for j, op in enumerate(circ.ops):
            o = ops[j]
            o.kind = KIND[op.kind]
            o.k = len(op.targets)
            for i, q in enumerate(map_qubits(op.targets, circ.n, order)):
                o.targets[i] = q
            o.c = len(op.controls)
            for i, q in enumerate(map_qubits(op.controls, circ.n, order)):
                o.controls[i] = q
            o.param = op.param
            if op.kind == "matrix":
                M, mp = _mat(op.matrix)
                self.mats.append(M)
                o.M = mp
        self.ops = ops
        self.s = qsv_circuit(circ.n, len(circ.ops), ops, circ.nparams)
        self.n = circ.n
        self.nparams = circ.nparams


class Plan:
    """qsv_plan: fused launch list, replayed through a HIP graph."""

    def __init__(self, circ, dtype_code_: int, fuse_k: int = 5, params_host=None, order="little"):
        self.c = circ if isinstance(circ, CircuitC) else CircuitC(circ, order)
        self.h = _vp()
        ph = None
        if params_host is not None:
            self._ph = np.ascontiguousarray(params_host, dtype=np.float64)
            ph = self._ph.ctypes.data_as(_D)
        _check(lib().qsv_plan_create(ctypes.byref(self.c.s), dtype_code_, fuse_k, ph,
                                     ctypes.byref(self.h)))

    def run(self, psi, params_dev=None, stream=None):
        _check(lib().qsv_plan_run(self.h, _ptr(psi), _ptr(params_dev), _stream(stream)))

    def info(self):
        n = ctypes.c_int()
        b = ctypes.c_double()
        f = ctypes.c_double()
        _check(lib().qsv_plan_info(self.h, ctypes.byref(n), ctypes.byref(b), ctypes.byref(f)))
        return n.value, b.value, f.value

    def __del__(self):
        if getattr(self, "h", None) and self.h.value and _lib is not None:
            _lib.qsv_plan_destroy(self.h)


class TrotterPlan(Plan):
    """qsv_trotter_plan_create: `steps` Trotter steps of length tau for the
    Pauli sum H (order 1 or 2), fused into blocks of at most fuse_k qubits."""

    def __init__(self, H, tau: float, steps: int, order: int, dtype_code_: int, fuse_k: int = 5):
        self.P = H if isinstance(H, PauliSum) else PauliSum(H)
        self.h = _vp()
        n = H.n
        _check(lib().qsv_trotter_plan_create(ctypes.byref(self.P.s), n, float(tau), int(steps),
                                             int(order), dtype_code_, fuse_k, ctypes.byref(self.h)))


class AdjointPlan:
    """qsv_adjoint_plan with its device workspace (a torch tensor)."""

    def __init__(self, circ, H, dtype_code_: int, fuse_k: int = 5, device="cuda", order="little"):
        import torch
        self.c = circ if isinstance(circ, CircuitC) else CircuitC(circ, order)
        self.H = H if isinstance(H, PauliSum) else PauliSum(H, order)
        self.h = _vp()
        wb = ctypes.c_size_t()
        _check(lib().qsv_adjoint_plan_create(ctypes.byref(self.c.s), ctypes.byref(self.H.s),
                                             dtype_code_, fuse_k, ctypes.byref(self.h),
                                             ctypes.byref(wb)))
        self.work_bytes = wb.value
        self.work = torch.empty((wb.value + 255) // 256 * 32, dtype=torch.float64, device=device)
        self.nparams = self.c.nparams
        self.device = device

    def run(self, params_dev, energy=None, grad=None, stream=None):
        import torch
        energy = energy if energy is not None else torch.empty(1, dtype=torch.float64,
                                                               device=self.device)
        grad = grad if grad is not None else torch.empty(max(self.nparams, 1), dtype=torch.float64,
                                                         device=self.device)
        _check(lib().qsv_adjoint_run(self.h, _ptr(params_dev), _ptr(self.work), _ptr(energy),
                                     _ptr(grad), _stream(stream)))
        return energy, grad[:self.nparams]

    def energy(self, params_dev, energy=None, stream=None):
        import torch
        energy = energy if energy is not None else torch.empty(1, dtype=torch.float64,
                                                               device=self.device)
        _check(lib().qsv_adjoint_energy(self.h, _ptr(params_dev), _ptr(self.work), _ptr(energy),
                                        _stream(stream)))
        return energy

    def state_ptr(self, slot=0):
        p = _vp()
        _check(lib().qsv_adjoint_state(self.h, _ptr(self.work), slot, ctypes.byref(p)))
        return p.value

    def __del__(self):
        if getattr(self, "h", None) and self.h.value and _lib is not None:
            _lib.qsv_adjoint_plan_destroy(self.h)


def _autograd_function():
    import torch

    class AdjointEnergy(torch.autograd.Function):
        """E(theta) = <psi(theta)|H|psi(theta)> with the gradient from the
        library's adjoint sweep (computed in forward, scaled in backward)."""

        @staticmethod
        def forward(ctx, params, plan):
            p = params.detach().to(torch.float64).contiguous()
            if not ctx.needs_input_grad[0]:
                # no gradient wanted: the forward sweep and the energy only
                return plan.energy(p)[0].clone()
            e, g = plan.run(p)
            ctx.save_for_backward(g.clone())
            return e[0].clone()

        @staticmethod
        def backward(ctx, grad_out):
            (g,) = ctx.saved_tensors
            return grad_out * g, None

    return AdjointEnergy


_AE = None


def adjoint_energy(params, plan):
    """Differentiable energy: torch.autograd sees dE/dtheta from the adjoint.
    Without a gradient to record (torch.no_grad() or params not requiring
    grad) only the forward sweep and the energy run."""
    import torch
    global _AE
    if _AE is None:
        _AE = _autograd_function()
    if not (torch.is_grad_enabled() and params.requires_grad):
        return plan.energy(params.detach().to(torch.float64).contiguous())[0].clone()
    return _AE.apply(params, plan)


def adjoint_gradient(circ, params_dev, H, dtype_code_: int, fuse_k: int, work, energy, grad,
                     stream=None, order="little"):
    """One-shot qsv_adjoint_gradient: plan, run and release in one call (it
    host-synchronises the stream).  work: a device tensor of at least
    adjoint_work_bytes(...) bytes."""
    c = circ if isinstance(circ, CircuitC) else CircuitC(circ, order)
    h = H if isinstance(H, PauliSum) else PauliSum(H, order)
    _check(lib().qsv_adjoint_gradient(ctypes.byref(c.s), _ptr(params_dev), ctypes.byref(h.s),
                                      dtype_code_, fuse_k, _ptr(work),
                                      work.numel() * work.element_size(), _ptr(energy),
                                      _ptr(grad), _stream(stream)))
    return energy, grad


def adjoint_work_bytes(circ, H, dtype_code_: int, fuse_k: int, order="little") -> int:
    """Workspace size the adjoint needs for (circ, H, dtype, fuse_k)."""
    c = circ if isinstance(circ, CircuitC) else CircuitC(circ, order)
    h = H if isinstance(H, PauliSum) else PauliSum(H, order)
    hp, wb = _vp(), ctypes.c_size_t()
    _check(lib().qsv_adjoint_plan_create(ctypes.byref(c.s), ctypes.byref(h.s), dtype_code_, fuse_k,
                                         ctypes.byref(hp), ctypes.byref(wb)))
    lib().qsv_adjoint_plan_destroy(hp)
    return wb.value


class BatchPlan:
    """qsv_batch_plan over a list of (circuit, Hamiltonian) instances, with its
    device workspace (a torch tensor).  Parameters and gradients of instance i
    are params[offsets[i]:offsets[i+1]] of the concatenated vectors."""

    def __init__(self, instances, dtype_code_: int, device="cuda", order="little"):
        import torch
        self.cs = [CircuitC(inst.circuit, order) for inst in instances]
        self.Hs = [PauliSum(inst.hamiltonian, order) for inst in instances]
        ca = (qsv_circuit * len(self.cs))(*[c.s for c in self.cs])
        ha = (qsv_pauli_sum * len(self.Hs))(*[h.s for h in self.Hs])
        self._ca, self._ha = ca, ha
        self.h = _vp()
        wb = ctypes.c_size_t()
        _check(lib().qsv_batch_plan_create(ca, ha, len(self.cs), dtype_code_, ctypes.byref(self.h),
                                           ctypes.byref(wb)))
        self.ninst = len(self.cs)
        off = (ctypes.c_int64 * (self.ninst + 1))()
        _check(lib().qsv_batch_offsets(self.h, off))
        self.offsets = np.array(off[:], dtype=np.int64)
        self.work = torch.empty((wb.value + 255) // 256 * 32, dtype=torch.float64, device=device)
        self.device = device

    def run(self, params_dev, energies=None, grads=None, stream=None):
        import torch
        energies = energies if energies is not None else torch.empty(
            self.ninst, dtype=torch.float64, device=self.device)
        grads = grads if grads is not None else torch.empty(
            max(int(self.offsets[-1]), 1), dtype=torch.float64, device=self.device)
        _check(lib().qsv_batch_run(self.h, _ptr(params_dev), _ptr(self.work), _ptr(energies),
                                   _ptr(grads), _stream(stream)))
        return energies, grads

    def tune(self, params_dev, energies, grads, stream=None):
        chosen = (ctypes.c_int * 3)()
        _check(lib().qsv_batch_tune(self.h, _ptr(params_dev), _ptr(self.work), _ptr(energies),
                                    _ptr(grads), _stream(stream), chosen))
        return chosen[0], chosen[1], chosen[2]

    def __del__(self):
        if getattr(self, "h", None) and self.h.value and _lib is not None:
            _lib.qsv_batch_plan_destroy(self.h)
