"""The C ABI without a GPU: the library loads, exports every function that
include/qsv.h declares, and rejects invalid arguments on the host before it
touches the device (no call here reaches a kernel)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def q():
    from paper_2202_07017_amd import qsv
    qsv.lib()
    return qsv


def header_functions():
    src = open(os.path.join(ROOT, "include", "qsv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qsv_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_function(q):
    names = header_functions()
    assert len(names) >= 25
    for name in names:
        assert hasattr(q.lib(), name), name
    assert set(names) == set(q.EXPORTED)


def test_version_and_sizes(q):
    assert q.lib().qsv_version().startswith(b"qsv")
    b = ctypes.c_size_t()
    assert q.lib().qsv_state_bytes(30, q.C64, ctypes.byref(b)) == q.OK and b.value == 8 << 30
    assert q.lib().qsv_state_bytes(32, q.C128, ctypes.byref(b)) == q.OK and b.value == 16 << 32
    assert q.lib().qsv_reduce_workspace_bytes(ctypes.byref(b)) == q.OK and b.value >= 16384


def call_gate(q, psi, n, dt, t, c, G=None):
    G = np.eye(2 ** max(len(t), 1), dtype=np.complex128) if G is None else G
    ti = (ctypes.c_int * max(len(t), 1))(*t)
    ci = (ctypes.c_int * max(len(c), 1))(*c)
    return q.lib().qsv_apply_gate(ctypes.c_void_p(psi), n, dt, ti, len(t), ci, len(c),
                                  G.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  None)


FAKE = 1 << 20  # never dereferenced: every call below fails validation first


@pytest.mark.parametrize("args,status,needle", [
    ((FAKE, 0, 1, (0,), ()), 1, "n = 0"),
    ((FAKE, 41, 1, (0,), ()), 1, "n = 41"),
    ((FAKE, 4, 3, (0,), ()), 1, "dtype"),
    ((None, 4, 1, (0,), ()), 1, "NULL"),
    ((FAKE + 8, 4, 1, (0,), ()), 1, "aligned"),
    ((FAKE, 4, 1, (4,), ()), 2, "qubit 4"),
    ((FAKE, 4, 1, (-1,), ()), 2, "qubit -1"),
    ((FAKE, 4, 1, (1, 1), ()), 2, "twice"),
    ((FAKE, 4, 1, (1,), (1,)), 2, "twice"),
    ((FAKE, 4, 1, (0, 1, 2), (3, 2)), 1, "exceeds"),
    ((FAKE, 8, 1, (0, 1, 2, 3, 4, 5), ()), 1, "k = 6"),
    ((FAKE, 4, 1, (), ()), 1, "k = 0"),
])
def test_apply_gate_validation(q, args, status, needle):
    psi, n, dt, t, c = args
    rc = call_gate(q, psi, n, dt, t, c)
    assert rc == status
    assert needle in q.lib().qsv_last_error().decode()


def test_other_validation(q):
    L = q.lib()
    assert L.qsv_init_basis(ctypes.c_void_p(FAKE), 4, 1, 16, None) == q.ERR_ARG
    assert L.qsv_norm2(ctypes.c_void_p(FAKE), 4, 1, None, None, None) == q.ERR_ARG
    x = np.array([1 << 5], np.uint64)
    z = np.array([0], np.uint64)
    cf = np.array([1.0])
    H = q.qsv_pauli_sum(1, x.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                        z.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                        cf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    rc = L.qsv_expectation(ctypes.c_void_p(FAKE), 4, 1, ctypes.byref(H), ctypes.c_void_p(FAKE),
                           ctypes.c_void_p(FAKE), None)
    assert rc == q.ERR_QUBIT and "qubit >= n" in L.qsv_last_error().decode()
    H.nterms = 0
    assert L.qsv_expectation(ctypes.c_void_p(FAKE), 4, 1, ctypes.byref(H), ctypes.c_void_p(FAKE),
                             ctypes.c_void_p(FAKE), None) == q.ERR_ARG
    assert L.qsv_apply_pauli_sum(ctypes.c_void_p(FAKE), ctypes.c_void_p(FAKE), 4, 1,
                                 ctypes.byref(H), None) == q.ERR_ARG


def test_circuit_validation(q):
    import workloads as W
    L = q.lib()
    bad = [W.Circuit(3, [W.Op("ry", (0,), param=2)], 1),          # param out of range
           W.Circuit(3, [W.Op("x", (0,), controls=(0,))]),         # repeated qubit
           W.Circuit(3, [W.Op("swap", (0,))]),                     # swap needs 2 targets
           W.Circuit(3, [W.Op("x", (3,))])]                         # qubit out of range
    for circ in bad:
        cc = q.CircuitC(circ)
        h = ctypes.c_void_p()
        assert L.qsv_plan_create(ctypes.byref(cc.s), 2, 5, None, ctypes.byref(h)) != q.OK
        assert not h.value
    cc = q.CircuitC(W.hea(3, 1))
    h = ctypes.c_void_p()
    assert L.qsv_plan_create(ctypes.byref(cc.s), 2, 6, None, ctypes.byref(h)) == q.ERR_ARG
    assert L.qsv_plan_create(ctypes.byref(cc.s), 5, 2, None, ctypes.byref(h)) == q.ERR_ARG


def test_binding_refuses_without_library(tmp_path, monkeypatch):
    from paper_2202_07017_amd import qsv
    monkeypatch.setattr(qsv, "_lib", None)
    monkeypatch.setattr(qsv, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no fallback"):
        qsv.lib()


@pytest.fixture
def forced_failure(monkeypatch):
    monkeypatch.setenv("QSV_TEST_FAIL_LAUNCH", "1")
    yield


def test_forced_launch_failure_reports_hip_error(q, forced_failure):
    """With QSV_TEST_FAIL_LAUNCH=1 every call that passes validation reports
    QSV_ERR_HIP with the launch-failure message before it enqueues anything;
    validation errors still come first.  The pointers are fake and never
    reached (the hook returns first), so this runs only where no GPU is."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("fake device pointers: the GPU variant of this test covers a real state")
    L = q.lib()
    P = ctypes.c_void_p(FAKE)
    assert call_gate(q, FAKE, 4, 1, (0,), (), np.array([[0, 1], [1, 0]], np.complex128)) == q.ERR_HIP
    assert "QSV_TEST_FAIL_LAUNCH" in L.qsv_last_error().decode()
    assert call_gate(q, FAKE, 4, 1, (4,), ()) == q.ERR_QUBIT  # validation first
    x = np.array([1], np.uint64)
    z = np.array([2], np.uint64)
    cf = np.array([1.0])
    H = q.qsv_pauli_sum(1, x.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                        z.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                        cf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    qs = (ctypes.c_int * 2)(0, 1)
    calls = [
        lambda: L.qsv_init_basis(P, 4, 1, 3, None),
        lambda: L.qsv_init_random(P, 4, 2, 7, P, None),
        lambda: L.qsv_norm2(P, 4, 1, P, P, None),
        lambda: L.qsv_expectation(P, 4, 1, ctypes.byref(H), P, P, None),
        lambda: L.qsv_inner(P, P, 4, 2, P, P, None),
        lambda: L.qsv_apply_pauli_sum(P, ctypes.c_void_p(FAKE * 2), 4, 1, ctypes.byref(H), None),
        lambda: L.qsv_probabilities(P, 4, 1, qs, 2, P, P, None),
        lambda: L.qsv_sample(P, 4, 1, P, 5, P, P, None),
        lambda: L.qsv_sample_seeded(P, 4, 1, 9, 5, P, P, None),
        lambda: L.qsv_frequencies(P, 5, 4, qs, 2, P, None),
        lambda: L.qsv_collapse(P, 4, 1, qs, 2, 1, P, None),
    ]
    for j, call in enumerate(calls):
        assert call() == q.ERR_HIP, j
        assert "QSV_TEST_FAIL_LAUNCH" in L.qsv_last_error().decode(), j


def test_expectation_launch_count(q):
    """Host-only query: one launch per pass over the state plus the final
    reduction; TFIM at n = 30 is five register passes (X on five qubits each,
    the first also the ZZ terms and, after its transpose, X on qubits 0..4); a
    diagonal-only sum at n >= 12 is one register pass."""
    import workloads as W
    assert q.expectation_launches(W.tfim_chain(30), 30, q.C64) == 6
    assert q.expectation_launches(W.pauli_sum(20, [("ZZ", (0, 19), 1.0), ("Z", (3,), 0.5)]), 20, q.C128) == 2
    assert q.expectation_launches(W.pauli_sum(5, [("Z", (0,), 1.0)]), 5, q.C64) == 2
    with pytest.raises(q.QsvError):
        q.expectation_launches(W.tfim_chain(30), 29, q.C64)
