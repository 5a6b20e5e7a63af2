"""Degenerate and boundary cases of the GPU path, through the C ABI, against
the CPU oracle: gates that span every qubit (k + c = n), identity gates (a
no-op that must leave the state bit-exact), non-unitary matrices on the VALU
and MFMA paths, MFMA launches of exactly one tile, empty plans, and Pauli
sums with identity and duplicated terms at one and two tiles."""
import numpy as np
import pytest

import workloads as W
from gpu_util import TOL, rand_state, raw_bits, say, to_gpu, to_np, torch_dtype

pytestmark = pytest.mark.gpu

DTYPES = ["c64", "c128"]


@pytest.fixture(scope="module")
def q():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2202_07017_amd import qsv
    qsv.lib()
    return qsv


def close(got, ref, name, what):
    err = np.max(np.abs(got - ref)) if got.size else 0.0
    assert err <= TOL[name], "%s %s: max|d| = %.3e" % (what, name, err)


def random_matrix(rng, d):
    return (rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))) / np.sqrt(2 * d)


def test_gates_spanning_every_qubit(q, orc):
    """k + c = n: the whole state is one group (or one controlled group)."""
    rng = np.random.default_rng(71)
    cases = [(1, (0,), ()), (2, (1, 0), ()), (3, (2, 0, 1), ()), (4, (3,), (0, 1, 2)),
             (4, (0, 2), (3, 1)), (5, (4, 2, 0, 1, 3), ()), (5, (1, 3, 0, 4), (2,)),
             (6, (5, 0), (1, 2, 3, 4))]
    for name in DTYPES:
        for n, t, c in cases:
            psi = rand_state(n, rng, name)
            G = W.haar_unitary(rng, 2 ** len(t))
            say("span", name, n, t, c)
            d = to_gpu(psi, name)
            q.qsv_apply_gate(d, t, c, G)
            close(to_np(d), orc.apply(psi, t, c, G), name, "span %s %s" % (t, c))


def test_identity_gates_are_bitexact_noops(q):
    rng = np.random.default_rng(72)
    for name in DTYPES:
        for n, t, c in [(1, (0,), ()), (7, (2, 5), ()), (7, (0,), (6,)), (12, (1, 4, 7, 9), ()),
                        (12, (0, 3, 5, 8, 11), ())]:
            psi = rand_state(n, rng, name)
            d = to_gpu(psi, name)
            before = raw_bits(d.cpu().numpy()).copy()
            say("identity", name, n, t, c)
            q.qsv_apply_gate(d, t, c, np.eye(2 ** len(t), dtype=np.complex128))
            assert np.array_equal(raw_bits(d.cpu().numpy()), before)


def test_non_unitary_matrices(q, orc):
    """eq. (1) is linear for any G: random complex and singular matrices on
    every kernel family (dense k <= 3, VALU k = 4, 5 and the matrix cores)."""
    import os
    rng = np.random.default_rng(73)
    proj = np.zeros((2, 2), np.complex128)
    proj[0, 0] = 1.0
    for name in DTYPES:
        n = 11
        psi = rand_state(n, rng, name)
        cases = [((3,), (), proj), ((0,), (), random_matrix(rng, 2)), ((9,), (2,), random_matrix(rng, 2)),
                 ((1, 8), (), random_matrix(rng, 4)), ((0, 5, 10), (), random_matrix(rng, 8)),
                 ((0, 1, 2, 3), (), random_matrix(rng, 16)), ((10, 2, 6, 4, 0), (), random_matrix(rng, 32))]
        for t, c, G in cases:
            for mfma in ["1", "0"]:
                os.environ["QSV_NO_MFMA"] = "0" if mfma == "1" else "1"
                say("non-unitary", name, t, c, mfma)
                d = to_gpu(psi, name)
                q.qsv_apply_gate(d, t, c, G)
                ref = orc.apply(psi, t, c, G)
                close(to_np(d), ref, name, "non-unitary %s" % (t,))
    os.environ.pop("QSV_NO_MFMA", None)


@pytest.mark.parametrize("k", [4, 5])
def test_mfma_single_tile(q, orc, k):
    """n = k + 6: the matrix-core launch has exactly one tile; n = k + 7: two."""
    rng = np.random.default_rng(74 + k)
    for name in DTYPES:
        for n in [k + 6, k + 7]:
            psi = rand_state(n, rng, name)
            for t in [tuple(range(k)), tuple(range(n - k, n)), tuple(int(v) for v in rng.choice(n, k, replace=False))]:
                G = W.haar_unitary(rng, 2 ** k)
                say("mfma tiles", name, n, t)
                d = to_gpu(psi, name)
                q.qsv_apply_gate(d, t, (), G)
                close(to_np(d), orc.apply(psi, t, (), G), name, "mfma n=%d %s" % (n, t))


def test_empty_and_noop_plans(q):
    import torch
    rng = np.random.default_rng(75)
    for name in DTYPES:
        dc = 1 if name == "c64" else 2
        n = 9
        psi = rand_state(n, rng, name)
        for circ in [W.Circuit(n, []),
                     W.Circuit(n, [W.Op("matrix", (3,), matrix=np.eye(2, dtype=np.complex128)),
                                   W.Op("matrix", (1, 7), matrix=np.eye(4, dtype=np.complex128))])]:
            for fuse in [1, 5]:
                say("empty plan", name, len(circ.ops), fuse)
                plan = q.Plan(circ, dc, fuse)
                d = to_gpu(psi, name)
                before = raw_bits(d.cpu().numpy()).copy()
                plan.run(d)
                torch.cuda.synchronize()
                assert np.array_equal(raw_bits(d.cpu().numpy()), before)


@pytest.mark.parametrize("n", [12, 13])
def test_pauli_identity_and_duplicate_terms(q, orc, n):
    """An identity term contributes c ||psi||^2, duplicated strings add, Y
    strings carry their phases; n = 12 is exactly one tile, n = 13 two."""
    rng = np.random.default_rng(76 + n)
    x = np.array([0, 0b101, 0b101, (1 << (n - 1)) | 1, 0b110, 0, 1 << 7], np.uint64)
    z = np.array([0, 0, 0, 1 << (n - 1), 0b110, 0b11, 1 << 3], np.uint64)
    c = np.array([0.7, -0.4, 0.25, 1.1, -0.6, 0.9, 0.3])
    H = W.PauliSum(n, x, z, c)
    scale = np.sum(np.abs(c))
    for name in DTYPES:
        psi = rand_state(n, rng, name)
        say("pauli edge", name, n)
        d = to_gpu(psi, name)
        e = q.qsv_expectation(d, H).cpu().numpy()
        ref = orc.expect(psi, H)
        assert abs(e[0] - ref.real) <= 1e-10 * scale, (e, ref)
        assert abs(e[1]) <= 1e-10 * scale
        out = to_gpu(np.zeros_like(psi), name)
        q.qsv_apply_pauli_sum(d, out, H)
        close(to_np(out) / scale, orc.apply_hamiltonian(psi, H) / scale, name, "H psi")


def test_forced_launch_failure_leaves_state_unchanged(q, monkeypatch):
    """QSV_TEST_FAIL_LAUNCH=1: gate, fused, plan, expectation and adjoint
    calls on real device buffers report QSV_ERR_HIP with the launch-failure
    message, enqueue nothing (the state keeps its bits), and work again once
    the variable is gone."""
    import torch
    n = 12
    rng = np.random.default_rng(5)
    for name in DTYPES:
        psi = to_gpu(rand_state(n, rng, name), name)
        before = psi.clone()
        G = W.haar_unitary(rng, 2)
        circ = W.random_u2_cz(n=n, depth=2, seed=3)
        plan = q.Plan(circ, 1 if name == "c64" else 2, 5)
        aplan = q.AdjointPlan(W.hea(n, 1), W.tfim_chain(n), 1 if name == "c64" else 2, 5)
        pdev = torch.zeros(2 * n, dtype=torch.float64, device="cuda")
        monkeypatch.setenv("QSV_TEST_FAIL_LAUNCH", "1")
        say("forced launch failure", name)
        calls = [lambda: q.qsv_apply_gate(psi, (3,), (), G),
                 lambda: q.qsv_apply_gate(psi, (0, 1, 2, 3, 4), (), W.haar_unitary(rng, 32)),
                 lambda: plan.run(psi),
                 lambda: q.qsv_expectation(psi, W.tfim_chain(n)),
                 lambda: q.qsv_norm2(psi),
                 lambda: aplan.run(pdev)]
        for call in calls:
            with pytest.raises(q.QsvError, match="QSV_TEST_FAIL_LAUNCH") as ei:
                call()
            assert ei.value.status == q.ERR_HIP
        torch.cuda.synchronize()
        assert torch.equal(torch.view_as_real(psi), torch.view_as_real(before))
        monkeypatch.delenv("QSV_TEST_FAIL_LAUNCH")
        q.qsv_apply_gate(psi, (3,), (), G)
        torch.cuda.synchronize()
        assert not torch.equal(torch.view_as_real(psi), torch.view_as_real(before))


def _device_to_host(ptr, nbytes):
    """Copy nbytes at a raw device pointer to the host (hipMemcpy, device to
    host), for buffers the library hands out as plain pointers."""
    import ctypes
    import torch
    torch.cuda.synchronize()
    try:
        hip = ctypes.CDLL("libamdhip64.so")
    except OSError:
        hip = ctypes.CDLL("/opt/rocm/lib/libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipMemcpy.restype = ctypes.c_int
    buf = np.empty(nbytes, dtype=np.uint8)
    assert hip.hipMemcpy(buf.ctypes.data, ptr, nbytes, 2) == 0
    return buf


def test_state_alloc_and_free(q, orc):
    """qsv_state_alloc / qsv_state_free (the allocation entry points for C
    callers): a basis state and a Hadamard on qubit 0 in the allocated
    buffer, read back and checked against the oracle; argument errors."""
    import ctypes
    import torch
    L = q.lib()
    n = 12
    H2 = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2)
    for name, code, npdt in (("c64", q.C64, np.complex64), ("c128", q.C128, np.complex128)):
        say("state alloc", name, n)
        p = ctypes.c_void_p()
        assert L.qsv_state_alloc(n, code, ctypes.byref(p)) == q.OK and p.value
        assert L.qsv_init_basis(p, n, code, 5, None) == q.OK
        tg = (ctypes.c_int * 1)(0)
        G = np.ascontiguousarray(H2)
        assert L.qsv_apply_gate(p, n, code, tg, 1, None, 0,
                                G.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None) == q.OK
        out = torch.empty(1, dtype=torch.float64, device="cuda")
        ws = q.reduce_workspace(out.device)
        assert L.qsv_norm2(p, n, code, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                           None) == q.OK
        got = _device_to_host(p.value, np.dtype(npdt).itemsize << n).view(npdt).astype(np.complex128)
        basis = np.zeros(1 << n, dtype=np.complex128)
        basis[5] = 1.0
        ref = orc.apply(basis, (0,), (), H2)
        close(got, ref, name, "allocated state")
        assert abs(float(out.cpu()[0]) - 1.0) < 1e-6
        assert L.qsv_state_free(p) == q.OK
    bad = ctypes.c_void_p()
    assert L.qsv_state_alloc(0, q.C64, ctypes.byref(bad)) == q.ERR_ARG
    assert L.qsv_state_alloc(12, 7, ctypes.byref(bad)) == q.ERR_ARG
    assert L.qsv_state_alloc(12, q.C64, None) == q.ERR_ARG
    assert L.qsv_state_free(None) == q.OK


def test_adjoint_state_slot(q, orc):
    """qsv_adjoint_state: after the forward sweep (qsv_adjoint_energy) slot 0
    of the workspace holds U(theta)|0>, equal to the oracle's circuit run;
    slots other than 0 and 1 are refused."""
    import ctypes
    import torch
    n, layers = 10, 3
    circ = W.hea(n, layers)
    H = W.tfim_chain(n)
    for name, code, npdt in (("c64", q.C64, np.complex64), ("c128", q.C128, np.complex128)):
        say("adjoint state slot", name, n)
        params = W.random_params(circ.nparams, 77)
        plan = q.AdjointPlan(circ, H, code, 5)
        pd = torch.from_numpy(params).to("cuda")
        e = plan.energy(pd)
        ptr = plan.state_ptr(0)
        got = _device_to_host(ptr, np.dtype(npdt).itemsize << n).view(npdt).astype(np.complex128)
        ref = orc.run(circ, params=params)
        close(got, ref, name, "adjoint slot 0")
        assert abs(float(e.cpu()[0]) - orc.expect(ref, H).real) <= 1e-5 * np.sum(np.abs(H.coeff))
        p = ctypes.c_void_p()
        assert q.lib().qsv_adjoint_state(plan.h, ctypes.c_void_p(plan.work.data_ptr()), 2,
                                         ctypes.byref(p)) == q.ERR_ARG
