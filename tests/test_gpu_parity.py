"""GPU parity of libqsv.so against the CPU oracle, through the C ABI.

Floating point: max |amplitude difference| <= 1e-12 (complex128) and
<= 1e-5 (complex64) against the complex128 oracle run on the same input
(for complex64 the input is the complex64 state widened exactly).
Permutation gates: bit-exact.  Expectation values: |dE| <= 1e-10 sum|c|.
"""
import itertools
import os

import numpy as np
import pytest

import workloads as W
from gpu_util import TOL, rand_state, raw_bits, say, to_gpu, to_np, torch_dtype

pytestmark = pytest.mark.gpu

DTYPES = ["c64", "c128"]
X2 = np.array([[0, 1], [1, 0]], np.complex128)
Z2 = np.array([[1, 0], [0, -1]], np.complex128)
SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], np.complex128)


@pytest.fixture(scope="module")
def q():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2202_07017_amd import qsv
    qsv.lib()
    return qsv


def check_close(got, ref, name, what=""):
    err = np.max(np.abs(got - ref)) if got.size else 0.0
    assert err <= TOL[name], "%s %s: max|d| = %.3e" % (what, name, err)


def gate_case(q, orc, psi, name, t, c, G):
    d = to_gpu(psi, name)
    q.qsv_apply_gate(d, t, c, G)
    got = to_np(d)
    ref = orc.apply(psi, t, c, G)
    check_close(got, ref, name, "t=%s c=%s" % (t, c))


def test_init_basis(q):
    import torch
    for name in DTYPES:
        for n in [1, 2, 5, 13]:
            for index in sorted({0, 1, (1 << n) - 1, (1 << n) // 3}):
                say("init_basis", name, n, index)
                d = torch.empty(1 << n, dtype=torch_dtype(name), device="cuda")
                d.fill_(complex(7, 7))
                q.qsv_init_basis(d, index)
                ref = np.zeros(1 << n, d.cpu().numpy().dtype)
                ref[index] = 1
                assert np.array_equal(raw_bits(d.cpu().numpy()), raw_bits(ref))


def test_init_random(q, orc):
    import torch
    for name in DTYPES:
        for n, seed in [(1, 3), (10, 5), (17, 1001)]:
            say("init_random", name, n, seed)
            d = torch.empty(1 << n, dtype=torch_dtype(name), device="cuda")
            q.qsv_init_random(d, seed)
            ref = orc.random_state(n, seed)
            got = to_np(d)
            rel = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
            assert rel <= (1e-14 if name == "c128" else 1e-7), rel


@pytest.mark.parametrize("n", [8, 9, 11])
def test_single_qubit_every_target(q, orc, n):
    """Uncontrolled single-qubit gates on every target at sizes with at least
    one block of 16-byte units (the lane-exchange sweep for low targets, the
    strided sweeps above), fixed matrices and device-side rotation angles, on
    one state and through the two-state path of a plan's rotations."""
    import torch
    rng = np.random.default_rng(40 + n)
    for name in DTYPES:
        psi = rand_state(n, rng, name)
        for t in range(n):
            G = W.haar_unitary(rng, 2)
            say("1q every target", name, n, t)
            gate_case(q, orc, psi, name, (t,), (), G)
        # rotations with device parameters: one RX, RY, RZ per qubit
        ops, npar = [], 0
        for t in range(n):
            for kind in ("rx", "ry", "rz"):
                ops.append(W.Op(kind, (t,), (), param=npar))
                npar += 1
        circ = W.Circuit(n, ops, npar)
        params = W.random_params(npar, 7)
        ref = orc.run(circ, params, psi0=psi)
        say("1q rotations every target", name, n)
        plan = q.Plan(circ, 1 if name == "c64" else 2, 1)
        d = to_gpu(psi, name)
        plan.run(d, torch.from_numpy(params).cuda())
        check_close(to_np(d), ref, name, "rotations")


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7])
def test_dense_gates_all_placements(q, orc, n):
    """Every (sampled) ordered placement of k <= 3 targets and c <= 2 controls."""
    rng = np.random.default_rng(100 + n)
    for name in DTYPES:
        psi = rand_state(n, rng, name)
        for k in range(1, min(n, 3) + 1):
            for c in range(0, min(n - k, 2) + 1):
                places = list(itertools.permutations(range(n), k + c))
                rng.shuffle(places)
                for qs in places[:24]:
                    say("dense", name, n, qs[:k], qs[k:])
                    gate_case(q, orc, psi, name, qs[:k], qs[k:], W.haar_unitary(rng, 2 ** k))


def test_permutations_bit_exact(q, orc):
    rng = np.random.default_rng(5)
    for name in DTYPES:
        for n in [1, 2, 3, 6, 9]:
            psi = rand_state(n, rng, name)
            psi[min(3, (1 << n) - 1)] = -0.0  # a signed zero must survive
            cases = [((j,), (), X2) for j in range(n)]
            if n >= 2:
                cases += [((1,), (0,), X2), ((0,), (n - 1,), X2), ((0, n - 1), (), SWAP),
                          ((n - 1, 0), (), SWAP)]
            if n >= 3:
                cases += [((2,), (0, 1), X2), ((0,), (1, 2), X2)]
                P = np.eye(8)[rng.permutation(8)].astype(np.complex128)
                cases += [((2, 0, 1), (), P), ((n - 1, 1, 0), (), P)]
            for t, c, G in cases:
                say("perm", name, n, t, c)
                d = to_gpu(psi, name)
                q.qsv_apply_gate(d, t, c, G)
                ref = orc.apply(psi, t, c, G).astype(np.complex64 if name == "c64" else np.complex128)
                assert np.array_equal(raw_bits(d.cpu().numpy()), raw_bits(ref)), (name, n, t, c)


def test_diagonal_gates(q, orc):
    rng = np.random.default_rng(6)
    for name in DTYPES:
        for n in [1, 2, 5, 9]:
            psi = rand_state(n, rng, name)
            cases = [((j,), (), Z2) for j in range(n)]
            cases += [((j,), (), np.diag(np.exp(1j * rng.uniform(0, 6, 2)))) for j in range(n)]
            if n >= 2:
                cases += [((1,), (0,), Z2), ((0,), (n - 1,), np.diag(np.exp([-0.3j, 0.3j]))),
                          ((0, n - 1), (), np.diag(np.exp(1j * rng.uniform(0, 6, 4)))),
                          ((n - 1, 0), (), np.diag([1, 1, 1, -1]).astype(np.complex128)),
                          ((0, 1), (), np.diag([1, 1j, 1, 1]).astype(np.complex128))]
            if n >= 5:
                cases += [((4, 0, 2), (1,), np.diag(np.exp(1j * rng.uniform(0, 6, 8))))]
            for t, c, G in cases:
                say("diag", name, n, t, c)
                gate_case(q, orc, psi, name, t, c, G)


@pytest.mark.parametrize("n", [10, 11, 12, 14])
def test_four_and_five_qubit_gates(q, orc, n):
    """k = 4, 5: matrix cores (uncontrolled, n >= k + 6) in both product
    forms (three real products, with the tiles per workgroup the host picks
    and forced to 1, 2 and 4, and one real-embedded product), and the VALU
    path."""
    rng = np.random.default_rng(200 + n)
    for name in DTYPES:
        psi = rand_state(n, rng, name)
        for k in [4, 5]:
            places = [tuple(range(k)), tuple(range(n - k, n)), tuple(reversed(range(k))),
                      (0, n - 1, 3, 7, 5)[:k], (1, 2, n - 1, 6, n - 3)[:k],
                      tuple(int(v) for v in rng.choice(n, k, replace=False))]
            for t in places:
                G = W.haar_unitary(rng, 2 ** k)
                for path in ["3m", "3m/1", "3m/2", "3m/4", "real", "valu"]:
                    os.environ["QSV_NO_MFMA"] = "1" if path == "valu" else "0"
                    os.environ["QSV_MFMA_FORM"] = path.split("/")[0]
                    if "/" in path:
                        os.environ["QSV_MFMA_TPB"] = path.split("/")[1]
                    say("k45", name, n, t, path)
                    gate_case(q, orc, psi, name, t, (), G)
                    os.environ.pop("QSV_MFMA_TPB", None)
                os.environ.pop("QSV_MFMA_FORM", None)
                ctl = [v for v in range(n) if v not in t][:1]
                say("k45 controlled", name, n, t, ctl)
                gate_case(q, orc, psi, name, t, tuple(ctl), G)
    os.environ.pop("QSV_NO_MFMA", None)
    os.environ.pop("QSV_MFMA_FORM", None)


@pytest.mark.parametrize("n", [10, 13])
def test_low_dense_gates_as_four_qubit_blocks(q, orc, n):
    """Dense 2- and 3-qubit gates with a target on the three lowest bits of
    the 16-byte unit index (complex128: qubits 0-2; complex64: qubits 1-3)
    run as G (x) I on the matrix cores; every target order, beside the
    vector-unit path, and sets that stay on the vector units."""
    rng = np.random.default_rng(250 + n)
    sets = [(0, 1), (0, n - 1), (1, 2), (3, 4), (2, n - 1), (4, 5), (0, 1, 2), (1, 2, n - 1),
            (0, 5, n - 1), (0, 2, 3), (2, 1, 4), (3, 6, 8)]
    for name in DTYPES:
        psi = rand_state(n, rng, name)
        for base in sets:
            for t in itertools.permutations(base):
                G = W.haar_unitary(rng, 2 ** len(t))
                for path in ["3m", "real", "valu"]:
                    os.environ["QSV_NO_MFMA"] = "1" if path == "valu" else "0"
                    os.environ["QSV_MFMA_FORM"] = path
                    say("low dense", name, n, t, path)
                    gate_case(q, orc, psi, name, t, (), G)
    os.environ.pop("QSV_NO_MFMA", None)
    os.environ.pop("QSV_MFMA_FORM", None)


def test_apply_fused(q, orc):
    rng = np.random.default_rng(8)
    for name in DTYPES:
        n = 13
        psi = rand_state(n, rng, name)
        blocks = []
        for k in [1, 2, 3, 4, 5, 5, 4, 2]:
            t = tuple(int(v) for v in rng.choice(n, k, replace=False))
            blocks.append((t, W.haar_unitary(rng, 2 ** k)))
        say("fused", name, [b[0] for b in blocks])
        d = to_gpu(psi, name)
        q.qsv_apply_fused(d, blocks)
        ref = psi
        for t, G in blocks:
            ref = orc.apply(ref, t, (), G)
        check_close(to_np(d), ref, name)


def test_observables(q, orc):
    rng = np.random.default_rng(9)
    for name in DTYPES:
        for n in [1, 3, 8, 12]:
            psi = rand_state(n, rng, name)
            d = to_gpu(psi, name)
            Hs = [W.random_pauli_sum(n, 11, seed=n), W.tfim_chain(n, 0.7)]
            if n >= 2:
                Hs.append(W.xxz_chain(n, 0.4))
            for H in Hs:
                say("expectation", name, n, len(H.coeff))
                e = q.qsv_expectation(d, H).cpu().numpy()
                ref = orc.expect(psi, H)
                scale = np.sum(np.abs(H.coeff))
                assert abs(e[0] - ref.real) <= 1e-10 * scale, (e, ref)
                assert abs(e[1]) <= 1e-10 * scale
                out = to_gpu(np.zeros_like(psi), name)
                q.qsv_apply_pauli_sum(d, out, H)
                check_close(to_np(out) / max(scale, 1), orc.apply_hamiltonian(psi, H) / max(scale, 1),
                            name, "H psi")
            say("norm/inner", name, n)
            nrm = q.qsv_norm2(d).cpu().numpy()[0]
            assert abs(nrm - orc.norm2(psi)) <= 1e-12
            phi = rand_state(n, rng, name)
            ip = q.qsv_inner(d, to_gpu(phi, name)).cpu().numpy()
            ref = orc.inner(psi, phi)
            assert abs(ip[0] - ref.real) <= 1e-12 and abs(ip[1] - ref.imag) <= 1e-12


@pytest.mark.parametrize("n", [13, 14, 17, 20])
def test_observables_tiled(q, orc, n):
    """n >= 12 runs the tiled passes: pass 0 on the low 12 qubits, further
    passes on high-qubit tiles, and the pair kernel for x masks wider than a
    tile (random Pauli strings)."""
    rng = np.random.default_rng(300 + n)
    for name in DTYPES:
        psi = rand_state(n, rng, name)
        d = to_gpu(psi, name)
        Hs = [W.tfim_chain(n, 0.9), W.xxz_chain(n, -0.6), W.random_pauli_sum(n, 40, seed=n),
              W.maxcut(n, [(0, n - 1), (3, 9), (n - 2, 1)])]
        for H in Hs:
            say("tiled expectation", name, n, len(H.coeff))
            e = q.qsv_expectation(d, H).cpu().numpy()
            ref = orc.expect(psi, H)
            scale = np.sum(np.abs(H.coeff))
            assert abs(e[0] - ref.real) <= 1e-10 * scale, (e, ref)
            assert abs(e[1]) <= 1e-10 * scale
            out = to_gpu(np.zeros_like(psi), name)
            q.qsv_apply_pauli_sum(d, out, H)
            check_close(to_np(out) / scale, orc.apply_hamiltonian(psi, H) / scale, name, "H psi")


def register_pass_sum(n, seed):
    """Pauli sums shaped for the register passes: diagonal strings anywhere,
    X/Y strings on one or two qubits >= 5 or on one or two of qubits 0..4 with
    random Z/Y factors elsewhere, plus terms the passes leave to the LDS tiles
    (three-qubit x masks, masks straddling qubits 4 and 5)."""
    rng = np.random.default_rng(seed)
    terms = [("", (), 0.3)]
    for _ in range(12):
        qs = [int(v) for v in rng.choice(n, int(rng.integers(1, 4)), replace=False)]
        terms.append(("Z" * len(qs), qs, float(rng.normal())))
    for lo in (False, True):
        for _ in range(10):
            pool = list(range(5)) if lo else list(range(5, n))
            xq = [int(v) for v in rng.choice(pool, int(rng.integers(1, 3)), replace=False)]
            letters = "".join(rng.choice(["X", "Y"]) for _ in xq)
            others = [v for v in range(n) if v not in xq]
            zq = [int(v) for v in rng.choice(others, int(rng.integers(0, 3)), replace=False)]
            terms.append((letters + "Z" * len(zq), xq + zq, float(rng.normal())))
    terms.append(("XXX", (1, 7, n - 1), 0.7))
    terms.append(("XY", (4, 5), -0.4))
    terms.append(("YZX", (0, 6, 9), 0.25))
    return W.pauli_sum(n, terms)


@pytest.mark.parametrize("n", [12, 15, 19])
def test_observables_register_passes(q, orc, n):
    """Expectation values through the register-tile passes (diagonal terms
    via the per-lane Walsh-Hadamard sums, strings on register qubits, strings
    on qubits 0..4 after the LDS transpose) and the LDS-tile fallback for the
    other terms, against the oracle; the imaginary part stays at rounding
    level (exactly 0 from the register passes)."""
    rng = np.random.default_rng(400 + n)
    for name in DTYPES:
        psi = rand_state(n, rng, name)
        d = to_gpu(psi, name)
        for seed in (1, 2, 3):
            H = register_pass_sum(n, 50 * n + seed)
            say("register-pass expectation", name, n, seed, len(H.coeff))
            e = q.qsv_expectation(d, H).cpu().numpy()
            ref = orc.expect(psi, H)
            scale = np.sum(np.abs(H.coeff))
            assert abs(e[0] - ref.real) <= 1e-10 * scale, (e, ref)
            assert abs(e[1]) <= 1e-10 * scale
            e2 = q.qsv_expectation_noalloc(d, H).cpu().numpy()
            assert np.array_equal(e, e2)


@pytest.mark.parametrize("n", [13, 19])
def test_observables_register_many_terms(q, orc, n):
    """A single X on every qubit (several register sets, the transposed set
    for qubits 0..4) with more diagonal strings than one register launch
    holds (48): Z on every qubit, every neighbouring ZZ, 30 random Z triples
    and the identity, so the diagonal terms split over launches and several
    register masks carry more than one five-term sign-table chunk."""
    rng = np.random.default_rng(900 + n)
    terms = [("", (), 0.5)]
    terms += [("X", (j,), float(rng.normal())) for j in range(n)]
    terms += [("Z", (j,), float(rng.normal())) for j in range(n)]
    terms += [("ZZ", (j, j + 1), float(rng.normal())) for j in range(n - 1)]
    for _ in range(30):
        qs = [int(v) for v in rng.choice(n, 3, replace=False)]
        terms.append(("ZZZ", qs, float(rng.normal())))
    H = W.pauli_sum(n, terms)
    assert q.expectation_launches(H, n, q.C64) >= 3
    for name in DTYPES:
        psi = rand_state(n, rng, name)
        d = to_gpu(psi, name)
        say("register-pass expectation, many terms", name, n, len(H.coeff))
        e = q.qsv_expectation(d, H).cpu().numpy()
        ref = orc.expect(psi, H)
        scale = np.sum(np.abs(H.coeff))
        assert abs(e[0] - ref.real) <= 1e-10 * scale, (e, ref)
        assert abs(e[1]) <= 1e-10 * scale


@pytest.mark.parametrize("n", [12, 16, 20])
def test_observables_span_passes(q, orc, n, monkeypatch):
    """Strings with arbitrary x masks (random strings, 70 strings on one
    mask, XORs of earlier masks, strings on qubits 0..5, diagonal strings, a
    Y on the top qubit), an XXZ chain and a Heisenberg chain with fields, at
    n = 12 (two tiles per span pass), 16 and 20:
    the default plan, the register-pass plans (QSV_EXPECT_PLAN=reg), span
    passes alone (=span) and one pass per x mask (QSV_NO_SPAN_PASS=1), each
    against the oracle."""
    from test_span_plan import span_sum
    rng = np.random.default_rng(1500 + n)
    heis = [(ab, (j, j + 1), 1.0) for j in range(n - 1) for ab in ("XX", "YY", "ZZ")]
    heis += [(c, (j,), float(rng.normal())) for j in range(n) for c in "XYZ"]
    models = [("span_sum", span_sum(n, 700 + n)), ("xxz", W.xxz_chain(n, 0.5)),
              ("heisenberg_fields", W.pauli_sum(n, heis))]
    variants = [("default", None, None), ("reg", "QSV_EXPECT_PLAN", "reg"), ("span", "QSV_EXPECT_PLAN", "span"),
                ("per-mask", "QSV_NO_SPAN_PASS", "1")]
    for mname, H in models:
        scale = np.sum(np.abs(H.coeff))
        counts = {}
        for vname, var, val in variants:
            if var:
                monkeypatch.setenv(var, val)
            counts[vname] = q.expectation_launches(H, n, q.C64)
            if var:
                monkeypatch.delenv(var)
        if mname == "span_sum" and n >= 16:  # at n = 12 every string fits a 12-qubit tile
            assert counts["default"] < counts["per-mask"], counts
        for name in DTYPES:
            psi = rand_state(n, rng, name)
            d = to_gpu(psi, name)
            ref = orc.expect(psi, H)
            for vname, var, val in variants:
                if var:
                    monkeypatch.setenv(var, val)
                say("expectation plans", mname, name, n, vname, "launches", counts[vname])
                e = q.qsv_expectation(d, H).cpu().numpy()
                if var:
                    monkeypatch.delenv(var)
                assert abs(e[0] - ref.real) <= 1e-10 * scale, (mname, vname, e, ref)
                assert abs(e[1]) <= 1e-10 * scale


def test_plan_random_circuit(q, orc):
    """Random U(2) layers with CZ pairs (n = 20, depth 10): every fusion width
    and graph replay against the oracle, plus <Z_0>."""
    import torch
    circ = W.random_u2_cz(n=20, depth=10, seed=1000)
    ref = orc.run(circ)
    Z0 = W.pauli_sum(20, [("Z", (0,), 1.0)])
    ez = orc.expect(ref, Z0).real
    for name in DTYPES:
        for fuse in [1, 2, 3, 5]:
            say("plan u2cz", name, "fuse", fuse)
            plan = q.Plan(circ, 1 if name == "c64" else 2, fuse)
            d = torch.empty(1 << 20, dtype=torch_dtype(name), device="cuda")
            outs = []
            for rep in range(2):
                q.qsv_init_basis(d, 0)
                plan.run(d)
                outs.append(d.clone())
            assert torch.equal(outs[0], outs[1]), "graph replay differs from capture run"
            check_close(to_np(d), ref, name, "fuse=%d" % fuse)
            e = q.qsv_expectation(d, Z0).cpu().numpy()[0]
            assert abs(e - ez) <= (1e-12 if name == "c128" else 1e-5)


def test_plan_rotations_and_pairs(q, orc):
    """Random pairs circuit (CNOT/CZ/CRZ) and the ansatz with device-side
    rotation angles (unbound) or host-bound angles (fused)."""
    import torch
    circ, params = W.random_u2_pairs(n=12, depth=6, seed=1001)
    ref = orc.run(circ, params)
    hea = W.hea(9, 3)
    hp = W.random_params(hea.nparams, 3)
    href = orc.run(hea, hp)
    for name in DTYPES:
        dc = 1 if name == "c64" else 2
        pd = torch.from_numpy(params).cuda()
        for fuse, bound in [(1, False), (5, False), (5, True), (3, True)]:
            say("plan pairs", name, fuse, bound)
            plan = q.Plan(circ, dc, fuse, params if bound else None)
            d = torch.empty(1 << 12, dtype=torch_dtype(name), device="cuda")
            q.qsv_init_basis(d, 0)
            plan.run(d, pd)
            check_close(to_np(d), ref, name)
            say("plan hea", name, fuse, bound)
            plan = q.Plan(hea, dc, fuse, hp if bound else None)
            d = torch.empty(1 << 9, dtype=torch_dtype(name), device="cuda")
            q.qsv_init_basis(d, 0)
            plan.run(d, torch.from_numpy(hp).cuda())
            check_close(to_np(d), href, name)


def test_adjoint_gradient(q, orc):
    import torch
    cases = [(W.hea(6, 3), W.tfim_chain(6)), (W.hea(11, 2), W.tfim_chain(11))]
    # controlled rotation, RX, shared parameter, fixed gates, Y terms
    c = W.Circuit(5, [W.Op("h", (0,)), W.Op("rx", (1,), param=0), W.Op("ry", (2,), param=1),
                      W.Op("rz", (3,), controls=(0,), param=2), W.Op("x", (4,), controls=(2,)),
                      W.Op("rx", (4,), param=0), W.Op("matrix", (1, 3), matrix=W.haar_unitary(
                          np.random.default_rng(1), 4)), W.Op("ry", (0,), controls=(1, 2), param=3),
                      W.Op("rz", (0,), param=1)], 4)
    cases.append((c, W.pauli_sum(5, [("XY", (0, 1), 0.7), ("ZZ", (2, 4), -1.1), ("Y", (3,), 0.4),
                                     ("X", (4,), 0.9)])))
    for circ, H in cases:
        p = W.random_params(circ.nparams, 17)
        E_ref, g_ref = orc.adjoint(circ, p, H)
        g_fd = orc.grad_finite_diff(circ, p, H)
        assert np.max(np.abs(g_fd - g_ref)) < 1e-6
        for name in DTYPES:
            for fuse in [1, 5]:
                say("adjoint", name, circ.n, circ.nparams, fuse)
                plan = q.AdjointPlan(circ, H, 1 if name == "c64" else 2, fuse)
                pd = torch.from_numpy(p).cuda()
                e, g = plan.run(pd)
                e, g = e.cpu().numpy()[0], g.cpu().numpy()
                if name == "c128":
                    assert abs(e - E_ref) < 1e-11
                    assert np.max(np.abs(g - g_ref)) < 1e-10
                    assert np.max(np.abs(g - g_fd)) < 1e-6
                else:
                    assert abs(e - E_ref) < 1e-4
                    assert np.max(np.abs(g - g_ref)) < 1e-4
                e2, g2 = plan.run(pd)  # graph replay, identical
                assert e2.cpu().numpy()[0] == e and np.array_equal(g2.cpu().numpy(), g)
                en = plan.energy(pd).cpu().numpy()[0]
                assert abs(en - E_ref) < (1e-11 if name == "c128" else 1e-4)


def every_form_circuit(n, ngates, seed):
    """Single-target gates of every matrix form the tile executor specialises
    (real: H, RY; swap: X; imaginary off-diagonal: Y, RX; real diagonal: Z;
    complex diagonal: S, T, RZ; general: Haar U(2)), each with 0, 1 or 2
    controls on random qubits, rotations sharing some parameters."""
    rng = np.random.default_rng(seed)
    s = np.diag([1, 1j]).astype(complex)
    t = np.diag([1, np.exp(0.25j * np.pi)]).astype(complex)
    ops, npar = [], 0
    for _ in range(ngates):
        kind = ["h", "x", "y", "z", "s", "t", "u", "rx", "ry", "rz"][rng.integers(10)]
        q = [int(v) for v in rng.choice(n, 1 + int(rng.integers(3)), replace=False)]
        tq, cs = (q[0],), tuple(q[1:])
        if kind in ("rx", "ry", "rz"):
            share = npar > 0 and rng.random() < 0.2
            ops.append(W.Op(kind, tq, controls=cs, param=int(rng.integers(npar)) if share else npar))
            npar += 0 if share else 1
        elif kind in ("s", "t", "u"):
            m = {"s": s, "t": t}.get(kind)
            ops.append(W.Op("matrix", tq, controls=cs, matrix=m if m is not None else W.haar_unitary(rng, 2)))
        else:
            ops.append(W.Op(kind, tq, controls=cs))
    return W.Circuit(n, ops, npar)


@pytest.mark.parametrize("n", [13, 15])
def test_adjoint_tiled_every_form(q, orc, n):
    """Cache-blocked adjoint over several tiles with gates of every form and
    control count, against the oracle's adjoint."""
    import torch
    circ = every_form_circuit(n, 160, 300 + n)
    H = W.random_pauli_sum(n, 12, seed=n)
    p = W.random_params(circ.nparams, 31 + n)
    E_ref, g_ref = orc.adjoint(circ, p, H)
    for name in DTYPES:
        say("adjoint every form", name, n, len(circ.ops), circ.nparams)
        plan = q.AdjointPlan(circ, H, 1 if name == "c64" else 2, 5)
        e, g = plan.run(torch.from_numpy(p).cuda())
        e, g = e.cpu().numpy()[0], g.cpu().numpy()
        scale = float(np.sum(np.abs(H.coeff)))
        tol = (1e-10 * scale, 1e-9 * scale) if name == "c128" else (2e-7 * scale, 2e-7 * scale)
        say("  |dE| %.3e  max|dgrad| %.3e  (sum|c| %.2f)" % (abs(e - E_ref), np.max(np.abs(g - g_ref)), scale))
        assert abs(e - E_ref) < tol[0], (e, E_ref)
        assert np.max(np.abs(g - g_ref)) < tol[1], np.max(np.abs(g - g_ref))


@pytest.mark.parametrize("n", [14, 16])
def test_adjoint_tiled_multi_tile(q, orc, n):
    """Cache-blocked adjoint (several tiles per pass, staircase passes) and the
    per-gate adjoint (QSV_NO_TILES=1) against the oracle's adjoint."""
    import torch
    circ, H = W.hea(n, 3), W.tfim_chain(n)
    circ.ops.insert(5, W.Op("rx", (n - 1,), controls=(2,), param=1))
    p = W.random_params(circ.nparams, 19 + n)
    E_ref, g_ref = orc.adjoint(circ, p, H)
    for name in DTYPES:
        for tiles in ["1", "0"]:
            os.environ["QSV_NO_TILES"] = "0" if tiles == "1" else "1"
            try:
                say("adjoint tiled" if tiles == "1" else "adjoint per-gate", name, n)
                plan = q.AdjointPlan(circ, H, 1 if name == "c64" else 2, 5)
            finally:
                os.environ.pop("QSV_NO_TILES", None)
            e, g = plan.run(torch.from_numpy(p).cuda())
            e, g = e.cpu().numpy()[0], g.cpu().numpy()
            scale = float(np.sum(np.abs(H.coeff)))
            # complex64 sweeps with FP64 accumulation: 1e-7 per unit of sum|c|
            tol = (1e-10, 1e-9) if name == "c128" else (1e-7 * scale, 1e-7 * scale)
            say("  |dE| %.3e  max|dgrad| %.3e" % (abs(e - E_ref), np.max(np.abs(g - g_ref))))
            assert abs(e - E_ref) < tol[0], (e, E_ref)
            assert np.max(np.abs(g - g_ref)) < tol[1], np.max(np.abs(g - g_ref))


def test_adjoint_autograd(q, orc):
    import torch
    circ, H = W.hea(5, 2), W.tfim_chain(5)
    p = W.random_params(circ.nparams, 4)
    plan = q.AdjointPlan(circ, H, 2, 5)
    theta = torch.tensor(p, device="cuda", requires_grad=True)
    say("autograd")
    E = q.adjoint_energy(theta, plan)
    (2.0 * E).backward()
    _, g_ref = orc.adjoint(circ, p, H)
    assert np.max(np.abs(theta.grad.cpu().numpy() - 2.0 * g_ref)) < 1e-10


def test_full_size_sampled(q, orc):
    """n = 30 (8 GiB complex64, 16 GiB complex128): each gate applied to the
    seeded random state, 96 output amplitudes compared with the oracle
    evaluated one by one on the same seeded input."""
    import torch
    n, seed = 30, 4242
    scale = 1.0 / np.sqrt(orc.random_norm2(n, seed))
    rng = np.random.default_rng(77)
    idx = np.concatenate([rng.integers(0, 1 << n, 90), [0, 1, (1 << n) - 1, (1 << n) - 2,
                                                       1 << 29, (1 << 29) - 1]]).astype(np.uint64)
    gates = [((t,), ()) for t in [0, 1, 2, 7, 15, 28, 29]]
    gates += [((0, 29), ()), ((3, 1), ()), ((29, 17), ()), ((0, 1, 2), ()), ((2, 28, 14), ()),
              ((29,), (0,)), ((0,), (29,)), ((5,), (3,)), ((0, 1, 2, 3, 4), ()),
              ((25, 26, 27, 28, 29), ()), ((0, 29, 9, 3, 20), ())]
    for name in DTYPES:
        d = torch.empty(1 << n, dtype=torch_dtype(name), device="cuda")
        for t, c in gates:
            G = W.haar_unitary(rng, 2 ** len(t))
            say("n30", name, t, c)
            q.qsv_init_random(d, seed)
            q.qsv_apply_gate(d, t, c, G)
            got = d[torch.from_numpy(idx.astype(np.int64)).cuda()].cpu().numpy().astype(np.complex128)
            ref = orc.apply_sampled_random(n, seed, scale, t, c, G, idx)
            err = np.max(np.abs(got - ref))
            assert err <= TOL[name] and err / np.max(np.abs(ref)) <= 1e-5, (name, t, c, err)
        # permutations at full size: out[i] == in[pi(i)] bit for bit
        for t, c in [((29,), ()), ((0,), ()), ((29,), (0,))]:
            say("n30 perm", name, t, c)
            q.qsv_init_random(d, seed)
            before = d[torch.from_numpy(idx.astype(np.int64)).cuda()].clone()
            q.qsv_apply_gate(d, t, c, X2)
            cm = sum(1 << v for v in c)
            src = np.where((idx & np.uint64(cm)) == np.uint64(cm), idx ^ np.uint64(1 << t[0]), idx)
            after = d[torch.from_numpy(src.astype(np.int64)).cuda()]
            assert torch.equal(torch.view_as_real(after), torch.view_as_real(before))
        norm = q.qsv_norm2(d).cpu().numpy()[0]
        assert abs(norm - 1.0) < (1e-12 if name == "c128" else 1e-5)
        del d
        torch.cuda.empty_cache()


def inverse_circuit(circ, params=None):
    """The circuit's inverse as data: ops reversed, every matrix daggered,
    rotations bound to -theta (a property check that holds at any size)."""
    ops = []
    for op in reversed(circ.ops):
        if op.kind == "matrix":
            ops.append(W.Op("matrix", op.targets, op.controls, matrix=op.matrix.conj().T))
        elif op.kind in ("rx", "ry", "rz"):
            ops.append(W.Op(op.kind, op.targets, op.controls, param=op.param))
        else:  # h, x, y, z, swap are their own inverses
            ops.append(W.Op(op.kind, op.targets, op.controls))
    inv = W.Circuit(circ.n, ops, circ.nparams)
    return inv, (None if params is None else -np.asarray(params))


@pytest.mark.parametrize("which", ["pairs28", "dense32"])
def test_full_size_fused_round_trip(q, orc, which):
    """Full workload sizes: the random-pairs circuit at n = 28 (fused up to 5
    qubits) and the random 1-3-qubit circuit at n = 32 (fused to 5-qubit MFMA
    blocks), each followed by its inverse, must return the seeded input; the
    result is checked amplitude by amplitude against the oracle's values of
    the seeded state at sampled indices, and the norm is checked too."""
    import torch
    if which == "pairs28":
        circ, params = W.random_u2_pairs(n=28, depth=20, seed=1001)
    else:
        circ, params = W.random_dense_123(n=32, depth=12, seed=1002), None
    inv, iparams = inverse_circuit(circ, params)
    n, seed = circ.n, 77
    scale = 1.0 / np.sqrt(orc.random_norm2(n, seed))
    rng = np.random.default_rng(5)
    idx = np.concatenate([rng.integers(0, 1 << n, 200), [0, (1 << n) - 1]]).astype(np.uint64)
    ref = orc.random_amps(seed, scale, idx)
    rms = 1.0 / np.sqrt(float(1 << n))  # typical |amplitude|
    for name in DTYPES:
        for fuse in [5, 3]:
            say("round trip", which, name, "fuse", fuse)
            dc = 1 if name == "c64" else 2
            fwd = q.Plan(circ, dc, fuse, params)
            bwd = q.Plan(inv, dc, fuse, iparams)
            d = torch.empty(1 << n, dtype=torch_dtype(name), device="cuda")
            q.qsv_init_random(d, seed)
            fwd.run(d)
            mid = q.qsv_norm2(d).cpu().numpy()[0]
            bwd.run(d)
            got = d[torch.from_numpy(idx.astype(np.int64)).cuda()].cpu().numpy().astype(np.complex128)
            err = np.max(np.abs(got - ref))
            # a few hundred gate applications: rounding grows like sqrt(#ops)
            # times the unit roundoff, relative to the typical amplitude
            tol = (1e-10 if name == "c128" else 1e-4) * rms
            assert abs(mid - 1.0) < (1e-12 if name == "c128" else 1e-4), mid
            assert err <= tol, (which, name, fuse, err)
            del d, fwd, bwd
            torch.cuda.empty_cache()


def test_n32_sampled(q, orc):
    """n = 32 (32 GiB complex64, 64 GiB complex128): single gates at low and
    high targets, a controlled gate and a 5-qubit MFMA block, sampled against
    the oracle evaluated one output at a time on the same seeded input."""
    import torch
    n, seed = 32, 4243
    scale = 1.0 / np.sqrt(orc.random_norm2(n, seed))
    rng = np.random.default_rng(78)
    idx = np.concatenate([rng.integers(0, 1 << n, 60), [0, (1 << n) - 1, 1 << 31, (1 << 31) - 1,
                                                       (1 << 32) - 2]]).astype(np.uint64)
    gates = [((0,), ()), ((31,), ()), ((30, 1), ()), ((31,), (0,)), ((0, 1, 2, 3, 4), ()),
             ((27, 28, 29, 30, 31), ()), ((0, 31, 16, 8, 24), ())]
    for name in DTYPES:
        d = torch.empty(1 << n, dtype=torch_dtype(name), device="cuda")
        for t, c in gates:
            G = W.haar_unitary(rng, 2 ** len(t))
            say("n32", name, t, c)
            q.qsv_init_random(d, seed)
            q.qsv_apply_gate(d, t, c, G)
            got = d[torch.from_numpy(idx.astype(np.int64)).cuda()].cpu().numpy().astype(np.complex128)
            ref = orc.apply_sampled_random(n, seed, scale, t, c, G, idx)
            err = np.max(np.abs(got - ref))
            assert err <= TOL[name] and err / np.max(np.abs(ref)) <= 1e-5, (name, t, c, err)
        del d
        torch.cuda.empty_cache()
