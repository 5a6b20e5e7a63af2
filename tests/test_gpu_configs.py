"""The seeded workload configurations at their full sizes, checked against the
CPU oracle (never against the GPU itself), through the C ABI.

* Random-pairs circuit, n = 28, depth 20 (Haar U(2) layers, CNOT/CZ/CRZ on a
  random matching): the whole final state, element by element, against the
  oracle's run of the same circuit on the same seeded input, unfused and
  fused to k = 2..5, complex64 and complex128.
* Random 1-3-qubit circuit, fused to k = 5 at n = 32: the input is a product
  phi (x) psi, psi a seeded 28-qubit state and phi a fixed state of 4 free
  qubits (the top four, or four in the middle), and the circuit acts on the
  other 28 qubits; every slice of the 32-qubit result must equal phi_j times
  the 28-qubit oracle result, and slices with phi_j = 0 must stay exactly 0.
  This exercises the 64-bit paths of 32-qubit states with low and high
  targets while the oracle runs at 28 qubits.
* Hardware-efficient ansatz, L = 8, n = 20: complex128 adjoint gradient (plan,
  one-shot call and autograd) against the oracle's adjoint (full vector), and
  against oracle central finite differences (h = 1e-6) and parameter shift
  on a seeded 16-parameter subset; n = 26 against the oracle's adjoint (full
  vector).  Complex64 errors against the oracle are printed and bounded.
* Batched workload (1024 instances): every instance with n <= 16 and 32
  seeded larger ones (n = 21 and n = 22 included) against the oracle's adjoint.
* Expectation values at n = 30 (the bench step's size): a product state
  built on the GPU, TFIM, XXZ, a Heisenberg chain with fields and random
  1-3-qubit strings, against the product-state closed form (pinned against
  the oracle in tests/test_product_formula.py).

Floating-point bars: complex128 max|d psi| and ||d psi||_2 <= 1e-12,
complex64 <= 1e-5 (both against the complex128 oracle); energies and
gradients as stated per test.  Every error is printed with its case.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import say, torch_dtype

pytestmark = pytest.mark.gpu

DTYPES = ["c64", "c128"]
CODE = {"c64": 1, "c128": 2}
TOL = {"c128": 1e-12, "c64": 1e-5}


@pytest.fixture(scope="module")
def q():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2202_07017_amd import qsv
    qsv.lib()
    return qsv


def diff_stats(got, ref_dev, scale=1.0):
    """(max |got - scale ref|, ||got - scale ref||_2) computed on the GPU in
    complex128 (ref_dev: the oracle's result uploaded once)."""
    import torch
    d = got.to(torch.complex128) - scale * ref_dev if scale != 1.0 else got.to(torch.complex128) - ref_dev
    return float(d.abs().max()), float(torch.linalg.vector_norm(d))


# ------------------------------------------------------------ n = 28 pairs

@pytest.fixture(scope="module")
def pairs28(orc):
    import torch
    circ, params = W.random_u2_pairs(n=28, depth=20, seed=1001)
    seed = 1001
    say("oracle: random-pairs circuit n=28 depth 20 (%d gates)" % len(circ.ops))
    ref = orc.run(circ, params, psi0=orc.random_state(28, seed))
    ref_dev = torch.from_numpy(ref).cuda()
    del ref
    return circ, params, seed, ref_dev


@pytest.mark.parametrize("name", DTYPES)
def test_pairs28_full_state_vs_oracle(q, pairs28, name):
    import torch
    circ, params, seed, ref_dev = pairs28
    pdev = torch.from_numpy(params).cuda()
    d = torch.empty(1 << 28, dtype=torch_dtype(name), device="cuda")
    for fuse in [1, 2, 3, 4, 5]:
        for bound in ([False, True] if fuse == 1 else [True]):
            plan = q.Plan(circ, CODE[name], fuse, params if bound else None)
            q.qsv_init_random(d, seed)
            plan.run(d, None if bound else pdev)
            mx, l2 = diff_stats(d, ref_dev)
            say("pairs28", name, "fuse", fuse, "bound" if bound else "device angles",
                "max|d| %.3e  ||d||_2 %.3e" % (mx, l2))
            assert mx <= TOL[name] and l2 <= TOL[name], (name, fuse, bound, mx, l2)
            del plan
    del d
    torch.cuda.empty_cache()


# ------------------------------------------------------ n = 32 product slices

PHI = {1: 0.5, 6: -0.5, 11: 0.5j, 12: -0.5j}  # 4 free qubits: 16 slices, |phi| = 1


@pytest.fixture(scope="module")
def dense28(orc):
    import torch
    circ = W.random_dense_123(n=28, depth=12, seed=1002)
    seed = 1002
    say("oracle: random 1-3-qubit circuit n=28 depth 12 (%d gates)" % len(circ.ops))
    ref = orc.run(circ, psi0=orc.random_state(28, seed))
    ref_dev = torch.from_numpy(ref).cuda()
    del ref
    return circ, seed, ref_dev


def remap(circ, n, f):
    ops = [W.Op(op.kind, tuple(f(t) for t in op.targets), tuple(f(c) for c in op.controls),
                op.param, op.matrix) for op in circ.ops]
    return W.Circuit(n, ops, circ.nparams)


@pytest.mark.parametrize("where", ["top", "middle"])
@pytest.mark.parametrize("name", DTYPES)
def test_dense32_product_slices_vs_oracle(q, dense28, name, where):
    """32-qubit state (32 GiB complex64 / 64 GiB complex128), circuit on 28
    qubits fused to 5-qubit blocks (matrix cores) and to 3-qubit blocks."""
    import torch
    circ28, seed, ref_dev = dense28
    if where == "top":        # free qubits 28..31, circuit on 0..27
        f = lambda t: t
    else:                     # free qubits 14..17, circuit on 0..13 and 18..31
        f = lambda t: t if t < 14 else t + 4
    circ = remap(circ28, 32, f)
    x28 = torch.empty(1 << 28, dtype=torch_dtype(name), device="cuda")
    q.qsv_init_random(x28, seed)
    x = torch.zeros(1 << 32, dtype=torch_dtype(name), device="cuda")

    def slices(v):
        if where == "top":
            return [v[j << 28:(j + 1) << 28] for j in range(16)]
        w = v.view(1 << 14, 16, 1 << 14)
        return [w[:, j, :] for j in range(16)]

    for fuse in [5, 3]:
        x.zero_()
        src = x28 if where == "top" else x28.view(1 << 14, 1 << 14)
        for j, ph in PHI.items():
            slices(x)[j].copy_(src * ph)
        plan = q.Plan(circ, CODE[name], fuse)
        plan.run(x)
        torch.cuda.synchronize()
        worst = (0.0, 0.0)
        for j, s in enumerate(slices(x)):
            if j in PHI:
                s = s.reshape(-1)
                mx, l2 = diff_stats(s, ref_dev, PHI[j])
                worst = (max(worst[0], mx), max(worst[1], l2))
                assert mx <= TOL[name] and l2 <= TOL[name], (name, where, fuse, j, mx, l2)
            else:
                assert bool((s == 0).all()), (name, where, fuse, j, "slice must stay zero")
        say("dense32", where, name, "fuse", fuse, "worst slice max|d| %.3e  ||d||_2 %.3e" % worst)
        del plan
    del x, x28
    torch.cuda.empty_cache()


# ------------------------------------------------------------------ HEA L = 8

def sub_params(P, seed, count=16):
    return np.sort(np.random.default_rng(seed).choice(P, size=count, replace=False))


@pytest.fixture(scope="module")
def hea20(orc):
    circ, H = W.hea(20, 8), W.tfim_chain(20)
    p = W.random_params(circ.nparams, 1003)
    say("oracle: HEA n=20 L=8 adjoint, finite differences and parameter shift on 16 parameters")
    E, g = orc.adjoint(circ, p, H)
    sub = sub_params(circ.nparams, 20)
    fd = orc.grad_finite_diff(circ, p, H, which=list(sub), h=1e-6)
    ps = orc.grad_param_shift(circ, p, H, which=list(sub))
    return circ, H, p, E, g, sub, fd, ps


def test_hea20_oracle_references_agree(hea20):
    """The three oracle gradients agree with each other (finite differences to
    O(h^2) + roundoff/h, parameter shift exactly)."""
    circ, H, p, E, g, sub, fd, ps = hea20
    assert np.max(np.abs(fd - g[sub])) <= 1e-7
    assert np.max(np.abs(ps - g[sub])) <= 1e-11


def test_hea20_adjoint_vs_oracle(q, hea20):
    import torch
    circ, H, p, E, g, sub, fd, ps = hea20
    scale = float(np.sum(np.abs(H.coeff)))  # 39
    pdev = torch.from_numpy(p).cuda()
    for name in DTYPES:
        plan = q.AdjointPlan(circ, H, CODE[name], 5)
        e, gg = plan.run(pdev)
        e, gg = float(e.cpu()[0]), gg.cpu().numpy()
        de, dg = abs(e - E), float(np.max(np.abs(gg - g)))
        say("hea20", name, "|dE| %.3e  max|dgrad| %.3e (vs oracle adjoint)" % (de, dg),
            "max|grad - FD| %.3e  max|grad - PS| %.3e" % (np.max(np.abs(gg[sub] - fd)),
                                                          np.max(np.abs(gg[sub] - ps))))
        if name == "c128":
            assert de <= 1e-10 * scale and dg <= 1e-10, (de, dg)
            assert np.max(np.abs(gg[sub] - fd)) <= 1e-6
            assert np.max(np.abs(gg[sub] - ps)) <= 1e-9
        else:
            # complex64 sweeps, FP64 accumulation: errors stated against the
            # complex128 oracle; bound 1e-7 per unit of sum|c|
            assert de <= 1e-7 * scale and dg <= 1e-7 * scale, (de, dg)
        # energy alone (forward sweep only)
        en = plan.energy(pdev)
        assert abs(float(en.cpu()[0]) - e) <= (1e-12 if name == "c128" else 1e-6) * scale


def test_hea20_one_shot_and_autograd(q, hea20):
    """qsv_adjoint_gradient (one call: plan, run, release) and the autograd
    function; energy only (no reverse sweep) without a gradient to record."""
    import torch
    circ, H, p, E, g, sub, fd, ps = hea20
    pdev = torch.from_numpy(p).cuda()
    for fuse in [5, 2]:
        wb = q.adjoint_work_bytes(circ, H, 2, fuse)
        work = torch.empty((wb + 255) // 256 * 32, dtype=torch.float64, device="cuda")
        en = torch.empty(1, dtype=torch.float64, device="cuda")
        gr = torch.empty(circ.nparams, dtype=torch.float64, device="cuda")
        say("one-shot adjoint n20 fuse", fuse, "work", wb)
        q.adjoint_gradient(circ, pdev, H, 2, fuse, work, en, gr)
        assert abs(float(en.cpu()[0]) - E) <= 1e-10 * 39
        assert np.max(np.abs(gr.cpu().numpy() - g)) <= 1e-10
        small = work[:max(wb // 8 - 64, 1)]
        with pytest.raises(q.QsvError, match="needs"):
            q.adjoint_gradient(circ, pdev, H, 2, fuse, small, en, gr)
    plan = q.AdjointPlan(circ, H, 2, 5)
    theta = pdev.clone().requires_grad_(True)
    Et = q.adjoint_energy(theta, plan)
    (3.0 * Et).backward()
    assert abs(float(Et.detach().cpu()) - E) <= 1e-10 * 39
    assert np.max(np.abs(theta.grad.cpu().numpy() - 3.0 * g)) <= 3e-10
    with torch.no_grad():
        E0 = q.adjoint_energy(theta, plan)
    assert abs(float(E0.cpu()) - E) <= 1e-10 * 39
    assert not E0.requires_grad


@pytest.fixture(scope="module")
def hea26(orc):
    circ, H = W.hea(26, 8), W.tfim_chain(26)
    p = W.random_params(circ.nparams, 1003)
    say("oracle: HEA n=26 L=8 adjoint (full vector, %d parameters)" % circ.nparams)
    E, g = orc.adjoint(circ, p, H)
    return circ, H, p, E, g


def test_hea26_adjoint_vs_oracle(q, hea26):
    import torch
    circ, H, p, E, g = hea26
    scale = float(np.sum(np.abs(H.coeff)))  # 51
    pdev = torch.from_numpy(p).cuda()
    for name in DTYPES:
        plan = q.AdjointPlan(circ, H, CODE[name], 5)
        e, gg = plan.run(pdev)
        e, gg = float(e.cpu()[0]), gg.cpu().numpy()
        de, dg = abs(e - E), float(np.max(np.abs(gg - g)))
        say("hea26", name, "|dE| %.3e  max|dgrad| %.3e (vs oracle adjoint)" % (de, dg))
        if name == "c128":
            assert de <= 1e-10 * scale and dg <= 1e-10, (de, dg)
        else:
            assert de <= 1e-7 * scale and dg <= 1e-7 * scale, (de, dg)
        del plan
        torch.cuda.empty_cache()


# ------------------------------------------------------------------- batched

def test_batched_workload_checked_subset(q, orc):
    """All 1024 instances in one batch (complex64); every instance with
    n <= 16 and a seeded sample of 32 larger ones (at least one each of
    n = 21 and n = 22) against the oracle's adjoint."""
    import torch
    insts = W.batched_hea()
    say("batch 1024 instances")
    plan = q.BatchPlan(insts, 1)
    params = torch.from_numpy(np.concatenate([i.params for i in insts])).cuda()
    e, g = plan.run(params)
    e, g = e.cpu().numpy(), g.cpu().numpy()
    assert np.all(np.isfinite(e)) and np.all(np.isfinite(g))
    small = [j for j, i in enumerate(insts) if i.circuit.n <= 16]
    large = [j for j, i in enumerate(insts) if i.circuit.n > 16]
    rng = np.random.default_rng(1004)
    pick = [next(j for j in large if insts[j].circuit.n == 21),
            next(j for j in large if insts[j].circuit.n == 22)]
    rest = [j for j in large if j not in pick]
    pick += [int(v) for v in rng.choice(rest, size=30, replace=False)]
    worst = {}
    for j in small + sorted(pick):
        inst = insts[j]
        n = inst.circuit.n
        E_ref, g_ref = orc.adjoint(inst.circuit, inst.params, inst.hamiltonian)
        gj = g[plan.offsets[j]:plan.offsets[j + 1]]
        scale = float(np.sum(np.abs(inst.hamiltonian.coeff)))
        de, dg = abs(e[j] - E_ref), float(np.max(np.abs(gj - g_ref)))
        w = worst.get(n, (0.0, 0.0))
        worst[n] = (max(w[0], de / scale), max(w[1], dg / scale))
        # complex64: worst measured instance 7e-8 per unit of sum|c|
        assert de <= 3e-7 * scale and dg <= 3e-7 * scale, (j, n, de, dg)
    for n in sorted(worst):
        say("batch n=%d worst |dE|/sum|c| %.3e  max|dgrad|/sum|c| %.3e" % ((n,) + worst[n]))
    assert len(small) > 400 and {21, 22} <= set(worst)


# ------------------------------------------- n = 30 expectation values

def product_expectation(H, vecs):
    """<H> on the product state (x)_q (a_q|0> + b_q|1>) (qubit q = bit q):
    sum_j c_j prod_q <sigma>_q with <X> = 2 Re(conj(a) b), <Y> = 2 Im(conj(a) b),
    <Z> = |a|^2 - |b|^2 and 1 for the identity factors (Sec. 3 Pauli
    strings; a closed form that holds at any size)."""
    one = {}
    for q, (a, b) in enumerate(vecs):
        w = np.conj(a) * b
        one[q] = (2 * w.real, 2 * w.imag, abs(a) ** 2 - abs(b) ** 2)
    tot = 0.0
    for x, z, c in zip(H.x_mask, H.z_mask, H.coeff):
        x, z, v = int(x), int(z), float(c)
        for q in range(len(vecs)):
            xb, zb = (x >> q) & 1, (z >> q) & 1
            if xb and zb:
                v *= one[q][1]
            elif xb:
                v *= one[q][0]
            elif zb:
                v *= one[q][2]
        tot += v
    return tot


def hamiltonians_for(n):
    rng = np.random.default_rng(3000 + n)
    heis = [(ab, (q, q + 1), 1.0) for q in range(n - 1) for ab in ("XX", "YY", "ZZ")]
    heis += [(c, (q,), float(rng.normal())) for q in range(n) for c in "XYZ"]
    mixed = [("", (), 0.3)]
    for _ in range(40):
        k = int(rng.integers(1, 4))
        qs = [int(v) for v in rng.choice(n, k, replace=False)]
        mixed.append(("".join(rng.choice(["X", "Y", "Z"]) for _ in range(k)), qs, float(rng.normal())))
    # strings of 7-10 factors spread over the register (x masks with many
    # qubits above 5: span passes), values large enough to test on a product
    # state
    spread = []
    for _ in range(48):
        k = min(n, int(rng.integers(7, 11)))
        qs = [int(v) for v in rng.choice(n, k, replace=False)]
        spread.append(("".join(rng.choice(["X", "Y", "X", "Y", "Z"]) for _ in range(k)), qs, float(rng.normal())))
    return [("tfim", W.tfim_chain(n, 0.8)), ("xxz", W.xxz_chain(n, 0.5)), ("heisenberg_fields", W.pauli_sum(n, heis)),
            ("mixed", W.pauli_sum(n, mixed)), ("spread", W.pauli_sum(n, spread))]


@pytest.mark.parametrize("n", [30, 32])
@pytest.mark.parametrize("name", DTYPES)
def test_expectation_n30_product_state(q, name, n, monkeypatch):
    """<psi|H|psi> at n = 30 (the bench step's size and launch configuration:
    register-tile passes, the LDS-tile and span passes for the rest) and at
    n = 32 on a product state built on the GPU by one Haar U(2) per qubit
    from |0...0>, against the closed form; TFIM, XXZ, a Heisenberg chain with
    fields, 40 random 1-3-qubit strings and 48 strings of 7-10 factors spread
    over all qubits.  At n = 30 also with the plan forced to register passes
    (QSV_EXPECT_PLAN=reg) and to span passes alone (=span).  The imaginary
    part stays at rounding level."""
    import torch
    rng = np.random.default_rng(3000 + n)
    Us = [W.haar_unitary(rng, 2) for _ in range(n)]
    psi = torch.empty(1 << n, dtype=torch_dtype(name), device="cuda")
    q.qsv_init_basis(psi, 0)
    for t in range(n):
        q.qsv_apply_gate(psi, (t,), (), Us[t])
    vecs = [U[:, 0] for U in Us]
    # measured per sum |c|: complex64 <= 1.8e-9 at n = 30 and <= 7.4e-8 at
    # n = 32 (the rounding of the 32 complex64 gate sweeps that build the
    # state), complex128 <= 1.6e-16
    tol = (1e-7 if n == 30 else 5e-7) if name == "c64" else 1e-13
    plans = ["default", "reg", "span"] if n == 30 else ["default"]
    for hname, H in hamiltonians_for(n):
        ref = product_expectation(H, vecs)
        scale = float(np.sum(np.abs(H.coeff)))
        for plan in plans:
            if plan != "default":
                monkeypatch.setenv("QSV_EXPECT_PLAN", plan)
            e = q.qsv_expectation(psi, H).cpu().numpy()
            nl = q.expectation_launches(H, n, CODE[name])
            if plan != "default":
                monkeypatch.delenv("QSV_EXPECT_PLAN")
            err = abs(e[0] - ref) / scale
            say("expectation product state", n, name, hname, plan, "launches", nl, "err/sum|c| %.2e" % err)
            assert err <= tol, (hname, plan, e, ref)
            assert abs(e[1]) <= tol * scale
    del psi
    torch.cuda.empty_cache()
