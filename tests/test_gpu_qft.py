"""GPU parity of the QFT workload (the quantum Fourier transform among the
paper's built-in circuits, Sec. 3): Hadamards, controlled phases (diagonal
launches) and swaps (bit-exact moves), unfused and fused, against the oracle
on seeded states, and at n = 30 against the closed-form transform of a basis
state, sampled."""
import numpy as np
import pytest

import workloads as W
from gpu_util import TOL, rand_state, raw_bits, say, to_gpu, to_np, torch_dtype

pytestmark = pytest.mark.gpu
DTYPES = ("c128", "c64")


@pytest.fixture(scope="module")
def q():
    import torch
    assert torch.cuda.is_available()
    from paper_2202_07017_amd import qsv
    qsv.lib()
    return qsv


def _code(q, name):
    return q.C128 if name == "c128" else q.C64


@pytest.mark.parametrize("name", DTYPES)
@pytest.mark.parametrize("n", [1, 5, 12, 16, 20])
@pytest.mark.parametrize("fuse", [1, 3, 5])
def test_qft_parity(q, orc, name, n, fuse):
    rng = np.random.default_rng(700 + n)
    psi = rand_state(n, rng, name)
    circ = W.qft(n)
    say("qft", name, n, fuse)
    d = to_gpu(psi, name)
    q.Plan(circ, _code(q, name), fuse).run(d)
    got = to_np(d)
    ref = orc.run(circ, psi0=psi)
    assert np.max(np.abs(got - ref)) <= TOL[name], np.max(np.abs(got - ref))


@pytest.mark.parametrize("name", DTYPES)
def test_qft_full_size_basis(q, name):
    """n = 30: QFT of |x> is exp(2 pi i x y / 2^n) / 2^(n/2); phases reduced
    with exact integer arithmetic; checked on sampled outputs."""
    import torch
    n, x = 30, 0x2A5F3C1
    N = 1 << n
    d = torch.empty(N, dtype=torch_dtype(name), device="cuda")
    rng = np.random.default_rng(30)
    y = np.concatenate([rng.integers(0, N, 200), [0, 1, N - 1, N // 2]]).astype(np.int64)
    want = np.exp(2j * np.pi * ((x * y) % N) / N) / np.sqrt(N)
    for fuse in (1, 5):
        say("qft n30", name, fuse)
        q.qsv_init_basis(d, x)
        q.Plan(W.qft(n), _code(q, name), fuse).run(d)
        got = d[torch.from_numpy(y).cuda()].cpu().numpy().astype(np.complex128)
        err = np.max(np.abs(got - want))
        assert err <= TOL[name] and err / np.max(np.abs(want)) <= 1e-5, (fuse, err)
    del d
    torch.cuda.empty_cache()


def _diag_circuit(n, seed):
    """Runs of diagonal gates (CZ, controlled phases with 1-2 controls, random
    two-qubit diagonals including non-unitary ones, Z, phases on low and high
    qubits) separated by Hadamards."""
    rng = np.random.default_rng(seed)
    c = W.Circuit(n)
    for layer in range(4):
        for _ in range(3 * n):
            kind = rng.integers(0, 5)
            qs = [int(v) for v in rng.permutation(n)[:3]]
            if kind == 0 and n >= 2:
                c.ops.append(W.Op("z", (qs[0],), controls=(qs[1],)))
            elif kind == 1 and n >= 3:
                ph = np.exp(1j * rng.uniform(0, 2 * np.pi))
                c.ops.append(W.Op("matrix", (qs[0],), controls=(qs[1], qs[2]),
                                  matrix=np.diag([1.0, ph]).astype(np.complex128)))
            elif kind == 2 and n >= 2:
                d = rng.standard_normal(4) + 1j * rng.standard_normal(4)
                c.ops.append(W.Op("matrix", (qs[0], qs[1]), matrix=np.diag(d).astype(np.complex128)))
            elif kind == 3:
                c.ops.append(W.Op("z", (qs[0],)))
            else:
                ph = np.exp(1j * rng.uniform(0, 2 * np.pi, 2))
                c.ops.append(W.Op("matrix", (qs[0],), matrix=np.diag(ph).astype(np.complex128)))
        c.ops.append(W.Op("h", (layer % n,)))
    return c


@pytest.mark.parametrize("name", DTYPES)
@pytest.mark.parametrize("n", [3, 7, 12, 17])
@pytest.mark.parametrize("fuse", [1, 3, 5])
def test_diagonal_runs(q, orc, name, n, fuse):
    """Plans merge consecutive diagonal launches into single sweeps; results
    match the oracle and the unmerged plan, with fewer launches."""
    import os
    circ = _diag_circuit(n, 40 + n)
    rng = np.random.default_rng(n)
    psi = rand_state(n, rng, name)
    ref = orc.run(circ, psi0=psi)
    say("diag runs", name, n, fuse)
    d = to_gpu(psi, name)
    merged = q.Plan(circ, _code(q, name), fuse)
    merged.run(d)
    got = to_np(d)
    os.environ["QSV_NO_DIAG_RUN"] = "1"
    try:
        plain = q.Plan(circ, _code(q, name), fuse)
    finally:
        del os.environ["QSV_NO_DIAG_RUN"]
    d2 = to_gpu(psi, name)
    plain.run(d2)
    scale = max(1.0, float(np.max(np.abs(ref))))
    assert np.max(np.abs(got - ref)) <= TOL[name] * scale, np.max(np.abs(got - ref))
    assert np.max(np.abs(to_np(d2) - ref)) <= TOL[name] * scale
    if n >= 7 and fuse == 1:
        assert merged.info()[0] < plain.info()[0], (merged.info(), plain.info())
    assert merged.info()[0] <= plain.info()[0]


def _swap_circuit(n, kind, seed):
    """Runs of SWAP gates: the bit reversal that closes the QFT, random swaps
    that chain into long cycles (two passes), swaps among qubits 0..5 only,
    among high qubits only, swaps that cancel, and runs cut by Hadamards."""
    rng = np.random.default_rng(seed)
    c = W.Circuit(n)
    if kind == "reverse":
        pairs = [(b, n - 1 - b) for b in range(n // 2)]
    elif kind == "random":
        pairs = [tuple(int(v) for v in rng.permutation(n)[:2]) for _ in range(2 * n)]
    elif kind == "low":
        pairs = [(0, 5), (1, 4), (2, 3), (0, 1)]
    elif kind == "high":
        pairs = [(n - 1, n - 3), (n - 2, n - 5), (n - 4, n - 6), (n - 1, n - 2)]
    elif kind == "cancel":
        pairs = [(1, n - 2), (3, 7), (3, 7), (1, n - 2)]
    else:  # "cut": three runs separated by Hadamards
        pairs = []
        for r in range(3):
            for _ in range(4):
                c.ops.append(W.Op("swap", tuple(int(v) for v in rng.permutation(n)[:2])))
            c.ops.append(W.Op("h", (int(rng.integers(0, n)),)))
        return c
    for a, b in pairs:
        c.ops.append(W.Op("swap", (a, b)))
    return c


@pytest.mark.parametrize("name", DTYPES)
@pytest.mark.parametrize("n", [12, 13, 17, 20])
@pytest.mark.parametrize("kind", ["reverse", "random", "low", "high", "cancel", "cut"])
def test_swap_runs(q, orc, name, n, kind):
    """Plans compose runs of consecutive swaps into qubit permutation passes
    (moves of raw bits): the result equals the oracle's gate-by-gate swaps
    exactly, and equals the plan that keeps the swaps separate bit for bit."""
    import os
    circ = _swap_circuit(n, kind, 900 + n)
    rng = np.random.default_rng(n)
    psi = rand_state(n, rng, name)
    if name == "c64":
        psi[3] = -0.0  # a signed zero survives moves
    ref = orc.run(circ, psi0=psi)
    say("swap runs", name, n, kind)
    d = to_gpu(psi, name)
    merged = q.Plan(circ, _code(q, name), 1)
    merged.run(d)
    os.environ["QSV_NO_SWAP_MERGE"] = "1"
    try:
        plain = q.Plan(circ, _code(q, name), 1)
    finally:
        del os.environ["QSV_NO_SWAP_MERGE"]
    d2 = to_gpu(psi, name)
    plain.run(d2)
    if kind != "cut":
        assert np.array_equal(to_np(d), ref)
    else:
        assert np.max(np.abs(to_np(d) - ref)) <= TOL[name]
    assert np.array_equal(raw_bits(d.cpu().numpy()), raw_bits(d2.cpu().numpy()))
    if kind in ("reverse", "random", "cancel"):
        assert merged.info()[0] < plain.info()[0], (merged.info(), plain.info())
    assert merged.info()[0] <= plain.info()[0]


def _phase_circuit(n, seed, rotations):
    """Hadamards, controlled phases (one and two controls), CZ, diagonal
    two-qubit matrices and, if asked, rotations with device parameters (RX,
    RZ: a standalone rotation on a deferred gate's qubit must come after it)
    in random order."""
    rng = np.random.default_rng(seed)
    c = W.Circuit(n)
    npar = 0
    for _ in range(8 * n):
        kind = int(rng.integers(0, 6 if rotations else 4))
        qs = [int(v) for v in rng.permutation(n)[:3]]
        if kind == 0:
            c.ops.append(W.Op("h", (qs[0],)))
        elif kind == 1:
            ph = np.exp(1j * rng.uniform(0, 2 * np.pi))
            ctl = (qs[1],) if rng.integers(0, 2) else (qs[1], qs[2])
            c.ops.append(W.Op("matrix", (qs[0],), controls=ctl,
                              matrix=np.diag([1.0, ph]).astype(np.complex128)))
        elif kind == 2:
            c.ops.append(W.Op("z", (qs[0],), controls=(qs[1],)))
        elif kind == 3:
            d = np.exp(1j * rng.uniform(0, 2 * np.pi, 4))
            c.ops.append(W.Op("matrix", (qs[0], qs[1]), matrix=np.diag(d).astype(np.complex128)))
        else:
            c.ops.append(W.Op("rx" if kind == 4 else "rz", (qs[0],), param=npar))
            npar += 1
    c.nparams = npar
    return c, W.random_params(npar, seed) if npar else None


@pytest.mark.parametrize("name", DTYPES)
@pytest.mark.parametrize("n", [7, 12, 16])
@pytest.mark.parametrize("fuse", [3, 4, 5])
@pytest.mark.parametrize("kind", ["qft", "phases", "rotations"])
def test_diagonal_deferral(q, orc, name, n, fuse, kind):
    """Fusion defers diagonal gates that do not fit an open block past the
    gates they commute with and packs them into diagonal blocks: results match
    the oracle and the plan that closes blocks at such gates, and the QFT
    takes fewer launches."""
    import os
    import torch
    if kind == "qft":
        circ, params = W.qft(n), None
    else:
        circ, params = _phase_circuit(n, 60 + n, kind == "rotations")
    rng = np.random.default_rng(n + 1)
    psi = rand_state(n, rng, name)
    ref = orc.run(circ, params, psi0=psi)
    say("diagonal deferral", name, n, fuse, kind)
    pdev = torch.from_numpy(params).cuda() if params is not None else None
    d = to_gpu(psi, name)
    deferred = q.Plan(circ, _code(q, name), fuse)
    deferred.run(d, pdev)
    os.environ["QSV_NO_DIAG_DEFER"] = "1"
    try:
        plain = q.Plan(circ, _code(q, name), fuse)
    finally:
        del os.environ["QSV_NO_DIAG_DEFER"]
    d2 = to_gpu(psi, name)
    plain.run(d2, pdev)
    assert np.max(np.abs(to_np(d) - ref)) <= TOL[name], np.max(np.abs(to_np(d) - ref))
    assert np.max(np.abs(to_np(d2) - ref)) <= TOL[name]
    if kind == "qft" and n >= 12:
        assert deferred.info()[0] < plain.info()[0], (deferred.info(), plain.info())


def _fold_circuit(n, seed):
    """Random single-qubit unitaries on every qubit (low, middle, high, qubit
    0) around runs of diagonal gates (CZ, controlled phases, diagonal
    two-qubit matrices), with controlled gates and Paulis (not foldable) in
    between."""
    rng = np.random.default_rng(seed)
    c = W.Circuit(n)
    for layer in range(3 * n):
        t = layer % n if layer < n else int(rng.integers(0, n))
        c.ops.append(W.Op("matrix", (t,), matrix=W.haar_unitary(rng, 2)))
        for _ in range(int(rng.integers(3, 7))):
            qs = [int(v) for v in rng.permutation(n)[:2]]
            if rng.random() < 0.5:
                c.ops.append(W.Op("z", (qs[0],), controls=(qs[1],)))
            else:
                d = np.exp(1j * rng.uniform(0, 2 * np.pi, 4))
                c.ops.append(W.Op("matrix", (qs[0], qs[1]), matrix=np.diag(d).astype(np.complex128)))
        r = rng.random()
        if r < 0.15:
            qs = [int(v) for v in rng.permutation(n)[:2]]
            c.ops.append(W.Op("matrix", (qs[0],), controls=(qs[1],), matrix=W.haar_unitary(rng, 2)))
        elif r < 0.25:
            c.ops.append(W.Op("x", (int(rng.integers(0, n)),)))
    return c


@pytest.mark.parametrize("name", DTYPES)
@pytest.mark.parametrize("n", [12, 13, 16, 20])
@pytest.mark.parametrize("kind", ["qft", "random"])
@pytest.mark.parametrize("fuse", [1, 5])
def test_gate_fold(q, orc, name, n, kind, fuse):
    """Plans apply a single-qubit gate next to a diagonal run in the run's
    sweep (the run's window of varying bits placed over the target): results
    match the oracle and the plan that keeps the gates separate."""
    import os
    circ = W.qft(n) if kind == "qft" else _fold_circuit(n, 70 + n)
    rng = np.random.default_rng(n + 2)
    psi = rand_state(n, rng, name)
    ref = orc.run(circ, psi0=psi)
    say("gate fold", name, n, kind, fuse)
    d = to_gpu(psi, name)
    folded = q.Plan(circ, _code(q, name), fuse)
    folded.run(d)
    os.environ["QSV_NO_GATE_FOLD"] = "1"
    try:
        plain = q.Plan(circ, _code(q, name), fuse)
    finally:
        del os.environ["QSV_NO_GATE_FOLD"]
    d2 = to_gpu(psi, name)
    plain.run(d2)
    scale = max(1.0, float(np.max(np.abs(ref))))
    assert np.max(np.abs(to_np(d) - ref)) <= TOL[name] * scale, np.max(np.abs(to_np(d) - ref))
    assert np.max(np.abs(to_np(d2) - ref)) <= TOL[name] * scale
    assert folded.info()[0] <= plain.info()[0]
    if kind == "qft" and fuse == 1 and n >= 16:
        assert folded.info()[0] < plain.info()[0], (folded.info(), plain.info())


def _swap_source(j, swaps):
    """Input index that output index j reads after the swaps are applied in
    order: the last swap acts first on the index."""
    j = np.asarray(j, dtype=np.int64).copy()
    for a, b in reversed(swaps):
        ba, bb = (j >> a) & 1, (j >> b) & 1
        j = j & ~((1 << a) | (1 << b)) | (ba << b) | (bb << a)
    return j


@pytest.mark.parametrize("name", DTYPES)
@pytest.mark.parametrize("kind", ["reverse", "random", "high"])
def test_swap_runs_full_size(q, name, kind):
    """n = 30: swap runs as qubit permutation passes on a state that holds
    its own index (complex64: low 24 bits in the real part, the rest in the
    imaginary part, both exact), checked on sampled outputs against the
    index the swaps map them to; the random run needs two passes."""
    import torch
    n = 30
    N = 1 << n
    rng = np.random.default_rng(31)
    if kind == "reverse":
        swaps = [(b, n - 1 - b) for b in range(n // 2)]
    elif kind == "random":
        swaps = [tuple(int(v) for v in rng.permutation(n)[:2]) for _ in range(40)]
    else:
        swaps = [(n - 1, n - 7), (n - 2, n - 9), (n - 3, 12), (n - 4, 0)]
    circ = W.Circuit(n, [W.Op("swap", s) for s in swaps])
    say("swap runs n30", name, kind)
    i = torch.arange(N, device="cuda", dtype=torch.int64)
    if name == "c64":
        d = torch.complex((i & 0xFFFFFF).to(torch.float32), (i >> 24).to(torch.float32))
    else:
        d = torch.complex(i.to(torch.float64), torch.zeros(N, device="cuda", dtype=torch.float64))
    del i
    plan = q.Plan(circ, _code(q, name), 1)
    plan.run(d)
    j = np.concatenate([rng.integers(0, N, 4096), [0, 1, N - 1, N // 2, 0x15555555, 0x2AAAAAAA]])
    got = d[torch.from_numpy(j).cuda()].cpu().numpy()
    if name == "c64":
        idx = got.real.astype(np.int64) | (got.imag.astype(np.int64) << 24)
    else:
        idx = got.real.astype(np.int64)
    want = _swap_source(j, swaps)
    assert np.array_equal(idx, want), np.flatnonzero(idx != want)[:8]
    assert plan.info()[0] <= 2
    del d
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name", DTYPES)
@pytest.mark.parametrize("fuse", [1, 5])
def test_plan_passes_graph_replay(q, orc, name, fuse):
    """A plan with every plan pass (a QFT: deferred diagonal gates, diagonal
    runs with gates in their sweeps, a qubit permutation pass) records a HIP
    graph on its first run and replays it on later runs: three runs on one
    state match the oracle's circuit applied three times, and a replay on a
    copy of an earlier state matches the run that produced the next one."""
    import torch
    n = 16
    circ = W.qft(n)
    rng = np.random.default_rng(5)
    psi = rand_state(n, rng, name)
    ref = psi
    for _ in range(3):
        ref = orc.run(circ, psi0=ref)
    say("plan passes replay", name, fuse)
    plan = q.Plan(circ, _code(q, name), fuse)
    d = to_gpu(psi, name)
    plan.run(d)
    first = d.clone()
    plan.run(d)
    second = d.clone()
    plan.run(d)
    assert np.max(np.abs(to_np(d) - ref)) <= 3 * TOL[name], np.max(np.abs(to_np(d) - ref))
    again = first.clone()
    plan.run(again)
    torch.cuda.synchronize()
    assert torch.equal(again, second), "replay differs from the recorded run"


@pytest.fixture(scope="module")
def qft26_reference(orc):
    """n = 26: the oracle's seeded random state and its QFT at sampled
    outputs y from the transform's definition, psi_out[y] = 2^(-n/2)
    sum_x psi_in[x] exp(+2 pi i x y / 2^n), with exact integer phases; x is
    split into 13-bit halves, so each output is a matrix-vector product."""
    n, seed = 26, 2602
    N, H = 1 << n, 1 << 13
    psi = orc.random_state(n, seed)
    M = psi.reshape(H, H)  # M[xh, xl] = psi[xh * 2^13 + xl]
    rng = np.random.default_rng(26)
    ys = np.concatenate([rng.integers(0, N, 6), [0, N - 1]]).astype(np.int64)
    h = np.arange(H, dtype=np.int64)
    want = np.empty(len(ys), dtype=np.complex128)
    for k, y in enumerate(ys):
        vl = np.exp(2j * np.pi * ((h * y) % N) / N)
        vh = np.exp(2j * np.pi * (((h << 13) * y) % N) / N)
        want[k] = np.dot(vh, M @ vl) / np.sqrt(N)
    return n, seed, ys, want


@pytest.mark.parametrize("name", DTYPES)
def test_qft_random_state_vs_dft(q, qft26_reference, name):
    """n = 26, a seeded random input (the device generator, equal to the
    oracle's): the QFT fused to k = 5 and unfused (every plan pass: deferred
    diagonal gates, runs with gates in their sweeps on window, lane and moved
    wave bits, the permutation pass) against the transform's definition at
    sampled outputs."""
    import torch
    n, seed, ys, want = qft26_reference
    for fuse in (1, 5):
        say("qft random n26", name, fuse)
        d = torch.empty(1 << n, dtype=torch_dtype(name), device="cuda")
        q.qsv_init_random(d, seed)
        q.Plan(W.qft(n), _code(q, name), fuse).run(d)
        got = d[torch.from_numpy(ys).cuda()].cpu().numpy().astype(np.complex128)
        err = np.max(np.abs(got - want))
        assert err <= TOL[name] * 1e-2, (fuse, err, np.max(np.abs(want)))
        del d
    torch.cuda.empty_cache()
