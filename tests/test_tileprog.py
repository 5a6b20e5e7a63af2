"""Host logic of the cache-blocked adjoint: the tile-program compiler
(paper_2202_07017_amd/csrc/tileprog.cpp) schedules single-target gates into
passes over tiles of m qubits and three-qubit steps.  A small C++ driver
(tests/tileprog_check.cpp) compiles a gate list with it, checks the
structure (every gate exactly once, tile masks, step shapes, step-local
targets and controls, rotation slots and their parameters) and executes the
passes on the CPU as their descriptors say.  The result must equal the
oracle applying the same gates in circuit order (eq. (1), Sec. 2): a gate
moved across one it does not commute with, a wrong step-local index or a
dropped gate changes the state."""
import os
import subprocess

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2202_07017_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("tileprog") / "tileprog_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I" + CSRC, os.path.join(ROOT, "tests", "tileprog_check.cpp"),
                    os.path.join(CSRC, "tileprog.cpp"), "-o", exe], check=True)
    return exe


def rot(kind, th):
    c, s = np.cos(th / 2), np.sin(th / 2)
    if kind == "rx":
        return np.array([[c, -1j * s], [-1j * s, c]])
    if kind == "ry":
        return np.array([[c, -s], [s, c]], dtype=complex)
    return np.diag([np.exp(-0.5j * th), np.exp(0.5j * th)])


FIXED = {"h": np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2),
         "x": np.array([[0, 1], [1, 0]], dtype=complex),
         "y": np.array([[0, -1j], [1j, 0]]),
         "z": np.diag([1, -1]).astype(complex),
         "s": np.diag([1, 1j]),
         "t": np.diag([1, np.exp(0.25j * np.pi)])}
GEN = {"rx": 5, "ry": 6, "rz": 7}


def random_gates(n, count, seed):
    """(kind code, target, controls, param, 2x2 matrix): fixed gates, Haar
    U(2) and rotations with 0-2 controls; a fifth of the rotations share an
    earlier parameter."""
    rng = np.random.default_rng(seed)
    out, npar, thetas = [], 0, []
    for _ in range(count):
        kind = ["h", "x", "y", "z", "s", "t", "u", "rx", "ry", "rz"][rng.integers(10)]
        q = [int(v) for v in rng.choice(n, 1 + int(rng.integers(3)), replace=False)]
        if kind in GEN:
            if npar and rng.random() < 0.2:
                p = int(rng.integers(npar))
            else:
                p, npar = npar, npar + 1
                thetas.append(rng.uniform(0, 2 * np.pi))
            out.append((GEN[kind], q[0], q[1:], p, rot(kind, thetas[p])))
        else:
            M = W.haar_unitary(rng, 2) if kind == "u" else FIXED[kind]
            out.append((0, q[0], q[1:], -1, M))
    return out


def hea_gates(n, layers, seed):
    rng = np.random.default_rng(seed)
    out, p = [], 0
    for _ in range(layers):
        for q in range(n):
            for kind in ("ry", "rz"):
                out.append((GEN[kind], q, [], p, rot(kind, rng.uniform(0, 2 * np.pi))))
                p += 1
        for q in range(n - 1):
            out.append((0, q + 1, [q], -1, FIXED["x"]))
    return out


def run_checker(exe, n, m, cap, gates, psi):
    lines = ["%d %d %d %d" % (n, m, cap, len(gates))]
    for kind, t, cs, p, M in gates:
        c = list(cs) + [0, 0]
        vals = " ".join("%.17g %.17g" % (z.real, z.imag) for z in np.asarray(M, complex).reshape(-1))
        lines.append("%d %d %d %d %d %d %s" % (kind, t, len(cs), c[0], c[1], p, vals))
    lines += ["%.17g %.17g" % (z.real, z.imag) for z in psi]
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    v = np.array(r.stdout.split(), dtype=np.float64).reshape(-1, 2)
    return v[:, 0] + 1j * v[:, 1]


@pytest.mark.parametrize("n,m,cap,count,seed", [
    (9, 6, 512, 160, 1), (11, 8, 512, 200, 2), (12, 7, 40, 200, 3),
    (8, 8, 16, 90, 4), (7, 12, 512, 60, 5), (10, 5, 512, 150, 6)])
def test_tile_program_matches_circuit_order(orc, checker, n, m, cap, count, seed):
    gates = random_gates(n, count, seed)
    rng = np.random.default_rng(100 + seed)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi /= np.linalg.norm(psi)
    got = run_checker(checker, n, m, cap, gates, psi)
    circ = W.Circuit(n, [W.Op("matrix", (t,), controls=tuple(cs), matrix=np.asarray(M, complex))
                         for _, t, cs, _, M in gates])
    ref = orc.run(circ, psi0=psi)
    assert np.max(np.abs(got - ref)) < 1e-12


@pytest.mark.parametrize("n,m,layers", [(10, 6, 4), (13, 8, 3)])
def test_tile_program_hea_ladder(orc, checker, n, m, layers):
    """The ladder ansatz the scheduler is tuned for (staircase passes)."""
    gates = hea_gates(n, layers, 7 + n)
    rng = np.random.default_rng(n)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi /= np.linalg.norm(psi)
    got = run_checker(checker, n, m, 512, gates, psi)
    circ = W.Circuit(n, [W.Op("matrix", (t,), controls=tuple(cs), matrix=np.asarray(M, complex))
                         for _, t, cs, _, M in gates])
    assert np.max(np.abs(got - orc.run(circ, psi0=psi))) < 1e-12


def test_checker_catches_a_reordered_gate(orc, checker):
    """The comparison is sensitive to gate order: with two adjacent gates
    that do not commute swapped in the input, the checker's result differs
    from the oracle's on the original order well above the tolerance (so a
    scheduling mistake of that kind cannot pass)."""
    n = 6
    gates = random_gates(n, 40, 9)
    rng = np.random.default_rng(11)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi /= np.linalg.norm(psi)

    def circ_of(gs):
        return W.Circuit(n, [W.Op("matrix", (t,), controls=tuple(cs), matrix=np.asarray(M, complex))
                             for _, t, cs, _, M in gs])

    ref = orc.run(circ_of(gates), psi0=psi)
    for k in range(len(gates) - 1):
        swapped = gates[:k] + [gates[k + 1], gates[k]] + gates[k + 2:]
        if np.max(np.abs(orc.run(circ_of(swapped), psi0=psi) - ref)) > 1e-6:
            break
    else:
        pytest.fail("no non-commuting adjacent pair in the seeded list")
    got = run_checker(checker, n, 4, 512, swapped, psi)
    assert np.max(np.abs(got - ref)) > 1e-6
