"""Host logic of gate fusion (paper_2202_07017_amd/csrc/fuse_plan.cpp): the
greedy planner groups the gates of a circuit into blocks of at most k qubits
(each one dense launch of eq. (1), Sec. 2) and, for k >= 3, defers diagonal
gates that do not fit an open block past the gates they commute with.  A
small C++ driver (tests/fuse_check.cpp) fuses a circuit, checks the items'
structure and applies the items in order and the gates in circuit order to
the same state: any reordering that does not commute (a diagonal gate moved
past a Hadamard on its qubit, a block emitted after the pool it precedes, a
rotation moved across a deferred gate) changes the result."""
import os
import subprocess

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2202_07017_amd", "csrc")
KIND = {"matrix": 0, "h": 1, "x": 2, "y": 3, "z": 4, "rx": 5, "ry": 6, "rz": 7, "swap": 8}
R2 = 1.0 / np.sqrt(2.0)
FIXED = {"h": np.array([[R2, R2], [R2, -R2]]), "x": np.array([[0, 1], [1, 0]]),
         "y": np.array([[0, -1j], [1j, 0]]), "z": np.diag([1.0, -1.0]),
         "swap": np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]])}


def build_checker(out, extra=()):
    subprocess.run(["g++", "-O2", "-std=c++17", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC] +
                   list(extra) + [os.path.join(ROOT, "tests", "fuse_check.cpp"),
                                  os.path.join(CSRC, "fuse_plan.cpp"), "-o", out], check=True)
    return out


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if os.environ.get("FUSE_CHECK_EXE"):  # a prebuilt checker (planted-mistake runs)
        return os.environ["FUSE_CHECK_EXE"]
    return build_checker(str(tmp_path_factory.mktemp("fuse") / "fuse_check"))


def op_matrix(op, params):
    if op.kind in FIXED:
        return FIXED[op.kind]
    if op.kind in ("rx", "ry", "rz"):
        t = params[op.param]
        c, s = np.cos(t / 2), np.sin(t / 2)
        return {"rx": np.array([[c, -1j * s], [-1j * s, c]]), "ry": np.array([[c, -s], [s, c]]),
                "rz": np.diag([np.exp(-0.5j * t), np.exp(0.5j * t)])}[op.kind]
    return op.matrix


def run(checker, circ, params, k, standalone, defer, env=None):
    lines = ["%d %d %d %d %d" % (circ.n, k, int(standalone), int(defer), len(circ.ops))]
    for op in circ.ops:
        m = np.asarray(op_matrix(op, params), dtype=np.complex128)
        head = [KIND[op.kind], len(op.targets), *op.targets, len(op.controls), *op.controls,
                op.param if op.param is not None and op.param >= 0 else -1]
        lines.append(" ".join(str(int(v)) for v in head))
        lines.append(" ".join("%.17g %.17g" % (v.real, v.imag) for v in m.ravel()))
    p = subprocess.run([checker], input="\n".join(lines) + "\n", capture_output=True, text=True, env=env)
    assert p.returncode == 0, p.stderr
    assert "runtime error" not in p.stderr and "Sanitizer" not in p.stderr, p.stderr
    return int(p.stdout.split()[1])


def random_circuit(n, seed, diag_heavy):
    """Hadamards, Paulis (some controlled), rotations, swaps, dense 2- and
    3-qubit unitaries, and (more of them when diag_heavy) diagonal gates: CZ,
    controlled phases with one or two controls, diagonal 2- and 3-qubit
    matrices."""
    rng = np.random.default_rng(seed)
    c = W.Circuit(n)
    npar = 0
    for _ in range(6 * n):
        qs = [int(v) for v in rng.permutation(n)[:3]]
        r = rng.random()
        if r < (0.55 if diag_heavy else 0.25):
            kind = int(rng.integers(0, 4))
            if kind == 0:
                c.ops.append(W.Op("z", (qs[0],), controls=(qs[1],)))
            elif kind == 1:
                ctl = (qs[1],) if rng.integers(0, 2) else (qs[1], qs[2])
                c.ops.append(W.Op("matrix", (qs[0],), controls=ctl,
                                  matrix=np.diag([1.0, np.exp(1j * rng.uniform(0, 6.3))])))
            else:
                m = 2 if kind == 2 else 3
                c.ops.append(W.Op("matrix", tuple(qs[:m]),
                                  matrix=np.diag(np.exp(1j * rng.uniform(0, 6.3, 1 << m)))))
        elif r < 0.7:
            c.ops.append(W.Op(["h", "x", "y"][int(rng.integers(0, 3))], (qs[0],),
                              controls=(qs[1],) if rng.random() < 0.2 else ()))
        elif r < 0.82:
            c.ops.append(W.Op(["rx", "ry", "rz"][int(rng.integers(0, 3))], (qs[0],), param=npar))
            npar += 1
        elif r < 0.9:
            c.ops.append(W.Op("swap", (qs[0], qs[1])))
        else:
            m = int(rng.integers(2, 4))
            c.ops.append(W.Op("matrix", tuple(qs[:m]), matrix=W.haar_unitary(rng, 1 << m)))
    c.nparams = npar
    return c, rng.uniform(0, 6.3, max(npar, 1))


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("standalone", [False, True])
def test_fusion_order_is_equivalent(checker, k, seed, standalone):
    n = 6 + seed % 3
    circ, params = random_circuit(n, 100 * k + seed, seed % 2 == 0)
    for defer in (False, True):
        run(checker, circ, params, k, standalone, defer)


@pytest.mark.parametrize("n", [6, 9, 11])
@pytest.mark.parametrize("k", [3, 4, 5])
def test_qft_deferral_keeps_order_and_packs(checker, n, k):
    """The QFT: deferral keeps the result and needs fewer items."""
    circ = W.qft(n)
    plain = run(checker, circ, np.zeros(1), k, True, False)
    deferred = run(checker, circ, np.zeros(1), k, True, True)
    assert deferred <= plain
    if n >= 9:
        assert deferred < plain, (deferred, plain)
