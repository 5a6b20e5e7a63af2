"""Host logic of the register-tile Pauli passes: the planner
(paper_2202_07017_amd/csrc/rpass_plan.cpp) sorts the strings of H into
register passes and a rest for the LDS-tile passes.  A small C++ driver
(tests/rpass_check.cpp) plans a Pauli sum, checks the structure of every
pass and evaluates it on the CPU as its descriptor says (tile insertion
masks, lane and register qubits, the transpose of the first pass, the lane,
tile and register parts of each string's sign, the half-sum coefficients,
the chunked sign tables of the diagonal strings).  The register passes'
value plus the oracle's value of the rest must equal the oracle's
<psi|H|psi> (Sec. 3, Hamiltonian expectation values): a wrong mask, sign,
phase, merge or a dropped or doubled string changes it."""
import os
import subprocess

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2202_07017_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if os.environ.get("RPASS_CHECK_EXE"):  # a prebuilt checker (planted-mistake runs)
        return os.environ["RPASS_CHECK_EXE"]
    exe = str(tmp_path_factory.mktemp("rpass") / "rpass_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I" + CSRC, "-I" + os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "rpass_check.cpp"), os.path.join(CSRC, "rpass_plan.cpp"),
                    "-o", exe], check=True)
    return exe


def run(checker, H, psi, tmp_path, env=None):
    path = str(tmp_path / "psi.bin")
    np.ascontiguousarray(psi, dtype=np.complex128).tofile(path)
    lines = ["%d %d" % (H.n, len(H.coeff))]
    lines += ["%d %d %.17g" % (int(x), int(z), float(c)) for x, z, c in zip(H.x_mask, H.z_mask, H.coeff)]
    p = subprocess.run([checker, path], input="\n".join(lines) + "\n", capture_output=True, text=True,
                       env=env)
    assert p.returncode == 0, p.stderr
    assert "runtime error" not in p.stderr and "Sanitizer" not in p.stderr, p.stderr
    out = dict(line.split(" ", 1) if " " in line else (line, "") for line in p.stdout.strip().splitlines())
    rest = [int(v) for v in out["rest"].split()]
    return int(out["passes"]), rest, float(out["energy"])


def sub(H, idx):
    idx = np.asarray(idx, dtype=np.int64)
    return W.PauliSum(H.n, H.x_mask[idx], H.z_mask[idx], H.coeff[idx])


def mixed_sum(n, seed):
    """Diagonal strings anywhere (more than one launch holds), single X and
    Y on every qubit, XX / YY / XY / YX on neighbours with and without Z
    factors elsewhere, non-neighbouring pairs, three-qubit strings, and
    pairs of qubit 4 with qubits above (cross-lane strings of the first
    pass, or left to the LDS tiles)."""
    rng = np.random.default_rng(seed)
    t = [("", (), 0.4)]
    for _ in range(60):
        qs = [int(v) for v in rng.choice(n, int(rng.integers(1, 4)), replace=False)]
        t.append(("Z" * len(qs), qs, float(rng.normal())))
    for q in range(n):
        t.append((str(rng.choice(["X", "Y"])), (q,), float(rng.normal())))
    for q in range(n - 1):
        for ab in ("XX", "YY", "XY", "YX"):
            if rng.random() < 0.6:
                t.append((ab, (q, q + 1), float(rng.normal())))
        if rng.random() < 0.5:
            others = [v for v in range(n) if v not in (q, q + 1)]
            zq = [int(v) for v in rng.choice(others, int(rng.integers(1, 3)), replace=False)]
            t.append(("XY" + "Z" * len(zq), [q, q + 1] + zq, float(rng.normal())))
        if rng.random() < 0.3:
            t.append(("ZX", (q, q + 1), float(rng.normal())))
    t.append(("XX", (1, 3), 0.3))
    t.append(("YY", (6, 9), -0.2))
    t.append(("XXX", (0, 7, n - 1), 0.7))
    t.append(("XX", (4, 5), 0.25))
    t += [("XX", (4, 7), 0.35), ("XY", (4, 6), -0.15), ("YX", (4, 9), 0.2), ("YYZ", (4, 8, 1), 0.1)]
    return W.pauli_sum(n, t)


@pytest.mark.parametrize("name,n", [("tfim", 12), ("tfim", 14), ("xxz", 13), ("heis_fields", 14),
                                    ("mixed", 12), ("mixed", 13), ("mixed", 15)])
def test_register_pass_plan_reproduces_expectation(checker, orc, tmp_path, name, n):
    if name == "tfim":
        H = W.tfim_chain(n, 0.7)
    elif name == "xxz":
        H = W.xxz_chain(n, 0.5)
    elif name == "heis_fields":
        rng = np.random.default_rng(n)
        t = [(ab, (q, q + 1), 1.0) for q in range(n - 1) for ab in ("XX", "YY", "ZZ")]
        t += [(c, (q,), float(rng.normal())) for q in range(n) for c in "XYZ"]
        H = W.pauli_sum(n, t)
    else:
        H = mixed_sum(n, 100 + n)
    psi = orc.random_state(n, 1234 + n)
    npass, rest, e_reg = run(checker, H, psi, tmp_path)
    assert npass >= 1
    e_rest = orc.expect(psi, sub(H, rest)).real if rest else 0.0
    ref = orc.expect(psi, H).real
    scale = float(np.sum(np.abs(H.coeff)))
    assert abs(e_reg + e_rest - ref) <= 1e-12 * scale, (e_reg, e_rest, ref)
    if name in ("tfim", "xxz", "heis_fields"):
        # every string of these models goes to the register passes (the
        # neighbour pair (4, 5) as a cross-lane string of the first pass)
        assert rest == [], [(j, int(H.x_mask[j]), int(H.z_mask[j])) for j in rest]
