"""Host logic of the span passes: the planner
(paper_2202_07017_amd/csrc/span_plan.cpp) groups Pauli strings with
arbitrary x masks into passes of up to five independent x masks each.  A
small C++ driver (tests/span_check.cpp) plans a Pauli sum, checks the
structure of every pass (tile insertion masks, group offsets, every index of
the state reached exactly once as base ^ lane ^ D(r)) and evaluates it on the
CPU as its descriptor says.  The span passes' value plus the oracle's value
of the strings they leave must equal the oracle's <psi|H|psi> (Sec. 3,
Hamiltonian expectation values): a wrong pivot, direction, sign part, Re/Im
choice or a dropped or doubled string changes it."""
import os
import subprocess

import numpy as np
import pytest

import workloads as W
from test_rpass_plan import sub

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2202_07017_amd", "csrc")


def build_checker(out, extra=()):
    subprocess.run(["g++", "-O2", "-std=c++17", "-I" + CSRC, "-I" + os.path.join(ROOT, "include")] + list(extra) +
                   [os.path.join(ROOT, "tests", "span_check.cpp"), os.path.join(CSRC, "span_plan.cpp"),
                    "-o", out], check=True)
    return out


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if os.environ.get("SPAN_CHECK_EXE"):  # a prebuilt checker (planted-mistake runs)
        return os.environ["SPAN_CHECK_EXE"]
    return build_checker(str(tmp_path_factory.mktemp("span") / "span_check"))


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


def span_sum(n, seed):
    """Random strings (I, X, Y, Z per qubit), several strings on one x mask
    with different z masks (more than one pass holds on one mask), masks
    that are XORs of earlier ones (dependent: a later pass), strings with x
    on qubits 0..5 only (left to other passes), Y factors on lane and pivot
    qubits."""
    rng = np.random.default_rng(seed)
    H = W.random_pauli_sum(n, 40, seed)
    xs, zs, cs = list(H.x_mask), list(H.z_mask), list(H.coeff)
    base_x = int(xs[0])
    for _ in range(40):  # one mask, 40 z masks (Y where z meets x)
        xs.append(base_x)
        zs.append(int(rng.integers(0, 1 << n)))
        cs.append(float(rng.normal()))
    for a, b in ((1, 2), (3, 4), (1, 5)):
        xs.append(int(xs[a]) ^ int(xs[b]))
        zs.append(int(rng.integers(0, 1 << n)))
        cs.append(float(rng.normal()))
    for q in (0, 3, 5):
        xs.append(1 << q)
        zs.append(int(rng.integers(0, 1 << n)))
        cs.append(float(rng.normal()))
    xs.append(1 << (n - 1))  # a single high qubit, Y
    zs.append(1 << (n - 1))
    cs.append(0.3)
    return W.PauliSum(n, np.asarray(xs, dtype=np.uint64), np.asarray(zs, dtype=np.uint64),
                      np.asarray(cs, dtype=np.float64))


@pytest.mark.parametrize("n", [12, 13, 15])
def test_span_plan_reproduces_expectation(checker, orc, tmp_path, n):
    H = span_sum(n, 300 + n)
    psi = orc.random_state(n, 4321 + n)
    npass, rest, e_span = run(checker, H, psi, tmp_path)
    assert npass >= 10
    # exactly the strings with no x bit at qubit 6 or above are left
    low = [j for j in range(len(H.coeff)) if int(H.x_mask[j]) >> 6 == 0]
    assert rest == low
    e_rest = orc.expect(psi, sub(H, rest)).real if rest else 0.0
    ref = orc.expect(psi, H).real
    scale = float(np.sum(np.abs(H.coeff)))
    assert abs(e_span + e_rest - ref) <= 1e-12 * scale, (e_span, e_rest, ref)


def test_span_plan_random_strings_pack_five_masks(checker, orc, tmp_path):
    """64 random strings on 16 qubits: distinct x masks, five per pass
    (13 passes) unless a mask depends on a pass's others."""
    n = 16
    H = W.random_pauli_sum(n, 64, 77)
    psi = orc.random_state(n, 78)
    npass, rest, e_span = run(checker, H, psi, tmp_path)
    keep = [j for j in range(64) if int(H.x_mask[j]) >> 6 != 0]
    assert npass <= (len(keep) + 4) // 5 + 2, npass
    e_rest = orc.expect(psi, sub(H, rest)).real if rest else 0.0
    ref = orc.expect(psi, H).real
    assert abs(e_span + e_rest - ref) <= 1e-12 * float(np.sum(np.abs(H.coeff)))
