"""Host logic of the span passes: the planner
(paper_2202_07017_amd/csrc/span_plan.cpp) groups Pauli strings with
arbitrary x masks into passes of up to five independent x masks each and
spreads strings on qubits 0..5 and diagonal strings over them.  A small C++
driver (tests/span_check.cpp) plans a Pauli sum, checks the structure of
every pass (tile insertion masks, group and diagonal offsets, every index of
the state reached exactly once as base ^ lane ^ D(r)) and evaluates it on the
CPU as its descriptor says.  The span passes' value must equal the oracle's
<psi|H|psi> (Sec. 3, Hamiltonian expectation values): a wrong pivot,
direction, sign part, Re/Im choice, lane partner or a dropped or doubled
string changes it."""
import os
import subprocess

import numpy as np
import pytest

import workloads as W

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
    out = dict(line.split(" ", 1) for line in p.stdout.strip().splitlines())
    return int(out["passes"]), float(out["energy"])


def span_sum(n, seed):
    """Random strings (I, X, Y, Z per qubit), several strings on one x mask
    with different z masks (more than one pass holds on one mask), masks
    that are XORs of earlier ones (dependent: a later pass), strings with x
    on qubits 0..5 only (lane strings), diagonal strings, Y factors on lane
    and pivot qubits."""
    rng = np.random.default_rng(seed)
    H = W.random_pauli_sum(n, 40, seed)
    xs, zs, cs = list(H.x_mask), list(H.z_mask), list(H.coeff)
    base_x = int(xs[0])
    for _ in range(70):  # one mask, 70 z masks (Y where z meets x): more than a pass holds
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
    for q in range(5):  # lane pairs (XX, YY, XY) with Z factors anywhere
        for zz in (0, 3 << q, int(rng.integers(0, 1 << n))):
            xs.append(3 << q)
            zs.append(zz)
            cs.append(float(rng.normal()))
    for _ in range(12):  # diagonal strings, and the identity
        xs.append(0)
        zs.append(int(rng.integers(0, 1 << n)))
        cs.append(float(rng.normal()))
    xs.append(0)
    zs.append(0)
    cs.append(0.5)
    xs.append(1 << (n - 1))  # a single high qubit, Y
    zs.append(1 << (n - 1))
    cs.append(0.3)
    return W.PauliSum(n, np.asarray(xs, dtype=np.uint64), np.asarray(zs, dtype=np.uint64),
                      np.asarray(cs, dtype=np.float64))


@pytest.mark.parametrize("n", [12, 13, 15])
def test_span_plan_reproduces_expectation(checker, orc, tmp_path, n):
    H = span_sum(n, 300 + n)
    psi = orc.random_state(n, 4321 + n)
    npass, e_span = run(checker, H, psi, tmp_path)
    high = len({int(x) for x in H.x_mask if int(x) >> 6})
    assert npass >= max(2, (high + 4) // 5), (npass, high)
    ref = orc.expect(psi, H).real
    scale = float(np.sum(np.abs(H.coeff)))
    assert abs(e_span - ref) <= 1e-12 * scale, (e_span, ref)


def test_span_plan_random_strings_pack_five_masks(checker, orc, tmp_path):
    """64 random strings on 16 qubits: distinct x masks, five per pass
    unless a mask depends on a pass's others; strings on qubits 0..5 only
    ride along."""
    n = 16
    H = W.random_pauli_sum(n, 64, 77)
    psi = orc.random_state(n, 78)
    npass, e_span = run(checker, H, psi, tmp_path)
    high = len({int(x) for x in H.x_mask if int(x) >> 6})
    assert npass <= (high + 4) // 5 + 2, (npass, high)
    ref = orc.expect(psi, H).real
    assert abs(e_span - ref) <= 1e-12 * float(np.sum(np.abs(H.coeff)))


@pytest.mark.parametrize("name", ["tfim", "xxz", "diag_only", "lane_only"])
def test_span_plan_models(checker, orc, tmp_path, name):
    """Whole model Hamiltonians through span passes alone: a TFIM and an XXZ
    chain (neighbour pairs on qubits 0..5 as lane strings, the others as
    directions, every ZZ diagonal), only diagonal strings (one pass, padded
    directions) and only strings on qubits 0..5."""
    n = 13
    rng = np.random.default_rng(5)
    if name == "tfim":
        H = W.tfim_chain(n, 0.7)
    elif name == "xxz":
        H = W.xxz_chain(n, 0.5)
    elif name == "diag_only":
        H = W.pauli_sum(n, [("ZZ", (q, (q + 3) % n), float(rng.normal())) for q in range(n)] + [("", (), 0.2)])
    else:
        H = W.pauli_sum(n, [(ab, (q, q + 1), float(rng.normal())) for q in range(5) for ab in ("XX", "YZ", "XY")])
    psi = orc.random_state(n, 31)
    npass, e_span = run(checker, H, psi, tmp_path)
    high = len({int(x) for x in H.x_mask if int(x) >> 6})
    assert npass == max(1, (high + 4) // 5), (npass, high)
    ref = orc.expect(psi, H).real
    assert abs(e_span - ref) <= 1e-12 * float(np.sum(np.abs(H.coeff)))
