"""Host logic of the qubit permutation passes: consecutive SWAP gates (Sec. 3
gate set) compose into one permutation of the bits of every amplitude index,
which plans apply in one in-place pass (an involution) or two.  A small C++
driver (tests/qperm_check.cpp) applies the swaps one after another to the
index vector, plans the composition
(paper_2202_07017_amd/csrc/qperm_plan.cpp), checks each pass's structure
and replays it tile by tile the way the kernel walks it; the result must
equal the sequential one exactly and every index must be written once per
pass."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2202_07017_amd", "csrc")


def build_checker(out, extra=()):
    subprocess.run(["g++", "-O2", "-std=c++17", "-I" + CSRC] + list(extra) +
                   [os.path.join(ROOT, "tests", "qperm_check.cpp"), os.path.join(CSRC, "qperm_plan.cpp"),
                    "-o", out], check=True)
    return out


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if os.environ.get("QPERM_CHECK_EXE"):  # a prebuilt checker (planted-mistake runs)
        return os.environ["QPERM_CHECK_EXE"]
    return build_checker(str(tmp_path_factory.mktemp("qperm") / "qperm_check"))


def run(checker, n, rl, swaps, env=None):
    text = "%d %d %d\n" % (n, rl, len(swaps)) + "".join("%d %d\n" % s for s in swaps)
    p = subprocess.run([checker], input=text, capture_output=True, text=True, env=env)
    assert p.returncode == 0, p.stderr
    assert "runtime error" not in p.stderr and "Sanitizer" not in p.stderr, p.stderr
    return int(p.stdout.split()[1])


def reversal(n):
    return [(b, n - 1 - b) for b in range(n // 2)]


@pytest.mark.parametrize("rl", [5, 6])
@pytest.mark.parametrize("n", [12, 13, 16])
def test_bit_reversal_is_one_pass(checker, n, rl):
    """The QFT's closing swaps reverse the bit order: an involution, one pass."""
    assert run(checker, n, rl, reversal(n)) == 1


@pytest.mark.parametrize("rl", [5, 6])
@pytest.mark.parametrize("seed", range(6))
def test_random_swap_sequences(checker, rl, seed):
    """Random swaps on any qubits (low, high, repeated, chained into long
    cycles): two passes unless the composition is an involution."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2 * rl, 17))
    swaps = [tuple(int(v) for v in rng.permutation(n)[:2]) for _ in range(int(rng.integers(2, 3 * n)))]
    assert run(checker, n, rl, swaps) in (1, 2)


def test_cycle_needs_two_passes(checker):
    """A 3-cycle of bits (two chained swaps) is not an involution."""
    assert run(checker, 14, 6, [(0, 7), (7, 13)]) == 2
    assert run(checker, 14, 6, [(8, 9), (9, 10), (10, 11)]) == 2


def test_swaps_that_cancel_need_no_pass(checker):
    assert run(checker, 12, 6, [(2, 9), (9, 2)]) == 0
    assert run(checker, 12, 6, [(0, 1), (1, 2), (0, 1), (1, 2), (0, 1), (1, 2)]) == 0


@pytest.mark.parametrize("swaps", [[(1, 4), (0, 5)], [(7, 9), (8, 11)], [(0, 11), (5, 6), (7, 8)]])
def test_tiles_inside_rows_and_above(checker, swaps):
    """Swaps among the row bits only (the tile is filled with other bits),
    among high bits only, and mixed."""
    assert run(checker, 12, 6, swaps) == 1
