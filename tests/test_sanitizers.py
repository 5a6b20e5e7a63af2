"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle (oracle/oracle.c) is driven through every entry point by
tests/oracle_sanitize_check.c, the tile-program compiler of the library
(paper_2202_07017_amd/csrc/tileprog.cpp) through tests/tileprog_check.cpp on
random gate lists, and the register-pass planner (csrc/rpass_plan.cpp)
through tests/rpass_check.cpp on mixed Pauli sums, the span-pass planner
(csrc/span_plan.cpp) through tests/span_check.cpp, the qubit permutation
planner (csrc/qperm_plan.cpp) through tests/qperm_check.cpp on swap runs, the
fusion planner (csrc/fuse_plan.cpp) through tests/fuse_check.cpp on random
circuits; all are built with g++/gcc and
-fsanitize=address,undefined -fno-sanitize-recover=all, so any out-of-bounds
access, use after free, leak or undefined behaviour aborts the run.  The
GPU code is not built here (GPU sanitizers are not available)."""
import os
import subprocess

import numpy as np
import pytest

import workloads as W
from test_rpass_plan import mixed_sum
from test_rpass_plan import run as run_rpass
from test_rpass_plan import sub
from test_tileprog import hea_gates, random_gates, run_checker

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2202_07017_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    subprocess.run(["gcc", "-O1", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-ffp-contract=off"] + SAN +
                   [os.path.join(ROOT, "tests", "oracle_sanitize_check.c"),
                    os.path.join(ROOT, "oracle", "oracle.c"), "-o", exe, "-lm"], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr


@pytest.fixture(scope="module")
def san_checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("tileprog_san") / "tileprog_check")
    subprocess.run(["g++", "-O1", "-std=c++17", "-I" + CSRC] + SAN +
                   [os.path.join(ROOT, "tests", "tileprog_check.cpp"),
                    os.path.join(CSRC, "tileprog.cpp"), "-o", exe], check=True)
    return exe


@pytest.mark.parametrize("n,m,cap,count,seed", [(9, 6, 512, 160, 1), (12, 7, 40, 200, 3),
                                                (7, 12, 512, 60, 5), (10, 4, 512, 150, 6)])
def test_tile_programs_under_sanitizers(orc, san_checker, n, m, cap, count, seed):
    gates = random_gates(n, count, seed)
    rng = np.random.default_rng(100 + seed)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi /= np.linalg.norm(psi)
    got = run_checker(san_checker, n, m, cap, gates, psi)
    circ = W.Circuit(n, [W.Op("matrix", (t,), controls=tuple(cs), matrix=np.asarray(M, complex))
                         for _, t, cs, _, M in gates])
    assert np.max(np.abs(got - orc.run(circ, psi0=psi))) < 1e-12


def test_tile_program_ladder_under_sanitizers(orc, san_checker):
    gates = hea_gates(11, 3, 18)
    rng = np.random.default_rng(3)
    psi = rng.normal(size=1 << 11) + 1j * rng.normal(size=1 << 11)
    psi /= np.linalg.norm(psi)
    got = run_checker(san_checker, 11, 8, 512, gates, psi)
    circ = W.Circuit(11, [W.Op("matrix", (t,), controls=tuple(cs), matrix=np.asarray(M, complex))
                          for _, t, cs, _, M in gates])
    assert np.max(np.abs(got - orc.run(circ, psi0=psi))) < 1e-12


def test_register_pass_planner_under_sanitizers(orc, tmp_path):
    exe = str(tmp_path / "rpass_check")
    subprocess.run(["g++", "-O1", "-std=c++17", "-I" + CSRC, "-I" + os.path.join(ROOT, "include")] + SAN +
                   [os.path.join(ROOT, "tests", "rpass_check.cpp"), os.path.join(CSRC, "rpass_plan.cpp"),
                    "-o", exe], check=True)
    for n in (12, 14):
        H = mixed_sum(n, 7 + n)
        psi = orc.random_state(n, 99 + n)
        _, rest, e_reg = run_rpass(exe, H, psi, tmp_path, env=ENV)
        e_rest = orc.expect(psi, sub(H, rest)).real if rest else 0.0
        assert abs(e_reg + e_rest - orc.expect(psi, H).real) <= 1e-12 * float(np.sum(np.abs(H.coeff)))


def test_span_pass_planner_under_sanitizers(orc, tmp_path):
    from test_span_plan import build_checker, span_sum
    from test_span_plan import run as run_span
    exe = build_checker(str(tmp_path / "span_check"), SAN)
    for n in (12, 14):
        H = span_sum(n, 11 + n)
        psi = orc.random_state(n, 55 + n)
        _, e_span = run_span(exe, H, psi, tmp_path, env=ENV)
        assert abs(e_span - orc.expect(psi, H).real) <= 1e-12 * float(np.sum(np.abs(H.coeff)))


def test_qubit_permutation_planner_under_sanitizers(tmp_path):
    from test_qperm_plan import build_checker, reversal
    from test_qperm_plan import run as run_qperm
    exe = build_checker(str(tmp_path / "qperm_check"), SAN)
    rng = np.random.default_rng(8)
    for n, rl in ((12, 6), (13, 5), (14, 6)):
        assert run_qperm(exe, n, rl, reversal(n), env=ENV) == 1
        swaps = [tuple(int(v) for v in rng.permutation(n)[:2]) for _ in range(3 * n)]
        assert run_qperm(exe, n, rl, swaps, env=ENV) in (0, 1, 2)


def test_fusion_planner_under_sanitizers(tmp_path):
    from test_fuse_plan import build_checker, random_circuit
    from test_fuse_plan import run as run_fuse
    exe = build_checker(str(tmp_path / "fuse_check"), SAN)
    for seed in range(4):
        circ, params = random_circuit(7, 900 + seed, seed % 2 == 0)
        for k in (2, 3, 5):
            run_fuse(exe, circ, params, k, seed % 2 == 1, True, env=ENV)
    run_fuse(exe, W.qft(9), np.zeros(1), 5, True, True, env=ENV)
