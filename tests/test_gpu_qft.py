"""GPU parity of the QFT workload (the quantum Fourier transform among the
paper's built-in circuits, Sec. 3): Hadamards, controlled phases (diagonal
launches) and swaps (bit-exact moves), unfused and fused, against the oracle
on seeded states, and at n = 30 against the closed-form transform of a basis
state, sampled."""
import numpy as np
import pytest

import workloads as W
from gpu_util import TOL, rand_state, say, to_gpu, to_np, torch_dtype

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
