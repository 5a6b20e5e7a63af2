"""qsv_expectation_noalloc (no workspace argument, partial sums in the
library's static per-GPU scratch) against qsv_expectation (caller workspace)
through the C ABI: two calls in a row on the same GPU, the second with a
smaller state, so stale partial sums of the first call would show; results
must equal qsv_expectation's bit for bit (same kernels, same summation order)
and the oracle within the expectation tolerance.  No torch allocation
happens inside the calls."""
import numpy as np
import pytest

import workloads as W
from gpu_util import say, to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2202_07017_amd import qsv
    qsv.lib()
    return qsv


@pytest.mark.parametrize("name", ["c64", "c128"])
def test_noalloc_expectation_matches_workspace_version(q, orc, name):
    import torch
    rng = np.random.default_rng(2027)
    # register passes (TFIM), span passes (random strings on 18 qubits), tile
    # passes, the small-state kernels; sizes shrink from call to call
    cases = [(20, W.tfim_chain(20)), (18, W.random_pauli_sum(18, 24, seed=7)),
             (13, W.random_pauli_sum(13, 9, seed=5)), (6, W.xxz_chain(6, 0.7))]
    for n, H in cases:
        psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
        psi /= np.linalg.norm(psi)
        if name == "c64":
            psi = psi.astype(np.complex64).astype(np.complex128)
        d = to_gpu(psi, name)
        ref = torch.empty(2, dtype=torch.float64, device="cuda")
        got = torch.full((2,), 7.0, dtype=torch.float64, device="cuda")
        q.qsv_expectation(d, H, out=ref)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        say("noalloc expectation", name, n, len(H.coeff))
        q.qsv_expectation_noalloc(d, H, out=got)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        g, r = got.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(g, r), (n, g, r)
        E = orc.expect(psi, H)
        scale = float(np.sum(np.abs(H.coeff)))
        assert abs(g[0] - E.real) <= 1e-10 * scale, (n, g[0], E)


def test_noalloc_rejects_bad_arguments(q):
    import ctypes
    L = q.lib()
    H = q.PauliSum(W.tfim_chain(4))
    assert L.qsv_expectation_noalloc(ctypes.c_void_p(1 << 20), 4, 1, ctypes.byref(H.s), None,
                                     None) == q.ERR_ARG
    assert L.qsv_expectation_noalloc(ctypes.c_void_p(1 << 20), 4, 3, ctypes.byref(H.s),
                                     ctypes.c_void_p(1 << 20), None) == q.ERR_ARG
