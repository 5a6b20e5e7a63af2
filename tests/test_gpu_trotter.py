"""GPU parity of Trotterised time evolution (Sec. 3: Hamiltonians evolved
with the Trotter decomposition): qsv_trotter_plan_create plans against the
oracle's Trotter product (matrix exponentials of each term) on seeded states,
unfused and fused; at n = 30 the pure-field evolution of |0...0> against its
closed form, and a symmetric forward/backward round trip of the TFIM against
the seeded input."""
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


def _hams(n):
    return {
        "tfim": W.tfim_chain(n, 0.9),
        "xxz": W.xxz_chain(n, 0.5),
        "maxcut": W.maxcut(n, [(i, (3 * i + 1) % n) for i in range(n) if i != (3 * i + 1) % n]),
        "mixed": W.pauli_sum(n, [("XYZ", [0, n // 2, n - 1], 0.9), ("YY", [1, 2], -0.4),
                                 ("", [], 0.3), ("ZXZYX", [0, 1, 2, 3, n - 1], 0.2)]),
    }


@pytest.mark.parametrize("name", DTYPES)
@pytest.mark.parametrize("n", [5, 12, 16])
@pytest.mark.parametrize("ham", ["tfim", "xxz", "maxcut", "mixed"])
@pytest.mark.parametrize("order,fuse", [(1, 1), (1, 5), (2, 3), (2, 5)])
def test_trotter_parity(q, orc, name, n, ham, order, fuse):
    H = _hams(n)[ham]
    rng = np.random.default_rng(800 + n)
    psi = rand_state(n, rng, name)
    say("trotter", name, n, ham, order, fuse)
    d = to_gpu(psi, name)
    q.TrotterPlan(H, 0.13, 3, order, 2 if name == "c128" else 1, fuse).run(d)
    ref = orc.trotter(psi, H, 0.13, 3, order)
    err = np.max(np.abs(to_np(d) - ref))
    assert err <= TOL[name], err


def test_trotter_errors(q):
    n = 8
    with pytest.raises(q.QsvError):
        q.TrotterPlan(W.pauli_sum(n, [("XXXXXX", list(range(6)), 1.0)]), 0.1, 1, 1, 2)
    with pytest.raises(q.QsvError):
        q.TrotterPlan(W.tfim_chain(n), 0.1, 1, 3, 2)
    with pytest.raises(q.QsvError):
        q.TrotterPlan(W.tfim_chain(n), 0.1, -1, 1, 2)
    p = q.TrotterPlan(W.tfim_chain(n), 0.1, 0, 2, 2)
    assert p.info()[0] == 0


def test_trotter_full_size(q, orc):
    """n = 30 complex64 and complex128: H = sum_i X_i (commuting, so Trotter is
    exact) from |0...0>: amplitude i = cos(t)^(n-w) (-i sin t)^w, w = popcount(i);
    then the TFIM, 2 symmetric steps forward and 2 with -tau, must return the
    seeded random state."""
    import torch
    n, t_step, steps = 30, 0.21, 2
    t = t_step * steps
    rng = np.random.default_rng(3030)
    idx = np.concatenate([rng.integers(0, 1 << n, 200), [0, (1 << n) - 1]]).astype(np.int64)
    w = np.array([bin(int(i)).count("1") for i in idx])
    want = np.cos(t) ** (n - w) * (-1j * np.sin(t)) ** w
    Hx = W.pauli_sum(n, [("X", [i], 1.0) for i in range(n)])
    seed = 99
    scale = 1.0 / np.sqrt(orc.random_norm2(n, seed))
    ref = orc.random_amps(seed, scale, idx.astype(np.uint64))
    for name in DTYPES:
        dc = 2 if name == "c128" else 1
        d = torch.empty(1 << n, dtype=torch_dtype(name), device="cuda")
        say("trotter n30 field", name)
        q.qsv_init_basis(d, 0)
        q.TrotterPlan(Hx, t_step, steps, 1, dc, 5).run(d)
        got = d[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.complex128)
        err = np.max(np.abs(got - want))
        assert err <= TOL[name] and err / np.max(np.abs(want)) <= 1e-5, err
        say("trotter n30 round trip", name)
        q.qsv_init_random(d, seed)
        H = W.tfim_chain(n, 0.7)
        q.TrotterPlan(H, 0.05, 2, 2, dc, 5).run(d)
        q.TrotterPlan(H, -0.05, 2, 2, dc, 5).run(d)
        got = d[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.complex128)
        err = np.max(np.abs(got - ref))
        assert err <= TOL[name] and err / np.max(np.abs(ref)) <= 1e-5, err
        del d
        torch.cuda.empty_cache()
