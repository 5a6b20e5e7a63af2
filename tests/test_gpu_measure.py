"""GPU parity of measurement (Sec. 3: simulated measurements sample the
state's Born probabilities): marginal probabilities and inverse-transform
shot sampling through the C ABI against the oracle on the same seeded inputs,
plus full-size (n = 30) checks against closed forms that hold at any size."""
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


def _u_gpu(u):
    import torch
    return torch.from_numpy(np.ascontiguousarray(u, dtype=np.float64)).cuda()


def _check_samples(psi, u, got, want, tol_rel):
    """Equal to the oracle except where t = u T lies within rounding of a
    boundary of the running sum; there the outcome must still bracket t and
    have nonzero probability."""
    p = np.abs(psi) ** 2
    C = np.cumsum(p)
    T = C[-1]
    bad = np.nonzero(got != want)[0]
    assert bad.size <= max(2, u.size // 1000), (bad.size, u.size)
    for s in bad:
        g = int(got[s])
        t = min(max(u[s], 0.0), 1.0) * T
        lo = C[g - 1] if g else 0.0
        assert p[g] > 0 and lo - tol_rel * T <= t <= C[g] + tol_rel * T, (s, g, int(want[s]))
    assert np.all(p[got] > 0)


@pytest.mark.parametrize("name", DTYPES)
@pytest.mark.parametrize("n,qubits", [(1, [0]), (4, [3, 0]), (6, [0, 1, 2, 3, 4, 5]),
                                      (9, [8, 7, 6, 5, 4, 3, 2, 1, 0]), (12, [11]), (12, [5, 0]),
                                      (13, [0, 1, 2, 3, 4, 5, 6, 7, 8, 9]), (17, [16, 2, 9]),
                                      (18, [0, 17, 3, 12, 6, 9, 1, 15, 4, 10, 13, 7, 2]),
                                      (20, [19, 18, 17, 16, 15, 14, 13, 12, 11, 10, 9, 8, 7, 6, 5, 4])])
def test_probabilities_parity(q, orc, name, n, qubits):
    rng = np.random.default_rng(500 + n)
    psi = rand_state(n, rng, name)
    say("probabilities", name, n, qubits)
    got = q.qsv_probabilities(to_gpu(psi, name), qubits).cpu().numpy()
    ref = orc.probabilities(psi, qubits)
    assert np.max(np.abs(got - ref)) <= 1e-13, np.max(np.abs(got - ref))


@pytest.mark.parametrize("name", DTYPES)
@pytest.mark.parametrize("n", [1, 3, 6, 7, 9, 10, 11, 16, 17, 20])
def test_sample_parity(q, orc, name, n):
    rng = np.random.default_rng(900 + n)
    psi = rand_state(n, rng, name)
    psi[::7] = 0                                      # zero-probability outcomes
    psi[1 % psi.size] *= 1e-6
    u = np.concatenate([W.uniforms(20000, 40 + n), [0.0, 1.0 - 2.0 ** -53, 1.0, -0.5, np.nan]])
    say("sample", name, n)
    got = q.qsv_sample(to_gpu(psi, name), _u_gpu(u)).cpu().numpy()
    want = orc.sample(psi, u)
    assert got.shape == want.shape and got.dtype == np.int64
    _check_samples(psi, u, got, want, 1e-13)


@pytest.mark.parametrize("name", DTYPES)
def test_sample_uniform_exact(q, name):
    """Equal superposition with n even: every weight and running sum is exact,
    so the outcome is floor(u 2^n) on every shot, grid points included."""
    import torch
    n = 14
    N = 1 << n
    psi = torch.full((N,), 2.0 ** (-n / 2), dtype=torch_dtype(name), device="cuda")
    u = np.concatenate([np.arange(0, N, 7) / N, W.uniforms(50000, 8)])
    say("sample uniform", name, n)
    got = q.qsv_sample(psi, _u_gpu(u)).cpu().numpy()
    assert np.array_equal(got, np.floor(u * N).astype(np.int64))


def test_sample_edges(q):
    """Zero vector -> 0; no shots -> nothing written; negative counts refused."""
    import torch
    z = torch.zeros(1 << 8, dtype=torch.complex128, device="cuda")
    assert q.qsv_sample(z, _u_gpu([0.0, 0.5, 0.99])).cpu().tolist() == [0, 0, 0]
    out = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    q.qsv_sample(z, _u_gpu(np.zeros(0)), out=out)
    assert out.item() == -7
    lib = q.lib()
    w = q.measure_workspace(8, 2, "cuda")
    st = lib.qsv_sample(q._ptr(z), 8, 2, q._ptr(w), -1, q._ptr(out), q._ptr(w), None)
    assert st != 0
    with pytest.raises(q.QsvError):
        q.qsv_probabilities(z, [3, 3])
    with pytest.raises(q.QsvError):
        q.qsv_probabilities(z, [8])


def _product_state(q, n, name, theta):
    """prod_q (cos(theta_q / 2)|0> + sin(theta_q / 2)|1>) built on the GPU."""
    import torch
    d = torch.empty(1 << n, dtype=torch_dtype(name), device="cuda")
    q.qsv_init_basis(d, 0)
    for j in range(n):
        c, s = np.cos(theta[j] / 2), np.sin(theta[j] / 2)
        q.qsv_apply_gate(d, [j], [], np.array([[c, -s], [s, c]], dtype=np.complex128))
    return d


def _product_cdf(i, p0):
    """C_i of a product distribution (p0[q] = weight of bit q = 0), by
    descending bits: every 1 bit of i adds the mass of the prefix with a 0
    there and anything below."""
    n = len(p0)
    acc, pref = 0.0, 1.0
    for b in range(n - 1, -1, -1):
        if (i >> b) & 1:
            acc += pref * p0[b]
            pref *= 1.0 - p0[b]
        else:
            pref *= p0[b]
    return acc + pref


def test_full_size_n30(q):
    """n = 30: the equal superposition (exact: floor(u 2^30)) in complex64 and
    complex128, then a product state in complex128 whose running sum has a
    closed form: every shot brackets u T, and marginals factorise."""
    import torch
    n = 30
    N = 1 << n
    u = W.uniforms(100000, 31)
    for name in DTYPES:
        say("n30 uniform", name)
        psi = torch.full((N,), 2.0 ** (-n / 2), dtype=torch_dtype(name), device="cuda")
        got = q.qsv_sample(psi, _u_gpu(u)).cpu().numpy()
        assert np.array_equal(got, np.floor(u * N).astype(np.int64))
        pr = q.qsv_probabilities(psi, [29, 0, 15]).cpu().numpy()
        assert np.all(pr == 0.125)
        del psi
        torch.cuda.empty_cache()
    theta = np.random.default_rng(32).uniform(0.3, 2.8, n)
    p0 = np.cos(theta / 2) ** 2
    say("n30 product c128")
    d = _product_state(q, n, "c128", theta)
    got = q.qsv_sample(d, _u_gpu(u[:20000])).cpu().numpy()
    T = float(q.qsv_norm2(d).cpu()[0])
    for s, g in enumerate(got):
        t = u[s] * T
        lo = _product_cdf(int(g) - 1, p0) if g else 0.0
        hi = _product_cdf(int(g), p0)
        assert lo - 1e-12 <= t <= hi + 1e-12, (s, int(g), lo, t, hi)
    for qs in ([29, 0, 15], list(range(10)) + list(range(20, 30)), [7]):
        say("n30 product marginal", qs)
        pr = q.qsv_probabilities(d, qs).cpu().numpy()
        m = len(qs)
        b = np.arange(1 << m)
        want = np.ones(1 << m)
        for j, qq in enumerate(qs):
            bit = (b >> (m - 1 - j)) & 1
            want *= np.where(bit == 0, p0[qq], 1 - p0[qq])
        assert np.max(np.abs(pr - want)) <= 1e-12, np.max(np.abs(pr - want))
    del d
    torch.cuda.empty_cache()


def test_full_size_n32_uniform(q):
    """n = 32 (32 GiB complex64, 64 GiB complex128): the equal superposition,
    exact in both precisions, samples floor(u 2^32) on every shot (outcome
    indices past 2^31) and every marginal entry is exactly 2^-m."""
    import torch
    n = 32
    N = 1 << n
    u = np.concatenate([W.uniforms(50000, 32), [0.5, 1.0 - 2.0 ** -40]])
    for name in DTYPES:
        say("n32 uniform", name)
        psi = torch.full((N,), 2.0 ** (-n / 2), dtype=torch_dtype(name), device="cuda")
        got = q.qsv_sample(psi, _u_gpu(u)).cpu().numpy()
        assert np.array_equal(got, np.floor(u * N).astype(np.int64))
        for qs in ([31], [0, 31, 16], list(range(31, 19, -1))):
            pr = q.qsv_probabilities(psi, qs).cpu().numpy()
            assert np.all(pr == 2.0 ** -len(qs))
        del psi
        torch.cuda.empty_cache()


@pytest.mark.parametrize("n,qubits", [(12, [0]), (12, [11, 0, 5]), (12, list(range(11, -1, -1))),
                                      (14, [13, 12, 11, 10, 9, 8, 7, 6, 5, 4, 3, 2, 1]), (30, [29, 0, 15])])
def test_frequencies_parity(q, orc, n, qubits):
    """Counts of GPU shots over a qubit subset equal the oracle's counts of the
    same shots exactly (the LDS path for 2^m <= 4096, the device path above)."""
    import torch
    rng = np.random.default_rng(70 + n)
    if n <= 20:
        psi = rand_state(n, rng, "c128")
        d = to_gpu(psi, "c128")
    else:
        d = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
        q.qsv_init_random(d, 7)
    u = W.uniforms(300000, 5 + n)
    say("frequencies", n, qubits)
    smp = q.qsv_sample(d, _u_gpu(u))
    got = q.qsv_frequencies(smp, n, qubits).cpu().numpy()
    want = orc.frequencies(n, smp.cpu().numpy(), qubits)
    assert np.array_equal(got, want) and got.sum() == u.size
    del d
    torch.cuda.empty_cache()


def test_frequencies_edges(q):
    import torch
    out = torch.full((4,), 9, dtype=torch.int64, device="cuda")
    q.qsv_frequencies(torch.zeros(0, dtype=torch.int64, device="cuda"), 5, [4, 1], out=out)
    assert out.cpu().tolist() == [0, 0, 0, 0]
    s = torch.tensor([3, 3, 0, 31], dtype=torch.int64, device="cuda")
    assert q.qsv_frequencies(s, 5, [1, 0]).cpu().tolist() == [1, 0, 0, 3]
    with pytest.raises(q.QsvError):
        q.qsv_frequencies(s, 5, [5])
    with pytest.raises(q.QsvError):
        q.qsv_frequencies(s, 5, [1, 1])


@pytest.mark.parametrize("name", DTYPES)
@pytest.mark.parametrize("n,qubits", [(1, [0]), (5, [4, 1]), (12, [0, 11, 6]), (20, [19, 3, 7, 12, 0])])
def test_collapse_parity(q, orc, name, n, qubits):
    """Collapse on the outcome's probability taken from qsv_probabilities on
    the device, against the oracle's projection with the oracle's marginal."""
    rng = np.random.default_rng(300 + n)
    psi = rand_state(n, rng, name)
    d = to_gpu(psi, name)
    pr = q.qsv_probabilities(d, qubits)
    b = int(np.argmax(pr.cpu().numpy()))
    say("collapse", name, n, qubits, b)
    q.qsv_collapse(d, qubits, b, pr[b:b + 1])
    ref = orc.collapse(psi, qubits, b, orc.probabilities(psi, qubits)[b])
    err = np.max(np.abs(to_np(d) - ref))
    assert err <= TOL[name], err
    assert abs(float(q.qsv_norm2(d).cpu()[0]) - 1.0) <= (1e-12 if name == "c128" else 1e-5)


def test_collapse_full_size_n30(q):
    """n = 30 complex64: a product state collapsed on qubits (29, 0, 15) with
    outcome 0b101 equals the product state with those qubits fixed to 1, 0, 1
    (closed form, sampled), and has unit norm."""
    import torch
    n = 30
    theta = np.random.default_rng(33).uniform(0.3, 2.8, n)
    d = _product_state(q, n, "c64", theta)
    qs, b = [29, 0, 15], 0b101
    pr = q.qsv_probabilities(d, qs)
    say("collapse n30")
    q.qsv_collapse(d, qs, b, pr[b:b + 1])
    rng = np.random.default_rng(34)
    idx = rng.integers(0, 1 << n, 300)
    idx = np.concatenate([idx, (idx | (1 << 29) | (1 << 15)) & ~1])   # half of them on the outcome
    got = d[torch.from_numpy(idx.astype(np.int64)).cuda()].cpu().numpy().astype(np.complex128)
    want = np.ones(idx.size, dtype=np.complex128)
    for j in range(n):
        bit = (idx >> j) & 1
        if j in qs:
            need = (b >> (2 - qs.index(j))) & 1
            want *= (bit == need)
        else:
            want *= np.where(bit == 0, np.cos(theta[j] / 2), np.sin(theta[j] / 2))
    assert np.max(np.abs(got - want)) <= 1e-5 * max(1.0, float(np.max(np.abs(want)))) + 1e-9
    assert abs(float(q.qsv_norm2(d).cpu()[0]) - 1.0) <= 1e-5
    del d
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name", DTYPES)
@pytest.mark.parametrize("n", [3, 11, 20])
def test_sample_seeded(q, orc, name, n):
    """Device-drawn uniforms (draw s of the seed's keyed SplitMix64 stream) give the oracle's
    outcomes for the oracle's own draw of the same counter-based stream."""
    rng = np.random.default_rng(950 + n)
    psi = rand_state(n, rng, name)
    psi[::7] = 0
    seed = 4242 + n
    say("sample seeded", name, n)
    got = q.qsv_sample_seeded(to_gpu(psi, name), seed, 30000).cpu().numpy()
    u = orc.seeded_uniforms(seed, 30000)
    _check_samples(psi, u, got, orc.sample(psi, u), 1e-13)
