"""Pins of the oracle's measurement sampling (Sec. 3: simulated measurements
draw outcomes from the state's Born probabilities) against mathematics that
does not come from the oracle: numpy reshapes of |psi|^2, exact closed forms of
the uniform and GHZ distributions, product-state factorisation, numpy's
sorted-search on a running sum, and a chi-square goodness-of-fit test.  A
swapped bit order, an exclusive/inclusive slip in the running sum, a >= for >
or a dropped imaginary part fails one of them.
"""
import numpy as np
import pytest
import scipy.stats

import workloads as W


def rand_state(n, seed):
    r = np.random.default_rng(seed)
    v = r.standard_normal(1 << n) + 1j * r.standard_normal(1 << n)
    return v / np.linalg.norm(v)


def marginal_by_reshape(psi, n, qubits):
    """|psi|^2 as an n-axis array (axis a = qubit n-1-a), summed over the other
    axes, measured axes ordered as listed, flattened with the first listed
    qubit most significant."""
    p = (np.abs(psi) ** 2).reshape([2] * n)
    keep = [n - 1 - q for q in qubits]
    drop = tuple(a for a in range(n) if a not in keep)
    s = p.sum(axis=drop)
    remaining = [a for a in range(n) if a in keep]          # ascending axis order
    s = np.transpose(s, [remaining.index(a) for a in keep])
    return s.reshape(-1)


@pytest.mark.parametrize("n,qubits", [(1, [0]), (3, [0, 1, 2]), (3, [2, 0]), (5, [1]),
                                      (5, [4, 0, 2]), (6, [3, 5, 0, 1]), (7, [6, 5, 4, 3, 2, 1, 0]),
                                      (13, [12, 0, 5, 7, 1, 9, 2, 11, 3, 10, 4, 8, 6])])
def test_probabilities_match_reshape(orc, n, qubits):
    psi = rand_state(n, 11 + n)
    got = orc.probabilities(psi, qubits)
    ref = marginal_by_reshape(psi, n, qubits)
    assert got.shape == (1 << len(qubits),)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-15)


def test_probabilities_product_state(orc):
    """A product state's marginal is the product of its one-qubit marginals."""
    n = 5
    r = np.random.default_rng(3)
    singles = []
    psi = np.ones(1, dtype=np.complex128)
    for q in range(n):                       # qubit q is bit q: kron puts later factors low
        a = r.standard_normal(2) + 1j * r.standard_normal(2)
        a /= np.linalg.norm(a)
        singles.append(np.abs(a) ** 2)
        psi = np.kron(a, psi)
    qubits = [3, 0, 4]
    got = orc.probabilities(psi, qubits)
    for b in range(8):
        bits = [(b >> (2 - j)) & 1 for j in range(3)]
        want = np.prod([singles[q][bit] for q, bit in zip(qubits, bits)])
        assert abs(got[b] - want) <= 1e-15


def test_probabilities_full_register_is_abs2(orc):
    n = 6
    psi = rand_state(n, 5)
    got = orc.probabilities(psi, list(range(n - 1, -1, -1)))   # qubit n-1 most significant
    assert np.array_equal(got, psi.real ** 2 + psi.imag ** 2)


def test_probabilities_reject_bad_qubits(orc):
    psi = rand_state(3, 1)
    for q in ([3], [0, 0], [-1]):
        with pytest.raises(ValueError):
            orc.probabilities(psi, q)


def test_sample_uniform_closed_form(orc):
    """Equal superposition of n qubits (n even: every |psi_i|^2 = 2^-n exactly,
    every running sum exact): outcome = floor(u 2^n), also on the grid points
    u = k 2^-n where a >= in place of > would return k - 1."""
    n = 8
    N = 1 << n
    psi = np.full(N, 2.0 ** (-n / 2), dtype=np.complex128)
    u = np.concatenate([np.arange(N) / N, W.uniforms(4000, 21)])
    got = orc.sample(psi, u)
    assert np.array_equal(got, np.floor(u * N).astype(np.int64))


def test_sample_basis_state_and_ghz(orc):
    n = 6
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[37] = -1j
    u = W.uniforms(500, 3)
    assert np.all(orc.sample(psi, u) == 37)
    ghz = np.zeros(1 << n, dtype=np.complex128)
    ghz[0] = ghz[-1] = 1 / np.sqrt(2)
    u = np.concatenate([np.linspace(0, 0.49, 50), np.linspace(0.51, 0.999999, 50)])
    got = orc.sample(ghz, u)
    assert np.array_equal(got, np.where(u < 0.5, 0, (1 << n) - 1))


def test_sample_matches_sorted_search(orc):
    """numpy's searchsorted (side='right') on a running sum is the smallest i
    with C_i > t; the oracle must agree on every shot."""
    for n, seed in ((1, 1), (4, 2), (9, 3), (12, 4)):
        psi = rand_state(n, seed)
        psi[::5] = 0                                   # zero-probability outcomes
        psi[3 % psi.size] *= 1e-9                      # a tiny one
        C = np.cumsum(np.abs(psi) ** 2)
        u = W.uniforms(3000, 100 + n)
        want = np.searchsorted(C, u * C[-1], side="right")
        got = orc.sample(psi, u)
        assert np.array_equal(got, want)
        assert np.all(np.abs(psi[got]) > 0)


def test_sample_edges(orc):
    """u >= 1 (and NaN) give the last outcome of nonzero probability; u < 0
    gives the first; the zero vector gives 0; no shots gives nothing."""
    psi = np.zeros(16, dtype=np.complex128)
    psi[[2, 9, 11]] = [0.6, 0.0, 0.8j]
    got = orc.sample(psi, [1.0, 2.5, np.nan, -0.5, 0.0])
    assert list(got) == [11, 11, 11, 2, 2]
    assert list(orc.sample(np.zeros(8, dtype=np.complex128), [0.0, 0.7])) == [0, 0]
    assert orc.sample(psi, np.zeros(0)).size == 0


def test_sample_frequencies_chi_square(orc):
    """Frequencies of 200000 seeded shots fit |psi|^2 (chi-square test at the
    1e-4 level; the seed is fixed, so the test is deterministic)."""
    n = 5
    psi = rand_state(n, 9)
    p = np.abs(psi) ** 2
    u = W.uniforms(200000, 77)
    counts = np.bincount(orc.sample(psi, u), minlength=1 << n)
    stat, pval = scipy.stats.chisquare(counts, p * u.size / p.sum())
    assert pval > 1e-4, (stat, pval)


def test_frequencies_match_bincount(orc):
    """Counts over a qubit subset equal numpy's bincount of the outcome bits
    extracted from each sample (first listed qubit most significant)."""
    n = 9
    r = np.random.default_rng(12)
    samples = r.integers(0, 1 << n, 5000)
    for qubits in ([0], [8, 0, 4], [3, 5, 7, 1], list(range(n - 1, -1, -1))):
        m = len(qubits)
        b = np.zeros(samples.size, dtype=np.int64)
        for j, qq in enumerate(qubits):
            b |= ((samples >> qq) & 1) << (m - 1 - j)
        want = np.bincount(b, minlength=1 << m)
        got = orc.frequencies(n, samples, qubits)
        assert np.array_equal(got, want) and got.sum() == samples.size
    assert orc.frequencies(n, np.zeros(0, dtype=np.int64), [2]).tolist() == [0, 0]


def test_collapse_matches_projector(orc):
    """Collapse equals the normalised projection (I (x) |b><b| (x) I) psi built
    from Kronecker products of 2x2 projectors; the result has unit norm and
    the measured qubits then give outcome b with probability 1."""
    n = 6
    psi = rand_state(n, 21)
    for qubits, b in (([0], 1), ([5, 2], 2), ([1, 3, 4], 5)):
        P = np.ones((1, 1))
        m = len(qubits)
        for q in range(n - 1, -1, -1):                 # qubit n-1 is the leftmost factor
            if q in qubits:
                bit = (b >> (m - 1 - qubits.index(q))) & 1
                P = np.kron(P, np.diag([1.0 - bit, float(bit)]))
            else:
                P = np.kron(P, np.eye(2))
        proj = P @ psi
        p = float(np.vdot(proj, proj).real)
        got = orc.collapse(psi, qubits, b, p)
        assert np.max(np.abs(got - proj / np.sqrt(p))) <= 1e-15
        assert abs(np.linalg.norm(got) - 1) <= 1e-14
        pr = orc.probabilities(got, qubits)
        assert abs(pr[b] - 1) <= 1e-14 and abs(pr.sum() - 1) <= 1e-14


def test_collapse_ghz_and_impossible(orc):
    n = 5
    ghz = np.zeros(1 << n, dtype=np.complex128)
    ghz[0] = ghz[-1] = 1 / np.sqrt(2)
    got = orc.collapse(ghz, [2], 1, 0.5)
    want = np.zeros(1 << n)
    want[-1] = 1.0
    assert np.max(np.abs(got - want)) <= 1e-15
    assert np.all(orc.collapse(ghz, [2], 1, 0.0) == 0)
    with pytest.raises(ValueError):
        orc.collapse(ghz, [2], 2, 0.5)


def test_seeded_uniforms_are_uniform(orc):
    """The counter-based uniforms (SplitMix64, whose output function is pinned
    against its published vector elsewhere) lie in [0, 1), differ per seed and
    pass a Kolmogorov-Smirnov test against U[0, 1)."""
    u = orc.seeded_uniforms(2024, 100000)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert scipy.stats.kstest(u, "uniform").pvalue > 1e-4
    v = orc.seeded_uniforms(2025, 100000)
    assert not np.array_equal(u[:100], v[:100])
    assert np.array_equal(orc.seeded_uniforms(2024, 10), u[:10])


def test_seeded_uniforms_of_nearby_seeds_are_different_sets(orc):
    """Streams of nearby seeds are not reorderings of each other: their
    sorted values differ and they share (almost) no value; the stream equals
    the published sequential generator restarted at its first output."""
    G, M = 0x9E3779B97F4A7C15, (1 << 64) - 1

    def mix(z):
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return z ^ (z >> 31)

    for seed in (0, 1, 1000, 2024):
        key = mix((seed + G) & M)
        want = [(mix((key + (s + 1) * G) & M) >> 11) / 2.0 ** 53 for s in range(200)]
        assert np.array_equal(orc.seeded_uniforms(seed, 200), np.array(want))
    count = 1 << 16
    for a, b in ((2024, 2025), (0, 1000), (0, 1), (6, 7), (1 << 40, (1 << 40) + 2)):
        ua, ub = orc.seeded_uniforms(a, count), orc.seeded_uniforms(b, count)
        assert not np.array_equal(np.sort(ua), np.sort(ub))
        assert np.intersect1d(ua, ub).size <= 2
