"""Pins of the CPU oracle against mathematics that does not come from the oracle.

The paper (Sec. 2, eq. (1)) prints no worked example and no amplitudes, so
every pin here is a closed form, an invariant, a textbook routine or a
brute-force Kronecker construction (oracle/brute.py) that shares no code
with oracle.c.  Each family is chosen so that a dropped term, a wrong sign,
a swapped index or a transposed matrix in oracle.c fails at least one test.
"""
import ctypes
import itertools

import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle import brute

RNG = np.random.default_rng(7)

H2 = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2)
X2 = brute.X
Z2 = brute.Z
CNOT_AS_X = X2


def rand_state(n, rng=RNG):
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return v / np.linalg.norm(v)


def bits_equal(a, b):
    return np.array_equal(np.asarray(a).view(np.uint64), np.asarray(b).view(np.uint64))


# ------------------------------------------------------------ eq. (1) apply

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_apply_matches_kronecker_all_placements(orc, n):
    """Every ordered placement of k targets and c controls, n <= 5."""
    psi = rand_state(n)
    for k in range(1, min(n, 3) + 1):
        for c in range(0, min(n - k, 2) + 1):
            for qs in itertools.permutations(range(n), k + c):
                t, ctl = qs[:k], qs[k:]
                if c == 2 and ctl[0] > ctl[1]:
                    continue
                G = W.haar_unitary(RNG, 2 ** k)
                got = orc.apply(psi, t, ctl, G)
                ref = brute.gate_unitary(n, t, ctl, G) @ psi
                assert np.max(np.abs(got - ref)) < 1e-13, (n, t, ctl)


@pytest.mark.parametrize("n", [6, 8, 10])
def test_apply_matches_kronecker_random(orc, n):
    rng = np.random.default_rng(n)
    psi = rand_state(n, rng)
    for _ in range(6):
        k = int(rng.integers(1, 6))
        c = int(rng.integers(0, min(3, n - k) + 1))
        t, ctl, G = W.random_gate(rng, n, k, c)
        # non-unitary matrices too: eq. (1) is linear in G
        G = G + 0.3 * (rng.standard_normal(G.shape) + 1j * rng.standard_normal(G.shape))
        got = orc.apply(psi, t, ctl, G)
        ref = brute.gate_unitary(n, t, ctl, G) @ psi
        assert np.max(np.abs(got - ref)) < 1e-12, (t, ctl)


def test_qubit_j_is_bit_j(orc):
    """X on qubit j of |0..0> gives amplitude 1 at index 2**j (bit exact)."""
    n = 7
    for j in range(n):
        psi = np.zeros(1 << n, np.complex128)
        psi[0] = 1
        out = orc.apply(psi, (j,), (), X2)
        ref = np.zeros_like(psi)
        ref[1 << j] = 1
        assert bits_equal(out, ref)


def test_first_target_is_msb(orc):
    """kron(A, B) on targets (a, b) equals A on a followed by B on b."""
    n = 5
    psi = rand_state(n)
    A, B = W.haar_unitary(RNG, 2), W.haar_unitary(RNG, 2)
    for a, b in [(0, 3), (4, 1), (2, 3)]:
        got = orc.apply(psi, (a, b), (), np.kron(A, B))
        ref = orc.apply(orc.apply(psi, (a,), (), A), (b,), (), B)
        assert np.max(np.abs(got - ref)) < 1e-14


def test_target_order_swap_is_conjugation_by_swap(orc):
    n = 4
    psi = rand_state(n)
    G = W.haar_unitary(RNG, 4)
    S = brute.gate_unitary(2, (0, 1), (), np.eye(4))  # identity sanity
    assert np.allclose(S, np.eye(4))
    SW = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], np.complex128)
    got = orc.apply(psi, (1, 3), (), G)
    ref = orc.apply(psi, (3, 1), (), SW @ G @ SW)
    assert np.max(np.abs(got - ref)) < 1e-14


def test_hadamard_everywhere_closed_form(orc):
    """H on every qubit: |0..0> -> uniform 2**(-n/2); on any psi the result is
    2**(-n/2) times the Sylvester Hadamard matrix times psi."""
    for n in [1, 3, 6, 9]:
        psi = np.zeros(1 << n, np.complex128)
        psi[0] = 1
        for q in range(n):
            psi = orc.apply(psi, (q,), (), H2)
        assert np.max(np.abs(psi - 2 ** (-n / 2))) < 1e-15
        phi = rand_state(n)
        out = phi
        for q in range(n):
            out = orc.apply(out, (q,), (), H2)
        ref = scipy.linalg.hadamard(1 << n) @ phi * 2 ** (-n / 2)
        assert np.max(np.abs(out - ref)) < 1e-13


def test_ghz_exact(orc):
    for n in [2, 5, 11]:
        psi = np.zeros(1 << n, np.complex128)
        psi[0] = 1
        psi = orc.apply(psi, (0,), (), H2)
        for q in range(n - 1):
            psi = orc.apply(psi, (q + 1,), (q,), X2)
        ref = np.zeros_like(psi)
        ref[0] = ref[-1] = 1 / np.sqrt(2)
        assert bits_equal(psi, ref)


def test_permutations_are_bit_exact_moves(orc):
    n = 6
    psi = rand_state(n)
    psi[5] = -0.0 + 0j  # signed zero must survive a move
    idx = np.arange(1 << n)
    SW = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], np.complex128)
    cases = [((2,), (), X2, idx ^ 4),
             ((0,), (3,), X2, np.where(idx & 8, idx ^ 1, idx)),
             ((1, 4), (), SW, np.where(((idx >> 1) & 1) != ((idx >> 4) & 1), idx ^ 0b10010, idx)),
             ((5,), (0, 2), X2, np.where((idx & 5) == 5, idx ^ 32, idx))]
    for t, c, G, src in cases:
        out = orc.apply(psi, t, c, G)
        assert bits_equal(out, psi[src]), (t, c)


def test_diagonal_and_controlled_phase(orc):
    n = 5
    psi = rand_state(n)
    idx = np.arange(1 << n)
    out = orc.apply(psi, (3,), (1,), Z2)  # CZ(1,3)
    sign = np.where(((idx >> 1) & 1) & ((idx >> 3) & 1), -1.0, 1.0)
    assert np.max(np.abs(out - sign * psi)) == 0.0


def test_norm_and_inverse(orc):
    n = 9
    rng = np.random.default_rng(3)
    psi = rand_state(n, rng)
    gates = [W.random_gate(rng, n, int(rng.integers(1, 4)), int(rng.integers(0, 2))) for _ in range(25)]
    out = psi
    for t, c, G in gates:
        out = orc.apply(out, t, c, G)
    assert abs(orc.norm2(out) - 1.0) < 1e-13
    back = out
    for t, c, G in reversed(gates):
        back = orc.apply(back, t, c, G.conj().T)
    assert np.max(np.abs(back - psi)) < 1e-13


def test_disjoint_gates_commute(orc):
    n = 6
    psi = rand_state(n)
    A, B = W.haar_unitary(RNG, 4), W.haar_unitary(RNG, 2)
    ab = orc.apply(orc.apply(psi, (0, 3), (), A), (5,), (2,), B)
    ba = orc.apply(orc.apply(psi, (5,), (2,), B), (0, 3), (), A)
    assert np.max(np.abs(ab - ba)) < 1e-15


def test_rejects_bad_qubits(orc):
    psi = rand_state(3)
    with pytest.raises(ValueError):
        orc.apply(psi, (3,), (), X2)
    with pytest.raises(ValueError):
        orc.apply(psi, (1,), (1,), X2)


# --------------------------------------------------------------- observables

def test_pauli_conventions_against_dense(orc):
    """Random Pauli sums: oracle expectation equals psi^dagger H psi with H
    built from Kronecker products of the 2x2 Pauli matrices."""
    for n in [1, 3, 6, 8]:
        H = W.random_pauli_sum(n, 12, seed=n)
        psi = rand_state(n)
        got = orc.expect(psi, H)
        M = brute.hamiltonian_dense(H)
        ref = np.vdot(psi, M @ psi)
        assert abs(got - ref) < 1e-12
        assert abs(got.imag) < 1e-12


def test_single_pauli_values(orc):
    """<0|Z|0> = 1, <1|Z|1> = -1, <+|X|+> = 1, <+i|Y|+i> = 1 (textbook)."""
    zero = np.array([1, 0], np.complex128)
    one = np.array([0, 1], np.complex128)
    plus = np.array([1, 1], np.complex128) / np.sqrt(2)
    plus_i = np.array([1, 1j], np.complex128) / np.sqrt(2)
    Zs, Xs, Ys = (W.pauli_sum(1, [(ch, (0,), 1.0)]) for ch in "ZXY")
    assert orc.expect(zero, Zs) == 1.0
    assert orc.expect(one, Zs) == -1.0
    assert abs(orc.expect(plus, Xs) - 1.0) < 1e-15
    assert abs(orc.expect(plus_i, Ys) - 1.0) < 1e-15
    assert abs(orc.expect(plus_i, Xs)) < 1e-15


def test_tfim_closed_forms(orc):
    for n in [2, 5, 10]:
        H = W.tfim_chain(n)
        zero = np.zeros(1 << n, np.complex128)
        zero[0] = 1
        plus = np.full(1 << n, 2 ** (-n / 2), np.complex128)
        ghz = np.zeros(1 << n, np.complex128)
        ghz[0] = ghz[-1] = 1 / np.sqrt(2)
        assert abs(orc.expect(zero, H) - (n - 1)) < 1e-13
        assert abs(orc.expect(plus, H) - n) < 1e-12
        assert abs(orc.expect(ghz, H) - (n - 1)) < 1e-13


def test_xxz_and_maxcut_closed_forms(orc):
    n = 6
    zero = np.zeros(1 << n, np.complex128)
    zero[0] = 1
    for delta in [0.0, 0.5, -1.3]:
        assert abs(orc.expect(zero, W.xxz_chain(n, delta)) - delta * (n - 1)) < 1e-13
    # MaxCut on a 4-cycle: basis state 0101 cuts every edge.
    edges = [(0, 1), (1, 2), (2, 3), (3, 0)]
    b = np.zeros(16, np.complex128)
    b[0b0101] = 1
    assert abs(orc.expect(b, W.maxcut(4, edges)) - 4.0) < 1e-15
    b0 = np.zeros(16, np.complex128)
    b0[0] = 1
    assert abs(orc.expect(b0, W.maxcut(4, edges))) < 1e-15


def test_z_diagonal_closed_form(orc):
    n = 7
    psi = rand_state(n)
    idx = np.arange(1 << n)
    for z in [1, 6, 0b1010011]:
        H = W.PauliSum(n, np.array([0], np.uint64), np.array([z], np.uint64), np.array([1.0]))
        par = np.array([bin(int(i) & z).count("1") & 1 for i in idx])
        ref = np.sum(np.abs(psi) ** 2 * (1 - 2 * par))
        assert abs(orc.expect(psi, H) - ref) < 1e-14


# ----------------------------------------------------------------- circuits

def test_run_matches_sequential_apply(orc):
    circ = W.random_u2_cz(n=6, depth=4, seed=11)
    psi = np.zeros(64, np.complex128)
    psi[0] = 1
    for op in circ.ops:
        G = op.matrix if op.kind == "matrix" else Z2
        psi = orc.apply(psi, op.targets, op.controls, G)
    assert bits_equal(orc.run(circ), psi)


def test_rotation_definitions(orc):
    """RX, RY, RZ = exp(-i theta P / 2) against scipy.linalg.expm; H and Y."""
    th = 0.7318
    circ = W.Circuit(1, [W.Op("rx", (0,), param=0)], 1)
    for kind, P in [("rx", brute.X), ("ry", brute.Y), ("rz", brute.Z)]:
        circ.ops[0].kind = kind
        ref = scipy.linalg.expm(-0.5j * th * P)
        for b in range(2):
            psi0 = np.zeros(2, np.complex128)
            psi0[b] = 1
            assert np.max(np.abs(orc.run(circ, [th], psi0) - ref[:, b])) < 1e-15
    for kind, M in [("h", H2), ("y", brute.Y), ("z", Z2)]:
        c2 = W.Circuit(1, [W.Op(kind, (0,))])
        psi0 = rand_state(1)
        assert np.max(np.abs(orc.run(c2, None, psi0) - M @ psi0)) < 1e-15


def test_swap_kind(orc):
    n = 4
    psi = rand_state(n)
    c = W.Circuit(n, [W.Op("swap", (0, 2))])
    idx = np.arange(16)
    src = np.where(((idx >> 0) & 1) != ((idx >> 2) & 1), idx ^ 0b101, idx)
    assert bits_equal(orc.run(c, None, psi), psi[src])


# ----------------------------------------------------------------- gradients

def test_one_qubit_gradient_closed_form(orc):
    """<Z> after RY(theta)|0> is cos(theta): derivative -sin(theta); same for
    RX; <X> after RZ(theta) on |+> is cos(theta)."""
    Zs = W.pauli_sum(1, [("Z", (0,), 1.0)])
    Xs = W.pauli_sum(1, [("X", (0,), 1.0)])
    for th in [0.3, 1.9, 4.4]:
        for kind in ["rx", "ry"]:
            c = W.Circuit(1, [W.Op(kind, (0,), param=0)], 1)
            assert abs(orc.energy(c, [th], Zs) - np.cos(th)) < 1e-15
            assert abs(orc.grad_param_shift(c, [th], Zs)[0] + np.sin(th)) < 1e-14
            assert abs(orc.grad_finite_diff(c, [th], Zs)[0] + np.sin(th)) < 1e-8
            E, g = orc.adjoint(c, [th], Zs)
            assert abs(E - np.cos(th)) < 1e-15 and abs(g[0] + np.sin(th)) < 1e-14
        c = W.Circuit(1, [W.Op("h", (0,)), W.Op("rz", (0,), param=0)], 1)
        assert abs(orc.energy(c, [th], Xs) - np.cos(th)) < 1e-15
        E, g = orc.adjoint(c, [th], Xs)
        assert abs(g[0] + np.sin(th)) < 1e-14


def test_gradients_agree_on_hea(orc):
    n, L = 5, 3
    circ = W.hea(n, L)
    p = W.random_params(circ.nparams, 5)
    H = W.tfim_chain(n)
    ps = orc.grad_param_shift(circ, p, H)
    fd = orc.grad_finite_diff(circ, p, H)
    E, adj = orc.adjoint(circ, p, H)
    assert abs(E - orc.energy(circ, p, H)) < 1e-13
    assert np.max(np.abs(ps - adj)) < 1e-12
    assert np.max(np.abs(fd - adj)) < 1e-7


def test_controlled_rotation_gradient(orc):
    """Adjoint on a CRZ (needs the zeroed control-off block) against finite
    differences; parameter shift refuses controlled rotations."""
    n = 3
    circ = W.Circuit(n, [W.Op("h", (0,)), W.Op("h", (1,)), W.Op("ry", (2,), param=1),
                         W.Op("rz", (1,), controls=(0,), param=0), W.Op("h", (1,))], 2)
    p = np.array([0.9, 0.4])
    H = W.pauli_sum(n, [("Z", (1,), 1.0), ("XZ", (0, 2), 0.5)])
    fd = orc.grad_finite_diff(circ, p, H)
    _, adj = orc.adjoint(circ, p, H)
    assert np.max(np.abs(fd - adj)) < 1e-8
    with pytest.raises(ValueError):
        orc.grad_param_shift(circ, p, H, which=[0])


# ------------------------------------------------------------- random state

def test_splitmix64_published_vector(orc):
    """SplitMix64 from seed 1234567: the first five outputs of the reference
    generator (state advanced by the golden gamma before each output)."""
    L = orc.lib()
    L.orc_splitmix64_at.restype = ctypes.c_uint64
    L.orc_splitmix64_at.argtypes = [ctypes.c_uint64]
    g = 0x9E3779B97F4A7C15
    got = [L.orc_splitmix64_at((1234567 + i * g) % 2 ** 64) for i in range(5)]
    assert got == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                   4593380528125082431, 16408922859458223821]


def test_random_state_properties(orc):
    n, seed = 14, 99
    psi = orc.random_state(n, seed)
    assert abs(np.sum(np.abs(psi) ** 2) - 1.0) < 1e-13
    s2 = orc.random_norm2(n, seed)
    raw = psi * np.sqrt(s2)
    assert np.all(np.abs(raw.real) <= 0.5) and np.all(np.abs(raw.imag) <= 0.5)
    assert abs(s2 / (1 << n) - 1 / 6) < 0.01  # E|u - 1/2|^2 = 1/12 per component
    idx = np.array([0, 1, 77, (1 << n) - 1], np.uint64)
    assert bits_equal(orc.random_amps(seed, 1 / np.sqrt(s2), idx), psi[idx.astype(np.int64)])
    assert not np.allclose(orc.random_state(n, seed + 1), psi)


def test_sampled_apply_matches_full(orc):
    n, seed = 12, 5
    psi = orc.random_state(n, seed)
    scale = 1 / np.sqrt(orc.random_norm2(n, seed))
    rng = np.random.default_rng(1)
    for k, c in [(1, 0), (2, 1), (3, 0), (5, 0)]:
        t, ctl, G = W.random_gate(rng, n, k, c)
        full = orc.apply(psi, t, ctl, G)
        idx = rng.integers(0, 1 << n, size=50).astype(np.uint64)
        got = orc.apply_sampled_random(n, seed, scale, t, ctl, G, idx)
        assert np.max(np.abs(got - full[idx.astype(np.int64)])) < 1e-15


class SplitMix64:
    """The sequential generator as published (Steele, Lea & Flood 2014): the
    state advances by the golden gamma, then the output function mixes it.
    Written here independently of the oracle's counter-based form."""
    G = 0x9E3779B97F4A7C15
    M = (1 << 64) - 1

    def __init__(self, state):
        self.s = state & self.M

    def next(self):
        self.s = (self.s + self.G) & self.M
        z = self.s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & self.M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & self.M
        return z ^ (z >> 31)


def test_sequential_splitmix64_published_vector():
    g = SplitMix64(1234567)
    assert [g.next() for _ in range(5)] == [6457827717110365317, 3203168211198807973,
                                            9817491932198370423, 4593380528125082431,
                                            16408922859458223821]


def stream(seed, count):
    """Draws 0..count-1 of a seed's stream: the generator restarted at the
    key = its own first output from the seed."""
    g = SplitMix64(SplitMix64(seed).next())
    return [g.next() for _ in range(count)]


def test_random_state_generator_definition(orc):
    """Amplitude i of the seeded state is (u(2i) - 1/2) + i (u(2i+1) - 1/2)
    with u(c) = top-53 bits of draw c of the seed's stream over 2**53, draws
    taken from the sequential published generator; the real parts are
    centred (mean ~ 0)."""
    for seed in (1234567, 0, 2 ** 64 - 1):
        draws = stream(seed, 64)
        u = [(d >> 11) / 2.0 ** 53 for d in draws]
        amps = orc.random_amps(seed, 1.0, np.arange(32, dtype=np.uint64))
        assert np.array_equal(amps.real, np.array(u[0::2]) - 0.5)
        assert np.array_equal(amps.imag, np.array(u[1::2]) - 0.5)
    n = 12
    s2 = orc.random_norm2(n, 1234567)
    psi = orc.random_state(n, 1234567) * np.sqrt(s2)
    assert abs(psi.real.mean()) < 0.02 and abs(psi.imag.mean()) < 0.02


def test_random_states_of_nearby_seeds_unrelated(orc):
    """States of seeds that differ in one low bit share no amplitude and are
    not images of each other under an X on any qubit, a complex conjugation
    or the two together (the structure a seed-xor-counter stream has)."""
    n = 10
    for seed in (0, 1000, 2024, 1234567):
        base = orc.random_state(n, seed)
        others = [orc.random_state(n, seed ^ d) for d in (1, 2, 3)]
        others.append(orc.random_state(n, seed + 1))
        idx = np.arange(1 << n)
        for o in others:
            assert np.intersect1d(np.abs(base.real), np.abs(o.real)).size == 0
            for flip in [0] + [1 << q for q in range(n)]:
                moved = o[idx ^ flip]
                for cand in (moved, np.conj(moved)):
                    # a relation up to a phase would give |overlap| = 1;
                    # unrelated 2^10-amplitude states give about 2^-5
                    assert abs(np.vdot(cand, base)) < 0.2
                    assert abs(np.sum(cand * base)) < 0.2
            assert abs(np.vdot(base, o)) < 0.2


def test_inner_product_convention(orc):
    """<a|b> conjugates its FIRST argument (the bra): closed forms
    <0|(i|0>) = i and (i<0|)|0> = -i, numpy's vdot on random complex vectors
    (real and imaginary parts, the chunked path from n = 11 on as well), and
    swapping the arguments conjugates the result exactly."""
    for n in (1, 3):
        e0 = np.zeros(1 << n, np.complex128)
        e0[0] = 1.0
        assert orc.inner(e0, 1j * e0) == 1j
        assert orc.inner(1j * e0, e0) == -1j
        e1 = np.zeros(1 << n, np.complex128)
        e1[1] = 1.0
        assert orc.inner(e0, e1) == 0
        assert orc.inner((1 + 2j) * e1, (3 - 1j) * e1) == (1 - 2j) * (3 - 1j)
    rng = np.random.default_rng(11)
    for n in (4, 10, 11, 13):
        a = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
        b = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
        b = b + 0.5j * a  # Im <a|b> gains 0.5 |a|^2: far from zero
        got, want = orc.inner(a, b), np.vdot(a, b)
        scale = np.sum(np.abs(a) * np.abs(b))
        assert abs(got.real - want.real) <= 1e-14 * scale
        assert abs(got.imag - want.imag) <= 1e-14 * scale
        assert abs(want.imag) > 1e-3 * scale
        assert orc.inner(b, a) == np.conj(got)
        assert abs(orc.inner(a, a).imag) <= 1e-15 * np.sum(np.abs(a) ** 2)


def test_apply_hamiltonian_against_dense(orc):
    n = 6
    H = W.random_pauli_sum(n, 9, seed=4)
    psi = rand_state(n)
    got = orc.apply_hamiltonian(psi, H)
    ref = brute.hamiltonian_dense(H) @ psi
    assert np.max(np.abs(got - ref)) < 1e-13
