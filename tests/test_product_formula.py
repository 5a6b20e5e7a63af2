"""Pin of the product-state closed form used by the n = 30 expectation test
(tests/test_gpu_configs.py): for a product state (x)_q (a_q|0> + b_q|1>) a
Pauli string's expectation is the product of single-qubit expectations
<X> = 2 Re(conj(a) b), <Y> = 2 Im(conj(a) b), <Z> = |a|^2 - |b|^2 (Sec. 3
Pauli strings).  Checked here against the oracle on small product states."""
import numpy as np

import workloads as W
from test_gpu_configs import hamiltonians_for, product_expectation


def test_product_formula_matches_oracle(orc):
    """The closed form above against the oracle on small product states (so
    the n = 30 check below rests on a pinned formula)."""
    n = 12
    rng = np.random.default_rng(5)
    vecs = [W.haar_unitary(rng, 2)[:, 0] for _ in range(n)]
    psi = np.array([1.0 + 0j])
    for q in range(n):  # qubit q = bit q: the highest qubit is the leftmost factor
        psi = np.kron(vecs[q], psi)
    for name, H in hamiltonians_for(n):
        ref = orc.expect(psi, H).real
        assert abs(product_expectation(H, vecs) - ref) <= 1e-12 * np.sum(np.abs(H.coeff)), name
