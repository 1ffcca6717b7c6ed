"""Pins of the oracle's controlled gates, measurement reads and Grover
closed form against things other than the oracle itself: brute-force
operators built from Kronecker products and projectors, truth tables,
closed forms of textbook states, and exact quantile counts."""
import numpy as np
import pytest

import circuits as C
import oracle

PX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PZ = np.diag([1.0, -1.0]).astype(np.complex128)


# ---------------------------------------------------------------- controls
@pytest.mark.parametrize("seed", range(4))
def test_controlled_vs_brute_force(seed):
    n = 7
    rng = np.random.Generator(np.random.PCG64(40 + seed))
    gates = [C.Gate((q,), C.haar_unitary(1, rng)) for q in range(n)]
    for _ in range(12):
        k = int(rng.integers(1, 4))
        nc = int(rng.integers(1, 4))
        qs = [int(v) for v in rng.choice(n, k + nc, replace=False)]
        vals = tuple(int(v) for v in rng.integers(0, 2, nc))
        gates.append(C.Gate(tuple(qs[:k]), C.haar_unitary(k, rng), tuple(qs[k:]), vals))
    got = oracle.apply_circuit(n, gates)
    ref = oracle.brute_force_state(n, gates)
    assert np.max(np.abs(got - ref)) < 1e-13


@pytest.mark.parametrize("c,t", [(0, 3), (3, 0), (5, 1)])
def test_controlled_x_is_cnot(c, t):
    n = 6
    rng = np.random.Generator(np.random.PCG64(7))
    prep = [C.Gate((q,), C.haar_unitary(1, rng)) for q in range(n)]
    a = oracle.apply_circuit(n, prep + [C.Gate((t,), C.X, (c,))])
    b = oracle.apply_circuit(n, prep + [C.Gate((c, t), C.CNOT)])
    assert np.max(np.abs(a - b)) < 1e-15


def test_toffoli_truth_table():
    n = 4
    g = C.Gate((2,), C.X, (0, 3))
    for x in range(1 << n):
        psi = oracle.basis_state(n, x)
        oracle.apply_gate(psi, n, g.qubits, g.matrix, g.cmask, g.cval)
        y = x ^ 4 if (x & 1) and (x & 8) else x
        assert psi[y] == 1 and np.count_nonzero(psi) == 1


def test_negative_control():
    n = 3
    g = C.Gate((1,), C.X, (0,), (0,))
    for x in range(1 << n):
        psi = oracle.basis_state(n, x)
        oracle.apply_gate(psi, n, g.qubits, g.matrix, g.cmask, g.cval)
        y = x ^ 2 if not (x & 1) else x
        assert psi[y] == 1


def test_controls_rejected_when_overlapping_targets():
    psi = oracle.basis_state(3, 0)
    with pytest.raises(ValueError):
        oracle.apply_gate(psi, 3, (1,), C.X, 0b010, 0b010)
    with pytest.raises(ValueError):
        oracle.apply_gate(psi, 3, (1,), C.X, 0b001, 0b100)   # value outside the mask


# ---------------------------------------------------------------- Pauli
def kron_pauli(n, xmask, zmask):
    """Dense Pauli operator; qubit q is bit q, so the Kronecker product runs
    from qubit n-1 (most significant) down to qubit 0."""
    op = np.eye(1, dtype=np.complex128)
    for q in reversed(range(n)):
        x, z = (xmask >> q) & 1, (zmask >> q) & 1
        m = PY if (x and z) else PX if x else PZ if z else np.eye(2)
        op = np.kron(op, m)
    return op


@pytest.mark.parametrize("seed", range(5))
def test_pauli_vs_kronecker(seed):
    n = 6
    psi = C.random_state_c64(n, seed).astype(np.complex128)
    rng = np.random.Generator(np.random.PCG64(seed))
    for _ in range(10):
        xm, zm = int(rng.integers(0, 1 << n)), int(rng.integers(0, 1 << n))
        ref = np.vdot(psi, kron_pauli(n, xm, zm) @ psi)
        got = oracle.pauli_expectation(psi, n, xm, zm)
        assert abs(got - ref) < 1e-14
        assert abs(got.imag) < 1e-14          # Hermitian


def test_pauli_closed_forms():
    n = 5
    zero = oracle.basis_state(n, 0)
    for q in range(n):
        assert oracle.pauli_expectation(zero, n, 0, 1 << q) == 1
        assert oracle.pauli_expectation(zero, n, 1 << q, 0) == 0
        assert oracle.pauli_expectation(zero, n, 1 << q, 1 << q) == 0
    ghz = oracle.apply_circuit(n, C.ghz_circuit(n))
    full = (1 << n) - 1
    assert abs(oracle.pauli_expectation(ghz, n, full, 0) - 1) < 1e-14           # X...X
    assert abs(oracle.pauli_expectation(ghz, n, full, 0b11) + 1) < 1e-14        # Y Y X X X
    assert abs(oracle.pauli_expectation(ghz, n, 0, 0b10010) - 1) < 1e-14        # Z Z
    assert abs(oracle.pauli_expectation(ghz, n, 0, 0b00100)) < 1e-14            # Z
    for th in (0.3, 1.1, 2.9):
        psi = oracle.apply_circuit(1, [C.Gate((0,), C.RY(th))])
        assert abs(oracle.pauli_expectation(psi, 1, 0, 1) - np.cos(th)) < 1e-15
        assert abs(oracle.pauli_expectation(psi, 1, 1, 0) - np.sin(th)) < 1e-15


# ---------------------------------------------------------------- marginals
def test_marginals_product_state_factorise():
    n = 6
    th = [0.2 + 0.4 * q for q in range(n)]
    psi = oracle.apply_circuit(n, [C.Gate((q,), C.RY(th[q])) for q in range(n)])
    qs = (4, 1, 2)
    p = oracle.marginal_probabilities(psi, n, qs)
    for o in range(8):
        e = 1.0
        for j, q in enumerate(qs):
            e *= np.sin(th[q] / 2) ** 2 if (o >> j) & 1 else np.cos(th[q] / 2) ** 2
        assert abs(p[o] - e) < 1e-15


def test_marginals_ghz_and_identity():
    n = 5
    ghz = oracle.apply_circuit(n, C.ghz_circuit(n))
    assert np.allclose(oracle.marginal_probabilities(ghz, n, (3, 0)), [0.5, 0, 0, 0.5], atol=1e-15)
    psi = C.random_state_c64(n, 3)
    p = oracle.marginal_probabilities(psi, n, tuple(range(n)))
    assert np.allclose(p, np.abs(psi.astype(np.complex128)) ** 2, rtol=1e-14, atol=0)
    rev = oracle.marginal_probabilities(psi, n, tuple(reversed(range(n))))
    assert np.array_equal(rev[oracle.bit_reverse(np.arange(1 << n), n)], p)


# ---------------------------------------------------------------- sampling
def test_sampling_basis_and_quantiles():
    n = 4
    psi = oracle.basis_state(n, 11)
    assert np.all(oracle.sample_indices(psi, C.uniforms(100, 1)) == 11)
    # p(0) = cos^2(pi/6) = 3/4 on qubit 0: the quantiles (j + 1/2)/1000 give exactly 750 zeros
    psi = oracle.apply_circuit(1, [C.Gate((0,), C.RY(np.pi / 3))])
    s = oracle.sample_indices(psi, (np.arange(1000) + 0.5) / 1000)
    assert np.count_nonzero(s == 0) == 750 and np.count_nonzero(s == 1) == 250


def test_sampling_ends():
    psi = np.zeros(8, dtype=np.complex128)
    psi[2] = psi[5] = np.sqrt(0.5)
    s = oracle.sample_indices(psi, np.array([0.0, 0.4999, 0.5, 0.99999999, 1.0]))
    assert s.tolist() == [2, 2, 5, 5, 5]


# ---------------------------------------------------------------- Grover
@pytest.mark.parametrize("n,marked,t", [(3, 5, 2), (5, 17, 4), (7, 100, 6)])
def test_grover_closed_form_vs_brute_force(n, marked, t):
    g = C.grover_circuit(n, marked, t)
    ref = oracle.brute_force_state(n, g)
    assert np.max(np.abs(ref - oracle.grover_amplitudes(n, marked, t, np.arange(1 << n)))) < 1e-13
    assert np.max(np.abs(ref - oracle.apply_circuit(n, g))) < 1e-13


def test_grover_success_near_one_at_optimal_iterations():
    n = 10
    t = int(np.floor(np.pi / 4 * np.sqrt(2 ** n)))
    p = abs(oracle.grover_amplitudes(n, 3, t, [3])[0]) ** 2
    assert p > 0.999
