"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: each test checks it against a
closed form, an invariant, a value the paper prints (tests/golden), or an
independent brute-force construction (Kronecker products + permutation).
"""
import json
import os

import numpy as np
import pytest

import circuits as C
import oracle

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


# --------------------------------------------------------------------------
# Gate definitions
# --------------------------------------------------------------------------
def test_hadamard_matches_paper():
    h = GOLDEN["hadamard"]
    assert np.allclose(C.H, np.array(h["entries"]) / np.sqrt(2), atol=0, rtol=1e-15)
    psi = oracle.basis_state(1, 0)
    oracle.apply_gate(psi, 1, (0,), C.H)
    assert np.allclose(psi, [1 / np.sqrt(2), 1 / np.sqrt(2)], atol=1e-16)


@pytest.mark.parametrize("name", ["H", "X", "Y", "Z", "SQRT_X", "SQRT_Y", "SQRT_W", "CZ", "CNOT"])
def test_gates_unitary(name):
    u = getattr(C, name)
    assert np.allclose(u @ u.conj().T, np.eye(u.shape[0]), atol=1e-15)


@pytest.mark.parametrize("sq,g", [("SQRT_X", "X"), ("SQRT_Y", "Y")])
def test_sqrt_gates_square(sq, g):
    s = getattr(C, sq)
    assert np.allclose(s @ s, getattr(C, g), atol=1e-15)


def test_sqrt_w():
    w = (C.X + C.Y) / np.sqrt(2)
    assert np.allclose(w @ w, np.eye(2), atol=1e-15)
    assert np.allclose(C.SQRT_W @ C.SQRT_W, w, atol=1e-15)
    expect = np.array([[(1 + 1j) / 2, -1j / np.sqrt(2)], [1 / np.sqrt(2), (1 + 1j) / 2]])
    assert np.allclose(C.SQRT_W, expect, atol=1e-15)


def test_rotations():
    th = 0.7
    assert np.allclose(C.RY(th) @ C.RY(-th), np.eye(2), atol=1e-15)
    assert np.allclose(C.RY(np.pi), [[0, -1], [1, 0]], atol=1e-15)
    assert np.allclose(C.RZ(th) @ C.RZ(th).conj().T, np.eye(2), atol=1e-15)
    assert np.allclose(C.CP(np.pi), C.CZ, atol=1e-15)


# --------------------------------------------------------------------------
# Oracle: single gates against closed forms
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,q,x", [(5, 0, 0), (5, 3, 9), (7, 6, 77), (9, 4, 300)])
def test_x_flips_bit(n, q, x):
    psi = oracle.basis_state(n, x)
    oracle.apply_gate(psi, n, (q,), C.X)
    expect = np.zeros(1 << n, dtype=np.complex128)
    expect[x ^ (1 << q)] = 1
    assert np.array_equal(psi, expect)


@pytest.mark.parametrize("c,t", [(0, 3), (3, 0), (2, 5), (5, 1)])
def test_cnot_both_orders(c, t):
    n = 6
    for x in range(1 << n):
        psi = oracle.basis_state(n, x)
        oracle.apply_gate(psi, n, (c, t), C.CNOT)
        y = x ^ (1 << t) if (x >> c) & 1 else x
        assert psi[y] == 1 and np.count_nonzero(psi) == 1


def test_group_map_is_bijection():
    """Every index belongs to exactly one group (Sec. IV: no conflicts between
    groups): the non-unitary gate 2*I must double every amplitude exactly once."""
    n = 8
    rng = np.random.default_rng(1)
    base = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    for qs in [(0,), (7,), (1, 6), (5, 0, 3), (2, 4, 6, 0), (7, 1, 3, 5, 0), (0, 1, 2, 3, 4, 5)]:
        psi = base.copy()
        oracle.apply_gate(psi, n, qs, 2 * np.eye(1 << len(qs)))
        assert np.array_equal(psi, 2 * base)


def test_tensor_product_identity():
    """Eq. 3: gates on disjoint qubits equal their Kronecker product; local bit 0
    is the low factor, so U1 on q1 then U2 on q2 == kron(U2, U1) on (q1, q2)."""
    rng = np.random.Generator(np.random.PCG64(3))
    n = 6
    u1, u2 = C.haar_unitary(1, rng), C.haar_unitary(2, rng)
    init = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    a = init.copy()
    oracle.apply_gate(a, n, (4,), u1)
    oracle.apply_gate(a, n, (0, 2), u2)
    b = init.copy()
    oracle.apply_gate(b, n, (4, 0, 2), np.kron(u2, u1))
    assert np.allclose(a, b, atol=1e-14)


# --------------------------------------------------------------------------
# Oracle against the brute-force full unitary (independent construction)
# --------------------------------------------------------------------------
def test_embed_gate_matches_definition_small():
    """The brute-force embedding itself, for a 2-qubit system written out by hand."""
    u = np.arange(4).reshape(2, 2) + 1j
    # U on qubit 1 of 2: kron(U, I) in the usual big-endian-of-bits layout of index = 2*b1 + b0
    assert np.allclose(oracle.embed_gate(2, (1,), u), np.kron(u, np.eye(2)))
    assert np.allclose(oracle.embed_gate(2, (0,), u), np.kron(np.eye(2), u))


@pytest.mark.parametrize("seed", range(6))
def test_oracle_vs_brute_force(seed):
    n = 7 if seed % 2 else 8
    gates = C.random_circuit(n, 12, max_k=4, seed=seed)
    init = seed * 11 % (1 << n)
    psi = oracle.apply_circuit(n, gates, init=init)
    ref = oracle.brute_force_state(n, gates, init=init)
    assert np.max(np.abs(psi - ref)) < 1e-12


def test_oracle_vs_brute_force_k6_unsorted():
    n = 8
    rng = np.random.Generator(np.random.PCG64(7))
    gates = [C.Gate((5, 0, 7, 2, 3, 6), C.haar_unitary(6, rng)), C.Gate((1, 4), C.haar_unitary(2, rng))]
    psi = oracle.apply_circuit(n, gates, init=3)
    assert np.max(np.abs(psi - oracle.brute_force_state(n, gates, init=3))) < 1e-12


def test_planted_transpose_is_caught():
    """A transposed matrix (a plausible bug) is detected by the brute-force pin."""
    n = 6
    rng = np.random.Generator(np.random.PCG64(5))
    u = C.haar_unitary(2, rng)
    good = oracle.brute_force_state(n, [C.Gate((1, 4), u)], init=5)
    bad = oracle.apply_circuit(n, [C.Gate((1, 4), u.T.copy())], init=5)
    assert np.max(np.abs(good - bad)) > 1e-3
    swapped = oracle.apply_circuit(n, [C.Gate((4, 1), u)], init=5)
    assert np.max(np.abs(good - swapped)) > 1e-3


# --------------------------------------------------------------------------
# Circuits with closed forms (Sec. VI)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 5, 12, 20])
def test_ghz_closed_form(n):
    gates = C.ghz_circuit(n)
    assert len(gates) == n  # Table 2, GHZ row: N gate ops in total
    psi = oracle.apply_circuit(n, gates)
    ref = oracle.ghz_amplitudes(n, range(1 << n))
    assert np.max(np.abs(psi - ref)) < 1e-15


@pytest.mark.parametrize("n,seed", [(3, 0), (7, 1), (10, 2), (12, 3), (14, 4)])
def test_qft_like_closed_form(n, seed):
    gates = C.qft_like_circuit(n)
    assert len(gates) == n * (n + 1) // 2
    x = C.qft_input_basis(n, seed)
    psi = oracle.apply_circuit(n, gates, init=x)
    ref = oracle.qft_like_amplitudes(n, x, np.arange(1 << n))
    assert np.max(np.abs(psi - ref)) < 1e-13
    assert np.allclose(np.abs(psi), 2 ** (-n / 2), atol=1e-13)


def test_qft_like_is_dft_of_bit_reversed_output():
    """The swap-free QFT of |x> equals the unitary DFT e^{2 pi i x y / N}/sqrt(N)
    read at bit-reversed y (numpy FFT as the independent reference)."""
    n = 9
    x = 333
    psi = oracle.apply_circuit(n, C.qft_like_circuit(n), init=x)
    e = np.zeros(1 << n)
    e[x] = 1
    dft = np.fft.ifft(e) * np.sqrt(1 << n)  # (1/sqrt N) sum_x' e^{+2 pi i x' y / N} e_x'
    rev = oracle.bit_reverse(np.arange(1 << n), n).astype(np.int64)
    assert np.max(np.abs(psi - dft[rev])) < 1e-13


def test_qft_count_golden():
    g = GOLDEN["qft_gate_count"]
    assert len(C.qft_like_circuit(g["n"])) == g["total"]


# --------------------------------------------------------------------------
# Norm (Eq. 1) and comparison statistics
# --------------------------------------------------------------------------
def test_norm_basis_and_uniform():
    assert oracle.norm_sq(oracle.basis_state(10, 77)) == 1.0
    n = 16
    psi = np.full(1 << n, 2 ** (-n / 2), dtype=np.complex128)
    assert oracle.norm_sq(psi) == 1.0  # exact: powers of two
    psi = np.arange(1 << 12, dtype=np.float64) + 0j
    assert oracle.norm_sq(psi) == float(np.sum(np.arange(1 << 12, dtype=np.float64) ** 2))


def test_norm_preserved_by_unitaries():
    n = 10
    psi = oracle.apply_circuit(n, C.random_circuit(n, 40, max_k=3, seed=9), init=5)
    assert abs(oracle.norm_sq(psi) - 1.0) < 1e-13


def test_compare_statistics():
    n = 8
    rng = np.random.default_rng(0)
    o = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    o /= np.linalg.norm(o)
    g = o.astype(np.complex64)
    r = oracle.compare(g, o)
    assert r["max_abs"] < 1e-7 and r["infidelity"] < 1e-12
    g2 = g.copy()
    g2[17] += np.complex64(1e-3)
    r2 = oracle.compare(g2, o)
    assert abs(r2["max_abs"] - 1e-3) < 1e-7
    # global phase is a fidelity-1 difference
    r3 = oracle.compare((o * np.exp(0.3j)).astype(np.complex64), o)
    assert r3["infidelity"] < 1e-12 and r3["max_abs"] > 1e-3
    # orthogonal states
    e0 = np.zeros(4, np.complex128); e0[0] = 1
    e1 = np.zeros(4, np.complex64); e1[1] = 1
    assert abs(oracle.compare(e1, e0)["infidelity"] - 1.0) < 1e-15


# --------------------------------------------------------------------------
# Paper-printed accounting (tests/golden)
# --------------------------------------------------------------------------
def test_flop_and_ai_accounting():
    """Useful flops per group of a k-qubit gate, 2^k (8 * 2^k - 2), gives the
    paper's 28 at k = 1; the paper's AI formula at numVals = 4 is exactly half
    of the read+write AI (8 * 2^k - 2) / 16 used for the roofline."""
    from paper_2602_09604_amd.accounting import flops_per_group, ai_read_write
    assert flops_per_group(1) == GOLDEN["flops_per_one_qubit_group"]["value"]

    def paper_ai(f, nv):
        return 2 * (3 * 2 ** (2 * f) + 2 ** f * (2 ** f - 1)) / (nv * 2 ** (f + 3))

    ai = GOLDEN["arithmetic_intensity"]
    assert round(paper_ai(3, ai["numVals"]), 2) == ai["f3_approx"] or abs(paper_ai(3, 4) - ai["f3_approx"]) < 0.01
    assert abs(paper_ai(1, ai["numVals"]) - ai["unfused_approx"]) < 0.01
    for f in range(1, 7):
        assert abs(2 * paper_ai(f, 4) - ai_read_write(f)) < 1e-12


# ---------------------------------------------------------------------------
# The comparison statistics themselves, on vectors exactly representable in
# complex64, against values worked out by hand.
# ---------------------------------------------------------------------------
def test_compare_statistics_by_hand():
    o = np.array([0.5, 0.5j, -0.5, 0.5], dtype=np.complex128)  # norm 1
    # g = 2 o: parallel, so no infidelity; |g - o| = |o|; <g|g> = 4
    r = oracle.compare((2 * o).astype(np.complex64), o)
    assert r["max_abs"] == 0.5 and r["rel_l2"] == 1.0
    assert r["infidelity"] == 0.0 and r["norm_drift"] == 3.0
    # one sign flipped: <o|g> = 0.25 + 0.25 - 0.25 + 0.25 = 0.5, fidelity 1/4;
    # the difference is 1 at one index, the norm unchanged
    g = np.array([0.5, 0.5j, 0.5, 0.5], dtype=np.complex64)
    r = oracle.compare(g, o)
    assert r["max_abs"] == 1.0 and r["rel_l2"] == 1.0
    assert r["infidelity"] == 0.75 and r["norm_drift"] == 0.0
    # a global phase i: fidelity 1, |i c - c| = sqrt(2) |c|
    r = oracle.compare((1j * o).astype(np.complex64), o)
    assert r["infidelity"] == 0.0 and r["norm_drift"] == 0.0
    assert abs(r["rel_l2"] - np.sqrt(2.0)) < 1e-15 and abs(r["max_abs"] - 0.5 * np.sqrt(2.0)) < 1e-15


def test_compare_streaming_equals_one_shot():
    rng = np.random.Generator(np.random.PCG64(17))
    o = rng.standard_normal(1000) + 1j * rng.standard_normal(1000)
    o /= np.linalg.norm(o)
    g = (o + 1e-4 * (rng.standard_normal(1000) + 1j * rng.standard_normal(1000))).astype(np.complex64)
    one = oracle.compare(g, o)
    acc = oracle.CompareAcc()
    for a, b in ((0, 137), (137, 600), (600, 1000)):
        acc.add(g[a:b], o[a:b])
    part = acc.result()
    for key in ("max_abs", "rel_l2", "infidelity", "norm_drift"):
        assert abs(part[key] - one[key]) <= 1e-12 * max(1.0, abs(one[key])), key
    # and against numpy written out directly
    gd = g.astype(np.complex128)
    assert abs(one["rel_l2"] - np.linalg.norm(gd - o)) < 1e-12
    assert abs(one["norm_drift"] - abs(np.vdot(gd, gd).real - 1.0)) < 1e-12
    fid = abs(np.vdot(o, gd)) ** 2 / (np.vdot(o, o).real * np.vdot(gd, gd).real)
    assert abs(one["infidelity"] - (1.0 - fid)) < 1e-12


# ---------------------------------------------------------------------------
# Probe projections (whole-state checks through a few inner products).
# ---------------------------------------------------------------------------
def test_probe_projections_definition_and_sensitivity():
    n = 9
    ph = C.probe_phases(n, 3, 4)
    unit = np.array([1, 1j, -1, -1j])
    # a basis state picks one entry: conj(i^e_x)
    for x in (0, 77, 511):
        e = np.zeros(1 << n, dtype=np.complex128)
        e[x] = 1.0
        assert np.allclose(oracle.probe_projections(e, ph), np.conj(unit[ph[:, x]]), atol=0, rtol=0)
    # a random state: the explicit probe vectors' inner products
    psi = C.random_state_c64(n, 5).astype(np.complex128)
    phi = unit[ph]
    assert np.max(np.abs(oracle.probe_projections(psi, ph) - phi.conj() @ psi)) < 1e-14
    # any deviation of norm 1e-4 moves some projection by more than 1e-5
    rng = np.random.Generator(np.random.PCG64(9))
    for _ in range(20):
        d = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
        d *= 1e-4 / np.linalg.norm(d)
        assert np.max(np.abs(oracle.probe_projections(psi + d, ph) - oracle.probe_projections(psi, ph))) > 1e-5


def test_probe_projections_of_batched_circuit_state():
    """The oracle path the batch golden file uses, for the batch's circuit
    family at a size the Kronecker brute force reaches."""
    rng = np.random.Generator(np.random.PCG64(4))
    n = 8
    gates = C.ansatz_circuit(n, rng.uniform(0, 2 * np.pi, size=(3, n, 2)))
    ph = C.probe_phases(n, 1000, 4)
    got = oracle.probe_projections(oracle.apply_circuit(n, gates), ph)
    ref = oracle.probe_projections(oracle.brute_force_state(n, gates), ph)
    assert np.max(np.abs(got - ref)) < 1e-12


@pytest.mark.parametrize("seed", range(3))
def test_diagonal_factors_against_brute_force(seed):
    """diagonal_factors against the Kronecker-product construction: from the
    uniform superposition every amplitude is 2^(-n/2) times the factor.  The
    mix holds a diagonal gate that is not symmetric in its qubits (so a
    swapped qubit order fails) and a controlled diagonal gate."""
    n = 7
    rng = np.random.Generator(np.random.PCG64(40 + seed))
    gates = []
    for _ in range(12):
        a, b = (int(v) for v in rng.choice(n, 2, replace=False))
        gates.append(C.Gate((a, b), C.CP(float(rng.uniform(0, 2 * np.pi)))))
    gates.append(C.Gate((1, 5), np.diag(np.exp(1j * np.array([0.1, 0.7, 1.9, 2.6])))))
    gates.append(C.Gate((3,), C.RZ(0.4), (0, 6), (1, 0)))
    gates += [C.Gate((q,), C.RZ(float(rng.uniform(0, 2 * np.pi)))) for q in range(n)]
    idx = np.arange(1 << n)
    psi = oracle.brute_force_state(n, [C.Gate((q,), C.H) for q in range(n)] + gates)
    f = oracle.diagonal_factors(gates, idx)
    assert np.max(np.abs(psi - f * 2.0 ** (-n / 2))) < 1e-13
    swapped = [C.Gate(tuple(reversed(g.qubits)), g.matrix, g.controls, g.control_values) if g.k == 2 else g
               for g in gates]
    assert np.max(np.abs(oracle.diagonal_factors(swapped, idx) - f)) > 1e-3
