"""Pins of the cut oracle (oracle/sf_cut.py) against the full-state oracle and
the Kronecker-product brute force, on ladders cut the same way as the
34-qubit 2x17 grid (between two columns, so only horizontal CZs cross)."""
import numpy as np
import pytest

import circuits as C
import oracle
from oracle import sf_cut


def ladder_left(rows, cols, cut_col):
    return [r * cols + c for r in range(rows) for c in range(cut_col)]


def test_cut_matches_full_oracle_2x6():
    rows, cols, depth = 2, 6, 8
    n = rows * cols
    gates = C.grid_circuit(rows, cols, depth, seed=3)
    left = ladder_left(rows, cols, 3)
    _, cross = sf_cut.split_circuit(gates, left, [q for q in range(n) if q not in left])
    assert len(cross) == 4  # two crossing couplers, patterns 0 and 1, twice each in 8 cycles
    idx = np.arange(1 << n, dtype=np.uint64)
    got = sf_cut.cut_amplitudes(n, gates, left, idx)
    ref = oracle.apply_circuit(n, gates)
    assert np.max(np.abs(got - ref)) < 1e-12


def test_cut_matches_brute_force_2x5():
    rows, cols, depth = 2, 5, 7
    n = rows * cols
    gates = C.grid_circuit(rows, cols, depth, seed=11)
    left = ladder_left(rows, cols, 2)
    got = sf_cut.cut_amplitudes(n, gates, left, np.arange(1 << n))
    ref = oracle.brute_force_state(n, gates)
    assert np.max(np.abs(got - ref)) < 1e-12


def test_cut_general_crossing_gates_and_basis_input():
    """Crossing gates other than CZ: a controlled phase, a uniformly
    controlled gate with Haar blocks and the left qubit listed second, and a
    CNOT controlled from the left; input a basis state other than |0>."""
    rng = np.random.Generator(np.random.PCG64(5))
    n = 9
    left = [0, 2, 4, 6]
    gates = []
    for _ in range(3):
        gates += [C.Gate((q,), C.haar_unitary(1, rng)) for q in range(n)]
        gates.append(C.Gate((2, 3), C.CP(0.7)))
        u0, u1 = C.haar_unitary(1, rng), C.haar_unitary(1, rng)
        m = np.zeros((4, 4), dtype=np.complex128)  # qubits (5, 4): local bit 1 is the left qubit 4
        m[0:2, 0:2] = u0
        m[2:4, 2:4] = u1
        gates.append(C.Gate((5, 4), m))
        gates.append(C.Gate((6, 7), C.CNOT))
        gates.append(C.Gate((0, 2), C.haar_unitary(2, rng)))
        gates.append(C.Gate((1, 8), C.haar_unitary(2, rng)))
    x = 0b101100110
    got = sf_cut.cut_amplitudes(n, gates, left, np.arange(1 << n), init=x)
    ref = oracle.apply_circuit(n, gates, init=x)
    assert np.max(np.abs(got - ref)) < 1e-12
    assert np.max(np.abs(ref - oracle.brute_force_state(n, gates, init=x))) < 1e-12


def test_cut_planted_block_swap_is_caught():
    rows, cols, depth = 2, 6, 8
    n = rows * cols
    gates = C.grid_circuit(rows, cols, depth, seed=3)
    left = ladder_left(rows, cols, 3)
    idx = np.arange(1 << n, dtype=np.uint64)
    bad = sf_cut.cut_amplitudes(n, gates, left, idx, blocks_fn=lambda b: (b[1], b[0]))
    ref = oracle.apply_circuit(n, gates)
    assert np.max(np.abs(bad - ref)) > 1e-3


def test_cut_rejects_gate_not_block_diagonal_in_left_qubit():
    # CNOT controlled from the right with its target on the left: not a sum of
    # two left projectors times right blocks
    gates = [C.Gate((0,), C.H), C.Gate((3, 1), C.CNOT)]
    with pytest.raises(ValueError):
        sf_cut.cut_amplitudes(4, gates, [0, 1], np.arange(16))


def test_grid34_cut_has_4096_paths():
    gates = C.grid_circuit(2, 17, 24, seed=0)
    left = ladder_left(2, 17, 9)
    labelled, cross = sf_cut.split_circuit(gates, left, [q for q in range(34) if q not in left])
    assert len(cross) == 12
    assert sum(1 for s, _ in labelled if s == "L") == 582
    assert sum(1 for s, _ in labelled if s == "R") == 516
    for a, b, (g0, g1) in cross:  # every crossing gate is a CZ: I and Z blocks
        assert np.array_equal(g0, np.eye(2)) and np.array_equal(g1, C.Z)
