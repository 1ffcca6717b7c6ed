"""Seeded input generators: gate counts and structure of the workloads."""
import numpy as np
import pytest

import circuits as C


@pytest.mark.parametrize("rows,cols,counts", [(4, 5, [8, 8, 8, 7]), (5, 6, [13, 12, 12, 12]), (2, 17, [16, 16, 9, 8])])
def test_coupler_patterns_are_matchings(rows, cols, counts):
    for p in range(4):
        edges = C.grid_couplers(rows, cols, p)
        assert len(edges) == counts[p]
        qs = [q for e in edges for q in e]
        assert len(qs) == len(set(qs))
        for a, b in edges:  # nearest neighbours
            ra, ca = divmod(a, cols)
            rb, cb = divmod(b, cols)
            assert abs(ra - rb) + abs(ca - cb) == 1


@pytest.mark.parametrize("rows,cols,depth,total", [(4, 5, 14, 389), (5, 6, 20, 845), (2, 17, 24, 1110)])
def test_grid_gate_counts(rows, cols, depth, total):
    g = C.grid_circuit(rows, cols, depth, seed=0)
    assert len(g) == total
    assert all(gate.k in (1, 2) for gate in g)


def test_grid_seeded_and_uniform():
    a = C.grid_circuit(4, 5, 14, seed=3)
    b = C.grid_circuit(4, 5, 14, seed=3)
    c = C.grid_circuit(4, 5, 14, seed=4)
    assert all(np.array_equal(x.matrix, y.matrix) and x.qubits == y.qubits for x, y in zip(a, b))
    assert any(not np.array_equal(x.matrix, y.matrix) for x, y in zip(a, c))


def test_batched_ansatz_shape():
    ns, circs = C.batched_ansatz(512, seed=0)
    assert len(ns) == 512 and min(ns) >= 10 and max(ns) <= 22
    assert all(len(c) == 8 * (3 * n - 1) for n, c in zip(ns, circs))
    total = sum(len(c) for c in circs)
    assert 150_000 < total < 240_000


def test_serialisation_roundtrip(tmp_path):
    g = C.random_circuit(9, 20, max_k=6, seed=1)
    p = tmp_path / "c.npz"
    C.save_npz(p, g, n=9)
    h = C.load_npz(p)
    assert all(x.qubits == y.qubits and np.array_equal(x.matrix, y.matrix) for x, y in zip(g, h))


def test_mirror_is_identity_product():
    g = C.random_circuit(4, 6, max_k=2, seed=2)
    m = C.mirror_circuit(g)
    assert len(m) == 12
    for a, b in zip(g, reversed(m[6:])):
        assert np.allclose(a.matrix @ b.matrix, np.eye(a.matrix.shape[0]))
