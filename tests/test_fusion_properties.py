"""Property-based checks of every fusion mode on random small circuits
(dense, pure-phase and controlled gates, random widths): the fused list must
act exactly like the gate list (oracle, complex128), keep every gate inside its
block, keep per-qubit order, and respect max_k."""
import os

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import circuits as C
import oracle
from paper_2602_09604_amd import sv

pytestmark = pytest.mark.skipif(not os.path.exists(sv.LIB_PATH), reason="libsv.so not built")


@st.composite
def circuits_st(draw):
    n = draw(st.integers(3, 8))
    seed = draw(st.integers(0, 2**31 - 1))
    rng = np.random.Generator(np.random.PCG64(seed))
    gates = []
    for _ in range(draw(st.integers(1, 40))):
        kind = draw(st.sampled_from(["dense", "dense", "phase", "cp", "ctrl"]))
        if kind == "dense":
            k = int(rng.integers(1, min(3, n) + 1))
            qs = tuple(int(v) for v in rng.choice(n, k, replace=False))
            gates.append(C.Gate(qs, C.haar_unitary(k, rng)))
        elif kind == "phase":
            gates.append(C.Gate((int(rng.integers(n)),), C.RZ(float(rng.uniform(0, 6.3)))))
        elif kind == "cp":
            a, b = (int(v) for v in rng.choice(n, 2, replace=False))
            gates.append(C.Gate((a, b), C.CP(float(rng.uniform(0, 6.3)))))
        else:
            k = 1
            nc = int(rng.integers(1, n))
            qs = [int(v) for v in rng.choice(n, k + nc, replace=False)]
            vals = tuple(int(v) for v in rng.integers(0, 2, nc))
            gates.append(C.Gate(tuple(qs[:k]), C.haar_unitary(k, rng), tuple(qs[k:]), vals))
    return n, gates


@settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(circuits_st(), st.sampled_from(["none", "greedy", "phase", "block", "learned"]), st.integers(1, 6))
def test_fusion_is_exact(case, fusion, max_k):
    n, gates = case
    max_k = min(max_k, n)
    fused, block_of = sv.sv_fuse(gates, n, sv.make_opts(max_k=max_k, fusion=fusion))
    assert len(block_of) == len(gates)
    assert block_of.min() >= 0 and block_of.max() < len(fused)
    widest = max(g.k for g in gates)
    def is_phase(g):
        m = np.asarray(g.matrix)
        return not g.controls and g.k <= 2 and np.allclose(m, np.diag(np.diag(m)))

    for i, g in enumerate(gates):
        if fusion in ("phase", "learned") and is_phase(g):
            continue  # a phase block is returned as canonical diagonal gates; block_of names the first
        f = fused[block_of[i]]
        span = set(f.qubits) | set(f.controls)
        assert set(g.qubits) <= span
        if not f.controls:
            assert set(g.controls) <= set(f.qubits)
    for f in fused:
        assert list(f.qubits) == sorted(f.qubits)
        if fusion != "none" and not f.controls:
            assert f.k <= max(max_k, widest, 2)
    for q in range(n):  # per-qubit order of the blocks that touch q (controls included)
        seq = [int(block_of[i]) for i, g in enumerate(gates) if q in g.qubits or q in g.controls]
        if fusion not in ("phase", "learned"):
            assert seq == sorted(seq)
    init = int(np.random.Generator(np.random.PCG64(len(gates))).integers(1 << n))
    ref = oracle.apply_circuit(n, gates, init=init)
    got = oracle.apply_circuit(n, fused, init=init)
    assert np.max(np.abs(ref - got)) < 1e-11


@st.composite
def wide_circuits_st(draw):
    """8..11 qubits, so that several qubits sit at bit 4 or above (and some below); many
    diagonal two-qubit gates (CZ, CP) among dense and controlled ones."""
    n = draw(st.integers(8, 11))
    seed = draw(st.integers(0, 2**31 - 1))
    rng = np.random.Generator(np.random.PCG64(seed))
    gates = []
    for _ in range(draw(st.integers(1, 50))):
        kind = draw(st.sampled_from(["dense", "dense", "cz", "cp", "phase", "ctrl"]))
        if kind == "dense":
            k = int(rng.integers(1, 3))
            qs = tuple(int(v) for v in rng.choice(n, k, replace=False))
            gates.append(C.Gate(qs, C.haar_unitary(k, rng)))
        elif kind in ("cz", "cp"):
            a, b = (int(v) for v in rng.choice(n, 2, replace=False))
            gates.append(C.Gate((a, b), C.CZ if kind == "cz" else C.CP(float(rng.uniform(0, 6.3)))))
        elif kind == "phase":
            gates.append(C.Gate((int(rng.integers(n)),), C.RZ(float(rng.uniform(0, 6.3)))))
        else:
            nc = int(rng.integers(1, 4))
            qs = [int(v) for v in rng.choice(n, 1 + nc, replace=False)]
            gates.append(C.Gate((qs[0],), C.haar_unitary(1, rng), tuple(qs[1:]),
                                tuple(int(v) for v in rng.integers(0, 2, nc))))
    return n, gates


@settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(wide_circuits_st(), st.integers(2, 6))
def test_blocks_with_controls_are_exact(case, max_k):
    """Learned fusion planned for a 30-qubit state at a matrix-core precision
    (where blocks may take control bits): every block is one gate or 2^c gates
    on the same targets with distinct control values, controls at bit 4 or
    above, at most 3; the fused list acts exactly like the gate list."""
    n, gates = case
    fused, block_of = sv.sv_fuse(gates, 30, sv.make_opts(max_k=max_k, fusion="learned", precision="fp16x3"))
    assert len(block_of) == len(gates)
    starts = sorted(set(int(b) for b in block_of))
    wide = {tuple(g.controls) for g in gates if g.controls}
    for a, b in zip(starts, starts[1:] + [len(fused)]):
        head = fused[a]
        c = len(head.controls)
        if c and tuple(head.controls) not in wide and b - a > 1:
            assert b - a == 1 << c and c <= 3 and min(head.controls) >= 4
            assert len({tuple(f.control_values) for f in fused[a:b]}) == b - a
            assert all(f.qubits == head.qubits and f.controls == head.controls for f in fused[a:b])
    init = int(np.random.Generator(np.random.PCG64(len(gates) + n)).integers(1 << n))
    ref = oracle.apply_circuit(n, gates, init=init)
    got = oracle.apply_circuit(n, fused, init=init)
    assert np.max(np.abs(ref - got)) < 1e-11
