"""Controlled gates (Eq. 4's indicator 1_c): fusion on the host (CPU, checked
through the oracle) and the controlled-gate kernel on the GPU, against the
oracle's gate-by-gate controlled application."""
import os

import numpy as np
import pytest

import circuits as C
import oracle
from paper_2602_09604_amd import sv

needs_lib = pytest.mark.skipif(not os.path.exists(sv.LIB_PATH), reason="libsv.so not built")


def controlled_mix(n, n_gates, seed, max_span=None):
    """Random dense and controlled gates; a controlled gate has 1..3 targets
    and 1..5 controls with random control values."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gates = []
    for _ in range(n_gates):
        if rng.random() < 0.5:
            k = int(rng.integers(1, 3))
            gates.append(C.Gate(tuple(int(v) for v in rng.choice(n, k, replace=False)), C.haar_unitary(k, rng)))
        else:
            k = int(rng.integers(1, 4))
            nc = int(rng.integers(1, 6))
            if max_span:
                nc = max(1, min(nc, max_span - k))
            qs = [int(v) for v in rng.choice(n, k + nc, replace=False)]
            vals = tuple(int(v) for v in rng.integers(0, 2, nc))
            gates.append(C.Gate(tuple(qs[:k]), C.haar_unitary(k, rng), tuple(qs[k:]), vals))
    return gates


# ------------------------------------------------------------------ host
@needs_lib
@pytest.mark.parametrize("fusion", ["none", "greedy", "phase", "block", "learned"])
@pytest.mark.parametrize("max_k", [2, 4, 6])
@pytest.mark.parametrize("seed", range(3))
def test_fusion_with_controls_equivalent(fusion, max_k, seed):
    n = 9
    gates = controlled_mix(n, 40, seed)
    fused, block_of = sv.sv_fuse(gates, n, sv.make_opts(max_k=max_k, fusion=fusion))
    assert len(block_of) == len(gates) and block_of.min() >= 0
    widest = max(g.k for g in gates)
    for f in fused:
        assert f.k <= max(max_k, widest) or fusion == "none"
        if f.controls:  # a kept controlled gate: wider than max_k with its controls, or unfused
            assert fusion == "none" or f.k + len(f.controls) > min(max_k, 6)
    init = 3 * seed + 1
    ref = oracle.apply_circuit(n, gates, init=init)
    got = oracle.apply_circuit(n, fused, init=init)
    assert np.max(np.abs(ref - got)) < 1e-12


@needs_lib
def test_narrow_controlled_gates_are_lifted():
    gates = [C.Gate((1,), C.X, (0,)), C.Gate((2,), C.Z, (0, 1), (1, 0))]
    fused, _ = sv.sv_fuse(gates, 4, sv.make_opts(max_k=3, fusion="greedy"))
    assert len(fused) == 1 and not fused[0].controls and fused[0].k == 3
    ref = oracle.apply_circuit(4, [C.Gate((q,), C.H) for q in range(4)] + gates)
    got = oracle.apply_circuit(4, [C.Gate((q,), C.H) for q in range(4)] + fused)
    assert np.max(np.abs(ref - got)) < 1e-14


@needs_lib
def test_wide_controlled_gate_blocks_its_controls():
    # the H on qubit 3 may not move across the MCZ that uses qubit 3 as a control
    gates = [C.Gate((0,), C.H), C.Gate((4,), C.Z, (0, 1, 2, 3)), C.Gate((3,), C.H), C.Gate((0,), C.X)]
    fused, block_of = sv.sv_fuse(gates, 5, sv.make_opts(max_k=2, fusion="greedy"))
    assert block_of[1] != block_of[0] and block_of[1] != block_of[2]
    for init in range(32):
        ref = oracle.apply_circuit(5, gates, init=init)
        assert np.max(np.abs(oracle.apply_circuit(5, fused, init=init) - ref)) < 1e-14


@needs_lib
@pytest.mark.parametrize("bad", [
    C.Gate((1,), C.X, (1,)),            # control is also a target
    C.Gate((1,), C.X, (7,)),            # control past n
])
def test_controlled_validation(bad):
    with pytest.raises(sv.SvError):
        sv.sv_fuse([bad], 4, sv.make_opts(max_k=2))


# ------------------------------------------------------------------ GPU
def prep(n, seed):
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    return [C.Gate((q,), C.haar_unitary(1, rng)) for q in range(n)]


@pytest.mark.gpu
@pytest.mark.parametrize("case", [
    # (n, targets, controls, values)
    (12, (0,), (1,), None),
    (12, (1,), (0,), None),               # control on bit 0
    (12, (5,), (0, 1, 2, 3), (1, 0, 1, 0)),
    (14, (0, 13), (6,), (0,)),
    (16, (3, 7, 11), (0, 15), None),
    (16, (2, 4, 6, 8), (0, 1), (0, 1)),
    (18, (0, 1, 2, 3, 4), (17,), None),
    (18, (12, 13, 14, 15, 16, 17), (0, 1, 2), (1, 1, 0)),
    (10, (9,), tuple(range(9)), None),    # one group (a multi-controlled gate on all qubits)
    (10, (0, 1, 2, 3, 4, 5), (6, 7, 8, 9), (0, 0, 0, 0)),  # k + c = n
    (20, (19,), (3,), None),
    (21, (10, 11), tuple(range(20, 21)), None),
])
def test_controlled_gate_kernel_vs_oracle(case):
    n, ts, cs, vals = case
    rng = np.random.Generator(np.random.PCG64(n + len(ts) + len(cs)))
    u = C.haar_unitary(len(ts), rng)
    gate = C.Gate(ts, u, cs, vals)
    ref = oracle.apply_circuit(n, prep(n, 1) + [gate])
    st = sv.State(n)
    try:
        st.apply_circuit(prep(n, 1), fusion="none")
        st.apply_controlled_gate(ts, u, cs, vals)
        r = oracle.compare(st.read(), ref)
        assert r["max_abs"] <= 1e-5 and r["infidelity"] <= 1e-6, r
    finally:
        st.free()


@pytest.mark.gpu
@pytest.mark.parametrize("fusion,prec", [("none", "fp32_valu"), ("greedy", "fp32_valu"), ("greedy", "fp16x3"),
                                         ("phase", "fp16x3"), ("greedy", "bf16x3"), ("block", "fp16x3"),
                                         ("block", "fp32_valu")])
@pytest.mark.parametrize("max_k", [3, 6])
def test_controlled_circuits_vs_oracle(fusion, prec, max_k):
    n = 18
    gates = prep(n, 2) + controlled_mix(n, 80, 5)
    ref = oracle.apply_circuit(n, gates)
    st = sv.State(n)
    try:
        s = st.apply_circuit(gates, max_k=max_k, fusion=fusion, precision=prec, stats=True)
        r = oracle.compare(st.read(), ref)
        assert r["max_abs"] <= 1e-5 and r["infidelity"] <= 1e-6, (s, r)
    finally:
        st.free()


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp16x3", "bf16x3", "fp32_mfma"])
@pytest.mark.parametrize("case", [
    # (n, targets, controls, values): k >= 4 controlled passes on the matrix cores
    (14, (2, 3, 5, 9), (12,), (1,)),
    (16, (0, 4, 5, 6, 7), (1, 15), (0, 1)),          # bit-0 target layout; a control on bit 1
    (18, (10, 11, 12, 13, 14, 15), (3, 7, 17), (1, 0, 1)),
    (18, (1, 2, 8, 9, 16, 17), (4, 5, 6), None),
    (13, (0, 1, 2, 3, 4, 5), (6,), (0,)),            # the smallest state with one tile left
    (26, (9, 14, 20, 25), (7, 12), (1, 1)),          # streaming stores
    (26, (0, 8, 16, 24, 25), (3, 22, 23), (0, 1, 0)),
])
def test_controlled_matrix_core_passes(case, prec):
    """Controlled k = 4..6 passes run on the matrix-core kernel (controls as
    extra fixed bits, the control values ORed into every group's base)."""
    n, ts, cs, vals = case
    rng = np.random.Generator(np.random.PCG64(7 * n + len(ts) + len(cs)))
    gates = [C.Gate(ts, C.haar_unitary(len(ts), rng), cs, vals),  # same control values: two launches
             C.Gate(tuple(reversed(ts)), C.haar_unitary(len(ts), rng), cs, vals)]
    ref = oracle.apply_circuit(n, prep(n, 3) + gates)
    st = sv.State(n)
    try:
        st.apply_circuit(prep(n, 3), fusion="none")
        s = st.apply_circuit(gates, fusion="none", precision=prec, stats=True, timing=True)
        assert s["variant_passes"][3] == 2, s  # both on the matrix-core kernel
        assert s["bytes"] == 2 * (16 << (n - len(cs)))
        r = oracle.compare(st.read(), ref)
        assert r["max_abs"] <= 1e-5 and r["infidelity"] <= 1e-6, r
    finally:
        st.free()


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp16x3", "bf16x3", "fp32_mfma"])
@pytest.mark.parametrize("case", [
    # (n, targets, controls, order of the control values given, values left out)
    (16, (2, 3, 5, 9), (12,), (1, 0), ()),
    (18, (0, 4, 5, 6, 7, 8), (9, 17), (0, 1, 2, 3), ()),
    (18, (10, 11, 12, 13, 14, 15), (7, 8, 16), (5, 0, 7, 2, 1, 6, 3, 4), ()),
    (26, (9, 14, 20, 25), (7, 12, 22), tuple(range(8)), ()),
    (18, (1, 2, 3, 4), (7, 8), (0, 1, 2, 3), (2,)),   # one value missing: one launch per value
    (18, (1, 2, 9), (7, 8, 17), tuple(range(8)), ()),  # k = 3: register launches, one per value
    (15, (0, 1, 2, 3, 4, 5), (12, 13, 14), tuple(range(8)), ()),  # smallest states: a few tiles per value
    (16, (1, 2, 3, 4, 5, 6), (13, 14, 15), (7, 6, 5, 4, 3, 2, 1, 0), ()),
])
def test_multiplexed_matrix_core_pass(case, prec):
    """One gate per control value on the same targets (what a fused block
    with controls becomes) runs as one matrix-core launch over the whole
    state; a group with a value missing, or with fewer than 4 targets, runs
    value by value."""
    n, ts, cs, order, missing = case
    rng = np.random.Generator(np.random.PCG64(5 * n + len(cs)))
    gates = []
    for v in order:
        if v in missing:
            continue
        vals = tuple((v >> t) & 1 for t in range(len(cs)))
        gates.append(C.Gate(ts, C.haar_unitary(len(ts), rng), cs, vals))
    ref = oracle.apply_circuit(n, prep(n, 4) + gates)
    st = sv.State(n)
    try:
        st.apply_circuit(prep(n, 4), fusion="none")
        s = st.apply_circuit(gates, fusion="none", precision=prec, stats=True, timing=True)
        if len(ts) < 4:
            assert s["passes"] == len(gates) and s["variant_passes"][1] == len(gates)
            assert s["bytes"] == 16 << n  # 2^c launches over 2^-c of the state each
        elif missing:
            assert s["passes"] == len(gates) and s["variant_passes"][3] == len(gates)
        else:
            assert s["passes"] == 1 and s["variant_passes"][3] == 1, s
            assert s["bytes"] == 16 << n
        r = oracle.compare(st.read(), ref)
        assert r["max_abs"] <= 1e-5 and r["infidelity"] <= 1e-6, r
    finally:
        st.free()


@pytest.mark.gpu
def test_controlled_pass_bytes_counted():
    n = 20
    st = sv.State(n)
    try:
        s = st.apply_circuit([C.Gate((5,), C.X, (16, 17, 18))], fusion="none", stats=True)
        assert s["passes"] == 1 and s["bytes"] == 16 << (n - 3)
    finally:
        st.free()


@pytest.mark.gpu
def test_controlled_bad_arguments():
    st = sv.State(6)
    try:
        with pytest.raises(sv.SvError):
            st.apply_controlled_gate((1,), C.X, (1,))
        with pytest.raises(sv.SvError):
            st.apply_controlled_gate((1,), C.X, (0,), (2,))
        with pytest.raises(sv.SvError):
            st.apply_controlled_gate((1,), C.X, (9,))
    finally:
        st.free()
