"""Diagonal specialisation: PHASE fusion (host, checked through the oracle)
and elementwise phase passes (GPU, against the oracle and closed forms)."""
import os

import numpy as np
import pytest

import circuits as C
import oracle
from paper_2602_09604_amd import sv

needs_lib = pytest.mark.skipif(not os.path.exists(sv.LIB_PATH), reason="libsv.so not built")


def phase_heavy_circuit(n, n_gates, seed):
    """Random mix: CZ, CP(theta), RZ, S/T-like phases, and dense Haar gates."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gates = []
    for _ in range(n_gates):
        r = rng.random()
        if r < 0.3:
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            gates.append(C.Gate((a, b), C.CP(float(rng.uniform(0, 2 * np.pi)))))
        elif r < 0.45:
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            gates.append(C.Gate((a, b), C.CZ))
        elif r < 0.6:
            gates.append(C.Gate((int(rng.integers(n)),), C.RZ(float(rng.uniform(0, 2 * np.pi)))))
        elif r < 0.65:  # a general 2-qubit diagonal phase gate
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            gates.append(C.Gate((a, b), np.diag(np.exp(1j * rng.uniform(0, 2 * np.pi, 4)))))
        else:
            k = int(rng.integers(1, 3))
            qs = tuple(int(x) for x in rng.choice(n, k, replace=False))
            gates.append(C.Gate(qs, C.haar_unitary(k, rng)))
    return gates


@needs_lib
@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("max_k", [2, 4, 6])
def test_phase_fusion_equivalent(seed, max_k):
    n = 9
    gates = phase_heavy_circuit(n, 60, seed)
    fused, block_of = sv.sv_fuse(gates, n, sv.make_opts(max_k=max_k, fusion="phase"))
    assert len(block_of) == len(gates) and block_of.min() >= 0
    assert all(f.k <= max_k for f in fused)
    init = seed * 7 % (1 << n)
    ref = oracle.apply_circuit(n, gates, init=init)
    got = oracle.apply_circuit(n, fused, init=init)
    assert np.max(np.abs(ref - got)) < 1e-12


@needs_lib
def test_phase_fusion_qft_few_blocks():
    """QFT-like: the controlled phases to qubits outside the current window
    become phase blocks, so the fused list is short."""
    n = 12
    gates = C.qft_like_circuit(n)
    fused, _ = sv.sv_fuse(gates, n, sv.make_opts(max_k=4, fusion="phase"))
    greedy, _ = sv.sv_fuse(gates, n, sv.make_opts(max_k=4, fusion="greedy"))
    x = C.qft_input_basis(n, 2)
    ref = oracle.qft_like_amplitudes(n, x, np.arange(1 << n))
    assert np.max(np.abs(oracle.apply_circuit(n, fused, init=x) - ref)) < 1e-12
    dense = [f for f in fused if not (f.k <= 2 and np.allclose(f.matrix, np.diag(np.diag(f.matrix))))]
    assert len(dense) <= n // 4 + 1, len(dense)
    assert len(dense) < len(greedy)


@needs_lib
def test_phase_fusion_canonical_gates_are_phases():
    gates = [C.Gate((0, 5), C.CP(0.3)), C.Gate((5, 0), C.CP(0.2)), C.Gate((2,), C.RZ(0.7))]
    fused, block_of = sv.sv_fuse(gates, 6, sv.make_opts(max_k=2, fusion="phase"))
    # one phase block: CP(0.5) on (0,5), a phase on qubit 2, global phase folded in
    assert len(fused) == 2 and set(block_of.tolist()) == {0}
    for f in fused:
        assert np.allclose(np.abs(np.diag(f.matrix)), 1) and np.allclose(f.matrix, np.diag(np.diag(f.matrix)))
    ref = oracle.apply_circuit(6, gates, init=37)
    assert np.max(np.abs(oracle.apply_circuit(6, fused, init=37) - ref)) < 1e-14


# ------------------------------------------------------------------ GPU
@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp32_valu", "fp16x3"])
def test_qft_phase_passes_closed_form(prec):
    n = 24
    x = C.qft_input_basis(n, 5)
    st = sv.State(n)
    try:
        st.set_basis(x)
        s = st.apply_circuit(C.qft_like_circuit(n), max_k=5, fusion="phase", precision=prec, timing=True)
        print(prec, "passes", s["passes"], "per family", s["variant_passes"], flush=True)
        assert s["variant_passes"][4] >= 1
        r = oracle.compare(st.read(), oracle.qft_like_amplitudes(n, x, np.arange(1 << n)))
        assert r["max_abs"] <= 1e-5 and r["infidelity"] <= 1e-6, r
    finally:
        st.free()


@pytest.mark.gpu
@pytest.mark.parametrize("seed", range(3))
def test_phase_heavy_random_circuits(seed):
    n = 18 + seed
    gates = [C.Gate((q,), C.H) for q in range(n)] + phase_heavy_circuit(n, 150, 100 + seed)
    ref = oracle.apply_circuit(n, gates)
    for K in (2, 5):
        st = sv.State(n)
        try:
            st.apply_circuit(gates, max_k=K, fusion="phase")
            r = oracle.compare(st.read(), ref)
            assert r["max_abs"] <= 1e-5 and r["infidelity"] <= 1e-6, (K, r)
        finally:
            st.free()


@pytest.mark.gpu
@pytest.mark.parametrize("n", [26, 28])
def test_phase_pass_all_pairs_one_sweep(n):
    """Controlled phases between random qubit pairs (every distance) plus
    one-qubit phases and a general diagonal two-qubit gate: the whole run is
    one phase pass, against the oracle's full state."""
    rng = np.random.Generator(np.random.PCG64(n))
    gates = [C.Gate((q,), C.H) for q in range(n)]
    phases = []
    for _ in range(160):
        a, b = (int(v) for v in rng.choice(n, 2, replace=False))
        phases.append(C.Gate((a, b), C.CP(float(rng.uniform(0, 2 * np.pi)))))
    for q in range(n):
        phases.append(C.Gate((q,), C.RZ(float(rng.uniform(0, 2 * np.pi)))))
    phases.append(C.Gate((0, n - 1), np.diag(np.exp(1j * rng.uniform(0, 2 * np.pi, 4)))))
    phases.append(C.Gate((9, n - 2), C.CZ))
    gates += phases
    ref = oracle.apply_circuit(n, gates)
    st = sv.State(n)
    try:
        s = st.apply_circuit(gates, max_k=1, fusion="phase", timing=True)
        print("phase passes", s["variant_passes"][4], "passes", s["passes"], flush=True)
        assert s["variant_passes"][4] == 1
        r = oracle.compare(st.read(), ref)
        print(r, flush=True)
        assert r["max_abs"] <= 1e-5 and r["infidelity"] <= 1e-6, r
    finally:
        st.free()


def phase_run(n, rng, pairs):
    gates = []
    for _ in range(pairs):
        a, b = (int(v) for v in rng.choice(n, 2, replace=False))
        gates.append(C.Gate((a, b), C.CP(float(rng.uniform(0, 2 * np.pi)))))
    gates += [C.Gate((q,), C.RZ(float(rng.uniform(0, 2 * np.pi)))) for q in range(n)]
    gates.append(C.Gate((0, n - 1), np.diag(np.exp(1j * rng.uniform(0, 2 * np.pi, 4)))))
    gates.append(C.Gate((9, n - 2), np.diag(np.exp(1j * rng.uniform(0, 2 * np.pi, 4)))))
    gates.append(C.Gate((n - 3, 1), C.CZ))
    return gates


@pytest.mark.gpu
@pytest.mark.parametrize("n", [30, 32])
def test_phase_pass_high_bits_sampled(n):
    """Above the low span one grid sweep covers (2^28 amplitudes) the pass
    walks the high index bits sweep by sweep.  From the uniform superposition
    every amplitude is 2^(-n/2) times the product of the diagonal entries its
    index selects (oracle.diagonal_factors): checked on 4096 random indices
    and the first and last 2^16 amplitudes, relative to 2^(-n/2)."""
    import torch
    rng = np.random.Generator(np.random.PCG64(300 + n))
    phases = phase_run(n, rng, 200)
    gates = [C.Gate((q,), C.H) for q in range(n)] + phases
    st = sv.State(n)
    try:
        s = st.apply_circuit(gates, max_k=6, fusion="phase", precision="fp32_valu", timing=True)
        assert s["variant_passes"][4] == 1
        scale = 2.0 ** (n / 2)
        worst, ms = 0.0, []
        idx = np.unique(rng.integers(0, 1 << n, 4096, dtype=np.uint64))
        got = np.array([st.read(int(i), 1)[0] for i in idx])
        blocks = [(idx, got)]
        for start in (0, (1 << n) - (1 << 16)):
            blocks.append((np.arange(start, start + (1 << 16), dtype=np.uint64), st.read(start, 1 << 16)))
        for ix, g in blocks:
            rel = np.abs(g.astype(np.complex128) * scale - oracle.diagonal_factors(phases, ix))
            worst = max(worst, float(rel.max()))
            ms.append(float(np.mean(rel ** 2)))
        print(n, "phase pass", s["variant_s"][4], "max rel", worst, "mean sq", max(ms), flush=True)
        assert worst <= 1e-5 and max(ms) <= 1e-10, (worst, ms)
    finally:
        st.free()
        del st
        torch.cuda.empty_cache()


@pytest.mark.gpu
@pytest.mark.parametrize("n", [1, 2, 5, 9, 10, 11, 13])
def test_phase_pass_small_states(n):
    """States smaller than one workgroup's span (idle threads) and the sizes
    where amplitude bit 9 and the block bits appear."""
    rng = np.random.Generator(np.random.PCG64(100 + n))
    psi0 = C.random_state_c64(n, 7 + n)
    gates = [C.Gate((q,), C.RZ(float(rng.uniform(0, 2 * np.pi)))) for q in range(n)]
    for _ in range(3 * n):
        if n < 2:
            break
        a, b = (int(v) for v in rng.choice(n, 2, replace=False))
        gates.append(C.Gate((a, b), C.CP(float(rng.uniform(0, 2 * np.pi)))))
    ref = psi0.astype(np.complex128)
    for g in gates:
        oracle.apply_gate(ref, n, g.qubits, g.matrix, g.cmask, g.cval)
    st = sv.State(n)
    try:
        st.write(0, psi0)
        s = st.apply_circuit(gates, max_k=1, fusion="phase", timing=True)
        assert s["variant_passes"][4] == 1
        r = oracle.compare(st.read(), ref)
        assert r["max_abs"] <= 1e-5 and r["infidelity"] <= 1e-6, (n, r)
    finally:
        st.free()


@pytest.mark.gpu
def test_grid_phase_fusion():
    n = 20
    gates = C.grid_circuit(4, 5, 14, seed=6)
    ref = oracle.apply_circuit(n, gates)
    for K in (4, 6):
        st = sv.State(n)
        try:
            st.apply_circuit(gates, max_k=K, fusion="phase", precision="fp16x3")
            r = oracle.compare(st.read(), ref)
            assert r["max_abs"] <= 1e-5 and r["infidelity"] <= 1e-6, (K, r)
        finally:
            st.free()
