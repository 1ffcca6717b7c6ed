"""Parity at the full sizes the benchmark runs (34 qubits, 128 GiB state;
32 qubits, 32 GiB), in the benchmark's launch configuration (fused to k = 6,
split-precision matrix cores), on sampled outputs the oracle computes one by
one, and on properties that hold at any size."""
import os
import sys

import numpy as np
import pytest

import circuits as C
import oracle

pytestmark = pytest.mark.gpu

ROWS, COLS, DEPTH = 2, 17, 24
N = ROWS * COLS
LEFT = [r * COLS + c for r in range(ROWS) for c in range(9)]       # columns 0..8: 18 qubits
RIGHT = [r * COLS + c for r in range(ROWS) for c in range(9, COLS)]  # columns 9..16: 16 qubits


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def factorised_grid(seed):
    """The 2x17 depth-24 grid circuit without the 12 CZs that cross between
    columns 8 and 9: its state is exactly a product of an 18-qubit and a
    16-qubit state."""
    gates = C.grid_circuit(ROWS, COLS, DEPTH, seed=seed)
    left, right = set(LEFT), set(RIGHT)
    kept = [g for g in gates if set(g.qubits) <= left or set(g.qubits) <= right]
    assert len(gates) - len(kept) == 12
    return kept


def half_states(gates):
    lpos = {q: i for i, q in enumerate(LEFT)}
    rpos = {q: i for i, q in enumerate(RIGHT)}
    def relabel(g, pos):
        return C.Gate(tuple(pos[q] for q in g.qubits), g.matrix, tuple(pos[q] for q in g.controls),
                      g.control_values)

    lg = [relabel(g, lpos) for g in gates if g.qubits[0] in lpos]
    rg = [relabel(g, rpos) for g in gates if g.qubits[0] in rpos]
    return oracle.apply_circuit(len(LEFT), lg), oracle.apply_circuit(len(RIGHT), rg)


def product_amplitudes(psi_l, psi_r, idx):
    idx = np.asarray(idx, dtype=np.uint64)
    il = np.zeros(idx.size, dtype=np.int64)
    ir = np.zeros(idx.size, dtype=np.int64)
    for i, q in enumerate(LEFT):
        il |= ((idx >> np.uint64(q)) & np.uint64(1)).astype(np.int64) << i
    for i, q in enumerate(RIGHT):
        ir |= ((idx >> np.uint64(q)) & np.uint64(1)).astype(np.int64) << i
    return psi_l[il] * psi_r[ir]


def sample_indices(n, seed, count=4096):
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.unique(rng.integers(0, 1 << n, size=count, dtype=np.uint64))


def read_samples(st, idx):
    return np.array([st.read(int(i), 1)[0] for i in idx], dtype=np.complex64)


@pytest.fixture(scope="module")
def state34():
    import torch
    from paper_2602_09604_amd import sv
    st = sv.State(N)
    yield st
    st.free()
    del st
    torch.cuda.empty_cache()


GOLD34 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "grid34_d24_s0_cut.npz")


@pytest.mark.parametrize("prec", ["fp16x3", "fp32_mfma", "fp32_valu", "bf16x3"])
def test_grid34_benchmark_circuit_against_cut_oracle(state34, prec):
    """The benchmarked circuit itself (2x17 grid, depth 24, seed 0, |0..0>,
    learned fusion to k <= 6 with control bits), against exact amplitudes the
    oracle computed by cutting the ladder between columns 8 and 9 (4096 paths
    of 18- and 16-qubit halves, tests/golden/make_grid34_cut.py): 4096 random
    indices and one contiguous block of 2^16."""
    with np.load(GOLD34, allow_pickle=False) as f:
        idx, ref, nr = f["idx"], f["amp"], int(f["n_random"])
    gates = C.grid_circuit(ROWS, COLS, DEPTH, seed=0)
    st = state34
    st.set_basis(0)
    stats = st.apply_circuit(gates, max_k=6, fusion="learned", precision=prec, stats=True)
    say(prec, "learned passes", stats["passes"], "gpu_s", stats["gpu_s"])
    acc = oracle.CompareAcc()
    acc.add(read_samples(st, idx[:nr]), ref[:nr])
    acc.add(st.read(int(idx[nr]), idx.size - nr), ref[nr:])
    r = acc.result()
    drift = abs(st.norm() - 1.0)
    rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    say(prec, r, "drift", drift, "rms amplitude", rms)
    assert r["max_abs"] <= 1e-5
    assert r["infidelity"] <= 1e-6  # fidelity estimated on the sampled amplitudes
    # |c| ~ 2^-17 here, so the absolute bar is loose; every sampled amplitude
    # must also be right to 1e-3 of the typical amplitude
    assert r["max_abs"] <= 1e-3 * rms
    # BF16X3 carries operands to ~16 bits and is outside this workload's
    # norm-drift bar (its drift is reported, not bounded)
    if prec != "bf16x3":
        assert drift <= 1e-5, drift


@pytest.mark.parametrize("prec,fusion", [("fp16x3", "greedy"), ("bf16x3", "greedy"), ("fp32_valu", "greedy"),
                                         ("fp16x3", "block"), ("fp16x3", "learned")])
def test_grid34_factorised_sampled(state34, prec, fusion):
    gates = factorised_grid(seed=5)
    psi_l, psi_r = half_states(gates)
    st = state34
    st.set_basis(0)
    stats = st.apply_circuit(gates, max_k=6, fusion=fusion, precision=prec, stats=True)
    say(prec, fusion, "passes", stats["passes"], "gpu_s", stats["gpu_s"])
    idx = sample_indices(N, 1)
    got = read_samples(st, idx)
    ref = product_amplitudes(psi_l, psi_r, idx)
    # a contiguous block too (coalesced read-back path)
    start = 123 << 20
    blk = st.read(start, 1 << 16)
    ref_blk = product_amplitudes(psi_l, psi_r, np.arange(start, start + (1 << 16), dtype=np.uint64))
    acc = oracle.CompareAcc()
    acc.add(got, ref)
    acc.add(blk, ref_blk)
    r = acc.result()
    say(prec, r)
    assert r["max_abs"] <= 1e-5
    assert r["infidelity"] <= 1e-6  # fidelity estimated on the sampled amplitudes
    # split BF16 carries the fused matrices to ~16 bits, which shows as a slow
    # norm drift over many k = 6 passes: reported, outside the drift bar;
    # FP16 (22 bits) and FP32 stay below 1e-5
    drift = abs(st.norm() - 1.0)
    say(prec, fusion, "drift", drift)
    if prec != "bf16x3":
        assert drift <= 1e-5, drift


@pytest.mark.parametrize("fusion", ["greedy", "learned"])
def test_grid34_mirror_returns_to_zero(state34, fusion):
    """C followed by C^dagger on the 34-qubit grid (12 cycles each way) must
    return |0...0> (learned fusion: blocks with controls included)."""
    gates = C.grid_circuit(ROWS, COLS, 12, seed=9)
    st = state34
    st.set_basis(0)
    st.apply_circuit(C.mirror_circuit(gates), max_k=6, fusion=fusion, precision="fp16x3")
    p0 = abs(complex(st.read(0, 1)[0])) ** 2
    norm = st.norm()
    say("mirror |psi_0|^2 =", p0, "norm", norm)
    assert p0 / norm >= 1 - 1e-6   # fidelity with |0...0>
    assert abs(norm - 1.0) <= 1e-5  # norm drift


@pytest.mark.parametrize("prec,fusion", [("fp16x3", "greedy"), ("bf16x3", "greedy"), ("fp16x3", "phase"),
                                         ("bf16x3", "phase"), ("fp32_valu", "phase")])
def test_qft32_closed_form_sampled(prec, fusion):
    """Config 3: 32-qubit QFT-like circuit from a seeded basis state, fused to
    k = 5 on split-precision matrix cores (and with the controlled phases as
    phase passes), against the closed form."""
    import torch
    from paper_2602_09604_amd import sv
    n = 32
    x = C.qft_input_basis(n, 0)
    st = sv.State(n)
    try:
        st.set_basis(x)
        stats = st.apply_circuit(C.qft_like_circuit(n), max_k=5, fusion=fusion, precision=prec, stats=True)
        say(prec, fusion, "passes", stats["passes"], "gpu_s", stats["gpu_s"])
        idx = sample_indices(n, 2)
        acc = oracle.CompareAcc()
        acc.add(read_samples(st, idx), oracle.qft_like_amplitudes(n, x, idx))
        start = 7 << 24
        acc.add(st.read(start, 1 << 16), oracle.qft_like_amplitudes(n, x, np.arange(start, start + (1 << 16))))
        r = acc.result()
        say(prec, r)
        assert r["max_abs"] <= 1e-5 and r["infidelity"] <= 1e-6
        assert abs(st.norm() - 1.0) <= 1e-5
    finally:
        st.free()
        del st
        torch.cuda.empty_cache()


def test_grid34_state_reads_on_product_state(state34):
    """State reads at the benchmark's 128 GiB size: on the factorised grid
    state (an 18-qubit left half times a 16-qubit right half) marginals and
    Pauli expectations factorise into the halves' oracle values, and sampled
    outcomes follow the marginal."""
    gates = factorised_grid(seed=7)
    psi_l, psi_r = half_states(gates)
    st = state34
    st.set_basis(0)
    st.apply_circuit(gates, max_k=6, fusion="block", precision="fp16x3")
    # marginal of five left-half and three right-half qubits
    ql = [LEFT[i] for i in (0, 3, 7, 11, 17)]
    qr = [RIGHT[i] for i in (2, 9, 15)]
    got = st.marginal_probs(ql + qr)
    pl = oracle.marginal_probabilities(psi_l, len(LEFT), [LEFT.index(q) for q in ql])
    pr = oracle.marginal_probabilities(psi_r, len(RIGHT), [RIGHT.index(q) for q in qr])
    ref = np.outer(pr, pl).reshape(-1)  # outcome bits: left qubits low, right qubits high
    say("marginal max diff", np.max(np.abs(got - ref)))
    assert np.max(np.abs(got - ref)) < 1e-5
    # Pauli strings: Z on a left qubit, X on a right qubit, Z Z across the halves, Y Y inside the left half
    a, b, c = LEFT[4], RIGHT[5], LEFT[9]
    terms = [(0, 1 << a), (1 << b, 0), (0, (1 << a) | (1 << b)), ((1 << a) | (1 << c), (1 << a) | (1 << c))]
    got = st.expect_pauli([t[0] for t in terms], [t[1] for t in terms])
    zl = oracle.pauli_expectation(psi_l, len(LEFT), 0, 1 << LEFT.index(a)).real
    xr = oracle.pauli_expectation(psi_r, len(RIGHT), 1 << RIGHT.index(b), 0).real
    zr = oracle.pauli_expectation(psi_r, len(RIGHT), 0, 1 << RIGHT.index(b)).real
    yy = oracle.pauli_expectation(psi_l, len(LEFT), (1 << LEFT.index(a)) | (1 << LEFT.index(c)),
                                  (1 << LEFT.index(a)) | (1 << LEFT.index(c))).real
    ref = np.array([zl, xr, zl * zr, yy])
    say("pauli", got, ref)
    assert np.max(np.abs(got - ref)) < 1e-5  # the state's own rounding (norm drift ~1e-6) bounds these
    # 20000 samples: the frequencies of the three right-half qubits' outcomes
    u = C.uniforms(20000, 11)
    idx = st.sample(u).astype(np.uint64)
    o = np.zeros(idx.size, dtype=np.int64)
    for j, q in enumerate(qr):
        o |= ((idx >> np.uint64(q)) & np.uint64(1)).astype(np.int64) << j
    freq = np.bincount(o, minlength=8) / idx.size
    sigma = np.sqrt(pr * (1 - pr) / idx.size)
    say("sample freq", freq, "expected", pr)
    assert np.all(np.abs(freq - pr) <= 5 * sigma + 1e-9)


def test_grid34_controlled_passes_sampled(state34):
    """Controlled passes at 34 qubits: multi-controlled gates inside each half
    of the factorised grid state keep it a product, so sampled amplitudes are
    checked against the halves' oracle states."""
    rng = np.random.Generator(np.random.PCG64(21))
    gates = factorised_grid(seed=8)
    ctl = [C.Gate((LEFT[2],), C.haar_unitary(1, rng), (LEFT[0], LEFT[9], LEFT[17]), (1, 0, 1)),
           C.Gate((RIGHT[3], RIGHT[12]), C.haar_unitary(2, rng), (RIGHT[0], RIGHT[15])),
           C.Gate((LEFT[5],), C.Z, tuple(LEFT[i] for i in (1, 4, 6, 8, 10, 12, 14, 16)))]
    psi_l, psi_r = half_states(gates + ctl)
    st = state34
    st.set_basis(0)
    st.apply_circuit(gates, max_k=6, fusion="block", precision="fp16x3")
    s = st.apply_circuit(ctl, fusion="none", stats=True)
    assert s["bytes"] == (16 << (N - 3)) + (16 << (N - 2)) + (16 << (N - 8))
    idx = sample_indices(N, 3)
    acc = oracle.CompareAcc()
    acc.add(read_samples(st, idx), product_amplitudes(psi_l, psi_r, idx))
    r = acc.result()
    say("controlled", r)
    assert r["max_abs"] <= 1e-5 and r["infidelity"] <= 1e-6
