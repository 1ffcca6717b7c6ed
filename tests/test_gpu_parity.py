"""GPU parity: the HIP path through the C ABI against the CPU complex128 oracle.

Bar (complex64 state, FP32 arithmetic): max |delta amplitude| <= 1e-5 and
infidelity <= 1e-6 against the oracle, on the same seeded inputs.
"""
import sys

import numpy as np
import pytest

import circuits as C
import oracle

pytestmark = pytest.mark.gpu

MAX_ABS = 1e-5
INFID = 1e-6


def _sv():
    from paper_2602_09604_amd import sv
    return sv


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check(psi_gpu, psi_ref, max_abs=MAX_ABS, infid=INFID):
    r = oracle.compare(psi_gpu, psi_ref)
    assert r["max_abs"] <= max_abs, r
    assert r["infidelity"] <= infid, r
    return r


def run_gpu(n, gates, init=0, **kw):
    sv = _sv()
    st = sv.State(n)
    try:
        if init:
            st.set_basis(init)
        st.apply_circuit(gates, **kw)
        return st.read()
    finally:
        st.free()


def random_state_circuit(n, seed):
    """A prefix circuit that spreads amplitude over the whole state."""
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    return [C.Gate((q,), C.haar_unitary(1, rng)) for q in range(n)]


TARGET_SETS = {
    # name: function (n, k) -> qubits (unsorted on purpose)
    "low_q0": lambda n, k: tuple(reversed(range(k))),
    "high_top": lambda n, k: tuple(range(n - 1, n - 1 - k, -1)),
    "mixed": lambda n, k: tuple(sorted({0, n - 1, *range(2, 2 + max(0, k - 2))}, key=lambda q: (q * 7) % 11))[:k],
    "mid": lambda n, k: tuple(range(3, 3 + k)),
    "low_no_q0": lambda n, k: tuple(range(1, 1 + k)),
}


@pytest.mark.parametrize("variant", ["reg", "lds", "auto", "shfl"])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("tname", list(TARGET_SETS))
def test_single_gate_variants(variant, k, tname):
    n = 14
    qs = TARGET_SETS[tname](n, k)
    assert len(set(qs)) == k and all(0 <= q < n for q in qs)
    rng = np.random.Generator(np.random.PCG64(k * 100 + len(tname)))
    gates = random_state_circuit(n, k) + [C.Gate(qs, C.haar_unitary(k, rng))]
    say("single gate", variant, k, tname, qs)
    got = run_gpu(n, gates, fusion="none", variant=variant)
    check(got, oracle.apply_circuit(n, gates))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 8, 9, 12])
def test_small_states_every_k(n):
    """Ragged sizes including n == k (every qubit a target) and n = 1."""
    for k in range(1, min(6, n) + 1):
        gates = random_state_circuit(n, n) + C.random_circuit(n, 6, max_k=k, min_k=k, seed=n * 10 + k)
        say("small", n, k)
        for variant in ("auto", "reg", "lds"):
            got = run_gpu(n, gates, fusion="none", variant=variant)
            check(got, oracle.apply_circuit(n, gates))


def test_config1_grid_unfused_full_state():
    """20-qubit 4x5 grid, depth 14, unfused: the plain FP32 baseline circuit."""
    n = 20
    gates = C.grid_circuit(4, 5, 14, seed=0)
    ref = oracle.apply_circuit(n, gates)
    for graph in (False, True):
        say("config1 graph", graph)
        got = run_gpu(n, gates, fusion="none", precision="fp32_valu", use_graph=graph)
        r = check(got, ref)
        say(r)


@pytest.mark.parametrize("own_stream", [False, True])
def test_graph_relaunch_and_replacement(own_stream, tmp_path):
    """use_graph keeps its graph: the same circuit again relaunches it, plain
    calls in between (which reuse the upload ring) leave its pass data alone,
    and a different circuit replaces it.  The state after the whole sequence
    matches the oracle, on the default stream and on a stream of its own."""
    import torch
    sv = _sv()
    n = 14
    a = random_state_circuit(n, 3) + C.random_circuit(n, 40, max_k=3, seed=21)
    b = C.random_circuit(n, 30, max_k=2, seed=22)
    arrays = {"a": sv.GateArray(a), "b": sv.GateArray(b)}
    runs = [("a", dict(max_k=5, fusion="greedy", precision="fp16x3", use_graph=True), 0),
            ("a", dict(max_k=5, fusion="greedy", precision="fp16x3", use_graph=True), 1),
            ("b", dict(max_k=4, fusion="phase"), None),
            ("a", dict(max_k=5, fusion="greedy", precision="fp16x3", use_graph=True), 1),
            ("a", dict(max_k=5, fusion="greedy", precision="fp32_valu", use_graph=True), 0),
            ("b", dict(max_k=3, fusion="block", use_graph=True), 0),
            ("b", dict(max_k=3, fusion="block", use_graph=True), 1),
            ("a", dict(max_k=5, fusion="greedy", precision="fp16x3", use_graph=True), 0)]
    st = sv.State(n, stream=torch.cuda.Stream() if own_stream else None)
    try:
        seq = []
        for name, kw, relaunched in runs:
            s = st.apply_circuit(arrays[name], stats=True, **kw)
            say(name, kw, "relaunched", s["graph_relaunched"], "fuse_s", s["fuse_s"])
            if relaunched is not None:
                assert s["graph_relaunched"] == relaunched
                if relaunched:  # the same call again: no fusion, no upload
                    assert s["fuse_s"] == 0.0 and s["passes"] > 0 and s["bytes"] > 0
            seq += a if name == "a" else b
        # reloading the tuned table (unchanged) bumps the planning epoch: the
        # next identical call plans again, then finds the same passes
        path = str(tmp_path / "tune.json")
        sv.sv_tune_save(path)
        sv.sv_tune_load(path)
        s = st.apply_circuit(arrays["a"], stats=True, **runs[-1][1])
        assert s["fuse_s"] > 0.0 and s["graph_relaunched"] == 1
        seq += a
        check(st.read(), oracle.apply_circuit(n, seq))
    finally:
        st.free()


def test_graph_relaunch_of_blocks_with_controls():
    """28 qubits, learned fusion at FP16X3 (blocks with control bits, one
    matrix-core launch per block): the kept graph, relaunched, gives the
    same state as plain launches, bit for bit, and keeps the norm."""
    import torch
    sv = _sv()
    n = 28
    gates = C.grid_circuit(4, 7, 10, seed=3)
    fused, block_of = sv.sv_fuse(gates, n, sv.make_opts(max_k=6, fusion="learned", precision="fp16x3"))
    assert any(f.controls for f in fused)
    arr = sv.GateArray(gates)
    kw = dict(max_k=6, fusion="learned", precision="fp16x3")
    st = sv.State(n)
    try:
        st.apply_circuit(arr, **kw)
        plain = st.read(0, 1 << 20)
        plain_hi = st.read((1 << n) - (1 << 20), 1 << 20)
        for rep in range(3):
            st.set_basis(0)
            s = st.apply_circuit(arr, use_graph=True, stats=True, **kw)
            say("graph rep", rep, "relaunched", s["graph_relaunched"], "passes", s["passes"])
            assert s["graph_relaunched"] == (rep > 0)
            assert np.array_equal(st.read(0, 1 << 20), plain)
            assert np.array_equal(st.read((1 << n) - (1 << 20), 1 << 20), plain_hi)
        assert abs(st.norm() - 1.0) < 1e-5
    finally:
        st.free()
        torch.cuda.empty_cache()


@pytest.mark.parametrize("max_k", [2, 3, 4, 5, 6])
def test_grid_fused_greedy(max_k):
    n = 20
    gates = C.grid_circuit(4, 5, 14, seed=1)
    ref = oracle.apply_circuit(n, gates)
    say("grid fused", max_k)
    check(run_gpu(n, gates, max_k=max_k, fusion="greedy"), ref)


@pytest.mark.parametrize("seed", range(4))
def test_random_circuits_fused(seed):
    n = 16 + seed
    gates = C.random_circuit(n, 60, max_k=3, seed=seed)
    ref = oracle.apply_circuit(n, gates, init=seed)
    for K in (3, 5):
        say("random fused", n, K)
        check(run_gpu(n, gates, init=seed, max_k=K), ref)


def test_ghz_closed_form_26():
    n = 26
    sv = _sv()
    st = sv.State(n)
    try:
        st.apply_circuit(C.ghz_circuit(n), fusion="none")
        idx = np.array([0, 1, 2, (1 << n) - 2, (1 << n) - 1, 12345, 1 << 25])
        got = np.array([st.read(int(i), 1)[0] for i in idx])
        assert np.max(np.abs(got - oracle.ghz_amplitudes(n, idx))) < 1e-6
        assert abs(st.norm() - 1) < 1e-6
    finally:
        st.free()


def test_qft_like_closed_form_24():
    n = 24
    x = C.qft_input_basis(n, 3)
    sv = _sv()
    st = sv.State(n)
    try:
        st.set_basis(x)
        st.apply_circuit(C.qft_like_circuit(n), max_k=5)
        psi = st.read()
        ref = oracle.qft_like_amplitudes(n, x, np.arange(1 << n))
        check(psi, ref)
    finally:
        st.free()


def test_norm_and_basis():
    sv = _sv()
    st = sv.State(12)
    try:
        assert st.norm() == 1.0
        st.set_basis(777)
        a = st.read()
        assert a[777] == 1 and np.count_nonzero(a) == 1
        v = (np.arange(1 << 12) % 7 + 1j * (np.arange(1 << 12) % 5)).astype(np.complex64)
        st.write(0, v)
        assert abs(st.norm() - float(np.sum(np.abs(v.astype(np.complex128)) ** 2))) < 1e-9 * np.sum(np.abs(v) ** 2)
        assert np.array_equal(st.read(100, 50), v[100:150])
    finally:
        st.free()


@pytest.mark.parametrize("n", [26, 27])
def test_norm_many_blocks_against_oracle(n):
    """sv_norm on a random, unnormalised 2^26..2^27-amplitude state (every one
    of the 2048 first-level blocks busy) against the oracle's pairwise FP64
    sum of the same complex64 values."""
    sv = _sv()
    psi = C.random_state_c64(n, n) * np.complex64(1.25)
    st = sv.State(n)
    try:
        st.write(0, psi)
        got = st.norm()
        ref = oracle.norm_sq(psi.astype(np.complex128))
        say("norm n=%d: gpu %.17g oracle %.17g" % (n, got, ref))
        # squares of complex64 parts are exact in FP64: only the summation
        # order differs (relative error ~ log2(2^n) * 2^-53)
        assert abs(got - ref) <= 1e-13 * ref
    finally:
        st.free()


def test_basis_on_streamed_state():
    """|index> on a 27-qubit state (the chunk-walk initialisation): the one
    amplitude set, odd and even indices, its neighbours zero, norm 1."""
    sv = _sv()
    n = 27
    st = sv.State(n)
    try:
        for index in ((1 << n) - 3, (1 << 26) + 2, 0, 12345):
            st.set_basis(index)
            lo = min(max(0, index - 4), (1 << n) - 8)
            got = st.read(lo, 8)
            want = np.zeros(8, dtype=np.complex64)
            want[index - lo] = 1.0
            assert np.array_equal(got, want), (index, got)
            assert st.norm() == 1.0
            assert np.count_nonzero(st.read((1 << n) - 4096, 4096)) == (1 if index >= (1 << n) - 4096 else 0)
    finally:
        st.free()


def test_fp16x3_range_guard():
    """FP16X3 scales amplitudes by 2^14: a state whose sum |c|^2 may exceed
    15, or a gate that is not unitary, is rejected before any pass runs."""
    sv = _sv()
    n = 14
    gates = C.grid_circuit(2, 7, 4, seed=1)
    st = sv.State(n)
    try:
        big = C.random_state_c64(n, 3) * np.complex64(5.0)  # sum |c|^2 = 25
        st.write(0, big)
        with pytest.raises(sv.SvError) as e:
            st.apply_circuit(gates, max_k=4, fusion="greedy", precision="fp16x3")
        assert e.value.code == sv.SV_EINVAL
        assert np.array_equal(st.read(), big)  # untouched
        # FP32 matrix cores take it
        st.apply_circuit(gates, max_k=4, fusion="greedy", precision="fp32_mfma")
        assert abs(st.norm() - 25.0) < 1e-4
        # a basis state is fine again, and so is a normalised written state
        st.set_basis(3)
        st.apply_circuit(gates, max_k=4, fusion="greedy", precision="fp16x3")
        st.write(0, big / np.complex64(5.0))
        st.apply_circuit(gates, max_k=4, fusion="greedy", precision="fp16x3")
        # a gate that is not unitary
        with pytest.raises(sv.SvError) as e:
            st.apply_circuit(gates + [C.Gate((0,), 2.0 * C.H)], max_k=4, precision="fp16x3")
        assert e.value.code == sv.SV_EINVAL
    finally:
        st.free()


def test_empty_circuit_and_identity_gates():
    """No gates: every fusion mode, with and without a graph or timing, leaves
    the state bit for bit as written and reports no passes.  Identity gates
    (dense, controlled, diagonal) keep it to rounding."""
    sv = _sv()
    n = 12
    st = sv.State(n)
    try:
        psi = C.random_state_c64(n, 4)
        st.write(0, psi)
        for kw in (dict(fusion="none"), dict(fusion="greedy", max_k=6), dict(fusion="learned", max_k=6),
                   dict(fusion="phase"), dict(fusion="block", use_graph=True), dict(fusion="greedy", timing=True)):
            s = st.apply_circuit([], stats=True, **kw)
            assert s["passes"] == 0 and s["gates_in"] == 0 and s["bytes"] == 0, (kw, s)
            assert np.array_equal(st.read(), psi), kw
        eye = [C.Gate((3,), np.eye(2)), C.Gate((0, 7), np.eye(4)), C.Gate((2, 9, 11), np.eye(8)),
               C.Gate((5,), np.eye(2), (1, 6), (1, 0)), C.Gate((4, 8), C.CP(0.0))]
        for kw in (dict(fusion="none"), dict(fusion="greedy", max_k=4, precision="fp16x3"),
                   dict(fusion="phase", max_k=2)):
            st.write(0, psi)
            st.apply_circuit(eye, **kw)
            check(st.read(), psi.astype(np.complex128))
    finally:
        st.free()


def test_validation_leaves_state_untouched():
    sv = _sv()
    st = sv.State(10)
    try:
        st.set_basis(5)
        for bad in ([C.Gate((10,), C.H)], [C.Gate((1, 1), C.CZ)], [C.Gate((0,), C.H), C.Gate((0, 1, 2, 3, 4, 5, 6), np.eye(128))]):
            with pytest.raises(sv.SvError) as e:
                st.apply_circuit(bad)
            assert e.value.code == sv.SV_EINVAL
        with pytest.raises(sv.SvError):
            sv.sv_read_amplitudes(st.h, 1000, 100)
        a = st.read()
        assert a[5] == 1 and np.count_nonzero(a) == 1
    finally:
        st.free()


def test_apply_gate_entry_point():
    n = 11
    rng = np.random.Generator(np.random.PCG64(4))
    gates = random_state_circuit(n, 2) + [C.Gate((7, 2, 0), C.haar_unitary(3, rng)), C.Gate((10,), C.H)]
    sv = _sv()
    st = sv.State(n)
    try:
        for g in gates:
            st.apply_gate(g.qubits, g.matrix)
        check(st.read(), oracle.apply_circuit(n, gates))
    finally:
        st.free()


def test_many_small_gates_wrap_the_arena():
    """More single-gate uploads than the staging ring holds."""
    n = 10
    gates = C.random_circuit(n, 900, max_k=6, min_k=6, seed=5)
    sv = _sv()
    st = sv.State(n)
    try:
        for g in gates:
            st.apply_gate(g.qubits, g.matrix)
        # 900 dense k = 6 passes in FP32: rounding grows like sqrt(passes) *
        # 2^-24 * sqrt(64) ~ 1.4e-5 relative, far inside the default bars
        check(st.read(), oracle.apply_circuit(n, gates))
    finally:
        st.free()


# --------------------------------------------------------------------------
# Matrix-core passes (k >= 4): FP32 MFMA and split BF16/FP16 (hi + lo)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["fp32_mfma", "bf16x3", "fp16x3"])
@pytest.mark.parametrize("k", [4, 5, 6])
@pytest.mark.parametrize("tname", list(TARGET_SETS))
def test_mfma_single_gate(prec, k, tname):
    n = 14
    qs = TARGET_SETS[tname](n, k)
    rng = np.random.Generator(np.random.PCG64(k * 1000 + len(tname) + len(prec)))
    gates = random_state_circuit(n, k) + [C.Gate(qs, C.haar_unitary(k, rng))]
    say("mfma single gate", prec, k, tname, qs)
    got = run_gpu(n, gates, fusion="none", precision=prec, variant="mfma")
    check(got, oracle.apply_circuit(n, gates))


SHFL_TARGETS = ([(t,) for t in range(1, 7)] + [(0, t) for t in range(1, 7)] + [(t, 0) for t in (3, 6)]
                + [(a, b) for a in range(1, 7) for b in range(a + 1, 7)] + [(6, 2), (5, 1)]
                + [(0, 1, 2), (0, 2, 5), (3, 0, 4), (1, 2, 3), (1, 3, 5), (5, 2, 4), (2, 4, 6), (0, 1, 6)])


@pytest.mark.parametrize("n", [9, 12])
@pytest.mark.parametrize("qs", SHFL_TARGETS)
def test_shuffle_kernel_all_lane_targets(n, qs):
    """Targets in bits 0..6 (k <= 3): partners by cross-lane permutes; the
    smallest state it runs on is 9 qubits; ineligible sets fall back to the
    register kernel."""
    sv = _sv()
    rng = np.random.Generator(np.random.PCG64(n * 100 + sum(qs) * 7 + qs[0]))
    gates = [C.Gate((q,), C.haar_unitary(1, rng)) for q in range(n)] + [C.Gate(qs, C.haar_unitary(len(qs), rng))]
    st = sv.State(n)
    try:
        st.apply_circuit(gates[:n], fusion="none")
        s = st.apply_circuit(gates[n:], fusion="none", variant="shfl", timing=True)
        assert s["variant_passes"][1] == 1  # the shuffle form, or the register form it falls back to
        check(st.read(), oracle.apply_circuit(n, gates))
    finally:
        st.free()


@pytest.mark.parametrize("qs", [(1,), (6,), (0, 4), (2, 5), (1, 5), (0, 2, 3), (1, 4, 5)])
def test_shuffle_kernel_streaming(qs):
    n = 26  # non-temporal loads and stores
    rng = np.random.Generator(np.random.PCG64(sum(qs) + 5))
    gates = [C.Gate((q,), C.haar_unitary(1, rng)) for q in range(n)] + [C.Gate(qs, C.haar_unitary(len(qs), rng))]
    check(run_gpu(n, gates, fusion="none", variant="shfl"), oracle.apply_circuit(n, gates))


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3", "fp32_mfma"])
@pytest.mark.parametrize("qs", [(2, 9, 14, 19, 23, 25), (0, 3, 9, 14, 20, 25), (1, 2, 9, 14, 20, 25),
                                (0, 1, 7, 12, 18, 24), (25, 3, 5, 8, 13, 17), (4, 2, 16, 0, 11)])
def test_mfma_low_target_streaming(prec, qs):
    """26 qubits (non-temporal streaming on): a target in bits 1..3 is moved to
    the lane-half bit of the split-precision layout; two such targets keep
    cached loads; bit 0 targets use the other layout."""
    n = 26
    rng = np.random.Generator(np.random.PCG64(sum(qs)))
    gates = [C.Gate((q,), C.haar_unitary(1, rng)) for q in range(n)] + [C.Gate(qs, C.haar_unitary(len(qs), rng))]
    say("mfma low target", prec, qs)
    got = run_gpu(n, gates, fusion="none", precision=prec, variant="mfma")
    check(got, oracle.apply_circuit(n, gates))


@pytest.mark.parametrize("prec", ["fp32_mfma", "bf16x3", "fp16x3"])
@pytest.mark.parametrize("max_k", [4, 5, 6])
def test_grid_fused_mfma(prec, max_k):
    n = 20
    gates = C.grid_circuit(4, 5, 14, seed=2)
    ref = oracle.apply_circuit(n, gates)
    say("grid fused mfma", prec, max_k)
    r = check(run_gpu(n, gates, max_k=max_k, fusion="greedy", precision=prec), ref)
    say(r)


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3"])
def test_qft_like_split_precision_closed_form(prec):
    """Config-3 analogue: QFT-like circuit from a seeded basis state, fused to
    k = 5, split-precision matrix cores; checked against the closed form."""
    n = 24
    x = C.qft_input_basis(n, 11)
    sv = _sv()
    st = sv.State(n)
    try:
        st.set_basis(x)
        st.apply_circuit(C.qft_like_circuit(n), max_k=5, precision=prec)
        r = check(st.read(), oracle.qft_like_amplitudes(n, x, np.arange(1 << n)))
        say(prec, r)
        assert abs(st.norm() - 1) < 1e-5
    finally:
        st.free()


def test_mfma_small_state_falls_back():
    """States too small for a 32-group tile run the VALU kernel instead."""
    n = 9
    rng = np.random.Generator(np.random.PCG64(8))
    gates = random_state_circuit(n, 1) + [C.Gate((0, 2, 4, 6, 8), C.haar_unitary(5, rng))]
    check(run_gpu(n, gates, fusion="none", precision="bf16x3", variant="mfma"), oracle.apply_circuit(n, gates))
