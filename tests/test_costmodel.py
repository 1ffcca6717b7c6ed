"""Learned fusion: model file handling (CPU), corpus + GPU training, what the
trained network gains over the same search without it and over greedy
max-k on held-out circuits, and parity of the partitions it picks (GPU)."""
import os
import struct

import numpy as np
import pytest

import circuits as C
import oracle
from partition_check import check_partition
from paper_2602_09604_amd import sv

needs_lib = pytest.mark.skipif(not os.path.exists(sv.LIB_PATH), reason="libsv.so not built")


@needs_lib
@pytest.mark.parametrize("blob", [
    b"",
    b"XXXX" + struct.pack("<4I", 1, 64, 40, 6849),
    struct.pack("<5I", 0x4D435653, 2, 64, 40, 6849),           # bad version
    struct.pack("<5I", 0x4D435653, 1, 32, 40, 6849),           # bad width
    struct.pack("<5I", 0x4D435653, 1, 64, 40, 6849) + b"\0" * 100,  # truncated
    struct.pack("<5I", 0x4D435653, 1, 64, 40, 6849) + struct.pack("<f", float("nan")) * 6849,
])
def test_cost_model_file_rejects_malformed(tmp_path, blob):
    p = tmp_path / "m.bin"
    p.write_bytes(blob)
    with pytest.raises(sv.SvError) as e:
        sv.sv_cost_model_load(str(p))
    assert e.value.code == sv.SV_EINVAL


@needs_lib
def test_cost_model_file_roundtrip_and_predict(tmp_path):
    """A hand-made parameter file: all weights zero except b3 = 1.5, so every
    prediction is 1.5; reload and predict through the ABI."""
    p = np.zeros(6849, dtype=np.float32)
    p[-1] = 1.5
    path = tmp_path / "m.bin"
    path.write_bytes(struct.pack("<5I", 0x4D435653, 1, 64, 40, 6849) + p.tobytes())
    sv.sv_cost_model_load(str(path))
    assert sv.sv_cost_model_predict(3, [0, 5, 9], 30, 0) == pytest.approx(1.5)
    out = tmp_path / "m2.bin"
    sv.sv_cost_model_save(str(out))
    assert out.read_bytes() == path.read_bytes()


@needs_lib
def test_learned_fusion_with_constant_model_is_valid(tmp_path):
    """With any installed model the learned partition is still a valid fusion:
    equal state through the oracle, coverage, per-qubit order."""
    p = np.zeros(6849, dtype=np.float32)
    p[-1] = -5.0
    path = tmp_path / "m.bin"
    path.write_bytes(struct.pack("<5I", 0x4D435653, 1, 64, 40, 6849) + p.tobytes())
    sv.sv_cost_model_load(str(path))
    n = 10
    gates = C.grid_circuit(2, 5, 10, seed=3)
    fused, block_of = sv.sv_fuse(gates, n, sv.make_opts(max_k=5, fusion="learned"))
    check_partition(gates, fused, block_of, 5)
    ref = oracle.apply_circuit(n, gates)
    assert np.max(np.abs(oracle.apply_circuit(n, fused) - ref)) < 1e-12


def test_high_target_augmentation():
    """Copies keep the label, k, the precision and n features and every
    target below bit 13; high targets move to distinct bits in [13, 34)."""
    from paper_2602_09604_amd import costmodel
    rng = np.random.Generator(np.random.PCG64(3))
    X = np.zeros((50, 40), dtype=np.float32)
    y = rng.standard_normal(50).astype(np.float32)
    for i in range(50):
        k = int(rng.integers(1, 7))
        X[i, 0], X[i, 1] = k / 6.0, 30 / 34.0
        X[i, 2 + rng.permutation(30)[:k]] = 1.0
        X[i, 36 + int(rng.integers(4))] = 1.0
    Xa, ya = costmodel.augment_high_targets(X, y, 3, np.random.Generator(np.random.PCG64(4)))
    assert Xa.shape == (200, 40) and np.array_equal(Xa[:50], X)
    moved = 0
    for c in range(1, 4):
        Xc, yc = Xa[50 * c:50 * (c + 1)], ya[50 * c:50 * (c + 1)]
        assert np.array_equal(yc, y)
        assert np.array_equal(Xc[:, :2], X[:, :2]) and np.array_equal(Xc[:, 36:], X[:, 36:])
        assert np.array_equal(Xc[:, 2:15], X[:, 2:15])  # bits 0..12 untouched
        assert np.array_equal(Xc[:, 2:36].sum(1), X[:, 2:36].sum(1))  # same number of targets
        assert set(np.unique(Xc)) <= {0.0, 1.0} | set(np.unique(X[:, :2]))
        moved += int(np.sum(Xc[:, 2 + 30:36]))  # bits 30..33 were never set in X
    assert moved > 0


@pytest.fixture(autouse=True)
def _no_model_after_test():
    """Tests here install models; none may leak into later tests."""
    yield
    if os.path.exists(sv.LIB_PATH):
        sv.sv_cost_model_clear()


@needs_lib
def test_cost_model_clear_restores_fewest_passes(tmp_path):
    """After sv_cost_model_clear the learned search keeps the fewest-pass
    candidate, whatever the model installed before preferred."""
    n = 12
    gates = C.grid_circuit(3, 4, 12, seed=4)
    fused0, _ = sv.sv_fuse(gates, n, sv.make_opts(max_k=5, fusion="learned"))
    p = np.zeros(6849, dtype=np.float32)
    p[-1] = 2.0
    path = tmp_path / "m.bin"
    path.write_bytes(struct.pack("<5I", 0x4D435653, 1, 64, 40, 6849) + p.tobytes())
    sv.sv_cost_model_load(str(path))
    sv.sv_cost_model_clear()
    with pytest.raises(sv.SvError):
        sv.sv_cost_model_predict(3, [0, 1, 2], n, 0)
    fused1, _ = sv.sv_fuse(gates, n, sv.make_opts(max_k=5, fusion="learned"))
    assert len(fused1) == len(fused0)
    assert [f.qubits for f in fused1] == [f.qubits for f in fused0]


def _best_time(st, gates, reps=3, **kw):
    """Best of reps of the summed pass durations (events around every pass):
    the partitions' device cost, without the idle gaps a small state leaves
    while the host encodes the next chunk of passes."""
    best, passes = 1e9, None
    for _ in range(reps):
        st.set_basis(0)
        s = st.apply_circuit(gates, stats=True, timing=True, **kw)
        best, passes = min(best, sum(s["variant_s"][1:])), s["passes"]
    return best, passes


@pytest.mark.gpu
def test_network_value_on_held_out_28_qubit_circuits(tmp_path):
    """What the trained network adds (Sec. IV-D: the best fused size depends
    on circuit and machine; Sec. VII-B).  A model trained on passes the
    simulator timed at 26 and 28 qubits runs the learned search on held-out
    28-qubit grid circuits, against the same search with no model (which
    keeps the fewest passes) and against greedy fusion at every max k.

    FP32 on the VALU kernels: a k = 6 pass is compute-bound (31.9 flop/B
    against a ridge of ~19.7), so fewer, larger passes are not the fastest;
    the network must beat both the no-model search and the best greedy K.
    Split FP16 on the matrix cores: every pass moves the same bytes at about
    the same speed, so there is nothing for the network to win: a tie with
    the no-model search (within 5 %, either way; the network may keep a
    partition with a few more passes that it prices the same)."""
    from paper_2602_09604_amd import costmodel
    st = sv.State(24)
    try:
        sv.sv_autotune(st.h, 0)
    finally:
        st.free()
    corpus = costmodel.collect_corpus(samples=1200, ns=(26, 28), seed=5, log=print)
    info = costmodel.train_cost_model(corpus, epochs=2000, lr=3e-3, seed=2, save_path=str(tmp_path / "m.bin"))
    print(info, flush=True)
    # a sanity bar on the ranking only (0.60-0.61 measured on two boxes with
    # this corpus size); the timed outcomes below are the test
    assert info["test_spearman"] > 0.5, info
    n = 28
    st = sv.State(n)
    try:
        for rows, cols, depth, seed in ((4, 7, 20, 78), (2, 14, 24, 79)):
            gates = C.grid_circuit(rows, cols, depth, seed=seed)
            for prec in ("fp32_valu", "fp16x3"):
                sv.sv_cost_model_load(str(tmp_path / "m.bin"))
                t_model, p_model = _best_time(st, gates, fusion="learned", max_k=6, precision=prec)
                assert abs(st.norm() - 1.0) <= 1e-5
                sv.sv_cost_model_clear()
                t_none, p_none = _best_time(st, gates, fusion="learned", max_k=6, precision=prec)
                greedy = {K: _best_time(st, gates, reps=2, fusion="greedy", max_k=K, precision=prec)
                          for K in (2, 3, 4, 5, 6)}
                t_greedy = min(v[0] for v in greedy.values())
                print("%dx%d %s: model %.4f s (%d passes), no model %.4f s (%d), best greedy %.4f s %s"
                      % (rows, cols, prec, t_model, p_model, t_none, p_none, t_greedy,
                         {K: (round(v[0], 4), v[1]) for K, v in greedy.items()}), flush=True)
                if prec == "fp32_valu":
                    assert t_model < t_none, (t_model, t_none)
                    assert t_model < t_greedy, (t_model, t_greedy)
                else:
                    assert t_model <= 1.05 * t_none and t_none <= 1.05 * t_model, (t_model, t_none)
                    assert t_model < t_greedy
    finally:
        st.free()


@pytest.mark.gpu
def test_learned_partition_parity_with_trained_model():
    """Partitions the trained network picks are checked amplitude by
    amplitude against the oracle (22 and 24 qubits, split and FP32)."""
    from paper_2602_09604_amd import costmodel
    corpus = costmodel.collect_corpus(samples=600, ns=(22, 24), seed=6)
    costmodel.train_cost_model(corpus, epochs=1000, lr=3e-3, seed=3)
    for n, rows, cols, depth, seed, prec in ((22, 2, 11, 16, 77, "bf16x3"), (24, 3, 8, 16, 78, "fp32_valu"),
                                             (24, 3, 8, 16, 78, "fp16x3")):
        gates = C.grid_circuit(rows, cols, depth, seed=seed)
        ref = oracle.apply_circuit(n, gates)
        st = sv.State(n)
        try:
            s = st.apply_circuit(gates, fusion="learned", max_k=6, precision=prec, stats=True)
            r = oracle.compare(st.read(), ref)
            print(n, prec, s["passes"], r, flush=True)
            assert r["max_abs"] <= 1e-5 and r["infidelity"] <= 1e-6, (n, prec, r)
        finally:
            st.free()
