"""Learned fusion: model file handling (CPU), corpus + GPU training + learned
partition parity and wall time against greedy max-k (GPU)."""
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


@pytest.mark.gpu
def test_corpus_training_and_learned_partition():
    import torch
    from paper_2602_09604_amd import costmodel
    st = sv.State(20)
    try:
        sv.sv_autotune(st.h, 0)
    finally:
        st.free()
    corpus = costmodel.collect_corpus(samples=900, ns=(22, 24), seed=5, log=print)
    info = costmodel.train_cost_model(corpus, epochs=1500, lr=3e-3, seed=2)
    print(info, flush=True)
    assert info["test_spearman"] > 0.6, info
    # learned partition on a held-out circuit: parity and wall time
    n = 22
    gates = C.grid_circuit(2, 11, 16, seed=77)
    ref = oracle.apply_circuit(n, gates)
    times = {}
    for name, kw in {"learned": dict(fusion="learned", max_k=6),
                     "greedy4": dict(fusion="greedy", max_k=4),
                     "greedy6": dict(fusion="greedy", max_k=6)}.items():
        st = sv.State(n)
        try:
            best = 1e9
            for _ in range(3):
                st.set_basis(0)
                s = st.apply_circuit(gates, precision="bf16x3", stats=True, **kw)
                best = min(best, s["gpu_s"])
            r = oracle.compare(st.read(), ref)
            assert r["max_abs"] <= 1e-5 and r["infidelity"] <= 1e-6, (name, r)
            times[name] = best
        finally:
            st.free()
    print(times, flush=True)
    assert times["learned"] <= 1.25 * min(times["greedy4"], times["greedy6"]), times
    # What the network adds over the fewest-passes rule: in FP32 on the VALU
    # kernels a k = 6 pass is compute-bound, so the fewest passes (the
    # largest-block partition at k = 6) is not the fastest; the network
    # prices that and picks smaller blocks.
    n = 24
    gates = C.grid_circuit(3, 8, 16, seed=78)
    ref = oracle.apply_circuit(n, gates)
    times = {}
    passes = {}
    for name, kw in {"learned": dict(fusion="learned", max_k=6), "block6": dict(fusion="block", max_k=6)}.items():
        st = sv.State(n)
        try:
            best = 1e9
            for _ in range(3):
                st.set_basis(0)
                s = st.apply_circuit(gates, precision="fp32_valu", stats=True, **kw)
                best = min(best, s["gpu_s"])
            r = oracle.compare(st.read(), ref)
            assert r["max_abs"] <= 1e-5 and r["infidelity"] <= 1e-6, (name, r)
            times[name] = best
            passes[name] = s["passes"]
        finally:
            st.free()
    print("fp32_valu", times, passes, flush=True)
    assert times["learned"] < 0.9 * times["block6"], (times, passes)
