"""Host-side checks of libsv.so that need no GPU: exported symbols, the FP64
fusion pass (checked through the oracle), validation and error codes."""
import ctypes
import os
import re

import numpy as np
import pytest

import circuits as C
import oracle
from partition_check import check_partition, sweeps
from paper_2602_09604_amd import sv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

needs_lib = pytest.mark.skipif(not os.path.exists(sv.LIB_PATH), reason="libsv.so not built")


def header_functions():
    text = open(os.path.join(ROOT, "include", "sv.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sv_[a-z0-9_]+)\s*\(", text)))


@needs_lib
def test_library_exports_every_declared_symbol():
    names = header_functions()
    assert len(names) >= 30
    L = ctypes.CDLL(sv.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(sv.exported_symbols())


@needs_lib
def test_version_and_last_error():
    assert b"libsv" in sv.lib().sv_version()
    assert isinstance(sv.lib().sv_last_error(), bytes)


# --------------------------------------------------------------------------
# Fusion (host FP64), checked against the unfused oracle
# --------------------------------------------------------------------------
def _check_partition(gates, fused, block_of, max_k):
    return check_partition(gates, fused, block_of, max_k)


@needs_lib
@pytest.mark.parametrize("max_k", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_greedy_fusion_equivalent(max_k, seed):
    n = 9
    gates = C.random_circuit(n, 40, max_k=min(2, max_k), seed=seed)
    fused, block_of = sv.sv_fuse(gates, n, sv.make_opts(max_k=max_k, fusion="greedy"))
    _check_partition(gates, fused, block_of, max_k)
    ref = oracle.apply_circuit(n, gates, init=seed)
    got = oracle.apply_circuit(n, fused, init=seed)
    assert np.max(np.abs(ref - got)) < 1e-12
    if max_k >= 2:
        assert len(fused) < len(gates)


@needs_lib
def test_greedy_fusion_grid_circuit():
    gates = C.grid_circuit(2, 5, 8, seed=1)
    n = 10
    ref = oracle.apply_circuit(n, gates)
    for K in (2, 4, 6):
        fused, block_of = sv.sv_fuse(gates, n, sv.make_opts(max_k=K))
        _check_partition(gates, fused, block_of, K)
        assert np.max(np.abs(oracle.apply_circuit(n, fused) - ref)) < 1e-12


@needs_lib
def test_fusion_vertical_product():
    """Two gates on the same qubit fuse into their matrix product (later gate on the left)."""
    rng = np.random.Generator(np.random.PCG64(0))
    a, b = C.haar_unitary(1, rng), C.haar_unitary(1, rng)
    fused, _ = sv.sv_fuse([C.Gate((3,), a), C.Gate((3,), b)], 5, sv.make_opts(max_k=1))
    assert len(fused) == 1
    assert np.allclose(fused[0].matrix, b @ a, atol=1e-15)


@needs_lib
def test_fusion_horizontal_tensor_product():
    """Eq. 3: gates on disjoint qubits fuse into the Kronecker product
    (ascending qubits, local bit 0 = lowest qubit = low Kronecker factor)."""
    rng = np.random.Generator(np.random.PCG64(1))
    a, b = C.haar_unitary(1, rng), C.haar_unitary(1, rng)
    fused, _ = sv.sv_fuse([C.Gate((4,), a), C.Gate((1,), b)], 6, sv.make_opts(max_k=2))
    assert len(fused) == 1 and fused[0].qubits == (1, 4)
    assert np.allclose(fused[0].matrix, np.kron(a, b), atol=1e-15)


@needs_lib
def test_fusion_none_sorts_targets():
    rng = np.random.Generator(np.random.PCG64(2))
    u = C.haar_unitary(3, rng)
    g = C.Gate((5, 0, 2), u)
    fused, block_of = sv.sv_fuse([g], 6, sv.make_opts(fusion="none"))
    assert fused[0].qubits == (0, 2, 5)
    a = oracle.apply_circuit(6, [g], init=13)
    b = oracle.apply_circuit(6, fused, init=13)
    assert np.max(np.abs(a - b)) < 1e-15


@needs_lib
def test_fusion_respects_blocking():
    """CNOT(0,1), H(1), X(0) with max_k = 1: H(1) cannot pass CNOT, so the
    single-qubit gates stay in separate blocks after it."""
    gates = [C.Gate((0, 1), C.CNOT), C.Gate((1,), C.H), C.Gate((0,), C.X)]
    fused, block_of = sv.sv_fuse(gates, 2, sv.make_opts(max_k=2))
    assert len(fused) == 1
    ref = oracle.apply_circuit(2, gates, init=1)
    assert np.max(np.abs(oracle.apply_circuit(2, fused, init=1) - ref)) < 1e-15


@needs_lib
def test_fusion_empty():
    fused, block_of = sv.sv_fuse([], 4, sv.make_opts())
    assert fused == [] and len(block_of) == 0


# --------------------------------------------------------------------------
# Validation
# --------------------------------------------------------------------------
@needs_lib
@pytest.mark.parametrize("gate,n", [
    (C.Gate((5,), C.H), 5),            # qubit out of range
    (C.Gate((-1,), C.H), 5),
    (C.Gate((1, 1), C.CZ), 5),         # repeated qubit
    (C.Gate((0, 1, 2), np.eye(8)), 2),  # k > n
])
def test_fuse_rejects_invalid_gates(gate, n):
    with pytest.raises(sv.SvError) as e:
        sv.sv_fuse([gate], n, sv.make_opts())
    assert e.value.code == sv.SV_EINVAL


@needs_lib
def test_fuse_rejects_bad_opts():
    with pytest.raises(sv.SvError):
        sv.sv_fuse([C.Gate((0,), C.H)], 2, sv.make_opts(max_k=7))
    o = sv.make_opts()
    o.timing = 2
    with pytest.raises(sv.SvError):
        sv.sv_fuse([C.Gate((0,), C.H)], 2, o)


@needs_lib
def test_fuse_rejects_k7_and_null_matrix():
    ga = sv.GateArray([C.Gate((0,), C.H)])
    ga.arr[0].k = 7
    out = ctypes.POINTER(sv.sv_gate)()
    n_out = ctypes.c_size_t()
    rc = sv.lib().sv_fuse(ga.ptr, 1, 8, None, ctypes.byref(out), ctypes.byref(n_out), None)
    assert rc == sv.SV_EINVAL
    ga = sv.GateArray([C.Gate((0,), C.H)])
    ga.arr[0].matrix = ctypes.cast(None, ctypes.POINTER(ctypes.c_double))
    rc = sv.lib().sv_fuse(ga.ptr, 1, 8, None, ctypes.byref(out), ctypes.byref(n_out), None)
    assert rc == sv.SV_EINVAL
    assert b"NULL" in sv.lib().sv_last_error()


@needs_lib
def test_null_handle_calls_fail_cleanly():
    L = sv.lib()
    assert L.sv_set_basis(None, 0) == sv.SV_EINVAL
    assert L.sv_norm(None, None) == sv.SV_EINVAL
    assert L.sv_free(None) == sv.SV_OK
    h = ctypes.c_void_p()
    assert L.sv_alloc(0, 0, ctypes.c_void_p(16), 1 << 20, None, ctypes.byref(h)) == sv.SV_EINVAL
    assert L.sv_alloc(41, 0, ctypes.c_void_p(16), 1 << 20, None, ctypes.byref(h)) == sv.SV_EINVAL
    assert L.sv_alloc(10, 1, ctypes.c_void_p(16), 1 << 20, None, ctypes.byref(h)) == sv.SV_EINVAL
    # buffer too small is rejected before any device call
    assert L.sv_alloc(20, 0, ctypes.c_void_p(16), 1 << 20, None, ctypes.byref(h)) == sv.SV_ENOMEM


@needs_lib
def test_cost_features_layout():
    f = sv.sv_cost_features(3, [0, 5, 33], 34, sv.SV_PREC_BF16X3)
    assert f.shape == (40,)
    assert abs(f[0] - 0.5) < 1e-7 and abs(f[1] - 1.0) < 1e-7
    assert f[2 + 0] == 1 and f[2 + 5] == 1 and f[2 + 33] == 1 and f[2:36].sum() == 3
    assert f[36:40].tolist() == [0, 0, 1, 0]


@needs_lib
@pytest.mark.parametrize("max_k", [2, 3, 4, 6])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_block_fusion_equivalent(max_k, seed):
    n = 9
    gates = C.random_circuit(n, 60, max_k=min(2, max_k), seed=seed)
    fused, block_of = sv.sv_fuse(gates, n, sv.make_opts(max_k=max_k, fusion="block"))
    _check_partition(gates, fused, block_of, max_k)
    ref = oracle.apply_circuit(n, gates, init=seed)
    assert np.max(np.abs(oracle.apply_circuit(n, fused, init=seed) - ref)) < 1e-12


@needs_lib
@pytest.mark.parametrize("rows,cols,depth", [(2, 5, 8), (3, 4, 12), (2, 17, 24)])
def test_block_fusion_fewer_passes_on_lattices(rows, cols, depth):
    """The largest-block partition needs fewer passes than first-come greedy
    on grid circuits (the 2x17 depth-24 grid: 53 against 79)."""
    n = rows * cols
    gates = C.grid_circuit(rows, cols, depth, seed=0)
    greedy, _ = sv.sv_fuse(gates, n, sv.make_opts(max_k=6, fusion="greedy"))
    fused, block_of = sv.sv_fuse(gates, n, sv.make_opts(max_k=6, fusion="block"))
    _check_partition(gates, fused, block_of, 6)
    assert len(fused) < len(greedy)
    if n <= 12:
        ref = oracle.apply_circuit(n, gates)
        assert np.max(np.abs(oracle.apply_circuit(n, fused) - ref)) < 1e-12
    if (rows, cols, depth) == (2, 17, 24):
        assert len(fused) <= 56, len(fused)


@needs_lib
def test_learned_without_model_keeps_fewest_passes():
    from paper_2602_09604_amd import costmodel  # noqa: F401  (no model is installed in the CPU suite)
    gates = C.grid_circuit(3, 4, 12, seed=2)
    n = 12
    counts = {f: sweeps(sv.sv_fuse(gates, n, sv.make_opts(max_k=5, fusion=f))[1]) for f in ("greedy", "block", "learned")}
    assert counts["learned"] <= min(counts["greedy"], counts["block"]), counts
    fused, _ = sv.sv_fuse(gates, n, sv.make_opts(max_k=5, fusion="learned"))
    ref = oracle.apply_circuit(n, gates)
    assert np.max(np.abs(oracle.apply_circuit(n, fused) - ref)) < 1e-12


@needs_lib
@pytest.mark.parametrize("case", ["random8_k5", "random12_k3", "grid4x3_k6"])
def test_beam_search_finds_fewer_passes(case):
    """Learned fusion without a model includes beam searches over
    largest-block passes; on these circuits it needs fewer passes than the
    largest-block rule, and its partition reaches the unfused state."""
    from paper_2602_09604_amd import costmodel  # noqa: F401  (no model is installed in the CPU suite)
    n, max_k, gates = {
        "random8_k5": (8, 5, lambda: C.random_circuit(8, 150, max_k=2, seed=5)),
        "random12_k3": (12, 3, lambda: C.random_circuit(12, 150, max_k=2, seed=4)),
        "grid4x3_k6": (12, 6, lambda: C.grid_circuit(4, 3, 30, seed=0)),
    }[case]
    gates = gates()
    block, _ = sv.sv_fuse(gates, n, sv.make_opts(max_k=max_k, fusion="block"))
    fused, block_of = sv.sv_fuse(gates, n, sv.make_opts(max_k=max_k, fusion="learned"))
    _check_partition(gates, fused, block_of, max_k)
    assert sweeps(block_of) < len(block), (sweeps(block_of), len(block))
    ref = oracle.apply_circuit(n, gates, init=3)
    assert np.max(np.abs(oracle.apply_circuit(n, fused, init=3) - ref)) < 1e-12


@needs_lib
def test_learned_fusion_on_34_qubit_grid():
    """The 2x17 depth-24 grid: 53 largest-block passes; the beam search alone
    reaches 49 and blocks with controls (CZs to outside qubits taken as
    control bits) at most 31 sweeps, with a valid partition."""
    gates = C.grid_circuit(2, 17, 24, seed=0)
    fused, block_of = sv.sv_fuse(gates, 34, sv.make_opts(max_k=6, fusion="learned", precision="fp16x3"))
    assert check_partition(gates, fused, block_of, 6) <= 31
    ctrl = [f for f in fused if f.controls]
    assert ctrl and all(min(f.controls) >= 4 and len(f.controls) <= 3 for f in ctrl)


@needs_lib
@pytest.mark.parametrize("rows,cols,depth,max_k,seed", [(3, 4, 12, 4, 0), (2, 6, 16, 5, 1), (3, 4, 20, 6, 2),
                                                         (4, 3, 14, 3, 3), (2, 5, 30, 6, 4)])
def test_blocks_with_controls_equivalent(rows, cols, depth, max_k, seed):
    """Blocks that take diagonal gates reaching outside qubits as controls
    (one fused gate per control value) reach the unfused state through the
    oracle; the grids are chosen so that such blocks occur.  The fusion is
    planned for a 30-qubit state (blocks take controls from 28 qubits up) and
    checked on the circuit's own qubits."""
    n = rows * cols
    gates = C.grid_circuit(rows, cols, depth, seed=seed)
    fused, block_of = sv.sv_fuse(gates, 30, sv.make_opts(max_k=max_k, fusion="learned", precision="fp16x3"))
    check_partition(gates, fused, block_of, max_k)
    assert any(f.controls for f in fused)
    block, _ = sv.sv_fuse(gates, 30, sv.make_opts(max_k=max_k, fusion="block"))
    assert sweeps(block_of) <= len(block)
    small, _ = sv.sv_fuse(gates, n, sv.make_opts(max_k=max_k, fusion="learned", precision="fp16x3"))
    assert not any(f.controls for f in small)  # below 28 qubits no block takes controls
    valu, _ = sv.sv_fuse(gates, 30, sv.make_opts(max_k=max_k, fusion="learned", precision="fp32_valu"))
    assert not any(f.controls for f in valu)  # nor where the matrix cores do not run the blocks
    ref = oracle.apply_circuit(n, gates, init=seed + 5)
    assert np.max(np.abs(oracle.apply_circuit(n, fused, init=seed + 5) - ref)) < 1e-12


@needs_lib
def test_block_split_rules():
    """Dense gates on (0, 1) interleaved with CZ(1, 9), CZ(0, 8) and CZ(0, 3),
    max_k = 3: qubits 8 and 9 (at or above bit 4) become controls of one
    block on (0, 1, 3); qubit 3 (below bit 4) stays a target.  Then single-qubit gates on 8
    and 9 form the second block."""
    rng = np.random.Generator(np.random.PCG64(11))
    u = lambda k: C.haar_unitary(k, rng)  # noqa: E731
    gates = [C.Gate((0, 1), u(2)), C.Gate((1, 9), C.CZ), C.Gate((0, 1), u(2)), C.Gate((0, 8), C.CZ),
             C.Gate((0, 3), C.CZ), C.Gate((0, 1), u(2)), C.Gate((9,), u(1)), C.Gate((8,), u(1))]
    fused, block_of = sv.sv_fuse(gates, 30, sv.make_opts(max_k=3, fusion="learned", precision="bf16x3"))
    assert check_partition(gates, fused, block_of, 3) == 2
    first = fused[0]
    assert first.controls == (8, 9) and first.qubits == (0, 1, 3)
    assert sorted(tuple(f.control_values) for f in fused[:4]) == [(0, 0), (0, 1), (1, 0), (1, 1)]
    assert list(block_of[:6]) == [0] * 6 and block_of[6] == block_of[7] == 4
    ref = oracle.apply_circuit(10, gates, init=77)
    assert np.max(np.abs(oracle.apply_circuit(10, fused, init=77) - ref)) < 1e-12


@needs_lib
def test_struct_layouts_match_binding():
    """The ctypes mirrors of the ABI structs have the library's sizes."""
    from paper_2602_09604_amd import sv
    import ctypes
    assert sv.sv_struct_size(0) == ctypes.sizeof(sv.sv_gate)
    assert sv.sv_struct_size(1) == ctypes.sizeof(sv.sv_run_opts)
    assert sv.sv_struct_size(2) == ctypes.sizeof(sv.sv_run_stats)
    assert sv.sv_struct_size(3) == 0 and sv.sv_struct_size(-1) == 0
