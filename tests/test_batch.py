"""Batched kernels (LDS-resident small circuits + level-synchronous large
ones, one captured graph) against the oracle, circuit by circuit."""
import json
import os
import sys

import numpy as np
import pytest

import circuits as C
import oracle
from paper_2602_09604_amd import sv

pytestmark = pytest.mark.gpu


def set_lds_limit(tmp_path, n):
    p = tmp_path / "t.json"
    p.write_text(json.dumps({"format": "libsv-tune-1", "batch_lds_max_n": n, "entries": []}))
    sv.sv_tune_load(str(p))


def level_passes(ns, circs, max_k=4, fusion="greedy"):
    return [len(sv.sv_fuse(c, n, sv.make_opts(max_k=max_k, fusion=fusion))[0]) for n, c in zip(ns, circs)]


def run_batch(ns, circs, max_k=4, fusion="greedy"):
    import torch
    stream = torch.cuda.current_stream()
    states = [sv.State(n, stream=stream) for n in ns]
    try:
        stats = sv.sv_batch_run([s.h for s in states], circs, sv.make_opts(max_k=max_k, fusion=fusion))
        out = [s.read() for s in states]
    finally:
        for s in states:
            s.free()
    return out, stats


@pytest.mark.parametrize("lds_limit", [14, 13, 11, 1])
def test_batched_ansatz_small(tmp_path, lds_limit):
    """24 circuits, n in [10, 16]: with limit 13 or 14 (128 KiB of LDS per
    workgroup, where the device allows it) the small ones stay in LDS and the
    rest go level by level; with limit 1 everything goes level by level."""
    set_lds_limit(tmp_path, lds_limit)
    ns, circs = C.batched_ansatz(24, seed=3, n_min=10, n_max=16)
    out, stats = run_batch(ns, circs)
    print("limit", lds_limit, "passes", stats["passes"], "launches", stats["launches"], "gpu_s", stats["gpu_s"],
          flush=True)
    assert stats["gates_in"] == sum(len(c) for c in circs)
    floor = sum(16 << n for n in ns)  # every state read and written once
    assert stats["bytes"] >= floor
    if lds_limit == 1:
        assert stats["bytes"] == sum((16 << n) * p for n, p in zip(ns, level_passes(ns, circs)))
    for n, c, got in zip(ns, circs, out):
        r = oracle.compare(got, oracle.apply_circuit(n, c))
        assert r["max_abs"] <= 1e-5 and r["infidelity"] <= 1e-6, (n, r)


def test_batched_ansatz_full_range(tmp_path):
    """A slice of the 512-circuit workload (n up to 22), fused to k = 4 .. 6,
    first-come greedy and largest-block partitions."""
    set_lds_limit(tmp_path, 12)
    ns, circs = C.batched_ansatz(512, seed=0)
    pick = [i for i in range(512) if ns[i] in (10, 13, 17, 22)][:8]
    sub_ns = [ns[i] for i in pick]
    sub = [circs[i] for i in pick]
    refs = [oracle.apply_circuit(n, c) for n, c in zip(sub_ns, sub)]
    for K, fusion in ((4, "greedy"), (6, "greedy"), (4, "block"), (5, "block")):
        out, stats = run_batch(sub_ns, sub, max_k=K, fusion=fusion)
        for n, got, ref in zip(sub_ns, out, refs):
            r = oracle.compare(got, ref)
            assert r["max_abs"] <= 1e-5 and r["infidelity"] <= 1e-6, (K, fusion, n, r)


def test_batch_matches_sequential_runs(tmp_path):
    """Same answer as sv_apply_circuit per circuit (the unbatched path)."""
    set_lds_limit(tmp_path, 12)
    ns, circs = C.batched_ansatz(6, seed=9, n_min=11, n_max=15)
    out, _ = run_batch(ns, circs)
    for n, c, got in zip(ns, circs, out):
        st = sv.State(n)
        try:
            st.apply_circuit(c, max_k=4)
            ref = st.read()
        finally:
            st.free()
        assert np.max(np.abs(got - ref)) < 1e-5


def test_batch_validation():
    st = sv.State(10)
    try:
        with pytest.raises(sv.SvError) as e:
            sv.sv_batch_run([st.h], [[C.Gate((10,), C.H)]])
        assert e.value.code == sv.SV_EINVAL
        assert sv.sv_batch_run([], [])["passes"] == 0
    finally:
        st.free()


GOLD512 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch512_projections.npz")


@pytest.mark.parametrize("max_k,fusion", [(4, "block"), (4, "greedy")])
def test_batch512_every_circuit_against_oracle_projections(max_k, fusion):
    """All 512 circuits of the batched workload in one sv_batch_run, each
    checked through 4 inner products with seeded probe vectors against the
    oracle's full states (tests/golden/make_batch512_projections.py).  A
    deviation d moves a projection by <phi|d> with mean square |d|^2, so
    |delta p| <= 1e-4 on 4 probes bounds |d| to about 1e-3 (infidelity
    about 1e-6) except with negligible probability; norms within 1e-5."""
    import torch
    with np.load(GOLD512, allow_pickle=False) as f:
        gold_ns, proj, norms = f["ns"], f["proj"], f["norm_sq"]
    ns, circs = C.batched_ansatz(512, seed=0)
    assert list(gold_ns) == ns
    stream = torch.cuda.current_stream()
    states = [sv.State(n, stream=stream) for n in ns]
    try:
        stats = sv.sv_batch_run([s.h for s in states], circs, sv.make_opts(max_k=max_k, fusion=fusion))
        print(fusion, max_k, "passes", stats["passes"], "launches", stats["launches"], "gpu_s", stats["gpu_s"],
              "bytes / floor", stats["bytes"] / sum(16 << n for n in ns), flush=True)
        worst = 0.0
        for c, (n, st) in enumerate(zip(ns, states)):
            psi = st.read()
            p = oracle.probe_projections(psi, C.probe_phases(n, 1000 + c, proj.shape[1]))
            d = float(np.max(np.abs(p - proj[c])))
            worst = max(worst, d)
            assert d <= 1e-4, (c, n, d)
            g2 = float(np.sum(np.abs(psi.astype(np.complex128)) ** 2))
            assert abs(g2 - norms[c]) <= 1e-5, (c, n, g2)
        print("worst projection difference", worst, flush=True)
    finally:
        for s in states:
            s.free()


def test_batch_lane_exchange_every_low_target_set():
    """Circuits of 18 and 19 qubits (at and above the size from which the
    batched level passes exchange across lanes), one per target set: every
    set of low targets on amplitude bits 1..3 with k = 1..4 and, with bit 0
    as a further target, k = 2..4; each circuit starts with a layer of random
    one-qubit gates so that the state is dense, then the gate on the set.
    Every circuit against the oracle."""
    rng = np.random.Generator(np.random.PCG64(2024))
    ns, circs = [], []
    for q0 in (False, True):
        for tm in range(1, 8):
            lows = [t + 1 for t in range(3) if (tm >> t) & 1]
            for k in range(1, 5):
                if len(lows) + q0 > k:
                    continue
                n = 18 + (len(circs) % 2)
                rest = [q for q in range(4, n) if q not in lows]
                qs = lows + ([0] if q0 else []) + [int(q) for q in rng.choice(rest, k - len(lows) - q0, replace=False)]
                rng.shuffle(qs)
                layer = [C.Gate((q,), C.haar_unitary(1, rng)) for q in range(n)]
                ns.append(n)
                circs.append(layer + [C.Gate(tuple(qs), C.haar_unitary(k, rng))])
    out, stats = run_batch(ns, circs, max_k=4, fusion="none")
    print("circuits", len(ns), "passes", stats["passes"], "launches", stats["launches"], flush=True)
    for n, c, got in zip(ns, circs, out):
        r = oracle.compare(got, oracle.apply_circuit(n, c))
        assert r["max_abs"] <= 1e-5 and r["infidelity"] <= 1e-6, ([g.qubits for g in c[-1:]], r)
