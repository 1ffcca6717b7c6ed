"""Benchmark: a 34-qubit random grid circuit (2x17 lattice, depth 24, 1110
gates) simulated on one MI355X through libsv.

Before the timed region: the autotuner times the kernel variants on a
scratch state; the simulator times its own passes (the cost-model corpus) and
trains the fusion cost model on the GPU.

One step = |0..0> initialisation, fusion + every gate pass of the circuit
(sv_apply_circuit), the FP64 norm reduction and a 2^20-amplitude read-back.
The timed region holds exactly --steps steps between device synchronisations.

Printed (one JSON line on stdout): gates/s of the configured path (default:
learned fusion, split-FP16 matrix cores), the roofline of the dominant pass
kernel (HIP events around every pass), the CPU oracle timed on a bounded
sample, and in `extra` the greedy max-k and plain unfused FP32 runs of the same
circuit on the same GPU plus the batched 512-circuit workload.  Progress goes
to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "gates/s + HBM GB/s (34q c64); fused+MFMA vs plain FP32 at infidelity≤1e-6"
HBM_PEAK_GBPS = 8000.0
VARIANT_NAMES = {1: "k_apply_reg", 2: "k_apply_lds", 3: "k_apply_mfma", 4: "k_phase"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name: str):
    import circuits as C
    if name == "grid34":
        return 34, C.grid_circuit(2, 17, 24, seed=0), "34-qubit 2x17 random grid, depth 24, |0..0>"
    if name == "grid30":
        return 30, C.grid_circuit(5, 6, 20, seed=0), "30-qubit 5x6 random grid, depth 20, |0..0>"
    if name == "grid20":
        return 20, C.grid_circuit(4, 5, 14, seed=0), "20-qubit 4x5 random grid, depth 14, |0..0>"
    raise SystemExit("unknown workload " + name)


def counter_traffic(kernel: str, workload_name: str, alg_bytes_per_launch: float):
    """HBM bytes per launch of `kernel`: the committed rocprofv3 counter
    summary's ratio of measured to algorithmic bytes over that kernel's
    launches, times this run's algorithmic bytes per launch; None when there
    is no summary or the kernel source has changed since the counters were
    taken."""
    import hashlib
    import re
    if kernel != "k_apply_mfma" or workload_name != "grid34":
        return None
    path = os.path.join(ROOT, "profiles", "k_apply_mfma_grid34.md")
    src = os.path.join(ROOT, "paper_2602_09604_amd", "csrc", "k_mfma.hip")
    try:
        text = open(path).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    m = re.search(r"traffic_ratio k_apply_mfma: ([0-9.e+]+)", text)
    s = re.search(r"k_mfma.hip sha256: ([0-9a-f]+)", text)
    if not m or not s or s.group(1) != sha:
        return None
    return float(m.group(1)) * alg_bytes_per_launch


def host_info() -> dict:
    """CPU model, logical CPUs and RAM of the host the oracle runs on."""
    model, mem = "unknown", 0
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                mem = int(line.split()[1]) * 1024
                break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "ram_GiB": round(mem / 2 ** 30, 1)}


GOLDEN = {"grid34": "grid34_d24_s0_cut.npz", "grid30": "grid30_d20_s0.npz"}


def accuracy_vs_oracle(st, workload_name: str):
    """Sampled amplitudes of the state against the stored oracle values for
    this workload (tests/golden: exact amplitudes the oracle computed, by a
    two-way cut of the 34-qubit ladder or on the full 30-qubit state), or
    None when there is no stored file."""
    import numpy as np
    name = GOLDEN.get(workload_name)
    path = os.path.join(ROOT, "tests", "golden", name) if name else None
    if not path or not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as f:
        idx, ref, nr = f["idx"], f["amp"], int(f["n_random"])
    got_r = np.array([st.read(int(i), 1)[0] for i in idx[:nr]], dtype=np.complex64)
    got_b = st.read(int(idx[nr]), idx.size - nr)
    got = np.concatenate([got_r, got_b]).astype(np.complex128)
    d = got - ref
    o2, g2 = float(np.vdot(ref, ref).real), float(np.vdot(got, got).real)
    fid = abs(np.vdot(ref, got)) ** 2 / (o2 * g2)
    return {"samples": int(idx.size), "max_abs": float(np.max(np.abs(d))),
            "rel_l2": float(np.sqrt(np.vdot(d, d).real / o2)), "sampled_infidelity": float(1.0 - fid),
            "reference": "tests/golden/" + name}


def issued_mfma_flops(gates, n: int, max_k: int, fusion: str, precision: str) -> dict:
    """Useful and issued flops of one run's matrix-core passes, from the
    partition sv_fuse returns for the same options (the model installed at
    the time of the call decides it, as in sv_apply_circuit).  A pass on k
    targets covering g groups is a real 4M-form GEMM of 2^(k+1) x 2^(k+1)
    by 2^(k+1) x g: 2 * 4^(k+1) * g flops per product, three products in the
    split modes; useful flops are g * 2^k (8 * 2^k - 2)."""
    from paper_2602_09604_amd import sv
    if precision == "fp32_valu":
        return {}
    prods = 1 if precision == "fp32_mfma" else 3
    fused, _ = sv.sv_fuse(gates, n, sv.make_opts(max_k=max_k, fusion=fusion, precision=precision))
    useful = issued = 0.0
    for g in fused:
        if g.k < 4:
            continue
        groups = 2.0 ** (n - g.k - len(g.controls))
        useful += groups * 2 ** g.k * (8 * 2 ** g.k - 2)
        issued += prods * 2.0 * 4.0 ** (g.k + 1) * groups
    return {"mfma_useful_flops": useful, "mfma_issued_flops": issued, "products_per_pass": prods}


def measured_ceilings(log) -> dict:
    """Bandwidth a plain device copy and an in-place read-modify-write reach
    on this GPU (torch's own kernels, 8 GiB tensors): the practical ceilings
    next to the 8 TB/s vendor peak."""
    import torch
    a = torch.empty(1 << 30, dtype=torch.complex64, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    nbytes = a.numel() * a.element_size()
    out = {}
    for label, fn, moved in (("copy", lambda: b.copy_(a), 2 * nbytes), ("rmw_inplace_scale", lambda: a.mul_(1.0),
                                                                          2 * nbytes)):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            fn()
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) * 1e-3 / 5
        out[label + "_GBps"] = moved / t / 1e9
    del a, b
    torch.cuda.empty_cache()
    log("ceilings:", out)
    return out


def library_sweeps(st, log) -> dict:
    """The library's own plainest sweeps of the benchmark state: the FP64 norm
    (read only) and a one-qubit gate on amplitude bit 0 (one contiguous
    read-modify-write stream, no gather), each the best of three.  They bound
    what a gate pass on this state can reach on this GPU."""
    import numpy as np
    import circuits as C
    h = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
    nbytes = 16.0 * (1 << st.n)
    best_pass, best_norm = 1e30, 1e30
    for _ in range(3):
        s = st.apply_circuit([C.Gate((0,), h)], fusion="none", precision="fp32_valu", stats=True, timing=True)
        best_pass = min(best_pass, s["gpu_s"])
        t0 = time.perf_counter()
        st.norm()
        best_norm = min(best_norm, time.perf_counter() - t0)
    out = {"one_qubit_bit0_pass_GBps": nbytes / best_pass / 1e9,
           "norm_read_GBps": nbytes / 2 / best_norm / 1e9, "state_qubits": st.n}
    log("library sweeps:", out)
    return out


def grid30_rows(log) -> dict:
    """The 30-qubit 5x6 depth-20 grid (845 gates): learned fusion in the
    split and FP32 modes and greedy max-k = 6, GPU time and accuracy against
    the oracle's stored full-state samples."""
    import torch
    from paper_2602_09604_amd import sv
    n, gates, _ = workload("grid30")
    garr = sv.GateArray(gates)
    st = sv.State(n)
    out = {}
    try:
        for fusion, K, prec in (("learned", 6, "fp16x3"), ("learned", 6, "fp32_mfma"), ("learned", 6, "fp32_valu"),
                                ("greedy", 6, "fp16x3"), ("greedy", 4, "fp32_valu")):
            best = None
            for _ in range(2):
                st.set_basis(0)
                r = st.apply_circuit(garr, fusion=fusion, max_k=K, precision=prec, stats=True)
                best = r if best is None or r["gpu_s"] < best["gpu_s"] else best
            row = {"passes": best["passes"], "gpu_s": best["gpu_s"], "gates_per_s_gpu": len(gates) / best["gpu_s"],
                   "alg_hbm_GBps": best["bytes"] / best["gpu_s"] / 1e9, "norm_drift": abs(st.norm() - 1.0)}
            a = accuracy_vs_oracle(st, "grid30")
            if a is not None:
                row["accuracy_vs_oracle"] = a
            out["%s%d_%s" % (fusion, K, prec)] = row
            log("grid30 %s k=%d %s:" % (fusion, K, prec), row)
    finally:
        st.free()
        del st
        torch.cuda.empty_cache()
    return out


def run_step(st, gates, opts_kw, sample):
    st.set_basis(0)
    stats = st.apply_circuit(gates, stats=True, **opts_kw)
    nrm = st.norm()
    st.read(0, sample)
    return stats, nrm


def cpu_baseline(seconds_hint: float = 20.0) -> dict:
    """The oracle (complex128, OpenMP, one gate at a time) on a 26-qubit 2x13
    grid of the same depth and gate set; gates/s scaled to 34 qubits by the
    state-size ratio 2^26 / 2^34 (the oracle's cost is linear in 2^n)."""
    import circuits as C
    import oracle
    n = 26
    gates = C.grid_circuit(2, 13, 24, seed=0)
    oracle.build()
    probe = gates[:40]
    t0 = time.perf_counter()
    oracle.apply_circuit(n, probe)
    per_gate = (time.perf_counter() - t0) / len(probe)
    count = max(40, min(len(gates), int(seconds_hint / max(per_gate, 1e-9))))
    t0 = time.perf_counter()
    oracle.apply_circuit(n, gates[:count])
    dt = time.perf_counter() - t0
    gps_n = count / dt
    # the other workloads, a few seconds each: the QFT-like circuit at 22
    # qubits (scaled to 32 by 2^-10) and the first 16 batched circuits
    qn = 22
    qft = C.qft_like_circuit(qn)
    t0 = time.perf_counter()
    oracle.apply_circuit(qn, qft, init=C.qft_input_basis(qn, 0))
    qdt = time.perf_counter() - t0
    ns, circs = C.batched_ansatz(512, seed=0)
    t0 = time.perf_counter()
    for nb, cb in list(zip(ns, circs))[:16]:
        oracle.apply_circuit(nb, cb)
    bdt = time.perf_counter() - t0
    return {
        "value": gps_n * 2.0 ** (n - 34),
        "unit": "gates/s",
        "cores": oracle.threads(),
        "kind": "oracle",
        "host": host_info(),
        "why_not_34q": "a 34-qubit complex128 oracle state is 256 GiB; the sample runs at 26 qubits and is scaled "
                       "(the oracle's cost is linear in 2^n)",
        "sample": "first %d gates of a 26-qubit 2x13 grid circuit (depth 24) in %.1f s = %.3g gates/s at 26 "
                  "qubits, scaled by 2^-8 to the 34-qubit state" % (count, dt, gps_n),
        "qft32_gates_per_s": len(qft) / qdt * 2.0 ** (qn - 32),
        "qft_sample": "22-qubit QFT-like circuit (%d gates) in %.2f s, scaled by 2^-10 to 32 qubits" % (len(qft), qdt),
        "batch_circuits_per_s": 16 / bdt,
        "batch_sample": "the first 16 of the 512 batched circuits in %.2f s" % bdt,
    }


def batch_figures(max_k: int) -> dict:
    """The 512-circuit batched workload: one captured graph (sv_batch_run)
    against one sv_apply_circuit launch sequence per circuit, both with the
    largest-block partition at max_k (k = 4 measured best: larger blocks make
    the batched VALU passes compute-bound)."""
    import torch
    import circuits as C
    from paper_2602_09604_amd import sv
    import ctypes
    ns, circs = C.batched_ansatz(512, seed=0)
    stream = torch.cuda.current_stream()
    states = [sv.State(n, stream=stream) for n in ns]
    try:
        opts = sv.make_opts(max_k=max_k, fusion="block")
        # marshal every gate list once, outside the timed regions
        arrays = [sv.GateArray(c) for c in circs]
        hs = (ctypes.c_void_p * 512)(*[s.h for s in states])
        cps = (ctypes.POINTER(sv.sv_gate) * 512)(*[a.ptr for a in arrays])
        counts = (ctypes.c_size_t * 512)(*[a.n for a in arrays])
        L = sv.lib()

        def batched():
            stt = sv.sv_run_stats()
            sv._check(L.sv_batch_run(hs, cps, counts, 512, ctypes.byref(opts), ctypes.byref(stt)))
            return stt.as_dict()

        batched()  # warm-up (code objects, allocator)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = batched()
        wall_batch = time.perf_counter() - t0
        for s, a in zip(states, arrays):  # warm-up of the per-circuit path
            sv._check(L.sv_apply_circuit(ctypes.c_void_p(s.h), a.ptr, a.n, ctypes.byref(opts), None))
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for s, a in zip(states, arrays):
            sv._check(L.sv_apply_circuit(ctypes.c_void_p(s.h), a.ptr, a.n, ctypes.byref(opts), None))
        e1.record(stream)
        torch.cuda.synchronize()
        wall_seq = time.perf_counter() - t0
        gpu_seq = e0.elapsed_time(e1) * 1e-3
        amps = sum(1 << n for n in ns)
        floor = sum(16 << n for n in ns)  # every state read once and written once
        return {
            "circuits": 512, "gates": int(st["gates_in"]), "passes": int(st["passes"]),
            "launches_in_graph": int(st["launches"]),
            "alg_hbm_bytes": int(st["bytes"]), "hbm_floor_bytes": floor,
            "alg_bytes_over_floor": st["bytes"] / floor,
            "batched_gpu_s": st["gpu_s"], "batched_wall_s": wall_batch, "batched_fuse_s": st["fuse_s"],
            "batched_circuits_per_s_gpu": 512 / st["gpu_s"],
            "batched_circuits_per_s_wall": 512 / wall_batch,
            "per_circuit_launches_wall_s": wall_seq, "per_circuit_launches_gpu_s": gpu_seq,
            "per_circuit_circuits_per_s_wall": 512 / wall_seq,
            "speedup_wall": wall_seq / wall_batch, "speedup_gpu": gpu_seq / st["gpu_s"],
            "total_amplitudes": amps,
        }
    finally:
        for s in states:
            s.free()


def profile_workload(name: str, tune_qubits: int) -> None:
    """One 32-qubit workload of other_workloads() (or the 30-qubit grid at a
    small greedy max k, whose passes are all k <= 3, or the 512-circuit
    batch, or the state reads at 32 qubits), after the autotuner, run twice (the second run is the one to
    read in a kernel trace).  It starts
    with a copy of known size (8 GiB read, 8 GiB written) that calibrates
    the HBM byte counters of rocprofv3 --pmc runs."""
    import torch
    import circuits as C
    from paper_2602_09604_amd import sv
    a = torch.empty(1 << 30, dtype=torch.complex64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    torch.cuda.empty_cache()
    scratch = sv.State(tune_qubits)
    sv.sv_autotune(scratch.h, 0)
    scratch.free()
    del scratch
    torch.cuda.empty_cache()
    if name == "batch512":  # the batched workload (its own warm-up run first)
        log("batch512:", batch_figures(4))
        return
    if name == "reads32":  # the state reads, each twice, on a 32-qubit entangled state
        st = sv.State(32)
        try:
            st.apply_circuit(C.grid_circuit(4, 8, 4, seed=0), max_k=5, fusion="greedy", precision="fp16x3")
            for rep in range(2):
                log("reads32 run %d:" % rep, state_reads(st, 32, reps=1))
        finally:
            st.free()
        return
    n = 32
    init = 0
    if name.startswith("grid30"):
        n = 30
        gates = C.grid_circuit(5, 6, 20, seed=0)
        kw = dict(max_k=int(name[-1]), fusion="greedy", precision="fp32_valu")
    elif name.startswith("qft32"):
        gates, init = C.qft_like_circuit(n), C.qft_input_basis(n, 0)
        kw = dict(max_k=5, fusion=name.split("_")[1], precision="fp16x3")
    elif name == "grover32":
        gates = C.grover_circuit(n, 0x2D2D2D2D, 3)
        kw = dict(max_k=6, fusion="greedy", precision="fp16x3")
    else:
        gates = C.quantum_volume_circuit(n, n, seed=0)
        kw = dict(max_k=6, fusion=name.split("_")[1], precision="fp16x3")
    st = sv.State(n)
    try:
        for rep in range(2):
            st.set_basis(init)
            s = st.apply_circuit(gates, stats=True, timing=True, **kw)
            log("%s run %d: %d passes %.3f s, per family %s" % (name, rep, s["passes"], s["gpu_s"],
                                                               {VARIANT_NAMES[v]: (s["variant_passes"][v],
                                                                                   round(s["variant_s"][v], 4))
                                                                for v in range(1, 5) if s["variant_passes"][v]}))
    finally:
        st.free()


def state_reads(st, n: int, reps: int = 3) -> dict:
    """Wall time of the synchronous state reads on an n-qubit state: one
    Pauli term, 8 terms sharing a flip mask (quads of elements), 8 terms
    with f = 1 (pairs inside an element), 8 diagonal terms, the marginal
    over 10 qubits and 100k inverse-CDF samples."""
    import numpy as np
    import torch
    import circuits as C
    state_bytes = 8.0 * (1 << n)

    def timed(fn, r=reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(r):
            fn()
        return (time.perf_counter() - t0) / r

    out = {}
    zm = np.array([(1 << t) | (1 << (t + 9)) for t in range(8)], dtype=np.uint64)
    cases = (("pauli_1_term", np.array([0b101 << 20], np.uint64), np.array([0b11], np.uint64)),
             ("pauli_8_terms_one_sweep", np.array([0b1011 << 20] * 8, dtype=np.uint64), zm),
             ("pauli_8_terms_flip_bit_0", np.ones(8, np.uint64), zm),
             ("pauli_8_diagonal_terms", np.zeros(8, np.uint64), zm))
    for name, xm, z in cases:
        t = timed(lambda: st.expect_pauli(xm, z))
        out[name] = {"s": t, "GBps": state_bytes / t / 1e9}
    t = timed(lambda: st.marginal_probs(tuple(range(0, 30, 3))))
    out["marginal_10_qubits"] = {"s": t, "GBps": state_bytes / t / 1e9}
    u = C.uniforms(100000, 0)
    t = timed(lambda: st.sample(u), r=2)
    out["sample_100k_shots"] = {"s": t, "shots_per_s": u.size / t}
    return out


def other_workloads() -> dict:
    """The paper's other circuit families at 30-32 qubits and the state
    reads, each timed on the GPU (device time of the passes; wall time of
    the synchronous reads)."""
    import numpy as np
    import torch
    import circuits as C
    from paper_2602_09604_amd import sv
    out = {}
    # the 20-qubit 4x5 depth-14 grid (8 MiB state, held in the caches):
    # launch-bound unfused (389 passes), so one launch per pass against the
    # kept graph relaunched, and block fusion; wall clock per circuit
    small = sv.State(20)
    try:
        g20 = sv.GateArray(C.grid_circuit(4, 5, 14, seed=0))
        for label, kw in (("unfused_launches", dict(fusion="none")),
                          ("unfused_graph", dict(fusion="none", use_graph=True)),
                          ("block6_graph", dict(fusion="block", max_k=6, precision="fp16x3", use_graph=True))):
            s = small.apply_circuit(g20, stats=True, **kw)  # captures the graph when asked
            small.norm()  # synchronises the state's stream
            t0 = time.perf_counter()
            for _ in range(5):
                small.set_basis(0)
                last = small.apply_circuit(g20, stats=True, **kw)
            small.norm()
            dt = (time.perf_counter() - t0) / 5
            out["grid20_" + label] = {"gates": g20.n, "passes": s["passes"], "wall_s": dt, "gates_per_s": g20.n / dt,
                                      "graph_relaunched": bool(last["graph_relaunched"])}
        log("grid20:", {k: v for k, v in out.items() if k.startswith("grid20")})
    finally:
        small.free()
        del small
    n = 32
    st = sv.State(n)
    try:
        x = C.qft_input_basis(n, 0)
        qft = C.qft_like_circuit(n)
        for fusion in ("greedy", "phase"):
            st.set_basis(x)
            s = st.apply_circuit(qft, max_k=5, fusion=fusion, precision="fp16x3", stats=True)
            out["qft32_" + fusion] = {"gates": len(qft), "passes": s["passes"], "gpu_s": s["gpu_s"],
                                      "gates_per_s_gpu": len(qft) / s["gpu_s"],
                                      "alg_hbm_frac": s["bytes"] / s["gpu_s"] / 1e9 / HBM_PEAK_GBPS}
            log("qft32 %s: %d passes %.3f s" % (fusion, s["passes"], s["gpu_s"]))
        marked, iters = 0x2D2D2D2D, 3
        grover = C.grover_circuit(n, marked, iters)
        for fusion in ("greedy", "learned"):
            st.set_basis(0)
            s = st.apply_circuit(grover, max_k=6, fusion=fusion, precision="fp16x3", stats=True)
            key = "grover32" if fusion == "greedy" else "grover32_learned"
            out[key] = {"gates": len(grover), "iterations": iters, "passes": s["passes"], "gpu_s": s["gpu_s"],
                        "gates_per_s_gpu": len(grover) / s["gpu_s"],
                        "alg_hbm_frac": s["bytes"] / s["gpu_s"] / 1e9 / HBM_PEAK_GBPS,
                        "marked_probability": abs(complex(st.read(marked, 1)[0])) ** 2}
            log(key + ":", out[key])
        # the network against the fewest-passes rule where they differ: FP32
        # on the VALU kernels, whose k = 6 passes are compute-bound
        grid = C.grid_circuit(4, 8, 20, seed=0)
        for fusion in ("learned", "block"):
            st.set_basis(0)
            s = st.apply_circuit(grid, max_k=6, fusion=fusion, precision="fp32_valu", stats=True)
            out["grid32_fp32_valu_" + fusion] = {"gates": len(grid), "passes": s["passes"], "gpu_s": s["gpu_s"],
                                                 "gates_per_s_gpu": len(grid) / s["gpu_s"]}
            log("grid32 fp32_valu %s:" % fusion, out["grid32_fp32_valu_" + fusion])
        qv = C.quantum_volume_circuit(n, n, seed=0)
        for fusion in ("greedy", "block", "learned"):
            st.set_basis(0)
            s = st.apply_circuit(qv, max_k=6, fusion=fusion, precision="fp16x3", stats=True)
            out["qv32_" + fusion] = {"gates": len(qv), "depth": n, "passes": s["passes"], "gpu_s": s["gpu_s"],
                                     "gates_per_s_gpu": len(qv) / s["gpu_s"],
                                     "alg_hbm_frac": s["bytes"] / s["gpu_s"] / 1e9 / HBM_PEAK_GBPS}
            log("qv32 %s:" % fusion, out["qv32_" + fusion])
        # state reads on the quantum-volume output
        out.update(state_reads(st, n))
        log("reads:", {k: out[k] for k in out if k.startswith(("pauli", "marginal", "sample"))})
    finally:
        st.free()
        del st
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="grid34")
    ap.add_argument("--max-k", type=int, default=6)
    ap.add_argument("--fusion", default="learned", choices=["none", "greedy", "learned", "block", "phase"])
    ap.add_argument("--precision", default="fp16x3", choices=["fp32_valu", "fp32_mfma", "bf16x3", "fp16x3"])
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (untuned defaults)")
    ap.add_argument("--tune-qubits", type=int, default=28)
    ap.add_argument("--corpus-samples", type=int, default=2400)
    ap.add_argument("--no-plain", action="store_true", help="skip the plain unfused FP32 comparison run")
    ap.add_argument("--no-greedy", action="store_true", help="skip the greedy max-k comparison run")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 512-circuit figures")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-others", action="store_true", help="skip the QFT / Grover / QV / state-read figures")
    ap.add_argument("--no-precisions", action="store_true",
                    help="skip the FP32 runs of the same circuit, the network-value runs and the 30-qubit rows")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--profile-workload", default=None,
                    choices=["qft32_greedy", "qft32_phase", "grover32", "qv32_greedy", "qv32_learned",
                             "grid30_greedy2", "grid30_greedy3", "batch512", "reads32"],
                    help="autotune, then run one 30/32-qubit workload twice (or the 512-circuit batch) and exit "
                         "(for rocprofv3 runs)")
    ap.add_argument("--profile-step", action="store_true",
                    help="counter-calibration copy + one untimed step, then exit (for rocprofv3 --pmc runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2602_09604_amd import sv

    if args.profile_workload:
        profile_workload(args.profile_workload, args.tune_qubits)
        return
    n, gates, desc = workload(args.workload)
    log("workload:", desc, "gates:", len(gates))
    if args.profile_step:
        # For hardware-counter runs: a copy of known size (8 GiB read + 8 GiB
        # written) to calibrate the byte counters, then one step of the
        # circuit with learned fusion and no cost model (so the fewest state
        # sweeps: blocks with controls, 2^c launches each over 2^-c of the
        # state, as in the timed run).
        a = torch.empty(1 << 30, dtype=torch.complex64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()
        st = sv.State(n)
        s = st.apply_circuit(gates, max_k=args.max_k, fusion="learned", precision=args.precision, stats=True)
        log("profile step: passes %d gpu %.3f s norm %.9f" % (s["passes"], s["gpu_s"], st.norm()))
        # the other pass kinds and the state reads, once each on the same state
        import numpy as np
        import circuits as C
        st.apply_controlled_gate((20,), C.X, (n - 1,))                 # touches half the state
        cps = [C.Gate((a, (a * 7 + 3) % n), C.CP(0.1 * a)) for a in range(n) if a != (a * 7 + 3) % n]
        st.apply_circuit(cps, max_k=2, fusion="phase")                 # one phase pass
        st.expect_pauli(np.array([0b101 << 20], np.uint64), np.array([0b11], np.uint64))
        st.marginal_probs(tuple(range(0, 30, 3)))
        st.sample(C.uniforms(1000, 0))
        torch.cuda.synchronize()
        log("profile step: controlled, phase and read kernels done")
        st.free()
        return
    extra = {}
    if not args.no_tune:
        t0 = time.perf_counter()
        scratch = sv.State(min(args.tune_qubits, n))
        sv.sv_autotune(scratch.h, 0)
        scratch.free()
        del scratch
        torch.cuda.empty_cache()
        extra["autotune_s"] = time.perf_counter() - t0
        log("autotune: %.1f s" % extra["autotune_s"])
    if args.fusion == "learned":
        from paper_2602_09604_amd import costmodel
        t0 = time.perf_counter()
        corpus = costmodel.collect_corpus(samples=args.corpus_samples, seed=0, log=log)
        info = costmodel.train_cost_model(corpus, epochs=4000, lr=3e-3, seed=0)
        info["corpus_s"] = time.perf_counter() - t0 - info["train_s"]
        extra["cost_model"] = info
        torch.cuda.empty_cache()
        log("cost model:", info)

    sample = 1 << 20
    st = sv.State(n)
    opts = dict(max_k=args.max_k, fusion=args.fusion, precision=args.precision, timing=True)
    garr = sv.GateArray(gates)  # the circuit as C structs, marshalled once
    for i in range(args.warmup):
        s, nrm = run_step(st, garr, opts, sample)
        log("warmup %d: passes %d gpu %.3f s norm %.9f" % (i, s["passes"], s["gpu_s"], nrm))

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    agg = None
    norms = []
    for i in range(args.steps):
        s, nrm = run_step(st, garr, opts, sample)
        norms.append(nrm)
        log("step %d: passes %d gpu %.3f s fuse %.3f s" % (i, s["passes"], s["gpu_s"], s["fuse_s"]))
        if agg is None:
            agg = s
        else:
            for key in ("gpu_s", "fuse_s", "useful_flops"):
                agg[key] += s[key]
            for v in range(5):
                agg["variant_s"][v] += s["variant_s"][v]
                agg["variant_passes"][v] += s["variant_passes"][v]
                agg["variant_bytes"][v] += s["variant_bytes"][v]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    gates_per_s = len(gates) / (wall / args.steps)
    passes = agg["variant_passes"]
    dom = max(range(1, 5), key=lambda v: agg["variant_s"][v])
    # launches differ in size when a block has controls (2^c launches, each
    # over 2^-c of the state): per-launch figures are averages over the
    # dominant kernel's launches, bytes / time over the same launches
    avg_launch = agg["variant_s"][dom] / max(1, passes[dom])
    bytes_per_launch = agg["variant_bytes"][dom] / max(1, passes[dom])
    achieved = bytes_per_launch / avg_launch / 1e9
    pass_time = sum(agg["variant_s"][1:5])
    extra.update({
        "passes_per_step": int(sum(passes) / args.steps),
        "state_sweeps_per_step": sum(agg["variant_bytes"][1:5]) / args.steps / (16.0 * (1 << n)),
        "alg_hbm_GBps_all_passes": sum(agg["variant_bytes"][1:5]) / pass_time / 1e9,
        "gpu_s_per_step": agg["gpu_s"] / args.steps,
        "fuse_s_per_step": agg["fuse_s"] / args.steps,
        "useful_tflops_per_s": agg["useful_flops"] / pass_time / 1e12,
        "norm_drift": max(abs(x - 1.0) for x in norms),
        "per_variant": {VARIANT_NAMES[v]: {"passes": int(passes[v]), "avg_ms": 1e3 * agg["variant_s"][v] / passes[v],
                                           "GBps": agg["variant_bytes"][v] / agg["variant_s"][v] / 1e9}
                        for v in range(1, 5) if passes[v]},
        "dominant_avg_launch_ms": 1e3 * avg_launch,
    })
    # the timed path's final state against the oracle's stored amplitudes
    acc = accuracy_vs_oracle(st, args.workload)
    if acc is not None:
        acc["norm_drift"] = extra["norm_drift"]
        extra["accuracy_vs_oracle"] = acc
        log("accuracy vs oracle:", acc)
    extra["library_sweeps"] = library_sweeps(st, log)
    extra["dominant_over_best_library_sweep"] = achieved / extra["library_sweeps"]["one_qubit_bit0_pass_GBps"]
    fl = issued_mfma_flops(gates, n, args.max_k, args.fusion, args.precision)
    if fl:
        mfma_s = agg["variant_s"][3] / args.steps
        fl.update({"mfma_pass_s_per_step": mfma_s, "mfma_useful_TFLOPs": fl["mfma_useful_flops"] / mfma_s / 1e12,
                   "mfma_issued_TFLOPs": fl["mfma_issued_flops"] / mfma_s / 1e12})
        extra["mfma_flops_per_step"] = fl
        log("mfma flops:", fl)

    if not args.no_greedy and args.fusion != "greedy":
        for mode in ("greedy", "block"):
            st.set_basis(0)
            g = st.apply_circuit(garr, fusion=mode, max_k=args.max_k, precision=args.precision, stats=True)
            extra[mode + "_max_k"] = {"max_k": args.max_k, "gpu_s": g["gpu_s"], "passes": g["passes"],
                                      "fuse_s": g["fuse_s"], "gates_per_s_gpu": len(gates) / g["gpu_s"]}
            log("%s max_k=%d: %d passes %.3f s" % (mode, args.max_k, g["passes"], g["gpu_s"]))
        # the learned search (candidates, beams, blocks with controls, and the
        # network) against first-come greedy blocks; network_value below
        # separates what the network itself adds
        extra["learned_search_over_greedy_gpu_time"] = agg["gpu_s"] / args.steps / extra["greedy_max_k"]["gpu_s"]
    if not args.no_precisions and args.fusion == "learned":
        # the paper's FP32 arithmetic on the same circuit and partition search,
        # and what the trained network adds: the same search with the model
        # removed keeps the fewest passes
        import tempfile
        tmp = tempfile.NamedTemporaryFile(suffix=".svcm", delete=False)
        tmp.close()
        sv.sv_cost_model_save(tmp.name)
        rows = {}
        try:
            for prec in dict.fromkeys((args.precision, "fp32_mfma", "fp32_valu")):
                for model in (True, False):
                    if model:
                        sv.sv_cost_model_load(tmp.name)
                    else:
                        sv.sv_cost_model_clear()
                    if prec == "fp32_mfma" and not model:
                        continue  # every matrix-core pass moves the same bytes: the FP16X3 pair shows the tie
                    st.set_basis(0)
                    r = st.apply_circuit(garr, fusion="learned", max_k=args.max_k, precision=prec, stats=True)
                    row = {"passes": r["passes"], "gpu_s": r["gpu_s"], "gates_per_s_gpu": len(gates) / r["gpu_s"],
                           "alg_hbm_GBps": r["bytes"] / r["gpu_s"] / 1e9, "norm_drift": abs(st.norm() - 1.0)}
                    a = accuracy_vs_oracle(st, args.workload)
                    if a is not None:
                        row["accuracy_vs_oracle"] = a
                    key = "%s_%s" % (prec, "model" if model else "no_model")
                    rows[key] = row
                    log("learned %s:" % key, row)
        finally:
            sv.sv_cost_model_load(tmp.name)
            os.unlink(tmp.name)
        extra["learned_by_precision"] = rows
        extra["network_value"] = {
            p_: {"model_over_no_model_gpu_time": rows[p_ + "_model"]["gpu_s"] / rows[p_ + "_no_model"]["gpu_s"],
                 "passes_model": rows[p_ + "_model"]["passes"], "passes_no_model": rows[p_ + "_no_model"]["passes"]}
            for p_ in dict.fromkeys((args.precision, "fp32_valu")) if p_ + "_no_model" in rows}
    if not args.no_plain:
        log("plain unfused FP32 run ...")
        st.set_basis(0)
        p = st.apply_circuit(gates, fusion="none", precision="fp32_valu", stats=True, timing=True)
        extra["plain_fp32_unfused"] = {
            "gates_per_s_gpu": len(gates) / p["gpu_s"], "gpu_s": p["gpu_s"], "passes": p["passes"],
            "alg_hbm_GBps": p["bytes"] / p["gpu_s"] / 1e9, "norm": st.norm(),
        }
        a = accuracy_vs_oracle(st, args.workload)
        if a is not None:
            extra["plain_fp32_unfused"]["accuracy_vs_oracle"] = a
        extra["speedup_vs_plain_fp32"] = gates_per_s / extra["plain_fp32_unfused"]["gates_per_s_gpu"]
        log("plain: %.3f s" % p["gpu_s"])
    st.free()
    del st
    torch.cuda.empty_cache()

    if not args.no_precisions and args.workload == "grid34":
        extra["grid30"] = grid30_rows(log)
        extra["measured_ceilings"] = measured_ceilings(log)

    if not args.no_batch:
        log("batched 512-circuit workload ...")
        extra["batch512"] = batch_figures(4)
        log("batch:", extra["batch512"])

    if not args.no_others:
        log("other workloads and state reads ...")
        extra["other_workloads_32q"] = other_workloads()

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(args.cpu_seconds)

    line = {
        "metric": METRIC,
        "value": gates_per_s,
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32_valu": "f32", "fp32_mfma": "f32", "bf16x3": "bf16x3+f32acc",
                  "fp16x3": "f16x3+f32acc"}[args.precision],
        "data": "synthetic",
        "config": {"workload": desc, "qubits": n, "gates": len(gates), "state": "complex64",
                   "fusion": args.fusion, "max_k": args.max_k, "precision": args.precision},
        "roofline": {"bound": "hbm", "kernel": VARIANT_NAMES[dom], "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": counter_traffic(VARIANT_NAMES[dom], args.workload, bytes_per_launch),
                     "algorithmic_bytes_per_launch": bytes_per_launch},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
