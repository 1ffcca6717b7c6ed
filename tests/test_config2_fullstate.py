"""30-qubit 5x6 grid (depth 20, 845 gates): greedy fusion swept over
max k = 2..6, FP32 VALU against FP32 MFMA and the split modes, plus the
largest-block and learned partitions, every result compared on the full
2^30-amplitude state with the complex128 oracle.

The oracle needs 16 GiB of host memory and minutes of CPU time, so this test
runs only when SV_LONG=1 is set:

    SV_LONG=1 python -m pytest tests/test_config2_fullstate.py -m gpu -s
"""
import os
import sys
import time

import numpy as np
import pytest

import circuits as C
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(os.environ.get("SV_LONG") != "1",
                                                  reason="long full-state run: set SV_LONG=1")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_config2_k_sweep_full_state():
    from paper_2602_09604_amd import sv
    n = 30
    gates = C.grid_circuit(5, 6, 20, seed=0)
    t0 = time.perf_counter()
    ref = oracle.basis_state(n, 0)
    for i in range(0, len(gates), 100):  # in slices, reporting progress (minutes of CPU work)
        oracle.apply_circuit(n, gates[i:i + 100], psi=ref)
        say("oracle: %d/%d gates, %.1f s" % (min(i + 100, len(gates)), len(gates), time.perf_counter() - t0))
    say("oracle: %.1f s on %d threads" % (time.perf_counter() - t0, oracle.threads()))
    st = sv.State(n)
    try:
        sv.sv_autotune(st.h, 0)
        rows = []
        runs = [(K, prec, "greedy") for K in (2, 3, 4, 5, 6) for prec in ("fp32_valu", "fp32_mfma", "bf16x3", "fp16x3")
                if K >= 4 or prec == "fp32_valu"]  # below k = 4 every precision runs the FP32 VALU kernels
        runs += [(K, "fp16x3", "block") for K in (5, 6)] + [(6, "fp32_mfma", "block"), (6, "fp16x3", "learned")]
        for K, prec, fusion in runs:
            if True:
                best = None
                for _ in range(2):
                    st.set_basis(0)
                    s = st.apply_circuit(gates, max_k=K, fusion=fusion, precision=prec, stats=True)
                    best = s if best is None or s["gpu_s"] < best["gpu_s"] else best
                acc = oracle.CompareAcc()
                chunk = 1 << 26
                for start in range(0, 1 << n, chunk):
                    acc.add(st.read(start, chunk), ref[start:start + chunk])
                r = acc.result()
                row = (K, prec, fusion, best["passes"], best["gpu_s"], best["bytes"] / best["gpu_s"] / 1e9,
                       len(gates) / best["gpu_s"], r["max_abs"], r["infidelity"], abs(st.norm() - 1))
                rows.append(row)
                say("K=%d %-9s %-7s passes %4d  %.4f s  %6.0f GB/s  %8.0f gates/s  max|d| %.2e  infid %.2e  "
                    "drift %.2e" % row)
                assert r["max_abs"] <= 1e-5 and r["infidelity"] <= 1e-6, row
    finally:
        st.free()
