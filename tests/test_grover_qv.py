"""The paper's other workloads (Table 2): Grover search with its
multi-controlled Z as a controlled pass, against the closed form, and
quantum-volume circuits against the oracle."""
import numpy as np
import pytest

import circuits as C
import oracle

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,marked,t,fusion,prec", [
    (12, 1234, 3, "none", "fp32_valu"),
    (16, 40000, 5, "greedy", "fp32_valu"),
    (20, 777777, 4, "greedy", "fp16x3"),
    (20, 3, 2, "phase", "fp16x3"),
    (20, 5, 6, "learned", "fp16x3"),
    (18, 77, 4, "block", "fp32_valu"),
])
def test_grover_full_state_closed_form(n, marked, t, fusion, prec):
    from paper_2602_09604_amd import sv
    st = sv.State(n)
    try:
        s = st.apply_circuit(C.grover_circuit(n, marked, t), max_k=6, fusion=fusion, precision=prec, stats=True)
        ref = oracle.grover_amplitudes(n, marked, t, np.arange(1 << n))
        r = oracle.compare(st.read(), ref)
        print(n, fusion, prec, "passes", s["passes"], r, flush=True)
        assert r["max_abs"] <= 1e-5 and r["infidelity"] <= 1e-6, r
    finally:
        st.free()


def test_grover_28_sampled_and_success_probability():
    from paper_2602_09604_amd import sv
    n, marked, t = 28, 0x5A5A5A5, 3
    st = sv.State(n)
    try:
        st.apply_circuit(C.grover_circuit(n, marked, t), max_k=6, fusion="greedy", precision="fp16x3")
        rng = np.random.Generator(np.random.PCG64(1))
        idx = np.unique(np.concatenate([[marked], rng.integers(0, 1 << n, 4000)]))
        got = np.array([st.read(int(i), 1)[0] for i in idx])
        acc = oracle.CompareAcc()
        acc.add(got, oracle.grover_amplitudes(n, marked, t, idx))
        r = acc.result()
        assert r["max_abs"] <= 1e-5 and r["infidelity"] <= 1e-6, r
        p = st.marginal_probs(tuple(range(10)))[marked & 1023]
        pm = abs(oracle.grover_amplitudes(n, marked, t, [marked])[0]) ** 2
        other = (1 - pm) * ((1 << (n - 10)) - 1) / ((1 << n) - 1)
        assert abs(p - (pm + other)) < 1e-6
    finally:
        st.free()


@pytest.mark.parametrize("n,depth,fusion,prec", [(16, 16, "greedy", "fp32_valu"), (20, 20, "learned", "fp16x3"),
                                                 (20, 12, "none", "fp32_valu"), (22, 10, "greedy", "bf16x3"),
                                                 (22, 16, "block", "fp16x3")])
def test_quantum_volume_vs_oracle(n, depth, fusion, prec):
    from paper_2602_09604_amd import sv
    gates = C.quantum_volume_circuit(n, depth, seed=n + depth)
    ref = oracle.apply_circuit(n, gates)
    st = sv.State(n)
    try:
        st.apply_circuit(gates, max_k=6, fusion=fusion, precision=prec)
        r = oracle.compare(st.read(), ref)
        assert r["max_abs"] <= 1e-5 and r["infidelity"] <= 1e-6, r
    finally:
        st.free()
