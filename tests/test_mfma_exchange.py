"""Passes with targets on amplitude bits 1..3 on streamed states (26 qubits
and more), where the lane-exchange kernels run: every low-target set (bits
1, 2, 3 alone, in pairs, all three), with and without bit 0 as a target --
matrix cores for k = 4..6 in FP32 / BF16 / FP16 plus controlled passes (one
control value, and all values of a block in one launch), and the FP32
register kernel for k = 1..3 (k = 4 with bit 0) -- each against the oracle
applying the same gate (Eq. 4) to the same random state."""
import sys

import numpy as np
import pytest

import circuits as C
import oracle

pytestmark = pytest.mark.gpu

N = 26
MAX_ABS, INFID = 1e-5, 1e-6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_2602_09604_amd import sv
    psi0 = C.random_state_c64(N, 26)
    st = sv.State(N)
    yield st, psi0, psi0.astype(np.complex128)
    st.free()
    del st
    torch.cuda.empty_cache()


def low_sets(prec, k, q0):
    all_tm = range(1, 8)
    tms = all_tm if (prec == "fp16x3" or k == 6) else (1, 6, 7)
    return [tm for tm in tms if not (q0 and k == 4 and bin(tm).count("1") > 2)]


def targets_for(tm, k, q0, rng):
    qs = [t + 1 for t in range(3) if (tm >> t) & 1]
    if q0:
        qs.append(0)
    rest = [q for q in range(4, N) if q not in qs]
    qs += [int(q) for q in rng.choice(rest, size=k - len(qs), replace=False)]
    rng.shuffle(qs)  # unsorted on purpose
    return tuple(qs)


def run_and_check(st, psi0, ref0, gates, prec, variant="mfma"):
    st.write(0, psi0)
    st.apply_circuit(gates, fusion="none", precision=prec, variant=variant)
    got = st.read()
    ref = ref0.copy()
    for g in gates:
        oracle.apply_gate(ref, N, g.qubits, g.matrix, g.cmask, g.cval)
    r = oracle.compare(got, ref)
    return r


@pytest.mark.parametrize("prec", ["fp32_mfma", "bf16x3", "fp16x3"])
@pytest.mark.parametrize("k", [4, 5, 6])
@pytest.mark.parametrize("q0", [False, True])
def test_low_target_sets(setup, prec, k, q0):
    st, psi0, ref0 = setup
    rng = np.random.Generator(np.random.PCG64(k * 10 + q0 + 100 * len(prec)))
    for tm in low_sets(prec, k, q0):
        qs = targets_for(tm, k, q0, rng)
        g = C.Gate(qs, C.haar_unitary(k, rng))
        r = run_and_check(st, psi0, ref0, [g], prec)
        say(prec, "k=%d" % k, "targets", qs, r)
        assert r["max_abs"] <= MAX_ABS and r["infidelity"] <= INFID, (qs, r)


@pytest.mark.parametrize("prec", ["fp32_mfma", "fp16x3"])
def test_low_targets_with_controls(setup, prec):
    """A controlled pass (controls at bits >= 4: the exchange still runs) for
    one control value, and a block's 2^c matrices on the same targets as one
    launch."""
    st, psi0, ref0 = setup
    rng = np.random.Generator(np.random.PCG64(7 + len(prec)))
    for qs, ctl in (((1, 2, 3, 20, 21, 22), (5, 17)), ((0, 2, 25, 18, 9), (4, 12, 23)), ((3, 1, 14, 19), (8,))):
        k = len(qs)
        one = [C.Gate(qs, C.haar_unitary(k, rng), ctl, tuple(int(v) for v in rng.integers(0, 2, len(ctl))))]
        block = [C.Gate(qs, C.haar_unitary(k, rng), ctl, tuple((v >> t) & 1 for t in range(len(ctl))))
                 for v in range(1 << len(ctl))]
        for gates in (one, block):
            r = run_and_check(st, psi0, ref0, gates, prec)
            say(prec, "targets", qs, "controls", ctl, "gates", len(gates), r)
            assert r["max_abs"] <= MAX_ABS and r["infidelity"] <= INFID, (qs, ctl, r)


@pytest.mark.parametrize("k,q0", [(1, False), (2, False), (3, False), (2, True), (3, True), (4, True)])
def test_register_low_target_sets(setup, k, q0):
    st, psi0, ref0 = setup
    rng = np.random.Generator(np.random.PCG64(50 + k * 10 + q0))
    kq = k - 1 if q0 else k  # targets that are not bit 0
    for tm in range(1, 8):
        if bin(tm).count("1") > kq:
            continue
        qs = targets_for(tm, k, q0, rng)
        g = C.Gate(qs, C.haar_unitary(k, rng))
        r = run_and_check(st, psi0, ref0, [g], "fp32_valu", variant="reg")
        say("reg k=%d" % k, "targets", qs, r)
        assert r["max_abs"] <= MAX_ABS and r["infidelity"] <= INFID, (qs, r)


@pytest.mark.parametrize("qs", [(6, 17), (5, 9, 14, 20), (0, 4, 9), (0, 5, 9, 14, 20), (20, 14, 0, 9, 5)])
def test_register_streamed_3m_forms(setup, qs):
    """The register kernel's 3M row products on a streamed state (no target
    on amplitude bits 1..3, so the plain register form runs, non-temporal):
    two and four element-space targets, without and with bit 0 as a target
    (k = 5 with bit 0 is the largest 3M form)."""
    st, psi0, ref0 = setup
    rng = np.random.Generator(np.random.PCG64(sum(qs) + len(qs)))
    g = C.Gate(qs, C.haar_unitary(len(qs), rng))
    r = run_and_check(st, psi0, ref0, [g], "fp32_valu", variant="reg")
    say("reg 3M targets", qs, r)
    assert r["max_abs"] <= MAX_ABS and r["infidelity"] <= INFID, (qs, r)
