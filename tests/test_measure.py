"""State reads on the GPU (Pauli expectations, marginal probabilities,
inverse-CDF sampling) against the oracle's plain definitions.  Inputs are
seeded random complex64 states written into the device state, and the same
complex64 values (widened to complex128) are handed to the oracle."""
import numpy as np
import pytest

import circuits as C
import oracle

pytestmark = pytest.mark.gpu


def load_state(n, seed):
    from paper_2602_09604_amd import sv
    psi = C.random_state_c64(n, seed)
    st = sv.State(n)
    st.write(0, psi)
    return st, psi.astype(np.complex128)


def random_terms(n, count, seed, shared_flip=None):
    rng = np.random.Generator(np.random.PCG64(seed))
    full = (1 << n) - 1
    x = rng.integers(0, 1 << n, size=count, dtype=np.uint64) & np.uint64(full)
    z = rng.integers(0, 1 << n, size=count, dtype=np.uint64) & np.uint64(full)
    if shared_flip is not None:
        x[:] = np.uint64(shared_flip)
    return x, z


@pytest.mark.parametrize("n", [1, 2, 5, 6, 7, 12, 17, 20])
def test_pauli_random_terms(n):
    st, psi = load_state(n, 10 + n)
    try:
        x, z = random_terms(n, 24, n)
        x[0] = z[0] = 0                 # identity: <psi|psi>
        x[1] = 0                        # a diagonal (Z-only) term
        got = st.expect_pauli(x, z)
        ref = np.array([oracle.pauli_expectation(psi, n, int(a), int(b)) for a, b in zip(x, z)])
        assert np.max(np.abs(ref.imag)) < 1e-12
        assert np.max(np.abs(got - ref.real)) < 1e-12, np.max(np.abs(got - ref.real))
    finally:
        st.free()


def test_pauli_many_terms_one_flip_split_into_sweeps():
    n = 14
    st, psi = load_state(n, 3)
    try:
        x, z = random_terms(n, 21, 9, shared_flip=0b10010000101)   # 3 sweeps of <= 8 terms
        got = st.expect_pauli(x, z)
        ref = np.array([oracle.pauli_expectation(psi, n, int(a), int(b)).real for a, b in zip(x, z)])
        assert np.max(np.abs(got - ref)) < 1e-12
    finally:
        st.free()


@pytest.mark.parametrize("flip", [0, 1, 0b10, (1 << 22) | (1 << 3) | 1, (1 << 20) | 0b110, (1 << 21) | (1 << 9)])
def test_pauli_long_walks_at_23_qubits(flip):
    """At 23 qubits every thread of the sweep walks 4 to 8 items, so the part
    of each term's sign that comes from the walk changes along it.  Per flip
    mask: 8, 3 and 2 terms in one sweep, z masks with bits in the thread's
    part, the walk's part (bits 20..22), bit 0 and the flip's own bits."""
    n = 23
    st, psi = load_state(n, 31)
    try:
        full = (1 << n) - 1
        rng = np.random.Generator(np.random.PCG64(flip + 7))
        z = [int(v) for v in rng.integers(0, 1 << n, size=8, dtype=np.uint64)]
        z[0], z[1], z[2], z[3] = 0, (1 << 22) | (1 << 21) | (1 << 20), full, flip | 1
        for count in (8, 3, 2):
            zs = z[:count]
            got = st.expect_pauli([flip] * count, zs)
            ref = np.array([oracle.pauli_expectation(psi, n, flip, b).real for b in zs])
            assert np.max(np.abs(got - ref)) < 1e-12, (count, np.max(np.abs(got - ref)))
    finally:
        st.free()


@pytest.mark.parametrize("flip", [0, 1, (1 << 26) | (1 << 2) | 1])
def test_pauli_chunk_walk_at_27_qubits(flip):
    """From 26 qubits up the sums walk the state in 32 KiB chunks per wave
    (two rounds of chunks at 27 qubits for every item kind): three terms
    per flip mask with z bits in the lane, step, wave and round fields and on
    bit 0, against the oracle on the same random state."""
    n = 27
    st, psi = load_state(n, 41)
    try:
        zs = [(1 << 25) | (1 << 3) | 1, (1 << 13) | (1 << 9), (1 << 26) | (1 << 20) | (1 << 6) | (1 << 1)]
        got = st.expect_pauli([flip] * 3, zs)
        ref = np.array([oracle.pauli_expectation(psi, n, flip, z).real for z in zs])
        assert np.max(np.abs(got - ref)) < 1e-12, (got, ref)
    finally:
        st.free()


def test_pauli_ghz_closed_forms_at_30_qubits():
    from paper_2602_09604_amd import sv
    n = 30
    st = sv.State(n)
    try:
        st.apply_circuit(C.ghz_circuit(n), max_k=4)
        full = (1 << n) - 1
        got = st.expect_pauli([full, full, 0, 0, 0], [0, 0b11, (1 << 29) | 1, 1 << 7, 0])
        assert np.allclose(got, [1, -1, 1, 0, 1], atol=1e-5), got
    finally:
        st.free()


def test_pauli_ghz_closed_forms_at_33_qubits():
    """Past 32 qubits (64-bit indices; every thread walks 8192 items): GHZ
    closed forms with Z and Y letters on the top qubit, quads and diagonal
    terms in one call."""
    from paper_2602_09604_amd import sv
    n = 33
    st = sv.State(n)
    try:
        st.apply_circuit(C.ghz_circuit(n), max_k=4)
        full = (1 << n) - 1
        top = 1 << (n - 1)
        got = st.expect_pauli([full, full, full, 0, 0, 0],
                              [0, top | 1, top | 0b110, top | (1 << 7), top, 0])
        assert np.allclose(got, [1, -1, 0, 1, 0, 1], atol=1e-5), got
    finally:
        st.free()


@pytest.mark.parametrize("n,qs", [(1, (0,)), (4, (3, 0)), (8, (0, 1, 2, 3, 4, 5, 6, 7)), (12, (11, 0, 5)),
                                  (16, (6, 7, 8)), (18, (2, 17, 9, 0, 12)),
                                  (20, (19, 18, 1, 3, 5, 7, 9, 11, 13, 15))])
def test_marginals(n, qs):
    st, psi = load_state(n, 20 + n)
    try:
        got = st.marginal_probs(qs)
        ref = oracle.marginal_probabilities(psi, n, qs)
        assert np.max(np.abs(got - ref)) < 1e-13
    finally:
        st.free()


def test_marginals_deterministic_and_bad_arguments():
    from paper_2602_09604_amd import sv
    st, _ = load_state(16, 4)
    try:
        a = st.marginal_probs((1, 9, 4))
        b = st.marginal_probs((1, 9, 4))
        assert np.array_equal(a, b)
        for bad in [(1, 1), (16,), tuple(range(11))]:
            with pytest.raises(sv.SvError):
                st.marginal_probs(bad)
    finally:
        st.free()


def check_samples(psi, u, got, exact_frac=0.999):
    """Each sample must be a valid inverse-CDF draw up to FP64 summation-order
    rounding, have p > 0, and almost all must equal the oracle's."""
    w = psi.real ** 2 + psi.imag ** 2
    cdf = np.cumsum(w)
    tot = cdf[-1]
    got = got.astype(np.int64)
    assert np.all((got >= 0) & (got < psi.size))
    assert np.all(w[got] > 0)
    tol = 1e-12 * tot
    t = u * tot
    lower = np.where(got > 0, cdf[np.maximum(got - 1, 0)], 0.0)
    assert np.all(lower <= t + tol)
    assert np.all((cdf[got] > t - tol) | (u >= 1 - 1e-12))
    ref = oracle.sample_indices(psi, u)
    assert np.mean(ref == got) >= exact_frac


@pytest.mark.parametrize("n", [1, 3, 12, 13, 16, 20])
def test_sampling_random_states(n):
    st, psi = load_state(n, 30 + n)
    try:
        u = C.uniforms(5000, n)
        check_samples(psi, u, st.sample(u))
    finally:
        st.free()


def test_sampling_sparse_state_and_ends():
    from paper_2602_09604_amd import sv
    n = 20
    st = sv.State(n)
    try:
        st.apply_circuit(C.ghz_circuit(n), max_k=4)
        u = np.concatenate([[0.0, 0.25, 0.4999, 0.5001, 1 - 1e-16], C.uniforms(2000, 7)])
        got = st.sample(u)
        assert set(np.unique(got).tolist()) <= {0, (1 << n) - 1}
        assert got[0] == 0 and got[-1 - 2000] == (1 << n) - 1
        frac = np.mean(got[5:] == 0)
        assert abs(frac - 0.5) < 0.05
    finally:
        st.free()


def test_sampling_basis_state_and_zero_state():
    from paper_2602_09604_amd import sv
    n = 15
    st = sv.State(n)
    try:
        st.set_basis(12345)
        assert np.all(st.sample(C.uniforms(300, 2)) == 12345)
        st.write(0, np.zeros(1 << n, dtype=np.complex64))
        with pytest.raises(sv.SvError):
            st.sample([0.5])
        with pytest.raises(sv.SvError):
            st.sample([1.0])
    finally:
        st.free()


def test_sampling_large_state_chunk_boundaries():
    """26 qubits: 2^14 chunks of 4096 amplitudes, several scan blocks."""
    n = 26
    st, psi = load_state(n, 5)
    try:
        u = C.uniforms(20000, 3)
        check_samples(psi, u, st.sample(u))
    finally:
        st.free()
