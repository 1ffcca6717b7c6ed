"""CPU complex128 oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it; the only module both sides use is ``circuits``
(seeded input generators, no state arithmetic).

Contents, each written from the paper's definitions:

* ``apply_circuit`` / ``apply_gate``: the plain gate-by-gate simulator of
  Sec. II-A, Eq. 4 (C, complex128, OpenMP over groups, ``sv_oracle.c``);
* ``norm_sq``: sum |c_i|^2 of Eq. 1 with pairwise FP64 summation;
* ``compare``: max |delta|, relative L2, infidelity and norm drift of a
  complex64 state against a complex128 one; ``probe_projections``: a state's
  inner products with seeded probe vectors (whole-state checks through a few
  stored numbers);
* ``full_unitary`` / ``brute_force_state``: an independent construction of
  the whole 2^n x 2^n circuit operator from Kronecker products (Eq. 3), a
  bit permutation and, for controlled gates, a diagonal projector, for
  n <= 10;
* ``diagonal_factors``: what a run of diagonal gates multiplies chosen
  amplitudes by (Eq. 4 with a diagonal matrix: the entry the index selects),
  for sampled checks of phase passes at any size;
* ``pauli_expectation``, ``marginal_probabilities``, ``sample_indices``:
  the plain definitions of what the state-reading kernels return;
* ``ghz_amplitudes``, ``qft_like_amplitudes``, ``grover_amplitudes``: closed
  forms of the GHZ, swap-free QFT and Grover circuits of Sec. VI;
* ``mlp``: float64 reference of the fusion cost model's network.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Iterable, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-shared", "-fPIC", "-std=c11", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.orc_apply_gate.argtypes = [dp, ctypes.c_int, ctypes.c_int, i32p, dp]
        lib.orc_apply_gate.restype = ctypes.c_int
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.orc_apply_controlled_gate.argtypes = [dp, ctypes.c_int, ctypes.c_int, i32p, dp,
                                                  ctypes.c_uint64, ctypes.c_uint64]
        lib.orc_apply_controlled_gate.restype = ctypes.c_int
        lib.orc_apply_circuit.argtypes = [dp, ctypes.c_int, ctypes.c_int64, i32p, i32p, i64p, dp, u64p, u64p]
        lib.orc_apply_circuit.restype = ctypes.c_int
        lib.orc_init_basis.argtypes = [dp, ctypes.c_int, ctypes.c_uint64]
        lib.orc_norm_sq.argtypes = [dp, ctypes.c_int64]
        lib.orc_norm_sq.restype = ctypes.c_double
        lib.orc_compare.argtypes = [ctypes.POINTER(ctypes.c_float), dp, ctypes.c_int64, dp]
        lib.orc_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def threads() -> int:
    return _load().orc_threads()


def basis_state(n: int, x: int = 0) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    _load().orc_init_basis(_dp(psi), n, x)
    return psi


def apply_gate(psi: np.ndarray, n: int, qubits: Sequence[int], matrix: np.ndarray,
               cmask: int = 0, cval: int = 0) -> None:
    """In place: Eq. 4 for one gate, acting only where (index & cmask) == cval."""
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous and psi.size == 1 << n
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    u = np.ascontiguousarray(matrix, dtype=np.complex128)
    assert u.shape == (1 << len(q), 1 << len(q))
    rc = _load().orc_apply_controlled_gate(_dp(psi), n, len(q), q.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                           _dp(u), cmask, cval)
    if rc != 0:
        raise ValueError("oracle rejected gate %r" % (tuple(qubits),))


def apply_circuit(n: int, gates, init: int = 0, psi: np.ndarray | None = None) -> np.ndarray:
    """Start from |init> (or from ``psi``, in place) and apply every gate in order."""
    from circuits import to_arrays
    if psi is None:
        psi = basis_state(n, init)
    if len(gates) == 0:
        return psi
    a = to_arrays(gates)
    mats = np.ascontiguousarray(a["mats"])
    rc = _load().orc_apply_circuit(
        _dp(psi), n, len(a["k"]),
        a["k"].ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        np.ascontiguousarray(a["qubits"]).ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        a["mat_off"].ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        _dp(mats),
        a["cmask"].ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
        a["cval"].ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    if rc != 0:
        raise ValueError("oracle rejected the circuit")
    return psi


def norm_sq(psi: np.ndarray) -> float:
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    return float(_load().orc_norm_sq(_dp(psi), psi.size))


class CompareAcc:
    """Streaming accumulator for ``compare`` over chunks of a large state."""

    def __init__(self):
        self.mx = 0.0
        self.d2 = self.o2 = self.g2 = 0.0
        self.ip = 0j
        self.count = 0

    def add(self, gpu_c64: np.ndarray, ref_c128: np.ndarray) -> None:
        g = np.ascontiguousarray(gpu_c64, dtype=np.complex64)
        o = np.ascontiguousarray(ref_c128, dtype=np.complex128)
        assert g.size == o.size
        out = np.zeros(6)
        _load().orc_compare(g.view(np.float32).ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                            _dp(o), g.size, _dp(out))
        self.mx = max(self.mx, out[0])
        self.d2 += out[1]
        self.o2 += out[2]
        self.g2 += out[3]
        self.ip += complex(out[4], out[5])
        self.count += g.size

    def result(self) -> dict:
        fid = abs(self.ip) ** 2 / (self.o2 * self.g2) if self.o2 > 0 and self.g2 > 0 else 0.0
        return {
            "max_abs": self.mx,
            "rel_l2": float(np.sqrt(self.d2 / self.o2)) if self.o2 > 0 else float("nan"),
            "infidelity": 1.0 - fid,
            "norm_drift": abs(self.g2 - 1.0),
            "count": self.count,
        }


def compare(gpu_c64: np.ndarray, ref_c128: np.ndarray) -> dict:
    acc = CompareAcc()
    acc.add(gpu_c64, ref_c128)
    return acc.result()


def probe_projections(psi: np.ndarray, phases: np.ndarray) -> np.ndarray:
    """<phi_r|psi> for probe vectors phi_r with entries i^e (e = phases[r, i]
    in {0, 1, 2, 3}): sum_i conj(i^e) psi_i, formed as the FP64 sums of psi
    over each exponent class.  A few such projections check a whole state
    against a stored reference: a deviation d moves each one by <phi_r|d>,
    whose mean square is |d|^2."""
    psi = np.asarray(psi).astype(np.complex128, copy=False)
    unit = np.array([1, 1j, -1, -1j])
    out = np.zeros(phases.shape[0], dtype=np.complex128)
    for r in range(phases.shape[0]):
        re = np.bincount(phases[r], weights=psi.real, minlength=4)
        im = np.bincount(phases[r], weights=psi.imag, minlength=4)
        out[r] = np.sum(np.conj(unit) * (re + 1j * im))
    return out


# ---------------------------------------------------------------------------
# Independent brute force: the whole circuit operator (n <= 10).
# ---------------------------------------------------------------------------
def embed_gate(n: int, qubits: Sequence[int], matrix: np.ndarray) -> np.ndarray:
    """2^n x 2^n operator of a gate: kron(I, U) puts U on the low k bits
    (Eq. 3 with identities), then a permutation matrix moves bit j to
    qubits[j] and the remaining bits, in ascending order, above them."""
    k = len(qubits)
    d = 1 << n
    op_low = np.kron(np.eye(1 << (n - k), dtype=np.complex128), np.asarray(matrix, dtype=np.complex128))
    rest = [q for q in range(n) if q not in qubits]
    order = list(qubits) + rest            # bit b of the "low" index <- state bit order[b]
    perm = np.zeros(d, dtype=np.int64)     # perm[x] = low-index of state index x
    for x in range(d):
        y = 0
        for b, q in enumerate(order):
            y |= ((x >> q) & 1) << b
        perm[x] = y
    p = np.zeros((d, d), dtype=np.complex128)
    p[perm, np.arange(d)] = 1.0            # p @ e_x = e_{perm[x]}
    return p.T @ op_low @ p


def embed_controlled(n: int, qubits: Sequence[int], matrix: np.ndarray, cmask: int, cval: int) -> np.ndarray:
    """Controlled operator D E + (I - D): E = embed_gate(...) and D the
    diagonal projector onto basis states whose control bits equal cval (it
    commutes with E because controls and targets are disjoint)."""
    e = embed_gate(n, qubits, matrix)
    if cmask == 0:
        return e
    d = np.array([1.0 if (x & cmask) == cval else 0.0 for x in range(1 << n)])
    return d[:, None] * e + np.diag(1.0 - d)


def full_unitary(n: int, gates) -> np.ndarray:
    if n > 10:
        raise ValueError("brute force is limited to n <= 10")
    u = np.eye(1 << n, dtype=np.complex128)
    for g in gates:
        u = embed_controlled(n, g.qubits, g.matrix, getattr(g, "cmask", 0), getattr(g, "cval", 0)) @ u
    return u


def brute_force_state(n: int, gates, init: int = 0) -> np.ndarray:
    return full_unitary(n, gates)[:, init].copy()


# ---------------------------------------------------------------------------
# Measurement (the expectation-value kernel of Sec. IV reads the state without
# writing it back; these are the plain definitions of what such reads return).
# ---------------------------------------------------------------------------
_PX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_PY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_PZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)



def diagonal_factors(gates, idx) -> np.ndarray:
    """For diagonal gates applied in order, the factor each amplitude index
    in ``idx`` is multiplied by: by Eq. 4 a diagonal U maps c_i to
    U[l, l] c_i, l the index's bits at the gate's qubits (qubits[j] -> bit j),
    and only where the controls match; the product over the gates."""
    idx = np.asarray(idx, dtype=np.uint64)
    out = np.ones(idx.shape, dtype=np.complex128)
    for g in gates:
        u = np.asarray(g.matrix, dtype=np.complex128)
        assert np.count_nonzero(u - np.diag(np.diag(u))) == 0, "diagonal gates only"
        l = np.zeros(idx.shape, dtype=np.int64)
        for j, q in enumerate(g.qubits):
            l |= ((idx >> np.uint64(q)) & np.uint64(1)).astype(np.int64) << j
        f = np.diag(u)[l]
        cmask, cval = int(getattr(g, "cmask", 0) or 0), int(getattr(g, "cval", 0) or 0)
        if cmask:
            on = (idx & np.uint64(cmask)) == np.uint64(cval)
            f = np.where(on, f, 1.0)
        out *= f
    return out

def pauli_expectation(psi: np.ndarray, n: int, xmask: int, zmask: int) -> complex:
    """<psi|P|psi> for the Pauli string with X on the qubits of xmask only, Z
    on those of zmask only and Y on those of both: every letter is applied to
    a copy of psi as a one-qubit gate (Eq. 4), then the inner product is
    taken in FP64.  Not normalised by <psi|psi>."""
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    phi = psi.copy()
    for q in range(n):
        x, z = (xmask >> q) & 1, (zmask >> q) & 1
        if x or z:
            apply_gate(phi, n, (q,), _PY if (x and z) else (_PX if x else _PZ))
    return complex(np.vdot(psi, phi))


def marginal_probabilities(psi: np.ndarray, n: int, qubits: Sequence[int]) -> np.ndarray:
    """p[o] = sum of |c_i|^2 over the indices i whose bit qubits[j] is bit j
    of o (Eq. 1's Born weights summed over the unmeasured qubits)."""
    psi = np.asarray(psi)
    i = np.arange(1 << n, dtype=np.int64)
    o = np.zeros(1 << n, dtype=np.int64)
    for j, q in enumerate(qubits):
        o |= ((i >> q) & 1) << j
    w = psi.real.astype(np.float64) ** 2 + psi.imag.astype(np.float64) ** 2
    return np.bincount(o, weights=w, minlength=1 << len(qubits))


def sample_indices(psi: np.ndarray, uniforms: np.ndarray) -> np.ndarray:
    """Inverse-CDF sampling of basis states from p_i = |c_i|^2 (FP64): for
    each u in [0, 1) the smallest i with p_0 + ... + p_i > u * sum(p); a
    value past the end (rounding) takes the last index with p_i > 0."""
    psi = np.asarray(psi)
    w = psi.real.astype(np.float64) ** 2 + psi.imag.astype(np.float64) ** 2
    cdf = np.cumsum(w)
    idx = np.searchsorted(cdf, np.asarray(uniforms, dtype=np.float64) * cdf[-1], side="right")
    last = int(np.flatnonzero(w)[-1])
    return np.minimum(idx, last).astype(np.int64)


# ---------------------------------------------------------------------------
# Closed forms (Sec. VI circuits).
# ---------------------------------------------------------------------------
def ghz_amplitudes(n: int, idx: Iterable[int]) -> np.ndarray:
    """GHZ from |0..0>: 1/sqrt(2) at indices 0 and 2^n - 1, zero elsewhere."""
    idx = np.asarray(list(idx), dtype=np.uint64)
    out = np.zeros(idx.size, dtype=np.complex128)
    out[(idx == 0) | (idx == np.uint64((1 << n) - 1))] = 1 / np.sqrt(2)
    return out


def bit_reverse(y: np.ndarray, n: int) -> np.ndarray:
    y = np.asarray(y, dtype=np.uint64)
    r = np.zeros_like(y)
    for t in range(n):
        r |= ((y >> np.uint64(t)) & np.uint64(1)) << np.uint64(n - 1 - t)
    return r


def qft_like_amplitudes(n: int, x: int, idx) -> np.ndarray:
    """Swap-free QFT of |x>: amp(y) = 2^{-n/2} exp(2 pi i (x * rev_n(y) mod 2^n) / 2^n).
    The phase numerator is formed exactly in 64-bit integers."""
    y = np.asarray(idx, dtype=np.uint64)
    mask = np.uint64((1 << n) - 1) if n < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    num = (np.uint64(x) * bit_reverse(y, n)) & mask
    phase = 2.0 * np.pi * num.astype(np.float64) / float(1 << n)
    return np.exp(1j * phase) * 2.0 ** (-n / 2)


def grover_amplitudes(n: int, marked: int, iterations: int, idx) -> np.ndarray:
    """Grover search from |0..0> after H on every qubit and t iterations of
    (phase flip of |marked>, then I - 2|s><s|): with sin(theta) = 2^(-n/2)
    the marked amplitude is (-1)^t sin((2t+1) theta) and every other one is
    (-1)^t cos((2t+1) theta) / sqrt(2^n - 1).  The sign is that of the
    diffusion written as -(2|s><s| - I), which H X MCZ X H implements."""
    idx = np.asarray(list(idx) if not isinstance(idx, np.ndarray) else idx, dtype=np.int64)
    th = np.arcsin(2.0 ** (-n / 2))
    a = np.sin((2 * iterations + 1) * th)
    b = np.cos((2 * iterations + 1) * th) / np.sqrt(2.0 ** n - 1)
    s = (-1.0) ** iterations
    return np.where(idx == marked, s * a, s * b).astype(np.complex128)
