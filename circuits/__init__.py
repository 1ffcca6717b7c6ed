"""Seeded synthetic circuit generators.

This module is the only code shared by the CPU oracle, the tests and the
benchmark.  It produces gate lists (qubits + dense matrix), seeded random
state vectors and seeded uniforms for sampling, and nothing else: no gate is
ever applied to a state here.

Conventions (fixed for the whole project):

* qubit ``q`` is bit ``q`` of the amplitude index (little-endian, 0-based;
  the paper counts qubits from 1 with stride ``2^i``, Sec. IV-C);
* a gate is ``Gate(qubits, matrix)`` with ``matrix`` a ``2^k x 2^k``
  complex128 array, row-major, acting as ``w = matrix @ v`` on the group
  vector of Eq. 4, where local bit ``j`` of the row/column index is the
  state bit ``qubits[j]``.  Qubits are *not* required to be sorted.

Every random draw uses ``numpy.random.Generator(PCG64(seed))`` so that the
oracle and the GPU path consume byte-identical circuits.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Gate", "H", "X", "Y", "Z", "SQRT_X", "SQRT_Y", "SQRT_W", "CZ", "CNOT",
    "CP", "RY", "RZ", "principal_sqrt_involution", "haar_unitary",
    "grid_circuit", "grid_couplers", "qft_like_circuit", "ghz_circuit",
    "batched_ansatz", "ansatz_circuit", "mirror_circuit", "random_circuit",
    "grover_circuit", "quantum_volume_circuit", "synthetic_fusion_circuit",
    "to_arrays", "from_arrays", "save_npz", "load_npz", "count_gates",
    "random_state_c64", "uniforms", "probe_phases",
]


@dataclass(frozen=True)
class Gate:
    """A k-qubit gate: local bit j of the matrix index is state bit qubits[j].

    ``controls`` (disjoint from ``qubits``) restrict the gate to the basis
    states whose control bits equal ``control_values`` (all ones when None);
    ``k`` counts the target qubits only."""

    qubits: Tuple[int, ...]
    matrix: np.ndarray
    controls: Tuple[int, ...] = ()
    control_values: Optional[Tuple[int, ...]] = None

    @property
    def k(self) -> int:
        return len(self.qubits)

    @property
    def cmask(self) -> int:
        m = 0
        for c in self.controls:
            m |= 1 << c
        return m

    @property
    def cval(self) -> int:
        vals = self.control_values if self.control_values is not None else (1,) * len(self.controls)
        v = 0
        for c, b in zip(self.controls, vals):
            v |= (int(b) & 1) << c
        return v

    def dagger(self) -> "Gate":
        return Gate(self.qubits, np.ascontiguousarray(self.matrix.conj().T), self.controls, self.control_values)


# ---------------------------------------------------------------------------
# Gate definitions.  Hadamard as printed in Sec. II-A; the square-root gates
# are principal square roots of the involutions X, Y and W = (X + Y)/sqrt(2).
# ---------------------------------------------------------------------------
_S2 = np.sqrt(2.0)

H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / _S2
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
W = (X + Y) / _S2


def principal_sqrt_involution(g: np.ndarray) -> np.ndarray:
    """Principal square root of an involution G (G @ G = I, eigenvalues +-1).

    sqrt(G) = (1+i)/2 * I + (1-i)/2 * G; squaring gives G because
    ((1+i)/2)^2 + ((1-i)/2)^2 = 0 and 2 * (1+i)/2 * (1-i)/2 = 1.
    """
    eye = np.eye(g.shape[0], dtype=np.complex128)
    return 0.5 * (1 + 1j) * eye + 0.5 * (1 - 1j) * g


SQRT_X = principal_sqrt_involution(X)
SQRT_Y = principal_sqrt_involution(Y)
SQRT_W = principal_sqrt_involution(W)
SINGLE_QUBIT_GRID_SET = (SQRT_X, SQRT_Y, SQRT_W)

CZ = np.diag([1, 1, 1, -1]).astype(np.complex128)

# CNOT with qubits=(control, target): local bit 0 = control, bit 1 = target.
CNOT = np.zeros((4, 4), dtype=np.complex128)
CNOT[0, 0] = CNOT[2, 2] = 1.0   # control = 0: identity
CNOT[3, 1] = CNOT[1, 3] = 1.0   # control = 1: flip the target


def CP(theta: float) -> np.ndarray:
    """Controlled phase: phase e^{i theta} on |11>."""
    return np.diag([1, 1, 1, np.exp(1j * theta)]).astype(np.complex128)


def RY(theta: float) -> np.ndarray:
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def RZ(phi: float) -> np.ndarray:
    return np.diag([np.exp(-0.5j * phi), np.exp(0.5j * phi)]).astype(np.complex128)


def haar_unitary(k: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random 2^k x 2^k unitary (QR of a complex Ginibre matrix, phases fixed)."""
    d = 1 << k
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / _S2
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return np.ascontiguousarray(q * ph[None, :])


# ---------------------------------------------------------------------------
# Circuits
# ---------------------------------------------------------------------------
def grid_couplers(rows: int, cols: int, pattern: int) -> List[Tuple[int, int]]:
    """Nearest-neighbour coupler pattern ``pattern`` (0..3) on a rows x cols lattice.

    Lattice qubit (r, c) is q = r * cols + c.  Patterns: 0 horizontal edges
    (r,c)-(r,c+1) with r+c even, 1 horizontal with r+c odd, 2 vertical edges
    (r,c)-(r+1,c) with r+c even, 3 vertical with r+c odd.  Each is a matching.
    """
    edges = []
    horizontal = pattern in (0, 1)
    parity = pattern % 2
    for r in range(rows):
        for c in range(cols):
            if (r + c) % 2 != parity:
                continue
            if horizontal and c + 1 < cols:
                edges.append((r * cols + c, r * cols + c + 1))
            if not horizontal and r + 1 < rows:
                edges.append((r * cols + c, (r + 1) * cols + c))
    return edges


def grid_circuit(rows: int, cols: int, depth: int, seed: int) -> List[Gate]:
    """Random grid circuit: per cycle t one gate from {sqrtX, sqrtY, sqrtW} on
    every qubit (uniform, seeded), then CZ on coupler pattern t mod 4."""
    n = rows * cols
    rng = np.random.Generator(np.random.PCG64(seed))
    choice = rng.integers(0, 3, size=(depth, n))
    gates: List[Gate] = []
    for t in range(depth):
        for q in range(n):
            gates.append(Gate((q,), SINGLE_QUBIT_GRID_SET[int(choice[t, q])]))
        for a, b in grid_couplers(rows, cols, t % 4):
            gates.append(Gate((a, b), CZ))
    return gates


def qft_like_circuit(n: int) -> List[Gate]:
    """QFT without the final swaps: for t = n-1 .. 0, H(q_t) then
    CP(pi / 2^j) on (q_t, q_{t-j}) for j = 1 .. t."""
    gates: List[Gate] = []
    for t in range(n - 1, -1, -1):
        gates.append(Gate((t,), H))
        for j in range(1, t + 1):
            gates.append(Gate((t, t - j), CP(np.pi / (2 ** j))))
    return gates


def qft_input_basis(n: int, seed: int) -> int:
    """Seeded basis-state input x for the QFT-like circuit."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return int(rng.integers(0, 2 ** n, dtype=np.uint64))


def ghz_circuit(n: int) -> List[Gate]:
    """H on qubit 0, then CNOT(q_i -> q_{i+1}) for i = 0 .. n-2 (n gates)."""
    gates = [Gate((0,), H)]
    for i in range(n - 1):
        gates.append(Gate((i, i + 1), CNOT))
    return gates


def ansatz_circuit(n: int, angles: np.ndarray) -> List[Gate]:
    """Layers of RY(theta) RZ(phi) on every qubit, each followed by a CNOT ladder."""
    layers = angles.shape[0]
    gates: List[Gate] = []
    for layer in range(layers):
        for q in range(n):
            gates.append(Gate((q,), RY(float(angles[layer, q, 0]))))
            gates.append(Gate((q,), RZ(float(angles[layer, q, 1]))))
        for i in range(n - 1):
            gates.append(Gate((i, i + 1), CNOT))
    return gates


def batched_ansatz(n_circuits: int, seed: int, n_min: int = 10, n_max: int = 22,
                   layers: int = 8) -> Tuple[List[int], List[List[Gate]]]:
    """Independent parameterised circuits with qubit counts uniform in [n_min, n_max]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = [int(v) for v in rng.integers(n_min, n_max + 1, size=n_circuits)]
    circs = []
    for n in ns:
        angles = rng.uniform(0.0, 2 * np.pi, size=(layers, n, 2))
        circs.append(ansatz_circuit(n, angles))
    return ns, circs


def mirror_circuit(gates: Sequence[Gate]) -> List[Gate]:
    """C followed by C^dagger (reverse order, conjugate-transposed matrices)."""
    return list(gates) + [g.dagger() for g in reversed(gates)]


def random_circuit(n: int, n_gates: int, max_k: int, seed: int,
                   min_k: int = 1) -> List[Gate]:
    """Haar-random k-qubit gates (k uniform in [min_k, max_k]) on random qubit
    subsets in random (unsorted) order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gates = []
    for _ in range(n_gates):
        k = int(rng.integers(min_k, min(max_k, n) + 1))
        qs = tuple(int(v) for v in rng.permutation(n)[:k])
        gates.append(Gate(qs, haar_unitary(k, rng)))
    return gates


def synthetic_fusion_circuit(n: int, n_gates: int, seed: int, q_min: int = 0) -> List[Gate]:
    """Synthetic one-qubit-gate benchmark in the spirit of Sec. VII-B: random
    one-qubit unitaries on qubits >= q_min, no controlled gates."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gates = []
    for _ in range(n_gates):
        q = int(rng.integers(q_min, n))
        gates.append(Gate((q,), haar_unitary(1, rng)))
    return gates


def grover_circuit(n: int, marked: int, iterations: int) -> List[Gate]:
    """Grover search on n qubits: H on all, then ``iterations`` x (oracle:
    X-conjugated multi-controlled Z marking ``marked``; diffusion:
    H X MCZ X H).  The multi-controlled Z is a Z on qubit n-1 controlled by
    qubits 0..n-2 (Table 2's multi-controlled Toffoli, with the target's H
    conjugation folded in)."""
    if n < 2:
        raise ValueError("Grover needs n >= 2")
    qs = tuple(range(n))
    mcz = Gate((n - 1,), Z, tuple(range(n - 1)))
    gates = [Gate((q,), H) for q in qs]
    for _ in range(iterations):
        for q in qs:
            if not (marked >> q) & 1:
                gates.append(Gate((q,), X))
        gates.append(mcz)
        for q in qs:
            if not (marked >> q) & 1:
                gates.append(Gate((q,), X))
        gates += [Gate((q,), H) for q in qs]
        gates += [Gate((q,), X) for q in qs]
        gates.append(mcz)
        gates += [Gate((q,), X) for q in qs]
        gates += [Gate((q,), H) for q in qs]
    return gates


def quantum_volume_circuit(n: int, depth: int, seed: int) -> List[Gate]:
    """Quantum-volume style: per layer a random qubit permutation is paired up
    and each pair gets random one-qubit unitaries, a CNOT, and random
    one-qubit unitaries again."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gates = []
    for _ in range(depth):
        perm = rng.permutation(n)
        for i in range(0, n - 1, 2):
            a, b = int(perm[i]), int(perm[i + 1])
            gates.append(Gate((a,), haar_unitary(1, rng)))
            gates.append(Gate((b,), haar_unitary(1, rng)))
            gates.append(Gate((a, b), CNOT))
            gates.append(Gate((a,), haar_unitary(1, rng)))
            gates.append(Gate((b,), haar_unitary(1, rng)))
    return gates


def count_gates(gates: Sequence[Gate]) -> dict:
    out: dict = {}
    for g in gates:
        out[g.k] = out.get(g.k, 0) + 1
    return out


# ---------------------------------------------------------------------------
# Serialisation: flat arrays, the layout both sides read.
# ---------------------------------------------------------------------------
def to_arrays(gates: Sequence[Gate]) -> dict:
    g = len(gates)
    ks = np.zeros(g, dtype=np.int32)
    qubits = np.full((g, 6), -1, dtype=np.int32)
    offs = np.zeros(g + 1, dtype=np.int64)
    for i, gate in enumerate(gates):
        ks[i] = gate.k
        qubits[i, : gate.k] = gate.qubits
        offs[i + 1] = offs[i] + (1 << (2 * gate.k))
    mats = np.zeros(int(offs[-1]), dtype=np.complex128)
    cmask = np.zeros(g, dtype=np.uint64)
    cval = np.zeros(g, dtype=np.uint64)
    for i, gate in enumerate(gates):
        mats[offs[i]:offs[i + 1]] = np.asarray(gate.matrix, dtype=np.complex128).reshape(-1)
        if gate.controls:
            cmask[i] = gate.cmask
            cval[i] = gate.cval
    return {"k": ks, "qubits": qubits, "mat_off": offs, "mats": mats, "cmask": cmask, "cval": cval}


def from_arrays(a: dict) -> List[Gate]:
    gates = []
    for i in range(len(a["k"])):
        k = int(a["k"][i])
        m = np.asarray(a["mats"][a["mat_off"][i]:a["mat_off"][i + 1]]).reshape(1 << k, 1 << k)
        cm = int(a["cmask"][i]) if "cmask" in a else 0
        cv = int(a["cval"][i]) if "cval" in a else 0
        ctl = tuple(q for q in range(64) if (cm >> q) & 1)
        gates.append(Gate(tuple(int(v) for v in a["qubits"][i, :k]), np.ascontiguousarray(m), ctl,
                          tuple((cv >> q) & 1 for q in ctl) if ctl else None))
    return gates


def save_npz(path, gates: Sequence[Gate], **meta) -> None:
    np.savez(path, **to_arrays(gates), **{k: np.asarray(v) for k, v in meta.items()})


def load_npz(path) -> List[Gate]:
    with np.load(path, allow_pickle=False) as f:
        return from_arrays({k: f[k] for k in ("k", "qubits", "mat_off", "mats", "cmask", "cval") if k in f})


def random_state_c64(n: int, seed: int) -> np.ndarray:
    """A seeded random normalised complex64 state (Gaussian real and
    imaginary parts, scaled in float64, then rounded to complex64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    v /= np.sqrt(np.sum(np.abs(v) ** 2))
    return v.astype(np.complex64)


def uniforms(count: int, seed: int) -> np.ndarray:
    """Seeded uniforms in [0, 1) (float64) for sampling."""
    return np.random.Generator(np.random.PCG64(seed)).random(count)


def probe_phases(n: int, seed: int, count: int = 4) -> np.ndarray:
    """Seeded exponents e in {0, 1, 2, 3}, shape (count, 2^n), uint8: the
    probe vectors phi_r with entries i^e used to compare two states through a
    few inner products <phi_r|psi> (a deviation d shows up in them with
    E|<phi|d>|^2 = |d|^2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, 4, size=(count, 1 << n), dtype=np.uint8)
