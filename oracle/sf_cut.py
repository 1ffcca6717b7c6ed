"""Exact amplitudes of a circuit too large for one complex128 state, by cutting
it into two halves -- TEST INFRASTRUCTURE ONLY (same rules as the rest of
``oracle``: only tests, the smoke check and the benchmark's CPU leg use it).

The qubits are split into a left set L and a right set R.  Every gate acts
inside L, inside R, or on one qubit a of L and one qubit b of R.  A crossing
gate must be block-diagonal in a (CZ, CP, any controlled gate whose control
is a), so that it is a sum of two product terms

    G = |0><0|_a (x) G_0(b)  +  |1><1|_a (x) G_1(b),

with G_v the 2x2 block of G where a = v (for CZ: G_0 = I, G_1 = Z).
Expanding every crossing gate this way writes the circuit operator as a sum
over paths p in {0,1}^c (c crossing gates) of products A_p (x) B_p, where A_p
is the left circuit with the projector |p_i><p_i| in place of crossing gate
i and B_p the right circuit with G_{p_i} in its place.  Both act on a product
basis input |x_L>|x_R>, so

    psi(x) = sum_p  (A_p |x_L>)[x's L bits] * (B_p |x_R>)[x's R bits].

Each half is simulated gate by gate with the plain Eq. 4 oracle
(``oracle.apply_circuit``: the projectors and blocks are ordinary 1-qubit
matrices to it), one path at a time.  Nothing is fused, truncated or
reordered; paths are summed in ascending order of p, in fixed chunks, so the
result does not depend on the number of worker processes.

Parity pins (tests/test_oracle_cut.py): on ladders small enough for the full
oracle and for the Kronecker-product brute force, every amplitude agrees to
1e-12; a planted swap of the two blocks is caught.
"""
from __future__ import annotations

import os
from typing import List, Sequence, Tuple

import numpy as np

_P = (np.diag([1.0, 0.0]).astype(np.complex128), np.diag([0.0, 1.0]).astype(np.complex128))


def crossing_blocks(gate, left: set) -> Tuple[int, int, Tuple[np.ndarray, np.ndarray]]:
    """(a, b, (G_0, G_1)) of a crossing gate: a its qubit in L, b its qubit
    in R, G_v the block of its matrix on b where a's bit is v.  Raises if the
    gate is not a controls-free 2-qubit gate block-diagonal in a."""
    if gate.k != 2 or gate.controls:
        raise ValueError("a crossing gate must be a 2-qubit gate without controls")
    q0, q1 = gate.qubits
    u = np.asarray(gate.matrix, dtype=np.complex128)
    # local index l = bit(q0) + 2 * bit(q1)
    if q0 in left:
        a, b, abit = q0, q1, 0
    else:
        a, b, abit = q1, q0, 1
    blocks = []
    for v in (0, 1):
        g = np.zeros((2, 2), dtype=np.complex128)
        for rb in (0, 1):
            for cb in (0, 1):
                r = (v << abit) | (rb << (1 - abit))
                c = (v << abit) | (cb << (1 - abit))
                g[rb, cb] = u[r, c]
        blocks.append(g)
    # block-diagonal in a: every entry that changes a's bit is zero
    for r in range(4):
        for c in range(4):
            if ((r >> abit) & 1) != ((c >> abit) & 1) and u[r, c] != 0:
                raise ValueError("crossing gate is not block-diagonal in its left qubit")
    return a, b, (blocks[0], blocks[1])


def split_circuit(gates: Sequence, left: Sequence[int], right: Sequence[int]):
    """Label every gate 'L', 'R' or 'X' (crossing); return the labelled list
    and the crossing gates' (a, b, blocks)."""
    ls, rs = set(left), set(right)
    out, cross = [], []
    for g in gates:
        qs = set(g.qubits) | set(g.controls)
        if qs <= ls:
            out.append(("L", g))
        elif qs <= rs:
            out.append(("R", g))
        else:
            out.append(("X", g))
            cross.append(crossing_blocks(g, ls))
    return out, cross


def _relabel(g, pos):
    import circuits as C
    return C.Gate(tuple(pos[q] for q in g.qubits), g.matrix, tuple(pos[q] for q in g.controls), g.control_values)


def path_circuits(labelled, cross, p: int, lpos: dict, rpos: dict, blocks_fn=None):
    """Left and right gate lists of path p (bit i of p picks term i of the
    i-th crossing gate)."""
    import circuits as C
    lg: List = []
    rg: List = []
    i = 0
    for side, g in labelled:
        if side == "L":
            lg.append(_relabel(g, lpos))
        elif side == "R":
            rg.append(_relabel(g, rpos))
        else:
            a, b, blocks = cross[i]
            if blocks_fn is not None:
                blocks = blocks_fn(blocks)
            v = (p >> i) & 1
            lg.append(C.Gate((lpos[a],), _P[v]))
            rg.append(C.Gate((rpos[b],), blocks[v]))
            i += 1
    return lg, rg


def _sub_index(idx: np.ndarray, qubits: Sequence[int]) -> np.ndarray:
    out = np.zeros(idx.size, dtype=np.int64)
    for i, q in enumerate(qubits):
        out |= ((idx >> np.uint64(q)) & np.uint64(1)).astype(np.int64) << i
    return out


def _paths_chunk(args):
    gates, left, right, idx, init, p0, p1, blocks_fn = args
    import oracle
    labelled, cross = split_circuit(gates, left, right)
    lpos = {q: i for i, q in enumerate(left)}
    rpos = {q: i for i, q in enumerate(right)}
    il, ir = _sub_index(idx, left), _sub_index(idx, right)
    xl = int(_sub_index(np.array([init], dtype=np.uint64), left)[0])
    xr = int(_sub_index(np.array([init], dtype=np.uint64), right)[0])
    acc = np.zeros(idx.size, dtype=np.complex128)
    for p in range(p0, p1):
        lg, rg = path_circuits(labelled, cross, p, lpos, rpos, blocks_fn)
        a = oracle.apply_circuit(len(left), lg, init=xl)
        b = oracle.apply_circuit(len(right), rg, init=xr)
        acc += a[il] * b[ir]
    return acc


def _worker_init():
    os.environ["OMP_NUM_THREADS"] = "1"


def cut_amplitudes(n: int, gates: Sequence, left: Sequence[int], idx, init: int = 0,
                   workers: int = 1, chunk: int = 64, blocks_fn=None) -> np.ndarray:
    """Amplitudes psi[idx] of ``gates`` applied to |init> on n qubits, by the
    two-way cut described above.  ``left`` lists the L qubits (R is the rest,
    ascending).  ``workers`` > 1 spreads fixed chunks of paths over that
    many single-threaded processes.  ``blocks_fn`` exists only so that a test
    can plant a mistake in the decomposition."""
    left = list(left)
    right = [q for q in range(n) if q not in set(left)]
    idx = np.asarray(idx, dtype=np.uint64)
    _, cross = split_circuit(gates, left, right)
    n_paths = 1 << len(cross)
    bounds = [(p, min(p + chunk, n_paths)) for p in range(0, n_paths, chunk)]
    jobs = [(list(gates), left, right, idx, init, p0, p1, blocks_fn) for p0, p1 in bounds]
    if workers <= 1:
        parts = [_paths_chunk(j) for j in jobs]
    else:
        import concurrent.futures as cf
        import multiprocessing as mp
        with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn"), initializer=_worker_init) as ex:
            parts = list(ex.map(_paths_chunk, jobs))
    out = np.zeros(idx.size, dtype=np.complex128)
    for part in parts:  # fixed order: ascending chunks of paths
        out += part
    return out
