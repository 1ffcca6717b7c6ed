"""Structural checks of a fused partition returned by sv_fuse (shared by the
fusion tests).  A block is one fused gate, or with controls 2^c fused gates
on the same targets and controls, one per control value; block_of names the
first fused gate of each gate's block."""
import numpy as np


def blocks_of(fused, block_of):
    """[(first, last + 1)] fused-gate ranges of the blocks, in order."""
    starts = sorted(set(int(b) for b in block_of))
    ends = starts[1:] + [len(fused)]
    return list(zip(starts, ends))


def check_partition(gates, fused, block_of, max_k):
    assert len(block_of) == len(gates)
    ranges = blocks_of(fused, block_of)
    assert ranges and ranges[0][0] == 0  # every fused gate belongs to a block
    for a, b in ranges:
        first = fused[a]
        assert 1 <= first.k <= max_k
        assert list(first.qubits) == sorted(first.qubits)
        c = len(first.controls)
        assert b - a == 1 << c, (a, b, c)
        assert not set(first.controls) & set(first.qubits)
        vals = set()
        for f in fused[a:b]:
            assert f.qubits == first.qubits and tuple(f.controls) == tuple(first.controls)
            vals.add(tuple(f.control_values) if f.controls else ())
        assert len(vals) == b - a  # one fused gate per control value
    for i, g in enumerate(gates):  # every gate's qubits are inside its block
        f = fused[block_of[i]]
        assert set(g.qubits) | set(g.controls) <= set(f.qubits) | set(f.controls)
    n = max(q for g in gates for q in g.qubits) + 1
    for q in range(n):  # per-qubit program order is preserved
        seq = [int(block_of[i]) for i, g in enumerate(gates) if q in g.qubits]
        assert seq == sorted(seq)
    return len(ranges)


def sweeps(block_of) -> int:
    """Number of state sweeps (blocks) of a partition."""
    return len(set(np.asarray(block_of).tolist()))
