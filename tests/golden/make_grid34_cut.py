"""Writes tests/golden/grid34_d24_s0_cut.npz: exact amplitudes of the
34-qubit 2x17 random grid circuit (depth 24, seed 0, |0..0>) -- the circuit
the benchmark runs -- on a sampled index set, computed only by the oracle.

The state (256 GiB in complex128) is never formed: the circuit is cut between
lattice columns 8 and 9 (qubits of columns 0..8 on the left, 18 qubits;
columns 9..16 on the right, 16 qubits).  The 12 CZs on the two couplers that
cross the cut each split into two product terms, so the amplitudes are a sum
over 4096 paths of products of an 18-qubit and a 16-qubit state, each
simulated gate by gate by the plain oracle (oracle/sf_cut.py).

Sample: 4096 indices drawn uniformly (PCG64 seed 34, duplicates removed,
sorted) plus the contiguous block [5 * 2^30, 5 * 2^30 + 2^16).

    python tests/golden/make_grid34_cut.py [--workers 8]

About 10 minutes on 8 cores.
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

ROWS, COLS, DEPTH, SEED = 2, 17, 24, 0
CUT_COL = 9
SAMPLE_SEED = 34
BLOCK_START = 5 << 30
BLOCK_LEN = 1 << 16
OUT = os.path.join(HERE, "grid34_d24_s0_cut.npz")


def sample_index_set(n):
    rng = np.random.Generator(np.random.PCG64(SAMPLE_SEED))
    rand = np.unique(rng.integers(0, 1 << n, size=4096, dtype=np.uint64))
    block = np.arange(BLOCK_START, BLOCK_START + BLOCK_LEN, dtype=np.uint64)
    return rand, block


def main():
    import circuits as C
    from oracle import sf_cut
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    n = ROWS * COLS
    gates = C.grid_circuit(ROWS, COLS, DEPTH, seed=SEED)
    left = [r * COLS + c for r in range(ROWS) for c in range(CUT_COL)]
    rand, block = sample_index_set(n)
    idx = np.concatenate([rand, block])
    t0 = time.perf_counter()
    amp = sf_cut.cut_amplitudes(n, gates, left, idx, workers=args.workers)
    dt = time.perf_counter() - t0
    np.savez(OUT, idx=idx, amp=amp, n_random=np.int64(rand.size),
             circuit=np.array("grid %dx%d depth %d seed %d, |0..0>" % (ROWS, COLS, DEPTH, SEED)),
             left=np.array(left, dtype=np.int32))
    print("wrote %s: %d amplitudes, sum |a|^2 over the block = %.6e, %.0f s on %d workers"
          % (OUT, idx.size, float(np.sum(np.abs(amp[rand.size:]) ** 2)), dt, args.workers))


if __name__ == "__main__":
    main()
