"""Writes tests/golden/grid30_d20_s0.npz: amplitudes of the 30-qubit 5x6
random grid circuit (depth 20, seed 0, |0..0>) on a sampled index set,
computed only by the oracle (the full 2^30-amplitude complex128 state, 16 GiB,
gate by gate, Eq. 4).

Sample: 8192 indices drawn uniformly (PCG64 seed 30, duplicates removed,
sorted) plus the contiguous block [3 * 2^27, 3 * 2^27 + 2^16).  The file also
records the exact norm of the oracle state.

    python tests/golden/make_grid30_samples.py

Needs about 17 GiB of host memory; tens of minutes on 8 cores.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

ROWS, COLS, DEPTH, SEED = 5, 6, 20, 0
SAMPLE_SEED = 30
BLOCK_START = 3 << 27
BLOCK_LEN = 1 << 16
OUT = os.path.join(HERE, "grid30_d20_s0.npz")


def sample_index_set(n):
    rng = np.random.Generator(np.random.PCG64(SAMPLE_SEED))
    rand = np.unique(rng.integers(0, 1 << n, size=8192, dtype=np.uint64))
    block = np.arange(BLOCK_START, BLOCK_START + BLOCK_LEN, dtype=np.uint64)
    return rand, block


def main():
    import circuits as C
    import oracle
    n = ROWS * COLS
    gates = C.grid_circuit(ROWS, COLS, DEPTH, seed=SEED)
    rand, block = sample_index_set(n)
    idx = np.concatenate([rand, block])
    t0 = time.perf_counter()
    psi = oracle.basis_state(n, 0)
    for i in range(0, len(gates), 50):
        oracle.apply_circuit(n, gates[i:i + 50], psi=psi)
        print("%d/%d gates, %.0f s" % (min(i + 50, len(gates)), len(gates), time.perf_counter() - t0), flush=True)
    amp = psi[idx.astype(np.int64)].copy()
    norm = oracle.norm_sq(psi)
    np.savez(OUT, idx=idx, amp=amp, n_random=np.int64(rand.size), norm_sq=np.float64(norm),
             circuit=np.array("grid %dx%d depth %d seed %d, |0..0>" % (ROWS, COLS, DEPTH, SEED)))
    print("wrote %s: %d amplitudes, norm %.15f, %.0f s on %d threads"
          % (OUT, idx.size, norm, time.perf_counter() - t0, oracle.threads()))


if __name__ == "__main__":
    main()
