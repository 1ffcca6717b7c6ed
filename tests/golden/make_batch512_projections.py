"""Writes tests/golden/batch512_projections.npz: for each of the 512
batched ansatz circuits (qubit counts uniform in [10, 22], 8 layers of
RY RZ per qubit each followed by a CNOT ladder, seed 0, |0..0>), the oracle's
state (Eq. 4, gate by gate, complex128) projected on 4 seeded probe vectors
with entries i^e (circuits.probe_phases, seed 1000 + circuit index): p_r =
sum_i conj(phi_r,i) psi_i, and the state's norm.  A GPU run of the whole
batch is then checked through the same projections of its own states.

    python tests/golden/make_batch512_projections.py

Minutes of CPU work (the full states of every circuit).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
OUT = os.path.join(HERE, "batch512_projections.npz")
PROBES = 4


def main():
    import circuits as C
    import oracle
    ns, circs = C.batched_ansatz(512, seed=0)
    proj = np.zeros((512, PROBES), dtype=np.complex128)
    norms = np.zeros(512)
    t0 = time.perf_counter()
    for c, (n, g) in enumerate(zip(ns, circs)):
        psi = oracle.apply_circuit(n, g)
        proj[c] = oracle.probe_projections(psi, C.probe_phases(n, 1000 + c, PROBES))
        norms[c] = oracle.norm_sq(psi)
        if c % 64 == 63:
            print("%d/512 circuits, %.0f s" % (c + 1, time.perf_counter() - t0), flush=True)
    np.savez(OUT, ns=np.array(ns), proj=proj, norm_sq=norms, probes=np.int64(PROBES))
    print("wrote %s in %.0f s" % (OUT, time.perf_counter() - t0))


if __name__ == "__main__":
    main()
