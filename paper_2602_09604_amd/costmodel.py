"""Timing corpus and GPU training of the fusion cost model.

The simulator times its own passes: for sampled (k, target qubits, n,
precision) one gate is applied through sv_apply_circuit with per-pass HIP
event timing, and the target is ln(pass seconds * 1e9 / 2^n).  Target sets
come half from uniform random subsets and half from the blocks that greedy
fusion builds on random grid circuits (the masks the partition search will
actually score).  Training runs the library's MLP kernels (sv_mlp_*); the
trained network is installed for SV_FUSE_LEARNED and can be saved.
"""
from __future__ import annotations

import math
import time
from typing import Dict, Sequence

import numpy as np

from . import sv

PRECISIONS = ("fp32_valu", "bf16x3", "fp16x3", "fp32_mfma")


def _grid_like_blocks(n: int, rng: np.random.Generator):
    """Qubit sets of greedily fused blocks of a random grid-like circuit on n qubits."""
    import circuits as C
    rows = 2 if n % 2 == 0 else 1
    cols = n // rows
    gates = C.grid_circuit(rows, cols, 6, seed=int(rng.integers(1 << 30)))
    if rows * cols < n:
        gates = [C.Gate(tuple(q + 1 for q in g.qubits), g.matrix) for g in gates]
    K = int(rng.integers(2, 7))
    fused, _ = sv.sv_fuse(gates, n, sv.make_opts(max_k=K))
    return [f.qubits for f in fused]


def collect_corpus(samples: int = 2400, ns: Sequence[int] = (26, 28, 30),
                   precisions: Sequence[str] = PRECISIONS, seed: int = 0, repeats: int = 3,
                   log=None) -> Dict[str, np.ndarray]:
    """Time `samples` single passes; returns X [samples, 40], y [samples] and the raw fields."""
    import circuits as C
    rng = np.random.Generator(np.random.PCG64(seed))
    per_n = [samples // len(ns) + (1 if i < samples % len(ns) else 0) for i in range(len(ns))]
    X, y, ks, masks, nn, precs, secs = [], [], [], [], [], [], []
    t0 = time.perf_counter()
    for n, count in zip(ns, per_n):
        st = sv.State(n)
        pool = []
        try:
            for i in range(count):
                if not pool:
                    pool = _grid_like_blocks(n, rng)
                if i % 3 == 0:
                    k = int(rng.integers(1, 7))
                    qs = tuple(int(q) for q in rng.permutation(n)[:k])
                else:
                    qs = pool.pop(int(rng.integers(len(pool))))
                    k = len(qs)
                prec = precisions[int(rng.integers(len(precisions)))]
                g = [C.Gate(qs, C.haar_unitary(k, rng))]
                best = math.inf
                for _ in range(repeats):
                    s = st.apply_circuit(g, fusion="none", precision=prec, timing=True)
                    best = min(best, s["gpu_s"])
                pid = sv.PRECISIONS[prec]
                X.append(sv.sv_cost_features(k, qs, n, pid))
                y.append(math.log(best * 1e9 / (1 << n)))
                ks.append(k)
                masks.append(sum(1 << q for q in qs))
                nn.append(n)
                precs.append(pid)
                secs.append(best)
                if (i + 1) % 200 == 0 and log:
                    log("corpus n=%d: %d/%d (%.1f s)" % (n, i + 1, count, time.perf_counter() - t0))
                if (i + 1) % 64 == 0:
                    st.set_basis(0)  # keep the state normalised and finite
        finally:
            st.free()
    return {"X": np.array(X, dtype=np.float32), "y": np.array(y, dtype=np.float32),
            "k": np.array(ks), "mask": np.array(masks, dtype=np.uint64), "n": np.array(nn),
            "precision": np.array(precs), "seconds": np.array(secs)}


def spearman(a, b) -> float:
    ra = np.argsort(np.argsort(a))
    rb = np.argsort(np.argsort(b))
    return float(np.corrcoef(ra, rb)[0, 1])


HIGH_BIT = 13  # targets from this bit up are gathered with strides of >= 64 KiB
MASK_BITS = 34  # target-mask features: bits 0..33, at feature 2 + bit


def augment_high_targets(X: np.ndarray, y: np.ndarray, copies: int, rng: np.random.Generator):
    """Append `copies` versions of every sample whose targets at or above
    HIGH_BIT are moved to other distinct bits in [HIGH_BIT, 34), label kept.
    Such passes run the same kernel form whichever high bits they use (the
    corpus shows a few percent between them), so the copies stop the network
    from keying on individual high bits, and it sees every high bit, also the
    ones above the state sizes the corpus was timed at."""
    out_x, out_y = [X], [y]
    high = np.arange(HIGH_BIT, MASK_BITS)
    for _ in range(copies):
        Xc = X.copy()
        for i in range(len(Xc)):
            bits = np.nonzero(Xc[i, 2:2 + MASK_BITS] > 0)[0]
            hi = bits[bits >= HIGH_BIT]
            if len(hi) == 0:
                continue
            Xc[i, 2 + hi] = 0.0
            Xc[i, 2 + rng.choice(high, size=len(hi), replace=False)] = 1.0
        out_x.append(Xc)
        out_y.append(y)
    return np.concatenate(out_x), np.concatenate(out_y)


def train_cost_model(corpus: Dict[str, np.ndarray], epochs: int = 4000, lr: float = 3e-3, seed: int = 0,
                     holdout: float = 0.2, install: bool = True, save_path: str | None = None,
                     check_every: int = 200, augment: int = 4) -> dict:
    """Train on the GPU with early stopping on a validation split (the
    parameters with the lowest validation error are kept), report the error on
    a separate test split and install the network as the fusion cost model.
    The training split is widened by `augment` copies with moved high targets
    (augment_high_targets); the validation and test splits are left as timed."""
    import torch
    X, y = corpus["X"], corpus["y"]
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    idx = rng.permutation(len(y))
    n_test = int(len(y) * holdout)
    n_val = n_test  # early-stopping split, disjoint from the reported test split
    te, va, tr = idx[:n_test], idx[n_test:n_test + n_val], idx[n_test + n_val:]
    x_tr, y_tr = augment_high_targets(X[tr], y[tr], augment, rng) if augment else (X[tr], y[tr])
    m = sv.Mlp(seed=seed)
    try:
        xd = torch.tensor(x_tr, device="cuda")
        yd = torch.tensor(y_tr, device="cuda")
        xt = torch.tensor(X[te], device="cuda") if n_test else None
        xv = torch.tensor(X[va], device="cuda") if n_val else None
        t0 = time.perf_counter()
        best = (math.inf, None, 0)
        done = 0
        loss = math.nan
        while done < epochs:
            step = min(check_every, epochs - done)
            loss = m.train(xd, yd, epochs=step, lr=lr)
            done += step
            if n_val:
                err = float(np.mean((m.forward(xv) - y[va]) ** 2))
                if err < best[0]:
                    best = (err, m.get_params(), done)
        if n_val and best[1] is not None:
            m.set_params(best[1])
        train_s = time.perf_counter() - t0
        out = {"train_mse": loss, "train_s": train_s, "epochs": epochs, "best_epoch": best[2],
               "samples": int(len(tr)), "augmented_samples": int(len(y_tr))}
        if n_test:
            pred = m.forward(xt)
            out["test_rmse"] = float(np.sqrt(np.mean((pred - y[te]) ** 2)))
            out["test_spearman"] = spearman(pred, y[te])
        if install:
            m.install()
            if save_path:
                sv.sv_cost_model_save(save_path)
        return out
    finally:
        m.free()
