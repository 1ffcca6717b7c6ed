"""Autotuner: table persistence (CPU) and tuned dispatch parity (GPU)."""
import json
import os

import numpy as np
import pytest

import circuits as C
import oracle
from paper_2602_09604_amd import sv

needs_lib = pytest.mark.skipif(not os.path.exists(sv.LIB_PATH), reason="libsv.so not built")


@needs_lib
def test_tune_file_roundtrip(tmp_path):
    p = tmp_path / "tune.json"
    p.write_text(json.dumps({"format": "libsv-tune-1",
                             "entries": [[0, 3, 0, 2, 2, 10, 1.5], [2, 6, 1, 0, 3, 12, 0.7]]}))
    sv.sv_tune_load(str(p))
    out = tmp_path / "out.json"
    sv.sv_tune_save(str(out))
    d = json.loads(out.read_text())
    entries = {tuple(e[:4]): e[4:6] for e in d["entries"]}
    assert entries[(0, 3, 0, 2)] == [2, 10]
    assert entries[(2, 6, 1, 0)] == [3, 12]


@needs_lib
@pytest.mark.parametrize("text", [
    "not json at all",
    '{"format": "other", "entries": []}',
    '{"format": "libsv-tune-1", "entries": [[9, 3, 0, 2, 2, 10, 1.5]]}',   # bad precision
    '{"format": "libsv-tune-1", "entries": [[0, 3, 0, 2, 7, 10, 1.5]]}',   # bad variant
    '{"format": "libsv-tune-1", "entries": [[0, 3, 0, 2, 2, 11, 1.5]]}',   # tile not built
    '{"format": "libsv-tune-1", "entries": [[0, 3, 0]]}',                  # truncated
])
def test_tune_file_rejects_malformed(tmp_path, text):
    p = tmp_path / "bad.json"
    p.write_text(text)
    with pytest.raises(sv.SvError) as e:
        sv.sv_tune_load(str(p))
    assert e.value.code == sv.SV_EINVAL


@needs_lib
def test_tune_missing_file():
    with pytest.raises(sv.SvError):
        sv.sv_tune_load("/nonexistent/tune.json")


@pytest.mark.gpu
def test_autotuned_dispatch_matches_oracle(tmp_path):
    st = sv.State(20)
    try:
        sv.sv_autotune(st.h, 0)
        sv.sv_tune_save(str(tmp_path / "t.json"))
        entries = json.loads((tmp_path / "t.json").read_text())["entries"]
        assert len(entries) > 40
        print("tuned classes:", len(entries), flush=True)
    finally:
        st.free()
    n = 18
    gates = C.grid_circuit(3, 6, 12, seed=4)
    ref = oracle.apply_circuit(n, gates)
    for prec in ("fp32_valu", "bf16x3"):
        for K in (2, 4, 6):
            st = sv.State(n)
            try:
                st.apply_circuit(gates, max_k=K, precision=prec)
                r = oracle.compare(st.read(), ref)
                assert r["max_abs"] <= 1e-5 and r["infidelity"] <= 1e-6, (prec, K, r)
            finally:
                st.free()
