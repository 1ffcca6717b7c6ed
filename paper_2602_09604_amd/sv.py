"""ctypes binding of libsv.so (argument marshalling only).

The functions keep the C names (``sv_alloc``, ``sv_apply_gate``, ...).  A
small ``State`` class pairs a handle with the torch tensor that owns the
device buffer.  PyTorch supplies device memory and the stream; every step of
gate application runs in the library's HIP kernels.  There is no CPU
fallback: if libsv.so is missing or no GPU is visible, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsv.so")

SV_OK, SV_EINVAL, SV_ENOMEM, SV_EDEVICE, SV_EUNSUPPORTED, SV_ESTATE = 0, -1, -2, -3, -4, -5
SV_C64 = 0
SV_PREC_FP32_VALU, SV_PREC_FP32_MFMA, SV_PREC_BF16X3, SV_PREC_FP16X3 = 0, 1, 2, 3
SV_FUSE_NONE, SV_FUSE_GREEDY, SV_FUSE_LEARNED, SV_FUSE_PHASE = 0, 1, 2, 3
SV_VARIANT_AUTO, SV_VARIANT_REG, SV_VARIANT_LDS, SV_VARIANT_MFMA = 0, 1, 2, 3
SV_MAX_K = 6
SV_COST_FEATURES = 40

PRECISIONS = {"fp32_valu": 0, "fp32_mfma": 1, "bf16x3": 2, "fp16x3": 3}
FUSIONS = {"none": 0, "greedy": 1, "learned": 2, "phase": 3, "block": 4}
VARIANTS = {"auto": 0, "reg": 1, "lds": 2, "mfma": 3, "shfl": 4}


class SvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("libsv error %d: %s" % (code, msg))
        self.code = code


class sv_gate(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("qubits", ctypes.c_int32 * SV_MAX_K),
                ("matrix", ctypes.POINTER(ctypes.c_double)), ("cmask", ctypes.c_uint64),
                ("cval", ctypes.c_uint64)]


class sv_run_opts(ctypes.Structure):
    _fields_ = [("max_k", ctypes.c_int32), ("fusion", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("variant", ctypes.c_int32), ("timing", ctypes.c_int32)]


class sv_run_stats(ctypes.Structure):
    _fields_ = [("gates_in", ctypes.c_uint64), ("passes", ctypes.c_uint64), ("bytes", ctypes.c_uint64),
                ("useful_flops", ctypes.c_double), ("fuse_s", ctypes.c_double), ("gpu_s", ctypes.c_double),
                ("variant_s", ctypes.c_double * 5), ("variant_passes", ctypes.c_uint64 * 5),
                ("graph_relaunched", ctypes.c_uint64), ("variant_bytes", ctypes.c_uint64 * 5),
                ("launches", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["variant_s"] = list(self.variant_s)
        d["variant_passes"] = list(self.variant_passes)
        d["variant_bytes"] = list(self.variant_bytes)
        return d


_lib = None
_vp = ctypes.c_void_p
_i32p = ctypes.POINTER(ctypes.c_int32)
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_u64p = ctypes.POINTER(ctypes.c_uint64)

_SIGS = {
    "sv_alloc": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
    "sv_free": (ctypes.c_int, [_vp]),
    "sv_set_basis": (ctypes.c_int, [_vp, ctypes.c_uint64]),
    "sv_num_qubits": (ctypes.c_int, [_vp]),
    "sv_apply_gate": (ctypes.c_int, [_vp, _i32p, ctypes.c_int, _dp]),
    "sv_apply_controlled_gate": (ctypes.c_int, [_vp, _i32p, ctypes.c_int, _dp, ctypes.c_int, _i32p, _i32p]),
    "sv_expect_pauli": (ctypes.c_int, [_vp, ctypes.c_size_t, _u64p, _u64p, _dp]),
    "sv_marginal_probs": (ctypes.c_int, [_vp, ctypes.c_int, _i32p, _dp]),
    "sv_sample": (ctypes.c_int, [_vp, ctypes.c_size_t, _dp, _u64p]),
    "sv_apply_circuit": (ctypes.c_int, [_vp, ctypes.POINTER(sv_gate), ctypes.c_size_t,
                                        ctypes.POINTER(sv_run_opts), ctypes.POINTER(sv_run_stats)]),
    "sv_fuse": (ctypes.c_int, [ctypes.POINTER(sv_gate), ctypes.c_size_t, ctypes.c_int,
                               ctypes.POINTER(sv_run_opts), ctypes.POINTER(ctypes.POINTER(sv_gate)),
                               ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(_i32p)]),
    "sv_fused_free": (ctypes.c_int, [ctypes.POINTER(sv_gate), ctypes.c_size_t, _i32p]),
    "sv_norm": (ctypes.c_int, [_vp, _dp]),
    "sv_norm_noalloc": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_size_t, _vp, _vp]),
    "sv_read_amplitudes": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.c_uint64, _fp]),
    "sv_write_amplitudes": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.c_uint64, _fp]),
    "sv_batch_run": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(ctypes.POINTER(sv_gate)),
                                    ctypes.POINTER(ctypes.c_size_t), ctypes.c_size_t,
                                    ctypes.POINTER(sv_run_opts), ctypes.POINTER(sv_run_stats)]),
    "sv_autotune": (ctypes.c_int, [_vp, ctypes.c_int]),
    "sv_tune_save": (ctypes.c_int, [ctypes.c_char_p]),
    "sv_tune_load": (ctypes.c_int, [ctypes.c_char_p]),
    "sv_mlp_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint64, _vp, ctypes.POINTER(_vp)]),
    "sv_mlp_free": (ctypes.c_int, [_vp]),
    "sv_mlp_num_params": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "sv_mlp_get_params": (ctypes.c_int, [_vp, _fp]),
    "sv_mlp_set_params": (ctypes.c_int, [_vp, _fp]),
    "sv_mlp_forward": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp]),
    "sv_mlp_loss_grad": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _fp, _fp]),
    "sv_mlp_adam_step": (ctypes.c_int, [_vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float]),
    "sv_mlp_train": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_float, _fp]),
    "sv_cost_model_install": (ctypes.c_int, [_vp]),
    "sv_cost_model_save": (ctypes.c_int, [ctypes.c_char_p]),
    "sv_cost_model_load": (ctypes.c_int, [ctypes.c_char_p]),
    "sv_cost_model_clear": (ctypes.c_int, []),
    "sv_cost_model_predict": (ctypes.c_int, [ctypes.c_int, _i32p, ctypes.c_int, ctypes.c_int, _dp]),
    "sv_cost_features": (ctypes.c_int, [ctypes.c_int, _i32p, ctypes.c_int, ctypes.c_int, _fp]),
    "sv_last_error": (ctypes.c_char_p, []),
    "sv_version": (ctypes.c_char_p, []),
    "sv_struct_size": (ctypes.c_size_t, [ctypes.c_int]),
}


def lib():
    """Load libsv.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsv.so is not built (run `python -m paper_2602_09604_amd.build`); "
                               "there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        for which, struct in enumerate((sv_gate, sv_run_opts, sv_run_stats)):
            if L.sv_struct_size(which) != ctypes.sizeof(struct):
                raise RuntimeError("%s layout differs from libsv.so (%d vs %d bytes); rebuild the library"
                                   % (struct.__name__, ctypes.sizeof(struct), L.sv_struct_size(which)))
        _lib = L
    return _lib


def exported_symbols() -> List[str]:
    return list(_SIGS)


def _check(rc: int) -> None:
    if rc != SV_OK:
        raise SvError(rc, lib().sv_last_error().decode())


# --------------------------------------------------------------------------
# Marshalling
# --------------------------------------------------------------------------
class GateArray:
    """A ctypes sv_gate array plus the matrix storage it points into."""

    def __init__(self, gates):
        self.n = len(gates)
        self.arr = (sv_gate * max(1, self.n))()
        sizes = [int(np.asarray(g.matrix).size) for g in gates]
        self.mats = np.empty(max(1, sum(sizes)), dtype=np.complex128)
        pos = 0
        base = self.mats.ctypes.data
        for i, g in enumerate(gates):
            qs = tuple(g.qubits)
            self.arr[i].k = len(qs)  # the library validates k (1..6) and rejects the call
            for j, q in enumerate(qs[:SV_MAX_K]):
                self.arr[i].qubits[j] = int(q)
            m = np.asarray(g.matrix, dtype=np.complex128).reshape(-1)
            self.mats[pos:pos + m.size] = m
            self.arr[i].matrix = ctypes.cast(base + 16 * pos, _dp)
            if getattr(g, "controls", ()):
                self.arr[i].cmask = g.cmask
                self.arr[i].cval = g.cval
            pos += m.size

    @property
    def ptr(self):
        return ctypes.cast(self.arr, ctypes.POINTER(sv_gate))


def make_opts(max_k: int = 4, fusion="greedy", precision="fp32_valu", use_graph: bool = False,
              variant="auto", timing: bool = False) -> sv_run_opts:
    o = sv_run_opts()
    o.max_k = int(max_k)
    o.fusion = FUSIONS[fusion] if isinstance(fusion, str) else int(fusion)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.use_graph = int(bool(use_graph))
    o.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    o.timing = int(bool(timing))
    return o


# --------------------------------------------------------------------------
# C-named wrappers
# --------------------------------------------------------------------------
def sv_alloc(n_qubits: int, dev_ptr: int, nbytes: int, stream_ptr: int) -> int:
    h = _vp()
    _check(lib().sv_alloc(n_qubits, SV_C64, _vp(dev_ptr), nbytes, _vp(stream_ptr), ctypes.byref(h)))
    return h.value


def sv_free(h: int) -> None:
    _check(lib().sv_free(_vp(h)))


def sv_set_basis(h: int, index: int) -> None:
    _check(lib().sv_set_basis(_vp(h), int(index)))


def sv_apply_gate(h: int, qubits: Sequence[int], matrix) -> None:
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    m = np.ascontiguousarray(matrix, dtype=np.complex128)
    _check(lib().sv_apply_gate(_vp(h), q.ctypes.data_as(_i32p), len(q), m.ctypes.data_as(_dp)))


def sv_apply_controlled_gate(h: int, qubits: Sequence[int], matrix, controls: Sequence[int],
                             control_values: Optional[Sequence[int]] = None) -> None:
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    m = np.ascontiguousarray(matrix, dtype=np.complex128)
    c = np.ascontiguousarray(controls, dtype=np.int32)
    v = None if control_values is None else np.ascontiguousarray(control_values, dtype=np.int32)
    _check(lib().sv_apply_controlled_gate(_vp(h), q.ctypes.data_as(_i32p), len(q), m.ctypes.data_as(_dp), len(c),
                                          c.ctypes.data_as(_i32p), None if v is None else v.ctypes.data_as(_i32p)))


def sv_expect_pauli(h: int, xmask, zmask) -> np.ndarray:
    x = np.ascontiguousarray(np.atleast_1d(np.asarray(xmask, dtype=np.uint64)))
    z = np.ascontiguousarray(np.atleast_1d(np.asarray(zmask, dtype=np.uint64)))
    if x.shape != z.shape:
        raise ValueError("xmask and zmask must have the same length")
    out = np.zeros(x.size, dtype=np.float64)
    _check(lib().sv_expect_pauli(_vp(h), x.size, x.ctypes.data_as(_u64p), z.ctypes.data_as(_u64p),
                                 out.ctypes.data_as(_dp)))
    return out


def sv_marginal_probs(h: int, qubits: Sequence[int]) -> np.ndarray:
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    out = np.zeros(1 << max(0, len(q)), dtype=np.float64)
    _check(lib().sv_marginal_probs(_vp(h), len(q), q.ctypes.data_as(_i32p), out.ctypes.data_as(_dp)))
    return out


def sv_sample(h: int, uniforms) -> np.ndarray:
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    out = np.zeros(u.size, dtype=np.uint64)
    _check(lib().sv_sample(_vp(h), u.size, u.ctypes.data_as(_dp), out.ctypes.data_as(_u64p)))
    return out


def sv_apply_circuit(h: int, gates, opts: Optional[sv_run_opts] = None, want_stats: bool = False) -> Optional[dict]:
    """`gates`: a list of circuits.Gate, or a GateArray marshalled once beforehand."""
    ga = gates if isinstance(gates, GateArray) else GateArray(gates)
    st = sv_run_stats() if want_stats else None
    _check(lib().sv_apply_circuit(_vp(h), ga.ptr, ga.n, ctypes.byref(opts) if opts is not None else None,
                                  ctypes.byref(st) if st is not None else None))
    return st.as_dict() if st is not None else None


def sv_fuse(gates, n_qubits: int, opts: Optional[sv_run_opts] = None):
    """Returns (fused gates as circuits.Gate list, block_of_gate array)."""
    from circuits import Gate
    ga = GateArray(gates)
    out = ctypes.POINTER(sv_gate)()
    n_out = ctypes.c_size_t()
    blk = _i32p()
    _check(lib().sv_fuse(ga.ptr, ga.n, n_qubits, ctypes.byref(opts) if opts is not None else None,
                         ctypes.byref(out), ctypes.byref(n_out), ctypes.byref(blk)))
    try:
        fused = []
        for i in range(n_out.value):
            g = out[i]
            k = g.k
            d = 1 << k
            m = np.ctypeslib.as_array(g.matrix, shape=(2 * d * d,)).copy().view(np.complex128).reshape(d, d)
            ctl = tuple(q for q in range(64) if (g.cmask >> q) & 1)
            fused.append(Gate(tuple(g.qubits[j] for j in range(k)), m, ctl,
                              tuple((g.cval >> q) & 1 for q in ctl) if ctl else None))
        block_of = np.ctypeslib.as_array(blk, shape=(len(gates),)).copy() if len(gates) else np.zeros(0, np.int32)
    finally:
        lib().sv_fused_free(out, n_out.value, blk)
    return fused, block_of


def sv_norm(h: int) -> float:
    v = ctypes.c_double()
    _check(lib().sv_norm(_vp(h), ctypes.byref(v)))
    return v.value


def sv_read_amplitudes(h: int, start: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.complex64)
    _check(lib().sv_read_amplitudes(_vp(h), start, count, out.view(np.float32).ctypes.data_as(_fp)))
    return out


def sv_write_amplitudes(h: int, start: int, values) -> None:
    v = np.ascontiguousarray(values, dtype=np.complex64)
    _check(lib().sv_write_amplitudes(_vp(h), start, v.size, v.view(np.float32).ctypes.data_as(_fp)))


def sv_batch_run(handles: Sequence[int], circuits, opts: Optional[sv_run_opts] = None) -> dict:
    """Run circuits[c] on handles[c] with the batched kernels; returns stats."""
    n = len(handles)
    arrays = [GateArray(c) for c in circuits]
    hs = (_vp * max(1, n))(*handles)
    cps = (ctypes.POINTER(sv_gate) * max(1, n))(*[a.ptr for a in arrays])
    counts = (ctypes.c_size_t * max(1, n))(*[a.n for a in arrays])
    st = sv_run_stats()
    _check(lib().sv_batch_run(hs, cps, counts, n, ctypes.byref(opts) if opts is not None else None,
                              ctypes.byref(st)))
    return st.as_dict()


class Mlp:
    """The cost-model network on the GPU (parameters and Adam state live in
    the library; inputs are torch float32 CUDA tensors)."""

    def __init__(self, width: int = 64, seed: int = 0, stream=None):
        import torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = _vp()
        _check(lib().sv_mlp_create(width, seed, _vp(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h.value
        n = ctypes.c_size_t()
        _check(lib().sv_mlp_num_params(_vp(self.h), ctypes.byref(n)))
        self.nparams = n.value

    def free(self):
        if self.h:
            lib().sv_mlp_free(_vp(self.h))
            self.h = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def get_params(self) -> np.ndarray:
        out = np.empty(self.nparams, dtype=np.float32)
        _check(lib().sv_mlp_get_params(_vp(self.h), out.ctypes.data_as(_fp)))
        return out

    def set_params(self, p) -> None:
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.nparams
        _check(lib().sv_mlp_set_params(_vp(self.h), p.ctypes.data_as(_fp)))

    @staticmethod
    def _dev(t, cols=None):
        import torch
        assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
        if cols is not None:
            assert t.dim() == 2 and t.shape[1] == cols
        return t

    def forward(self, x) -> np.ndarray:
        import torch
        x = self._dev(x, SV_COST_FEATURES)
        y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        _check(lib().sv_mlp_forward(_vp(self.h), _vp(x.data_ptr()), x.shape[0], _vp(y.data_ptr())))
        return y.cpu().numpy()

    def loss_grad(self, x, t):
        x = self._dev(x, SV_COST_FEATURES)
        t = self._dev(t)
        loss = ctypes.c_float()
        g = np.empty(self.nparams, dtype=np.float32)
        _check(lib().sv_mlp_loss_grad(_vp(self.h), _vp(x.data_ptr()), _vp(t.data_ptr()), x.shape[0],
                                      ctypes.byref(loss), g.ctypes.data_as(_fp)))
        return float(loss.value), g

    def adam_step(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
        _check(lib().sv_mlp_adam_step(_vp(self.h), lr, beta1, beta2, eps))

    def train(self, x, t, epochs: int, lr: float) -> float:
        x = self._dev(x, SV_COST_FEATURES)
        t = self._dev(t)
        loss = ctypes.c_float()
        _check(lib().sv_mlp_train(_vp(self.h), _vp(x.data_ptr()), _vp(t.data_ptr()), x.shape[0], epochs, lr,
                                  ctypes.byref(loss)))
        return float(loss.value)

    def install(self) -> None:
        _check(lib().sv_cost_model_install(_vp(self.h)))


def sv_cost_model_save(path: str) -> None:
    _check(lib().sv_cost_model_save(os.fsencode(path)))


def sv_cost_model_load(path: str) -> None:
    _check(lib().sv_cost_model_load(os.fsencode(path)))


def sv_cost_model_clear() -> None:
    _check(lib().sv_cost_model_clear())


def sv_cost_model_predict(k: int, qubits, n: int, precision: int) -> float:
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    out = ctypes.c_double()
    _check(lib().sv_cost_model_predict(k, q.ctypes.data_as(_i32p), n, precision, ctypes.byref(out)))
    return out.value


def sv_autotune(h: int, budget_ms: int = 0) -> None:
    _check(lib().sv_autotune(_vp(h), int(budget_ms)))


def sv_tune_save(path: str) -> None:
    _check(lib().sv_tune_save(os.fsencode(path)))


def sv_tune_load(path: str) -> None:
    _check(lib().sv_tune_load(os.fsencode(path)))


def sv_cost_features(k: int, qubits, n: int, precision: int) -> np.ndarray:
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    out = np.zeros(SV_COST_FEATURES, dtype=np.float32)
    _check(lib().sv_cost_features(k, q.ctypes.data_as(_i32p), n, precision, out.ctypes.data_as(_fp)))
    return out


def sv_struct_size(which: int) -> int:
    """sizeof(sv_gate), sizeof(sv_run_opts), sizeof(sv_run_stats) for which 0, 1, 2."""
    return int(lib().sv_struct_size(which))


# --------------------------------------------------------------------------
# Convenience: a state that owns its torch buffer
# --------------------------------------------------------------------------
class State:
    """An n-qubit complex64 state in a torch tensor on the current GPU."""

    def __init__(self, n: int, device: str = "cuda", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: libsv has no CPU path")
        self.n = n
        self.buf = torch.empty(1 << n, dtype=torch.complex64, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.buf.device)
        self.h = sv_alloc(n, self.buf.data_ptr(), self.buf.numel() * 8, self.stream.cuda_stream)

    def free(self) -> None:
        if self.h:
            sv_free(self.h)
            self.h = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def set_basis(self, x: int) -> None:
        sv_set_basis(self.h, x)

    def apply_gate(self, qubits, matrix) -> None:
        sv_apply_gate(self.h, qubits, matrix)

    def apply_controlled_gate(self, qubits, matrix, controls, control_values=None) -> None:
        sv_apply_controlled_gate(self.h, qubits, matrix, controls, control_values)

    def expect_pauli(self, xmask, zmask) -> np.ndarray:
        return sv_expect_pauli(self.h, xmask, zmask)

    def marginal_probs(self, qubits) -> np.ndarray:
        return sv_marginal_probs(self.h, qubits)

    def sample(self, uniforms) -> np.ndarray:
        return sv_sample(self.h, uniforms)

    def apply_circuit(self, gates, max_k: int = 4, fusion="greedy", precision="fp32_valu",
                      use_graph: bool = False, variant="auto", stats: bool = False, timing: bool = False):
        opts = make_opts(max_k, fusion, precision, use_graph, variant, timing)
        return sv_apply_circuit(self.h, gates, opts, stats or timing)

    def norm(self) -> float:
        return sv_norm(self.h)

    def read(self, start: int = 0, count: Optional[int] = None) -> np.ndarray:
        if count is None:
            count = (1 << self.n) - start
        return sv_read_amplitudes(self.h, start, count)

    def write(self, start: int, values) -> None:
        sv_write_amplitudes(self.h, start, values)
