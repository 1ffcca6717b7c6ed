"""sv_norm_noalloc (the allocation-free norm: partials in the library's static
per-device scratch, result to a device double) against sv_norm on the same
states, through the C ABI: two calls in a row, the second on a smaller
state, so the second reads scratch the first left behind."""
import ctypes
import sys

import numpy as np
import pytest

import circuits as C

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def norm_noalloc(st, stream_ptr):
    import torch
    from paper_2602_09604_amd import sv
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    rc = sv.lib().sv_norm_noalloc(ctypes.c_void_p(st.buf.data_ptr()), st.n, st.buf.numel() * st.buf.element_size(),
                                  ctypes.c_void_p(stream_ptr), ctypes.c_void_p(out.data_ptr()))
    sv._check(rc)
    torch.cuda.current_stream().synchronize()
    return float(out.item())


@pytest.mark.parametrize("n_big,n_small", [(24, 13), (27, 5), (12, 1)])
def test_norm_noalloc_matches_sv_norm_twice(n_big, n_small):
    import torch
    from paper_2602_09604_amd import sv
    stream = torch.cuda.current_stream()
    for step, (n, seed) in enumerate(((n_big, 1), (n_small, 2))):
        st = sv.State(n, stream=stream)
        try:
            psi = C.random_state_c64(n, seed) * np.complex64(1.5)  # norm 2.25, not 1
            st.write(0, psi)
            ref = st.norm()
            say("n=%d call %d: sv_norm %.17g" % (n, step, ref))
            got = norm_noalloc(st, stream.cuda_stream)
            say("n=%d call %d: sv_norm_noalloc %.17g" % (n, step, got))
            # same kernels, same partial count and order: the same double
            assert got == ref, (got, ref)
            exact = float(np.sum(psi.real.astype(np.float64) ** 2 + psi.imag.astype(np.float64) ** 2))
            assert abs(got - exact) <= 1e-12 * exact
        finally:
            st.free()


def test_norm_noalloc_rejects_bad_arguments():
    import torch
    from paper_2602_09604_amd import sv
    L = sv.lib()
    st = sv.State(10)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    host = np.zeros(1, dtype=np.float64)
    try:
        nb = st.buf.numel() * st.buf.element_size()
        buf, o = ctypes.c_void_p(st.buf.data_ptr()), ctypes.c_void_p(out.data_ptr())
        assert L.sv_norm_noalloc(buf, 41, nb, None, o) == sv.SV_EINVAL
        assert L.sv_norm_noalloc(buf, 0, nb, None, o) == sv.SV_EINVAL
        assert L.sv_norm_noalloc(buf, 11, nb, None, o) == sv.SV_EINVAL   # buffer too small for 11 qubits
        assert L.sv_norm_noalloc(None, 10, nb, None, o) == sv.SV_EINVAL
        assert L.sv_norm_noalloc(buf, 10, nb, None, ctypes.c_void_p(host.ctypes.data)) == sv.SV_EINVAL
    finally:
        st.free()
