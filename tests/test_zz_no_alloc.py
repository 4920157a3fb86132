"""The allocation-free reduction (lbfast_reduce_noalloc) against lbfast_reduce
on the same states, through the C ABI: two calls in a row, the second on a
smaller state, for every storage format.  Both run the same two-pass kernels
in the same order, so the sums agree bit for bit."""
import ctypes

import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


def _state(shape, storage, seed):
    from paper_2609_09160_amd import Solver, inputs
    s = Solver(shape, 0.7, storage=storage)
    s.set_moments(inputs.random_state(shape, seed=seed))
    s.step(3)
    return s


def _noalloc(s, out_dev):
    import torch
    from paper_2609_09160_amd import _lib
    lib = _lib.load()
    sc = (ctypes.c_float * 10)(*[float(v) for v in s.scales()])
    _lib.check(lib.lbfast_reduce_noalloc(ctypes.c_void_p(s.state_ptr()), s.params.storage,
                                         s.N, sc, ctypes.c_void_p(out_dev.data_ptr()),
                                         ctypes.c_void_p(s.stream.cuda_stream)))
    torch.cuda.synchronize()
    return out_dev.cpu().numpy().copy()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s", "bf16s", "f16su"])
def test_noalloc_reduce_matches_reduce(storage):
    import torch
    out_dev = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
    for shape, seed in (((130, 48, 40), 11), ((20, 12, 9), 12)):
        say(f"noalloc reduce: {storage} {shape}")
        s = _state(shape, storage, seed)
        want = s.reduce()
        got = _noalloc(s, out_dev)
        s.close()
        assert np.array_equal(got, want), (got, want)


def test_noalloc_reduce_rejects_bad_arguments():
    import torch
    from paper_2609_09160_amd import _lib
    lib = _lib.load()
    out_dev = torch.zeros(5, dtype=torch.float64, device="cuda")
    st = torch.zeros(10 * 64, dtype=torch.float32, device="cuda")
    vp = ctypes.c_void_p
    null_stream = vp(None)
    # n_sites beyond the supported maximum
    rc = lib.lbfast_reduce_noalloc(vp(st.data_ptr()), _lib.LBF_F32, int(5e9), None,
                                   vp(out_dev.data_ptr()), null_stream)
    assert rc == _lib.LBF_E_ARG and b"4e9" in lib.lbfast_last_error()
    # host output
    host = (ctypes.c_double * 5)()
    rc = lib.lbfast_reduce_noalloc(vp(st.data_ptr()), _lib.LBF_F32, 64, None,
                                   ctypes.cast(host, vp), null_stream)
    assert rc == _lib.LBF_E_ARG
    # 16-bit storage without its scales
    rc = lib.lbfast_reduce_noalloc(vp(st.data_ptr()), _lib.LBF_F16S, 64, None,
                                   vp(out_dev.data_ptr()), null_stream)
    assert rc == _lib.LBF_E_ARG
