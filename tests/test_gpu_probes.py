"""The library's copy probes (the bandwidth ceilings the step is measured
against) move every byte: exact copies at a full-tile size and at a ragged one
whose last block is partly empty."""
import ctypes

import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,nplanes", [(1 << 16, 10), (2 * 70001, 10), (2 * 333, 3), (2, 1)])
def test_copy_probes_are_exact(n, nplanes):
    import torch
    from paper_2609_09160_amd import _lib
    lib = _lib.load()
    g = torch.Generator(device="cpu").manual_seed(n + nplanes)
    a = torch.rand(nplanes * n, generator=g).cuda()
    guard = torch.full((nplanes * n + 64,), -7.0, device="cuda")
    stream = torch.cuda.current_stream()
    S = ctypes.c_void_p(stream.cuda_stream)
    A, B = ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(guard.data_ptr())
    _lib.check(lib.lbfast_planes_probe(A, B, n, nplanes, S))
    torch.cuda.synchronize()
    assert torch.equal(guard[:nplanes * n], a)
    assert bool((guard[nplanes * n:] == -7.0).all())
    if (nplanes * n) % 4 == 0:
        guard.fill_(-7.0)
        _lib.check(lib.lbfast_copy_probe(A, B, nplanes * n // 4, S))
        torch.cuda.synchronize()
        assert torch.equal(guard[:nplanes * n], a)
        assert bool((guard[nplanes * n:] == -7.0).all())
