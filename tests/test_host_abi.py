"""Host-side checks of the C ABI (no GPU needed): exported symbols, buffer
sizing against the paper's memory model, and argument validation that must
happen before any device call."""
import ctypes
import os
import threading

import pytest

from paper_2609_09160_amd import _lib

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "memory_footprint_512.txt")


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def _golden():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


def test_exports_every_declared_symbol(lib):
    names = _lib.declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert lib.lbfast_abi_version() == 1


def test_params_layout_matches_header():
    # offsets fixed by the C struct in include/lbfast.h
    P = _lib.LbfastParams
    assert ctypes.sizeof(P) == 152
    assert P.nx.offset == 24 and P.tau.offset == 48 and P.scale.offset == 80


def test_memory_model_matches_paper(lib):
    """Section 3: 512^3 moment form = 20 GB (FP64) / 10 GB (FP32) double
    buffered, against 38/54 (FP64) and 19/27 (FP32) for population schemes."""
    g = _golden()
    GiB = float(2 ** 30)
    N = 512 ** 3
    for st, b, tag in (("f64", 8, "fp64"), ("f32", 4, "fp32")):
        p = _lib.make_params((512, 512, 512), 0.6, storage=st)
        two = 2 * lib.lbfast_buffer_bytes(ctypes.byref(p))
        assert two / GiB == g[f"{tag}_moment_GB"]
        assert N * 38 * b / GiB == g[f"{tag}_d3q19_GB"]
        assert N * 54 * b / GiB == g[f"{tag}_d3q27_GB"]
    assert round(100 * (1 - 20 / 38), 1) == g["saving_vs_d3q19_percent"]
    assert round(100 * (1 - 20 / 54), 1) == g["saving_vs_d3q27_percent"]
    for st in ("f16s", "bf16s"):
        p = _lib.make_params((512, 512, 512), 0.6, storage=st)
        assert 2 * lib.lbfast_buffer_bytes(ctypes.byref(p)) / GiB == 5.0
    # the split-velocity form: ten 16-bit moment planes plus three low words
    p = _lib.make_params((512, 512, 512), 0.6, storage="f16su")
    assert lib.lbfast_buffer_bytes(ctypes.byref(p)) == N * 13 * 2


@pytest.mark.parametrize("lattice,rounding,code,needle", [
    (19, "stochastic", _lib.LBF_E_ARG, "nearest"),
    ("27h", "stochastic", _lib.LBF_E_ARG, "nearest"),
])
def test_split_storage_validation(lib, lattice, rounding, code, needle):
    p = _lib.make_params((32, 8, 8), 0.7, lattice=lattice, storage="f16su", rounding=rounding)
    assert lib.lbfast_buffer_bytes(ctypes.byref(p)) == 0
    rc, msg = _create(lib, p)
    assert rc == code and needle in msg


def _create(lib, p, bufs=(None, None)):
    h = ctypes.c_void_p()
    rc = lib.lbfast_create(ctypes.byref(p), None, bufs[0], bufs[1], ctypes.byref(h))
    return rc, lib.lbfast_last_error().decode()


@pytest.mark.parametrize("mutate,code,needle", [
    (lambda p: setattr(p, "tau", 0.5), _lib.LBF_E_ARG, "tau"),
    (lambda p: setattr(p, "tau", float("nan")), _lib.LBF_E_ARG, "tau"),
    (lambda p: setattr(p, "lattice", 15), _lib.LBF_E_ARG, "lattice"),
    (lambda p: setattr(p, "lattice", 28), _lib.LBF_E_ARG, "lattice"),
    (lambda p: setattr(p, "storage", 7), _lib.LBF_E_ARG, "storage"),
    (lambda p: setattr(p, "nx", 0), _lib.LBF_E_ARG, "extent"),
    (lambda p: setattr(p, "struct_size", 8), _lib.LBF_E_ARG, "struct_size"),
    (lambda p: p.bc.__setitem__(0, 1), _lib.LBF_E_UNSUPPORTED, "y axis"),
    (lambda p: p.bc.__setitem__(1, 3), _lib.LBF_E_ARG, "bc"),
    (lambda p: (p.bc.__setitem__(1, 1), setattr(p, "ny", 1)), _lib.LBF_E_ARG, "walled"),
    (lambda p: p.scale.__setitem__(3, 1.0), _lib.LBF_E_ARG, "16-bit"),
    (lambda p: (setattr(p, "storage", 2), p.scale.__setitem__(3, 3.0)), _lib.LBF_E_ARG,
     "power of two"),
    (lambda p: p.reserved.__setitem__(2, 1), _lib.LBF_E_ARG, "reserved"),
    (lambda p: setattr(p, "rounding", 3), _lib.LBF_E_ARG, "rounding"),
    (lambda p: setattr(p, "rounding", 2), _lib.LBF_E_ARG, "16-bit storage only"),
    (lambda p: p.force.__setitem__(1, float("inf")), _lib.LBF_E_ARG, "force"),
])
def test_validation_before_device(lib, mutate, code, needle):
    p = _lib.make_params((8, 8, 8), 0.8)
    mutate(p)
    rc, msg = _create(lib, p)
    assert rc == code, msg
    assert needle in msg
    assert lib.lbfast_buffer_bytes(ctypes.byref(p)) == 0


def test_buffer_arguments(lib):
    p = _lib.make_params((8, 8, 8), 0.8)
    rc, msg = _create(lib, p, (ctypes.c_void_p(4096), None))
    assert rc == _lib.LBF_E_ARG and "both" in msg
    rc, msg = _create(lib, p, (ctypes.c_void_p(4096), ctypes.c_void_p(4096)))
    assert rc == _lib.LBF_E_ARG and "differ" in msg
    rc, msg = _create(lib, p, (ctypes.c_void_p(4096 + 8), ctypes.c_void_p(8192)))
    assert rc == _lib.LBF_E_ARG and "aligned" in msg
    assert lib.lbfast_create(ctypes.byref(p), None, None, None, None) == _lib.LBF_E_ARG


def test_null_handle_calls(lib):
    assert lib.lbfast_step(None, 1) == _lib.LBF_E_ARG
    assert lib.lbfast_sync(None) == _lib.LBF_E_ARG
    assert lib.lbfast_set_launch(None, 8, 0) == _lib.LBF_E_ARG
    assert lib.lbfast_set_block_order(None, 1) == _lib.LBF_E_ARG
    assert lib.lbfast_destroy(None) == _lib.LBF_OK


def test_last_error_is_per_thread(lib):
    p = _lib.make_params((8, 8, 8), 0.3)
    _create(lib, p)
    main_msg = lib.lbfast_last_error().decode()
    other = {}

    def worker():
        other["msg"] = lib.lbfast_last_error().decode()

    t = threading.Thread(target=worker)
    t.start()
    t.join()
    assert "tau" in main_msg and other["msg"] == ""


@pytest.mark.parametrize("lattice", [19, 27, "27h"])
def test_valid_params_without_gpu_report_device_error(lib, lattice):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    p = _lib.make_params((8, 8, 8), 0.8, lattice=lattice)
    assert p.lattice == {19: 19, 27: 27, "27h": 270}[lattice]
    assert lib.lbfast_buffer_bytes(ctypes.byref(p)) == 10 * 8 ** 3 * 4
    rc, msg = _create(lib, p)
    assert rc == _lib.LBF_E_DEVICE and msg


@pytest.mark.parametrize("args,needle", [((4096, 8192, 100, 8, 4, 0, 1), "nx"),
                                         ((4096, 8192, 128, 12, 4, 0, 1), "ny"),
                                         ((4096, 8192, 128, 8, 4, 0, 0), "zchunk"),
                                         ((4096, 8192, 128, 8, 0, 0, 1), "nz"),
                                         ((4096, 8192, 128, 8, 4, 4, 1), "layout"),
                                         ((4100, 8192, 128, 8, 4, 3, 1), "aligned"),
                                         ((0, 8192, 128, 8, 4, 3, 1), "null")])
def test_zmarch_probe_validation(lib, args, needle):
    # rejected on the host before any device call (the pointers are never used)
    a, b, nx, ny, nz, layout, zchunk = args
    rc = lib.lbfast_zmarch_probe(ctypes.c_void_p(a or None), ctypes.c_void_p(b), nx, ny, nz,
                                 layout, zchunk, None)
    assert rc == _lib.LBF_E_ARG
    assert needle in lib.lbfast_last_error().decode()


@pytest.mark.parametrize("n,nplanes,needle", [(3, 10, "even"), (0, 10, "even"),
                                              (8, 0, "nplanes"), (8, 11, "nplanes")])
def test_planes_probe_validation(lib, n, nplanes, needle):
    # rejected on the host before any device call (the pointers are never used)
    rc = lib.lbfast_planes_probe(ctypes.c_void_p(4096), ctypes.c_void_p(8192), n, nplanes, None)
    assert rc == _lib.LBF_E_ARG
    assert needle in lib.lbfast_last_error().decode()
