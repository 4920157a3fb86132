"""ctypes binding of liblbfast.so (include/lbfast.h): argument marshalling only.

The library must have been built (`python -m paper_2609_09160_amd.build`, or
`__graft_entry__.build()`); there is no fallback path.
"""
import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbfast.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "lbfast.h")
HEADERS = (HEADER, os.path.join(os.path.dirname(_HERE), "include", "lbfast_measure.h"))

# constants mirrored from include/lbfast.h
LBF_OK, LBF_E_ARG, LBF_E_UNSUPPORTED, LBF_E_NOMEM = 0, -1, -2, -3
LBF_E_DEVICE, LBF_E_NONFINITE, LBF_E_STATE = -4, -5, -6
LBF_D3Q19, LBF_D3Q27, LBF_D3Q27H = 19, 27, 270
LBF_F64, LBF_F32, LBF_F16S, LBF_BF16S, LBF_F16SU = 0, 1, 2, 3, 4
LBF_PERIODIC, LBF_WALLS = 0, 1
LBF_ROUND_AUTO, LBF_ROUND_NEAREST, LBF_ROUND_STOCHASTIC = 0, 1, 2
ROUNDING = {"auto": LBF_ROUND_AUTO, "nearest": LBF_ROUND_NEAREST,
            "stochastic": LBF_ROUND_STOCHASTIC}

STORAGE = {"f64": LBF_F64, "f32": LBF_F32, "f16s": LBF_F16S, "bf16s": LBF_BF16S,
           "f16su": LBF_F16SU}
LATTICE = {19: LBF_D3Q19, 27: LBF_D3Q27, "19": LBF_D3Q19, "27": LBF_D3Q27, "27h": LBF_D3Q27H,
           LBF_D3Q27H: LBF_D3Q27H}
STATUS_NAMES = {0: "LBF_OK", -1: "LBF_E_ARG", -2: "LBF_E_UNSUPPORTED", -3: "LBF_E_NOMEM",
                -4: "LBF_E_DEVICE", -5: "LBF_E_NONFINITE", -6: "LBF_E_STATE"}


class LbfastParams(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("lattice", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("bc", ctypes.c_int32 * 3),
                ("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("tau", ctypes.c_double), ("force", ctypes.c_double * 3),
                ("scale", ctypes.c_float * 10), ("rounding", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 7)]


class LbfastPhaseParams(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("reserved0", ctypes.c_int32),
                ("sigma", ctypes.c_double), ("width", ctypes.c_double),
                ("diffusivity", ctypes.c_double), ("rho_l", ctypes.c_double),
                ("rho_h", ctypes.c_double), ("tau_l", ctypes.c_double), ("tau_h", ctypes.c_double)]


class LbfastError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load():
    """Load liblbfast.so (or the file named by LBFAST_LIB, for comparing
    builds); raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("LBFAST_LIB") or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build the HIP library first "
                          "(python -m paper_2609_09160_amd.build)")
    lib = ctypes.CDLL(path)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    P = ctypes.POINTER(LbfastParams)
    sig = {
        "lbfast_abi_version": ([], i32),
        "lbfast_buffer_bytes": ([P], ctypes.c_size_t),
        "lbfast_create": ([P, vp, vp, vp, ctypes.POINTER(vp)], i32),
        "lbfast_destroy": ([vp], i32),
        "lbfast_set_moments": ([vp, vp, i32, i32], i32),
        "lbfast_get_moments": ([vp, vp, i32, i32], i32),
        "lbfast_set_force_field": ([vp, vp, i32], i32),
        "lbfast_step": ([vp, i64], i32),
        "lbfast_sync": ([vp], i32),
        "lbfast_reduce": ([vp, ctypes.POINTER(ctypes.c_double)], i32),
        "lbfast_reduce_noalloc": ([vp, i32, i64, ctypes.POINTER(ctypes.c_float), vp, vp], i32),
        "lbfast_state_ptr": ([vp, ctypes.POINTER(vp)], i32),
        "lbfast_get_scales": ([vp, ctypes.POINTER(ctypes.c_float)], i32),
        "lbfast_set_launch": ([vp, i32, i32], i32),
        "lbfast_set_lane_sites": ([vp, i32], i32),
        "lbfast_set_block_order": ([vp, i32], i32),
        "lbfast_last_error": ([], ctypes.c_char_p),
        "lbfast_stream_probe": ([vp, vp, i64, i32, vp], i32),
        "lbfast_copy_probe": ([vp, vp, i64, vp], i32),
        "lbfast_planes_probe": ([vp, vp, i64, i32, vp], i32),
        "lbfast_zmarch_probe": ([vp, vp, i32, i32, i32, i32, i32, vp], i32),
        "lbfast_enable_two_phase": ([vp, ctypes.POINTER(LbfastPhaseParams)], i32),
        "lbfast_set_phase": ([vp, vp, i32, i32], i32),
        "lbfast_get_phase": ([vp, vp, i32, i32], i32),
        "lbfast_forward_checkpointed": ([vp, i64, i64, vp], i32),
        "lbfast_adjoint_work_bytes": ([vp, i64], ctypes.c_size_t),
        "lbfast_adjoint": ([vp, i64, i64, vp, vp, vp, vp, vp], i32),
        "lbfast_set_adjoint_launch": ([vp, i32, i32], i32),
    }
    for name, (args, res) in sig.items():
        if path != LIB_PATH and not hasattr(lib, name):
            continue  # an alternate build may predate a symbol
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(rc):
    if rc != LBF_OK:
        raise LbfastError(rc, load().lbfast_last_error().decode(errors="replace"))
    return rc


def declared_functions():
    """Names of the functions include/lbfast.h and include/lbfast_measure.h
    declare."""
    text = "".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbfast_[a-z0-9_]+)\s*\(", text)))


def make_params(shape, tau, lattice=19, storage="f32", bc=(0, 0, 0), force=(0.0, 0.0, 0.0),
                scale=None, rounding="auto"):
    p = LbfastParams()
    p.struct_size = ctypes.sizeof(LbfastParams)
    p.lattice = LATTICE.get(lattice, lattice if isinstance(lattice, int) else -1)
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    for a in range(3):
        p.bc[a] = int(bc[a])
        p.force[a] = float(force[a])
    p.nx, p.ny, p.nz = (int(v) for v in shape)
    p.tau = float(tau)
    for k in range(10):
        p.scale[k] = 0.0 if scale is None else float(scale[k])
    p.rounding = ROUNDING[rounding] if isinstance(rounding, str) else int(rounding)
    return p
