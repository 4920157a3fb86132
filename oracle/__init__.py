"""FP64 CPU oracle for the moment-represented regularized LBM step.

TEST INFRASTRUCTURE.  Only `tests/`, `__graft_entry__.smoke()` and the CPU
baseline leg of `bench.py` may import this package.  It shares no code with
the GPU library (`paper_2609_09160_amd`) and imports nothing from it; inputs
reach both sides as plain arrays.

Contents
  * `PopulationOracle` -- ctypes wrapper of `lbm_oracle.c`: the full
    population regularized LBM that the moment form of the paper is equivalent
    to (Eq. (3) with the populations of Eq. (4), Guo source Eq. (9), moments
    corrected as in Eq. (8)).
  * `moment_form` -- independent NumPy evaluation of the moment-space update
    Eq. (7) + Eq. (8) with generic Hermite tensors (tiny grids).
  * `lattice_tables(Q)` -- the velocity set the C oracle uses.
  * `two_phase` -- the two-component variant (phase field by the conservative
    Allen-Cahn equation, Eq. (2), capillary force, flow step with a force
    that changes every step) and the Laplace measurement.
  * `adjoint` -- FP64 discrete adjoint of the population oracle.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    i64, dp, ip = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_lattice.argtypes = [ctypes.c_int, ip, dp]
    lib.oracle_lattice.restype = ctypes.c_int
    lib.oracle_init.argtypes = [ctypes.c_int, i64, i64, i64, dp, dp, dp]
    lib.oracle_moments.argtypes = [ctypes.c_int, i64, i64, i64, dp, dp, dp]
    lib.oracle_collide.argtypes = [ctypes.c_int, i64, i64, i64, ctypes.c_double, dp, dp, dp]
    lib.oracle_stream.argtypes = [ctypes.c_int, i64, i64, i64, ip, dp, dp]
    lib.oracle_run.argtypes = [ctypes.c_int, i64, i64, i64, ip, ctypes.c_double, dp, dp,
                               dp, i64]
    lib.oracle_grad.argtypes = [i64, i64, i64, ip, dp, dp]
    lib.oracle_lap.argtypes = [i64, i64, i64, ip, dp, dp]
    d = ctypes.c_double
    lib.oracle_phase_step.argtypes = [i64, i64, i64, ip, dp, dp, d, d, d, dp]
    lib.oracle_capillary_force.argtypes = [i64, i64, i64, ip, dp, d, d, dp, dp]
    lib.oracle_contrast_force.argtypes = [i64, i64, i64, ip, dp, dp, d, d, d, d, dp]
    lib.oracle_collide_var.argtypes = [ctypes.c_int, i64, i64, i64, dp, dp, dp, dp, dp]
    lib.oracle_moments_var.argtypes = [ctypes.c_int, i64, i64, i64, dp, dp, dp, dp]
    lib.oracle_init_var.argtypes = [ctypes.c_int, i64, i64, i64, dp, dp, dp, dp]
    for f in ("oracle_init", "oracle_moments", "oracle_collide", "oracle_stream",
              "oracle_run", "oracle_grad", "oracle_lap", "oracle_phase_step",
              "oracle_capillary_force", "oracle_contrast_force", "oracle_collide_var",
              "oracle_moments_var", "oracle_init_var"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


D3Q27H = 270  # lattice code: the D3Q27 velocity set with the complete Hermite basis


def lattice_code(Q):
    """(code for the C library, number of velocities) of 19, 27 or "27h"."""
    if Q in ("27h", "D3Q27h", D3Q27H):
        return D3Q27H, 27
    Q = int(Q)
    if Q not in (19, 27):
        raise ValueError(f"unknown velocity set {Q!r}")
    return Q, Q


def threads() -> int:
    """OpenMP threads the oracle's loops use (OMP_NUM_THREADS or all cores)."""
    return _load().oracle_threads()


def set_threads(n: int) -> None:
    """Use n OpenMP threads in the oracle's later loops."""
    lib = _load()
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = None
    lib.oracle_set_threads(int(n))


def lattice_tables(Q):
    """(c[Q,3] int, w[Q] float64) of the oracle's velocity set."""
    lib = _load()
    code, Q = lattice_code(Q)
    c = np.zeros((Q, 3), dtype=np.int32)
    w = np.zeros(Q, dtype=np.float64)
    q = lib.oracle_lattice(code, c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(w))
    if q != Q:
        raise ValueError(f"unknown velocity set Q={Q}")
    return c.astype(np.int64), w


class PopulationOracle:
    """Full-population FP64 regularized LBM on an (nx, ny, nz) grid.

    State: populations f[Q, nz, ny, nx].  `Q` is 19, 27 or "27h" (the D3Q27
    set with the complete Hermite basis).  `force` is None (zero), a length-3
    uniform vector, or a [3, nz, ny, nx] field (static in time).  `bc` is a
    per-axis (x, y, z) tuple: 0 periodic, 1 halfway bounce-back walls.
    """

    def __init__(self, Q, shape, tau, bc=(0, 0, 0), force=None):
        self.lattice, self.Q = lattice_code(Q)
        self.nx, self.ny, self.nz = (int(v) for v in shape)
        self.N = self.nx * self.ny * self.nz
        self.tau = float(tau)
        self.bc = np.ascontiguousarray(np.asarray(bc, dtype=np.int32))
        self.F = None
        if force is not None:
            F = np.asarray(force, dtype=np.float64)
            if F.shape == (3,):
                F = np.broadcast_to(F[:, None], (3, self.N))
            self.F = np.ascontiguousarray(F.reshape(3, self.N))
        self.f = np.zeros((self.Q, self.N), dtype=np.float64)
        self._scratch = np.zeros_like(self.f)
        self._lib = _load()

    def _dims(self):
        return self.nx, self.ny, self.nz

    def set_moments(self, m):
        """Populations whose corrected moments are m[10, nz, ny, nx] (or [10, N])."""
        m = np.ascontiguousarray(np.asarray(m, dtype=np.float64).reshape(10, self.N))
        rc = self._lib.oracle_init(self.lattice, *self._dims(), _dp(m), _dp(self.F), _dp(self.f))
        assert rc == 0

    def moments(self):
        """Corrected moments [10, nz, ny, nx] of the current populations."""
        m = np.zeros((10, self.N), dtype=np.float64)
        rc = self._lib.oracle_moments(self.lattice, *self._dims(), _dp(self.f), _dp(self.F), _dp(m))
        assert rc == 0
        return m.reshape(10, self.nz, self.ny, self.nx)

    def step(self, n=1):
        bcp = self.bc.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        rc = self._lib.oracle_run(self.lattice, *self._dims(), bcp, self.tau, _dp(self.F),
                                  _dp(self.f), _dp(self._scratch), int(n))
        assert rc == 0

    def post_collision(self):
        """Post-collision populations f*[Q, N] of the current state."""
        out = np.zeros_like(self.f)
        rc = self._lib.oracle_collide(self.lattice, *self._dims(), self.tau, _dp(self.f),
                                      _dp(self.F), _dp(out))
        assert rc == 0
        return out
