"""Python front end of the C ABI: device memory and streams come from torch,
every step of the method runs in liblbfast.so."""
import ctypes

import numpy as np

from . import _lib
from ._lib import check

N_MOMENTS = 10
MOMENT_NAMES = ("p*", "ux", "uy", "uz", "a2xx", "a2yy", "a2zz", "a2xy", "a2xz", "a2yz")


class Solver:
    """One moment-represented LBM lattice on one GPU.

    shape = (nx, ny, nz); lattice in {19, 27, "27h"} ("27h": the D3Q27 set
    with the complete Hermite basis); storage in {"f64", "f32", "f16s", "bf16s",
    "f16su"} ("f16su": FP16 with the velocity split over two 16-bit words);
    bc = per-axis 0 (periodic) / 1 (walls, y only); force = uniform body force;
    rounding = "auto" (FP16 to nearest, BF16 stochastic), "nearest" or
    "stochastic" (16-bit storage: how the step rounds p* and u).
    The two flip/flop moment buffers are torch allocations on `device`, the
    launches go to torch's current stream of that device.
    """

    def __init__(self, shape, tau, lattice=19, storage="f32", bc=(0, 0, 0),
                 force=(0.0, 0.0, 0.0), scale=None, device=None, rounding="auto"):
        import torch
        self._torch = torch
        self.lib = _lib.load()
        self.shape = tuple(int(v) for v in shape)
        self.N = self.shape[0] * self.shape[1] * self.shape[2]
        self.storage = storage
        self.compute_dtype = torch.float64 if storage == "f64" else torch.float32
        self.device = torch.device(device if device is not None else "cuda")
        self.params = _lib.make_params(self.shape, tau, lattice, storage, bc, force, scale,
                                       rounding)
        nbytes = self.lib.lbfast_buffer_bytes(ctypes.byref(self.params))
        if nbytes == 0:
            check(_lib.LBF_E_ARG)
        self._bufs = [torch.empty(nbytes, dtype=torch.uint8, device=self.device) for _ in range(2)]
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        check(self.lib.lbfast_create(ctypes.byref(self.params),
                                     ctypes.c_void_p(self.stream.cuda_stream),
                                     ctypes.c_void_p(self._bufs[0].data_ptr()),
                                     ctypes.c_void_p(self._bufs[1].data_ptr()), ctypes.byref(h)))
        self.h = h
        self._force_field = None

    # -- state -----------------------------------------------------------------
    def _as_moments(self, m):
        torch = self._torch
        if isinstance(m, np.ndarray):
            m = torch.from_numpy(np.ascontiguousarray(m))
        if m.dtype not in (torch.float64, torch.float32):
            raise TypeError("moments must be float64 or float32")
        if m.numel() != N_MOMENTS * self.N:
            raise ValueError(f"expected 10 x {self.N} values, got {tuple(m.shape)}")
        return m.contiguous()

    def set_moments(self, m):
        """m: [10, nz, ny, nx] (or [10, N]) float64/float32, host or device."""
        torch = self._torch
        m = self._as_moments(m)
        dt = _lib.LBF_F64 if m.dtype == torch.float64 else _lib.LBF_F32
        on_dev = 1 if m.is_cuda else 0
        check(self.lib.lbfast_set_moments(self.h, ctypes.c_void_p(m.data_ptr()), dt, on_dev))
        if on_dev:
            self.sync()

    def moments(self, dtype=None, out=None):
        """Current state as a device tensor [10, nz, ny, nx] (float64 default)."""
        torch = self._torch
        dtype = dtype or torch.float64
        nx, ny, nz = self.shape
        if out is None:
            out = torch.empty((N_MOMENTS, nz, ny, nx), dtype=dtype, device=self.device)
        dt = _lib.LBF_F64 if out.dtype == torch.float64 else _lib.LBF_F32
        check(self.lib.lbfast_get_moments(self.h, ctypes.c_void_p(out.data_ptr()), dt, 1))
        return out

    def moments_host(self, dtype=np.float64):
        nx, ny, nz = self.shape
        out = np.empty((N_MOMENTS, nz, ny, nx), dtype=dtype)
        dt = _lib.LBF_F64 if dtype == np.float64 else _lib.LBF_F32
        check(self.lib.lbfast_get_moments(self.h, out.ctypes.data_as(ctypes.c_void_p), dt, 0))
        return out

    def set_force_field(self, F):
        """Per-site force [3, nz, ny, nx] device tensor of the compute dtype (kept
        alive by this object), or None for the uniform force."""
        torch = self._torch
        if F is None:
            check(self.lib.lbfast_set_force_field(self.h, None, 0))
            self._force_field = None
            return
        F = F.to(device=self.device, dtype=self.compute_dtype).contiguous()
        if F.numel() != 3 * self.N:
            raise ValueError("force field must have 3 x N values")
        dt = _lib.LBF_F64 if F.dtype == torch.float64 else _lib.LBF_F32
        check(self.lib.lbfast_set_force_field(self.h, ctypes.c_void_p(F.data_ptr()), dt))
        self._force_field = F

    def set_launch(self, tile_rows=0, z_chunk=0, lane_sites=0):
        """Launch shape: rows per tile, z-planes per workgroup, x-sites per
        lane (0 keeps the current value).  Sites per lane are applied first."""
        if lane_sites:
            check(self.lib.lbfast_set_lane_sites(self.h, int(lane_sites)))
        check(self.lib.lbfast_set_launch(self.h, int(tile_rows), int(z_chunk)))

    def set_block_order(self, order=0):
        """Workgroup order over the XCDs: 0 automatic, 1 hardware order,
        2 contiguous tile ranges per XCD (same results bit for bit)."""
        check(self.lib.lbfast_set_block_order(self.h, int(order)))

    def set_adjoint_launch(self, sites=0, tile_rows=0):
        """Launch shape of the adjoint step (0 = automatic)."""
        check(self.lib.lbfast_set_adjoint_launch(self.h, int(sites), int(tile_rows)))

    def scales(self):
        out = (ctypes.c_float * 10)()
        check(self.lib.lbfast_get_scales(self.h, out))
        return np.array(out[:], dtype=np.float32)

    # -- time stepping -----------------------------------------------------------
    def step(self, n=1):
        check(self.lib.lbfast_step(self.h, int(n)))

    def sync(self):
        check(self.lib.lbfast_sync(self.h))

    def reduce(self):
        """FP64 [sum p*, sum ux, sum uy, sum uz, 1/2 sum |u|^2]."""
        out = (ctypes.c_double * 5)()
        rc = self.lib.lbfast_reduce(self.h, out)
        check(rc)
        return np.array(out[:])

    # -- two-component variant -------------------------------------------------------
    def enable_two_phase(self, sigma, width, diffusivity, rho=(1.0, 1.0), tau=None):
        """Two-component variant: phase field by the conservative Allen-Cahn
        equation, capillary force, and densities rho = (light, heavy) and
        relaxation times tau = (light, heavy) blended in the phase field
        (tau: one value for both phases, default the solver's tau).  The
        solver's uniform force is read as a body acceleration."""
        pp = _lib.LbfastPhaseParams()
        pp.struct_size = ctypes.sizeof(_lib.LbfastPhaseParams)
        pp.sigma, pp.width, pp.diffusivity = float(sigma), float(width), float(diffusivity)
        pp.rho_l, pp.rho_h = (float(v) for v in rho)
        t = self.params.tau if tau is None else tau
        pp.tau_l, pp.tau_h = (float(v) for v in (t if np.ndim(t) else (t, t)))
        check(self.lib.lbfast_enable_two_phase(self.h, ctypes.byref(pp)))

    def set_phase(self, phi):
        """phi: [nz, ny, nx] (or N) float64/float32, host or device."""
        torch = self._torch
        if isinstance(phi, np.ndarray):
            phi = torch.from_numpy(np.ascontiguousarray(phi))
        if phi.dtype not in (torch.float64, torch.float32) or phi.numel() != self.N:
            raise ValueError("phi must be N float64/float32 values")
        phi = phi.contiguous()
        dt = _lib.LBF_F64 if phi.dtype == torch.float64 else _lib.LBF_F32
        check(self.lib.lbfast_set_phase(self.h, ctypes.c_void_p(phi.data_ptr()), dt,
                                        1 if phi.is_cuda else 0))
        self.sync()

    def phase(self, dtype=None):
        """Current phase field as a device tensor [nz, ny, nx] (float64 default)."""
        torch = self._torch
        nx, ny, nz = self.shape
        out = torch.empty((nz, ny, nx), dtype=dtype or torch.float64, device=self.device)
        dt = _lib.LBF_F64 if out.dtype == torch.float64 else _lib.LBF_F32
        check(self.lib.lbfast_get_phase(self.h, ctypes.c_void_p(out.data_ptr()), dt, 1))
        return out

    # -- discrete adjoint ----------------------------------------------------------
    def buffer_bytes(self):
        return self._bufs[0].numel()

    def forward_checkpointed(self, nsteps, every):
        """Advance nsteps, saving the state every `every` steps; returns the
        checkpoint tensor (ceil(nsteps/every) state buffers) for adjoint()."""
        torch = self._torch
        nseg = (int(nsteps) + int(every) - 1) // int(every) if nsteps > 0 and every > 0 else 0
        ckpt = torch.empty(max(nseg, 1) * self.buffer_bytes(), dtype=torch.uint8,
                           device=self.device)
        check(self.lib.lbfast_forward_checkpointed(self.h, int(nsteps), int(every),
                                                   ctypes.c_void_p(ckpt.data_ptr())))
        return ckpt

    def adjoint(self, nsteps, every, ckpt, lam_T, want_m0=True):
        """Reverse sweep over the nsteps run by forward_checkpointed: for
        lam_T = dJ/dm(T) (10 x N), returns (dJ/dF [3, nz, ny, nx],
        dJ/dm(0) [10, nz, ny, nx] or None), in the compute dtype."""
        torch = self._torch
        nx, ny, nz = self.shape
        lam_T = lam_T.to(device=self.device, dtype=self.compute_dtype).contiguous()
        if lam_T.numel() != N_MOMENTS * self.N:
            raise ValueError("lam_T must have 10 x N values")
        gF = torch.empty((3, nz, ny, nx), dtype=self.compute_dtype, device=self.device)
        lam0 = torch.empty((N_MOMENTS, nz, ny, nx), dtype=self.compute_dtype,
                           device=self.device) if want_m0 else None
        wb = self.lib.lbfast_adjoint_work_bytes(self.h, int(every))
        if wb == 0:
            check(_lib.LBF_E_ARG)
        work = torch.empty(wb, dtype=torch.uint8, device=self.device)
        check(self.lib.lbfast_adjoint(self.h, int(nsteps), int(every),
                                      ctypes.c_void_p(ckpt.data_ptr()),
                                      ctypes.c_void_p(lam_T.data_ptr()),
                                      ctypes.c_void_p(gF.data_ptr()),
                                      ctypes.c_void_p(lam0.data_ptr() if want_m0 else None),
                                      ctypes.c_void_p(work.data_ptr())))
        self.sync()
        del work
        return gF, lam0

    def state_ptr(self):
        p = ctypes.c_void_p()
        check(self.lib.lbfast_state_ptr(self.h, ctypes.byref(p)))
        return p.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.lbfast_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
