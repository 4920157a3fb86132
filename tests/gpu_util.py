"""Shared helpers of the GPU tests: run the HIP path and the CPU oracle on the
same seeded inputs and measure their difference."""
import sys

import numpy as np

GROUPS = ((0, 1), (1, 4), (4, 10))  # p*, u, a2


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_run(shape, tau, m0, steps, lattice=19, storage="f64", bc=(0, 0, 0), force=(0, 0, 0),
            Ffield=None, launch=None, scale=None, rounding="auto"):
    """Run the HIP path; returns host float64 moments [10, nz, ny, nx]."""
    import torch
    from paper_2609_09160_amd import Solver
    s = Solver(shape, tau, lattice=lattice, storage=storage, bc=bc, force=force, scale=scale,
               rounding=rounding)
    if launch:
        s.set_launch(*launch)
    s.set_moments(np.ascontiguousarray(m0))
    if Ffield is not None:
        s.set_force_field(torch.as_tensor(Ffield, device="cuda"))
    s.step(steps)
    out = s.moments().cpu().numpy()
    s.close()
    return out


def stored_planes(words, nplanes, N):
    """The binary16 words of a 16-bit state as [nplanes, N], plane by plane,
    from the layout the library documents: planes 4j .. 4j + 3 interleaved
    site by site in words [4jN, (4j + 4)N), plane 4j first (the lowest 16
    bits of each 64-bit word); two planes left over interleaved the same way
    after the groups; a last single plane on its own."""
    words = np.asarray(words).reshape(-1)[:nplanes * N]
    out = np.empty((nplanes, N), dtype=words.dtype)
    q4 = nplanes & ~3
    for j in range(q4 // 4):
        grp = words[4 * j * N:(4 * j + 4) * N].reshape(N, 4)
        for c in range(4):
            out[4 * j + c] = grp[:, c]
    k = q4
    if nplanes - q4 >= 2:
        pair = words[q4 * N:(q4 + 2) * N].reshape(N, 2)
        out[q4], out[q4 + 1] = pair[:, 0], pair[:, 1]
        k = q4 + 2
    if k < nplanes:
        out[k] = words[k * N:(k + 1) * N]
    return out


def oracle_run(shape, tau, m0, steps, lattice=19, bc=(0, 0, 0), force=None):
    import oracle
    o = oracle.PopulationOracle(lattice, shape, tau, bc=bc, force=force)
    o.set_moments(m0)
    o.step(steps)
    return o.moments()


_CACHE = {}


def lattice_number(Q):
    """An integer for seeds and labels: 19, 27, or 270 for "27h"."""
    return 270 if Q == "27h" else int(Q)


def solenoidal_oracle_1000(Q, n=64, tau=0.6):
    """Oracle moments after 1000 steps of the n^3 solenoidal workload (cached:
    several storage types compare against the same reference)."""
    key = (Q, n, tau)
    if key not in _CACHE:
        m0 = __import__("paper_2609_09160_amd.inputs", fromlist=["x"]).solenoidal_field((n, n, n))
        _CACHE[key] = (m0, oracle_run((n, n, n), tau, m0, 1000, lattice=Q))
    return _CACHE[key]


def oracle_site_update(crop, Q, tau):
    """One oracle step at the centre of a 3x3x3 neighbourhood [10, 3, 3, 3]
    (z, y, x): the pull at the centre reads only its 26 neighbours, so a
    periodic 3^3 box gives the exact update of that site."""
    import oracle
    o = oracle.PopulationOracle(Q, (3, 3, 3), tau)
    o.set_moments(np.ascontiguousarray(crop))
    o.step(1)
    return o.moments()[:, 1, 1, 1]


def state_rel_err(got, want):
    """max|got - want| over all moments / max|want| over all moments, and the
    same for the velocity group alone; rounding scales with the state's
    magnitude, so a moment that has decayed far below the others is judged
    against the state, not against itself."""
    st = float(np.abs(got - want).max() / np.abs(want).max())
    vel = float(np.abs(got[1:4] - want[1:4]).max() / np.abs(want[1:4]).max())
    return max(st, vel)


def group_rel_err(got, want):
    """Max over the groups (p*, u, a2) of max|got - want| / max|want in group|
    (a sub-array of fewer than 10 moments is one group)."""
    err = 0.0
    for lo, hi in (GROUPS if len(want) == 10 else ((0, len(want)),)):
        ref = np.abs(want[lo:hi]).max()
        d = np.abs(got[lo:hi] - want[lo:hi]).max()
        err = max(err, d / ref if ref > 0 else d)
    return err


def u_rel_l2(got, want):
    return float(np.linalg.norm(got[1:4] - want[1:4]) / np.linalg.norm(want[1:4]))
