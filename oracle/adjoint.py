"""FP64 CPU discrete adjoint of the population oracle.

TEST INFRASTRUCTURE (see the package docstring).  The paper does not treat
differentiation; what is differentiated here is the oracle's own discrete
model, in its population form (the form the moment update of Eq. (7) + Eq. (8)
is equivalent to):

  f(0)   = Init(m0, F):  f_i = w_i [a0 + c_i.(u - F/2)/cs^2
                                   + H2_i:(a2 - (F u + u F)/2)/(2 cs^4)]
  f(t+1) = Stream(Collide(f(t), F)), with, at every site,
           moments (Eq. (5) corrected as in Eq. (8)): p = sum f,
             u = sum c f + F/2, a2 = sum H2 f + (F u + u F)/2;
           Collide (Eq. (3) with Eqs. (4), (6), (9)):
             f*_i = w_i [p + c_i.u/cs^2 + H2_i:u u/(2 cs^4)]
                  + (1 - omega) w_i H2_i:(a2 - u u)/(2 cs^4)
                  + (1/2) w_i [(c_i - u).F/cs^2 + (c_i.u)(c_i.F)/cs^4];
           Stream: pull with periodic wrap, or halfway bounce-back
             f_i(x, t+1) = f*_{-i}(x) where x - c_i lies beyond a wall;
  m(T)   = moments(f(T)),  rho = 1, F static in time.

Given g = dJ/dm(T) (10 planes, second-order planes by stored component),
`adjoint()` returns dJ/dF (3 planes) and dJ/dm0 (10 planes) by transposing
each of these maps by hand, in population space (Q values per site).  The GPU
path differentiates the moment form instead, so the two share no algebra.
The forward trajectory comes from the C oracle; only u(t) is kept.
"""
import numpy as np

from . import PopulationOracle, lattice_tables

CS2 = 1.0 / 3.0


def _tables(Q):
    c, w = lattice_tables(Q)
    c = c.astype(np.float64)
    H2 = np.einsum("ia,ib->iab", c, c) - CS2 * np.eye(3)[None]
    return c, w, H2


def stream_source_index(Q, shape, bc):
    """Flat index into fpost[Q, N] of the value that streaming delivers to
    f[i, x] (pull from x - c_i; on a walled axis, beyond the wall, the
    opposite direction at x itself).  The map is a permutation of Q*N."""
    c, _ = lattice_tables(Q)
    nx, ny, nz = shape
    N = nx * ny * nz
    opp = np.array([int(np.nonzero((c == -c[i]).all(axis=1))[0][0]) for i in range(Q)])
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pos = (x.ravel(), y.ravel(), z.ravel())
    n = (nx, ny, nz)
    site = np.arange(N)
    idx = np.empty((Q, N), dtype=np.int64)
    for i in range(Q):
        src = [pos[a] - c[i, a] for a in range(3)]
        outside = np.zeros(N, dtype=bool)
        for a in range(3):
            if bc[a]:
                outside |= (src[a] < 0) | (src[a] >= n[a])
            else:
                src[a] = np.mod(src[a], n[a])
        flat = np.where(outside, 0, src[0] + nx * (src[1] + ny * src[2]))
        idx[i] = np.where(outside, opp[i] * N + site, i * N + flat)
    return idx


def _sym_from_stored(g):
    """Full symmetric 3x3 gradient from the gradient of the 6 stored
    components (an off-diagonal stored value stands for two entries)."""
    G = np.empty((3, 3) + g.shape[1:])
    G[0, 0], G[1, 1], G[2, 2] = g[0], g[1], g[2]
    G[0, 1] = G[1, 0] = 0.5 * g[3]
    G[0, 2] = G[2, 0] = 0.5 * g[4]
    G[1, 2] = G[2, 1] = 0.5 * g[5]
    return G


def _stored_from_full(G):
    """Gradient of the 6 stored components from the full-tensor gradient."""
    return np.stack([G[0, 0], G[1, 1], G[2, 2], G[0, 1] + G[1, 0], G[0, 2] + G[2, 0],
                     G[1, 2] + G[2, 1]])


def _moments_transpose(c, H2, gp, gu, GA, u, F):
    """Transpose of the corrected moments at every site.  (gp, gu, GA) are the
    gradients with respect to p, u and the full a2; returns dJ/df [Q, N] and
    the contribution to dJ/dF [3, N] (u = j + F/2, a2 = Pi + (F u + u F)/2)."""
    gu_tot = gu + np.einsum("abn,bn->an", GA, F)  # a2 depends on u
    lam_f = gp[None] + c @ gu_tot + H2.reshape(-1, 9) @ GA.reshape(9, -1)
    gF = 0.5 * gu_tot + np.einsum("abn,bn->an", GA, u)
    return lam_f, gF


def _collide_transpose(c, w, H2, omega, lam_post, u, F):
    """Transpose of Collide with respect to (p, u, full a2) at every site, and
    the direct dependence of the Guo term on F."""
    ell = w[:, None] * lam_post  # w_i dJ/df*_i
    gp = ell.sum(axis=0)
    Lc = c.T @ ell                                          # sum ell c
    LH = (H2.reshape(-1, 9).T @ ell).reshape(3, 3, -1)      # sum ell H2
    Lcc = np.einsum("ia,ib,in->abn", c, c, ell)             # sum ell c c
    LHu = np.einsum("abn,bn->an", LH, u)
    gu = Lc / CS2 + omega * LHu / CS2**2 \
        + 0.5 * (-gp[None] * F / CS2 + np.einsum("abn,bn->an", Lcc, F) / CS2**2)
    GA = (1.0 - omega) * LH / (2.0 * CS2**2)
    gF = 0.5 * ((Lc - gp[None] * u) / CS2 + np.einsum("abn,bn->an", Lcc, u) / CS2**2)
    return gp, gu, GA, gF


def _init_transpose(c, w, H2, lam_f0, u0, F):
    ell = w[:, None] * lam_f0
    Lc = c.T @ ell
    LH = (H2.reshape(-1, 9).T @ ell).reshape(3, 3, -1)
    g0 = np.empty((10,) + ell.shape[1:])
    g0[0] = ell.sum(axis=0)
    g0[1:4] = Lc / CS2 - np.einsum("abn,bn->an", LH, F) / (2.0 * CS2**2)
    g0[4:10] = _stored_from_full(LH / (2.0 * CS2**2))
    gF = -Lc / (2.0 * CS2) - np.einsum("abn,bn->an", LH, u0) / (2.0 * CS2**2)
    return g0, gF


def forward(Q, shape, tau, m0, F, steps, bc=(0, 0, 0)):
    """m(T) of the C oracle (FP64), [10, N]."""
    nx, ny, nz = shape
    o = PopulationOracle(Q, shape, tau, bc=bc, force=F)
    o.set_moments(m0)
    o.step(steps)
    return o.moments().reshape(10, nx * ny * nz)


def adjoint(Q, shape, tau, m0, F, steps, gT, bc=(0, 0, 0)):
    """(dJ/dF [3, N], dJ/dm0 [10, N]) for dJ/dm(T) = gT [10, N]."""
    nx, ny, nz = shape
    N = nx * ny * nz
    F = np.ascontiguousarray(np.asarray(F, dtype=np.float64).reshape(3, N))
    m0 = np.ascontiguousarray(np.asarray(m0, dtype=np.float64).reshape(10, N))
    gT = np.asarray(gT, dtype=np.float64).reshape(10, N)
    c, w, H2 = _tables(Q)
    omega = 1.0 / tau
    idx = stream_source_index(Q, shape, bc)
    # forward sweep: velocities u(t), t = 0..T
    o = PopulationOracle(Q, shape, tau, bc=bc, force=F)
    o.set_moments(m0)
    U = np.empty((steps + 1, 3, N))
    for t in range(steps + 1):
        U[t] = o.moments().reshape(10, N)[1:4]
        if t < steps:
            o.step(1)
    # seed: the moments of f(T)
    lam_f, gF = _moments_transpose(c, H2, gT[0], gT[1:4], _sym_from_stored(gT[4:10]), U[steps], F)
    for t in range(steps - 1, -1, -1):
        lam_post = np.empty(Q * N)
        lam_post[idx.ravel()] = lam_f.ravel()  # Stream is a permutation
        gp, gu, GA, gF_s = _collide_transpose(c, w, H2, omega, lam_post.reshape(Q, N), U[t], F)
        lam_f, gF_m = _moments_transpose(c, H2, gp, gu, GA, U[t], F)
        gF += gF_s + gF_m
    g0, gF_i = _init_transpose(c, w, H2, lam_f, m0[1:4], F)
    gF += gF_i
    return gF, g0
