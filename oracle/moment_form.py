"""Brute-force NumPy evaluation of the moment-space update, FP64.

TEST INFRASTRUCTURE (see the package docstring).  Independent of the C
population oracle: it has its own velocity-set construction and evaluates the
paper's moment-form equations literally, with generic Hermite tensors
H^(0) = 1, H^(1)_a = c_a, H^(2)_ab = c_a c_b - cs^2 d_ab (section 2):

  Eq. (7): a*^(n)(x, t+1) = sum_i H^(n)_i [ w_i sum_{m=0..2} H^(m)_i .
           (a_eq^(m) + (1 - omega) a_neq^(m))(x - c_i, t) / (cs^(2m) m!)
           + S_i(x - c_i, t) / 2 ]
  with a_eq = (p*, u, u u), a_neq = (0, 0, a2 - u u) (Eq. (6)) and S_i the
  Guo term of Eq. (9); then Eq. (8): a0 = a*0, u = a*1 + F/(2 rho),
  a2 = a*2 + (F u + u F)/(2 rho), with u the updated velocity and F at the
  destination (force at the updated time).

Walls (per axis, halfway bounce-back): where x - c_i lies beyond a wall the
pulled population is the one of the opposite direction at x itself.  Meant
for grids of at most a few thousand sites (Python loops over directions and
tensor orders, NumPy over sites).
"""
import itertools
import math

import numpy as np

CS2 = 1.0 / 3.0


def velocity_set(Q):
    """Textbook D3Q19 / D3Q27: c in {-1,0,1}^3 (|c|^2 <= 2 for Q=19)."""
    weights = {19: {0: 1 / 3, 1: 1 / 18, 2: 1 / 36},
               27: {0: 8 / 27, 1: 2 / 27, 2: 1 / 54, 3: 1 / 216}}[Q]
    cs, ws = [], []
    for c in itertools.product((-1, 0, 1), repeat=3):
        c2 = sum(v * v for v in c)
        if c2 in weights:
            cs.append(c)
            ws.append(weights[c2])
    return np.array(cs, dtype=np.int64), np.array(ws, dtype=np.float64)


def hermite(c):
    """[H0, H1[3], H2[3,3]] for one velocity c."""
    c = np.asarray(c, dtype=np.float64)
    return [np.float64(1.0), c.copy(), np.outer(c, c) - CS2 * np.eye(3)]


def _full(m):
    """moments [10, ...] -> (a0, a1[3,...], a2[3,3,...])."""
    a0 = m[0]
    a1 = m[1:4]
    a2 = np.empty((3, 3) + m.shape[1:])
    for (a, b), k in {(0, 0): 4, (1, 1): 5, (2, 2): 6, (0, 1): 7, (0, 2): 8, (1, 2): 9}.items():
        a2[a, b] = m[k]
        a2[b, a] = m[k]
    return a0, a1, a2


def _pack(a0, a1, a2):
    return np.stack([a0, a1[0], a1[1], a1[2], a2[0, 0], a2[1, 1], a2[2, 2],
                     a2[0, 1], a2[0, 2], a2[1, 2]])


def _contract(Hm, am):
    """H^(m) : a^(m) over the tensor indices, sites broadcast."""
    if np.ndim(Hm) == 0:
        return Hm * am
    if np.ndim(Hm) == 1:
        return np.tensordot(Hm, am, axes=(0, 0))
    return np.tensordot(Hm, am, axes=([0, 1], [0, 1]))


def _guo(c, w, u, F, rho):
    """Eq. (9) as printed: w [ (c_a - u_a)/cs^2 + (c.u) c_a / cs^4 ] F_a / rho."""
    cu = sum(c[b] * u[b] for b in range(3))
    s = sum(((c[a] - u[a]) / CS2 + cu * c[a] / CS2 ** 2) * F[a] for a in range(3))
    return w * s / rho


def step(m, Q, tau, F=None, bc=(0, 0, 0), rho=1.0):
    """One update of the moment state m[10, nz, ny, nx]; returns the new state."""
    m = np.asarray(m, dtype=np.float64)
    shape = m.shape[1:]
    c, w = velocity_set(Q)
    omega = 1.0 / tau
    F = np.zeros(3) if F is None else np.asarray(F, dtype=np.float64)
    if F.shape == (3,):
        F = np.broadcast_to(F[:, None, None, None], (3,) + shape)
    else:
        F = F.reshape((3,) + shape)
    a0, u, a2 = _full(m)
    uu = np.einsum("a...,b...->ab...", u, u)
    a_eq = [a0, u, uu]
    a_neq = [np.zeros_like(a0), np.zeros_like(u), a2 - uu]

    # post-collision population at every (source) site, per direction
    post = []
    for i in range(len(c)):
        H = hermite(c[i])
        g = np.zeros(shape)
        for mo in range(3):
            g = g + _contract(H[mo], a_eq[mo] + (1.0 - omega) * a_neq[mo]) / (
                CS2 ** mo * math.factorial(mo))
        g = w[i] * g + 0.5 * _guo(c[i], w[i], u, F, rho)
        post.append(g)

    # pull: value at x comes from x - c_i; array axes are (z, y, x)
    opp = [int(np.flatnonzero((c == -c[i]).all(axis=1))[0]) for i in range(len(c))]
    n_axes = (shape[2], shape[1], shape[0])
    pulled = []
    for i in range(len(c)):
        g = post[i]
        for a in range(3):
            g = np.roll(g, shift=int(c[i][a]), axis=2 - a)
        solid = np.zeros(shape, dtype=bool)
        for a in range(3):
            if bc[a] and c[i][a] != 0:
                idx = np.arange(n_axes[a])
                edge = (idx - c[i][a] < 0) | (idx - c[i][a] >= n_axes[a])
                sel = [None, None, None]
                sel[2 - a] = slice(None)
                solid |= np.broadcast_to(edge[tuple(sel)], shape)
        g = np.where(solid, post[opp[i]], g)
        pulled.append(g)

    # projection on H^(n), Eq. (5)/(7)
    s0 = np.zeros(shape)
    s1 = np.zeros((3,) + shape)
    s2 = np.zeros((3, 3) + shape)
    for i in range(len(c)):
        H = hermite(c[i])
        s0 = s0 + H[0] * pulled[i]
        s1 = s1 + H[1][:, None, None, None] * pulled[i]
        s2 = s2 + H[2][:, :, None, None, None] * pulled[i]

    # correction, Eq. (8)
    u_new = s1 + F / (2.0 * rho)
    a2_new = s2 + (np.einsum("a...,b...->ab...", F, u_new)
                   + np.einsum("a...,b...->ab...", u_new, F)) / (2.0 * rho)
    return _pack(s0, u_new, a2_new)


def run(m, Q, tau, nsteps, F=None, bc=(0, 0, 0)):
    for _ in range(nsteps):
        m = step(m, Q, tau, F=F, bc=bc)
    return m
