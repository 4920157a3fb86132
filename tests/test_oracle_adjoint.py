"""Pins of the FP64 CPU adjoint (oracle/adjoint.py) against facts that do not
come from its own algebra: central finite differences of the C oracle's
forward model, and the exact gradients that mass and momentum conservation
impose on linear objectives (any state, any force)."""
import numpy as np
import pytest

from paper_2609_09160_amd import inputs


def _case(shape, seed):
    N = int(np.prod(shape))
    rng = np.random.default_rng(seed)
    m0 = inputs.random_state(shape, seed=seed + 1).reshape(10, N)
    F = 1e-3 * rng.standard_normal((3, N))
    return rng, m0, F


@pytest.mark.parametrize("bc", [(0, 0, 0), (0, 1, 0), (1, 1, 1)])
@pytest.mark.parametrize("Q", [19, 27])
def test_adjoint_matches_finite_differences(oracle_mod, Q, bc):
    """J = r.m(T) + |u(T)|^2/2 on a 6x5x4 grid, 12 steps, random state and a
    force of 1e-3 (so the force terms of every transposed map carry weight
    ~1e-3 of the gradient): the directional derivatives along random unit
    directions in F and in m0 equal central differences of the forward model
    (step 1e-5, truncation ~1e-10, rounding ~1e-9 of J) to 1e-6 relative.
    A dropped term, a wrong sign or a transposed index in any transposed
    step (streaming, collision, Guo term, moment correction, initialisation)
    moves the result by far more."""
    from oracle import adjoint as A
    shape = (6, 5, 4)
    N = int(np.prod(shape))
    rng, m0, F = _case(shape, 7 * Q + sum(bc))
    r = rng.standard_normal((10, N))
    tau, steps = 0.7, 12

    def J(m):
        return float((r * m).sum() + 0.5 * (m[1:4] ** 2).sum())

    mT = A.forward(Q, shape, tau, m0, F, steps, bc)
    gT = r.copy()
    gT[1:4] += mT[1:4]
    gF, g0 = A.adjoint(Q, shape, tau, m0, F, steps, gT, bc)
    eps = 1e-5
    for _ in range(3):
        for which in ("F", "m0"):
            d = rng.standard_normal((3 if which == "F" else 10, N))
            d /= np.linalg.norm(d)
            if which == "F":
                Jp = J(A.forward(Q, shape, tau, m0, F + eps * d, steps, bc))
                Jm = J(A.forward(Q, shape, tau, m0, F - eps * d, steps, bc))
                ad = float((gF * d).sum())
            else:
                Jp = J(A.forward(Q, shape, tau, m0 + eps * d, F, steps, bc))
                Jm = J(A.forward(Q, shape, tau, m0 - eps * d, F, steps, bc))
                ad = float((g0 * d).sum())
            fd = (Jp - Jm) / (2 * eps)
            assert abs(fd - ad) <= 1e-6 * abs(ad), (which, fd, ad)


@pytest.mark.parametrize("Q", [19, 27])
def test_adjoint_of_conserved_totals(oracle_mod, Q):
    """Periodic domain: sum p* is invariant and sum u(t+1) = sum u(t) + sum F
    exactly (half the force enters at the source, half in the correction), for
    any state.  So for J = r.sum u(T) + s sum p*(T) (uniform r, s) the exact
    gradients are dJ/dF = T r, dJ/du0 = r, dJ/dp0 = s, dJ/da2 = 0 at every
    site.  Catches a wrong weight on either half of the force, or a leak
    between the moment groups."""
    from oracle import adjoint as A
    shape = (5, 4, 3)
    N = int(np.prod(shape))
    _, m0, F = _case(shape, 40 + Q)
    steps = 9
    r = np.array([0.3, -1.1, 0.7])
    s = 0.9
    gT = np.zeros((10, N))
    gT[0] = s
    gT[1:4] = r[:, None]
    gF, g0 = A.adjoint(Q, shape, 0.8, m0, F, steps, gT)
    assert np.abs(gF - steps * r[:, None]).max() <= 1e-13
    assert np.abs(g0[0] - s).max() <= 1e-13
    assert np.abs(g0[1:4] - r[:, None]).max() <= 1e-13
    assert np.abs(g0[4:]).max() <= 1e-13


@pytest.mark.parametrize("Q", [19, 27])
def test_streaming_map_is_a_permutation(oracle_mod, Q):
    """Halfway bounce-back and periodic wrap move every post-collision value
    to exactly one place, so the transpose of streaming is its inverse."""
    from oracle import adjoint as A
    for bc in ((0, 0, 0), (0, 1, 0), (1, 1, 1)):
        idx = A.stream_source_index(Q, (4, 3, 5), bc)
        assert np.array_equal(np.sort(idx.ravel()), np.arange(idx.size))
