"""The algebra of the two-iteration (s-step, s = 2) CG, restated in numpy
and pinned to the oracle's Hestenes-Stiefel PLCG.

The GPU kernels form Y = [p, Bp, B^2 p, r/6, B r/6] with B = A/6 - I
(A = -M), sum 12 moments instead of the 15 Gram products (B is symmetric,
so <B^a u, B^b v> depends on a + b only), and run two CG iterations on
5-vectors with Ahat v = v + S v. This test performs the same steps with
numpy on small periodic grids and checks that
* the moment Gram equals Y^T Y;
* after 2k (and 2k + 1) iterations the iterate equals the oracle's PLCG
  iterate after as many iterations, to rounding.
"""
import numpy as np
import pytest

import oracle


def gidx(a, b):
    return a * 5 - a * (a - 1) // 2 + (b - a)


def gmom(a, b):
    """Moment holding Gram entry (a, b), a <= b (p-block 0..2, rhat-block 3..4)."""
    if b <= 2:
        return a + b
    if a <= 2:
        return 5 + a + (b - 3)
    return 9 + (a - 3) + (b - 3)


def B_op(v):
    """B = A/6 - I = -(sum of the six periodic neighbours)/6."""
    s = sum(np.roll(v, sh, ax) for ax in range(3) for sh in (1, -1))
    return -s / 6.0


def moments(Y):
    p, bp, b2p, rh, brh = Y
    return np.array([np.vdot(p, p), np.vdot(p, bp), np.vdot(bp, bp), np.vdot(bp, b2p),
                     np.vdot(b2p, b2p), np.vdot(p, rh), np.vdot(p, brh), np.vdot(bp, brh),
                     np.vdot(b2p, brh), np.vdot(rh, rh), np.vdot(rh, brh), np.vdot(brh, brh)])


def gram_from_moments(m):
    G = np.zeros((5, 5))
    for a in range(5):
        for b in range(a, 5):
            G[a, b] = G[b, a] = m[gmom(a, b)]
    return G


def ahat(v):
    return np.array([v[0], v[1] + v[0], v[1], v[3], v[3]])


def two_iteration_cg(b, n_iter):
    """x after n_iter iterations of the two-iteration form from x = 0."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r / 6.0
    it = 0
    while it < n_iter:
        Y = [p, B_op(p), None, r / 6.0, None]
        Y[2] = B_op(Y[1])
        Y[4] = B_op(Y[3])
        G = gram_from_moments(moments(Y))
        xv = np.zeros(5)
        rv = np.array([0.0, 0, 0, 1, 0])
        pv = np.array([1.0, 0, 0, 0, 0])
        rr = rv @ G @ rv
        for _ in range(min(2, n_iter - it)):
            ap = ahat(pv)
            al = rr / (pv @ G @ ap)
            xv = xv + al * pv
            rv = rv - al * ap
            rr2 = rv @ G @ rv
            pv = rv + (rr2 / rr) * pv
            rr = rr2
            it += 1
        Ym = np.stack(Y)
        x = x + np.tensordot(xv, Ym, 1)
        r = 6.0 * np.tensordot(rv, Ym, 1)
        p = np.tensordot(pv, Ym, 1)
    return x


def rhs(N, seed):
    rng = np.random.default_rng(seed)
    b = rng.standard_normal((N, N, N))
    return b - b.mean()


@pytest.mark.parametrize("N", [6, 9, 12])
def test_moment_gram_equals_products(N):
    rng = np.random.default_rng(N)
    p, r = rng.standard_normal((2, N, N, N))
    Y = [p, B_op(p), B_op(B_op(p)), r / 6.0, B_op(r / 6.0)]
    G = np.array([[np.vdot(u, v) for v in Y] for u in Y])
    Gm = gram_from_moments(moments(Y))
    assert np.abs(G - Gm).max() <= 1e-12 * np.abs(G).max()


@pytest.mark.parametrize("N,n_iter", [(8, 2), (8, 7), (10, 12), (12, 13), (12, 30)])
def test_iterates_equal_the_oracle_plcg(N, n_iter):
    b = rhs(N, seed=N + n_iter)
    x = two_iteration_cg(b, n_iter)
    ref, it, _ = oracle.pcg(b, thr=0.0, max_iter=n_iter)
    assert it == n_iter
    # the same Krylov iterate, to rounding amplified by the conditioning
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)
    # and a genuine solve: the residual falls with the iterations
    res = np.linalg.norm(b + oracle.apply_M(x)) / np.linalg.norm(b)
    assert res < 1.0
