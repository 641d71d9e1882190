"""Pins of the oracle's stencil and linear solver against independent
mathematics: closed-form eigenvectors, a Kronecker-sum sparse matrix, a
dense direct solve and an FFT diagonalisation."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from conftest import fft_poisson

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def kron_laplacian(N):
    """Periodic 3-D second-difference matrix built as a Kronecker sum of the
    1-D circulant [1, -2, 1] (an independent construction of M)."""
    e = np.ones(N)
    d1 = sp.diags([e[:-1], -2 * e, e[:-1]], [-1, 0, 1], format="lil")
    d1[0, N - 1] = 1.0
    d1[N - 1, 0] = 1.0
    d1 = d1.tocsr()
    I = sp.identity(N, format="csr")
    return (sp.kron(sp.kron(d1, I), I) + sp.kron(sp.kron(I, d1), I)
            + sp.kron(sp.kron(I, I), d1)).tocsr()


@pytest.mark.parametrize("N", [4, 6, 9])
def test_apply_M_matches_kronecker_sum(oracle_lib, N):
    rng = np.random.default_rng(N)
    x = rng.standard_normal((N, N, N))
    got = oracle_lib.apply_M(x).ravel()
    ref = kron_laplacian(N) @ x.ravel()
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)


def test_stencil_row_from_paper(oracle_lib):
    g = json.load(open(os.path.join(GOLDEN, "paper_values.json")))["stencil_row"]
    N = 7
    e = np.zeros((N, N, N))
    e[3, 2, 5] = 1.0
    col = oracle_lib.apply_M(e)
    assert col[3, 2, 5] == g["diagonal"]
    assert np.count_nonzero(col) == g["nonzeros_per_row"]
    nz = col[col != 0]
    assert sorted(nz.tolist()).count(g["offdiagonal"]) == 6


@pytest.mark.parametrize("k", [(1, 0, 0), (0, 2, 1), (3, 1, 2)])
def test_apply_M_plane_wave_eigenvalue(oracle_lib, k):
    """M cos(2 pi k.n / N) = -sum_d 2 (1 - cos(2 pi k_d / N)) cos(2 pi k.n / N)."""
    N = 10
    i, j, l = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    th = 2 * np.pi * (k[0] * i + k[1] * j + k[2] * l) / N
    x = np.cos(th)
    lam = sum(2 * (1 - np.cos(2 * np.pi * kd / N)) for kd in k)
    np.testing.assert_allclose(oracle_lib.apply_M(x), -lam * x, atol=1e-12)


def test_apply_M_symmetric_and_kills_constants(oracle_lib):
    rng = np.random.default_rng(3)
    N = 8
    a, b = rng.standard_normal((2, N, N, N))
    lhs = np.vdot(a, oracle_lib.apply_M(b))
    rhs = np.vdot(oracle_lib.apply_M(a), b)
    assert abs(lhs - rhs) < 1e-10
    assert np.abs(oracle_lib.apply_M(np.ones((N, N, N)))).max() == 0.0


@pytest.mark.parametrize("N", [4, 6, 8])
def test_pcg_matches_dense_direct_solve(oracle_lib, N):
    """(-M) x = b for mean-zero b against LU of the dense regularised matrix
    -M + 11^T / G, whose solution on mean-zero b is the mean-zero x."""
    rng = np.random.default_rng(10 + N)
    G = N ** 3
    b = rng.standard_normal(G)
    b -= b.mean()
    A = -kron_laplacian(N).toarray() + np.ones((G, G)) / G
    ref = np.linalg.solve(A, b)
    x, it, ok = oracle_lib.pcg(b.reshape(N, N, N), thr=1e-14 * np.linalg.norm(b))
    assert ok
    x = x.ravel() - x.mean()
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("N", [12, 20, 32])
def test_pcg_matches_fft_solution(oracle_lib, N):
    rng = np.random.default_rng(N)
    q = rng.standard_normal((N, N, N))
    q -= q.mean()
    h = 0.4
    b = 4 * np.pi * q / h
    x, it, ok = oracle_lib.pcg(b, thr=1e-14 * np.linalg.norm(b))
    assert ok
    ref = fft_poisson(q, h)
    assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)


def test_jacobi_pcg_equals_plain_cg(oracle_lib):
    """A constant-diagonal Jacobi preconditioner leaves the CG iterates
    unchanged (Appendix B preconditioner on a stencil with diagonal -6): the
    iteration count and the iterate agree with unpreconditioned CG."""
    N = 12
    rng = np.random.default_rng(5)
    b = rng.standard_normal(N ** 3)
    b -= b.mean()
    A = -kron_laplacian(N)
    thr = 1e-10 * np.linalg.norm(b)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = r @ r
    k = 0
    while np.sqrt(rr) > thr:
        w = A @ p
        al = rr / (p @ w)
        x += al * p
        r -= al * w
        k += 1
        rr_new = r @ r
        if np.sqrt(rr_new) <= thr:
            break
        p = r + (rr_new / rr) * p
        rr = rr_new
    xo, it, ok = oracle_lib.pcg(b.reshape(N, N, N), thr=thr)
    assert ok and it == k
    np.testing.assert_allclose(xo.ravel(), x, atol=1e-12 * np.abs(x).max())


def test_pcg_stopping_rule_is_tight(oracle_lib):
    N = 10
    rng = np.random.default_rng(7)
    b = rng.standard_normal((N, N, N))
    b -= b.mean()
    thr = 1e-6 * np.linalg.norm(b)
    x, it, ok = oracle_lib.pcg(b, thr=thr)
    assert ok and it > 2
    r = b + oracle_lib.apply_M(x)
    assert np.linalg.norm(r) <= thr * (1 + 1e-6)
    x2, it2, ok2 = oracle_lib.pcg(b, thr=thr, max_iter=it - 1)
    assert not ok2 and it2 == it - 1
    assert np.linalg.norm(b + oracle_lib.apply_M(x2)) > thr


def test_pcg_max_norm_mode(oracle_lib):
    N = 10
    rng = np.random.default_rng(8)
    b = rng.standard_normal((N, N, N))
    b -= b.mean()
    x, it, ok = oracle_lib.pcg(b, thr=1e-8, norm=oracle_lib.NORM_ABSMAX)
    assert ok
    assert np.abs(b + oracle_lib.apply_M(x)).max() <= 1e-8


def test_pcg_zero_rhs_converges_immediately(oracle_lib):
    x, it, ok = oracle_lib.pcg(np.zeros((6, 6, 6)), thr=1e-12)
    assert ok and it == 0 and not x.any()


@pytest.mark.parametrize("box,h", [(20.64, 0.172), (10.0, 0.333), (10.0, 0.1)])
def test_grid_size_matches_paper(oracle_lib, box, h):
    g = json.load(open(os.path.join(GOLDEN, "paper_values.json")))["grid_points_per_side"]
    expect = {(e["box"], e["h"]): e["N"] for e in g}
    assert oracle_lib.grid_n(box, h) == expect[(box, h)]
