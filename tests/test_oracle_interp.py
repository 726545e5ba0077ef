"""Pins of the oracle's column ID and butterfly factorization (CPU).

The column ID (oracle/interp.py) is pinned by what the mathematics fixes:
  - a block of exact rank r keeps r columns and is reproduced to rounding;
  - R11^-1 R12 is the least-squares fit of the other columns by the skeleton;
  - the residual obeys |A - A(:, J) P|_2 <= |R22|_F <= sqrt(K - k) tol |A|_2;
  - the pivot order is the greedy one: a pure-Python Gram-Schmidt selection of
    the longest remaining residual column, on tiny blocks;
  - the degenerate blocks (no columns, no rows, all zeros, full rank).
The factorization (oracle/factorize.py) is pinned by the applied factor set:
exact for a matrix of exact low rank, within the per-block bound otherwise, and
against the dense transform on the flat torus.  Planted mistakes show the pins bite.
"""
import numpy as np
import pytest

from oracle import butterfly as ob
from oracle import factorize as ofz
from oracle import interp as oi
from oracle import modes as om


def _spectrum(rng, M, K, sv):
    U = np.linalg.qr(rng.standard_normal((M, len(sv))))[0]
    V = np.linalg.qr(rng.standard_normal((K, len(sv))))[0]
    return (U * sv) @ V.T


@pytest.mark.parametrize("M,K,r", [(60, 20, 7), (20, 40, 9), (33, 33, 1), (200, 64, 40)])
def test_exact_rank_block(M, K, r):
    rng = np.random.default_rng(M + K + r)
    A = rng.standard_normal((M, r)) @ rng.standard_normal((r, K))
    J, P, ident = oi.column_id(A, 1e-10)
    assert not ident and len(J) == r and P.shape == (r, K)
    assert np.array_equal(P[:, J], np.eye(r))
    assert np.linalg.norm(A - A[:, J] @ P) <= 1e-12 * np.linalg.norm(A)


def test_t_is_the_least_squares_fit():
    rng = np.random.default_rng(3)
    A = _spectrum(rng, 80, 30, np.geomspace(1.0, 1e-12, 30))
    J, P, _ = oi.column_id(A, 1e-6)
    k = len(J)
    Jc = np.setdiff1d(np.arange(30), J)
    T_ls = np.linalg.lstsq(A[:, J], A[:, Jc], rcond=None)[0]
    assert 0 < k < 30
    assert np.allclose(P[:, Jc], T_ls, rtol=0, atol=1e-8 * np.abs(T_ls).max())


@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-9])
def test_residual_bound(tol):
    rng = np.random.default_rng(int(-np.log10(tol)))
    M, K = 120, 50
    A = _spectrum(rng, M, K, np.geomspace(1.0, 1e-14, K))
    J, P, ident = oi.column_id(A, tol)
    k = len(J)
    assert not ident
    res = np.linalg.norm(A - A[:, J] @ P, 2)
    assert res <= np.sqrt(K - k) * tol * np.linalg.norm(A, 2)
    # and the rank is not larger than needed: sigma_{k+1} of A is below the cut
    sv = np.linalg.svd(A, compute_uv=False)
    assert sv[min(k, K - 1)] <= np.sqrt(K) * tol * np.abs(A).max() * np.sqrt(M)


def _greedy_pivots(A, k):
    """Pure-Python Businger-Golub selection: repeatedly take the column whose
    residual (after removing the span of the chosen ones) is longest."""
    M, K = len(A), len(A[0])
    R = [[A[i][c] for i in range(M)] for c in range(K)]   # residual columns
    chosen = []
    for _ in range(k):
        best, bn = -1, -1.0
        for c in range(K):
            if c in chosen:
                continue
            s = sum(x * x for x in R[c])
            if s > bn:
                best, bn = c, s
        chosen.append(best)
        q = R[best]
        qn = sum(x * x for x in q) ** 0.5
        q = [x / qn for x in q]
        for c in range(K):
            if c not in chosen:
                d = sum(q[i] * R[c][i] for i in range(M))
                R[c] = [R[c][i] - d * q[i] for i in range(M)]
    return chosen


@pytest.mark.parametrize("seed", range(6))
def test_pivot_order_is_greedy(seed):
    rng = np.random.default_rng(100 + seed)
    M, K, r = 9, 7, 4
    A = rng.standard_normal((M, r)) @ rng.standard_normal((r, K)) * rng.uniform(0.5, 2.0, K)
    J, P, ident = oi.column_id(A, 1e-10)
    assert len(J) == r
    assert list(J) == _greedy_pivots(A.tolist(), r)


def test_degenerate_blocks():
    J, P, ident = oi.column_id(np.zeros((5, 0)), 1e-8)
    assert ident and J.size == 0 and P is None
    J, P, ident = oi.column_id(np.zeros((0, 4)), 1e-8)
    assert not ident and J.size == 0 and P.shape == (0, 4)
    J, P, ident = oi.column_id(np.zeros((6, 4)), 1e-8)
    assert not ident and J.size == 0 and P.shape == (0, 4)
    rng = np.random.default_rng(9)
    J, P, ident = oi.column_id(rng.standard_normal((30, 6)), 1e-8)
    assert ident and np.array_equal(J, np.arange(6)) and P is None


def _trees(rng, n, m, L, k=2):
    """Random complete k-ary trees: any partition is a valid input to the algebra."""
    nb = k ** L
    perm = rng.permutation(n).astype(np.int32)
    xoff = np.linspace(0, n, nb + 1).round().astype(np.int64)
    koff = np.linspace(0, m, nb + 1).round().astype(np.int64)
    return perm, xoff, koff


@pytest.mark.parametrize("n,m,L,r,k", [(64, 48, 2, 5, 2), (96, 40, 3, 9, 2), (80, 64, 1, 6, 4), (128, 96, 2, 10, 4)])
def test_factorization_of_exact_low_rank(n, m, L, r, k):
    rng = np.random.default_rng(n + m + L)
    Phi = rng.standard_normal((n, r)) @ rng.standard_normal((r, m))
    perm, xoff, koff = _trees(rng, n, m, L, k)
    fs = ofz.butterfly_factorization(Phi, perm, xoff, koff, L, 1e-11, arity=k)
    assert fs["rank"].max() <= r
    c = rng.standard_normal((m, 3))
    f = rng.standard_normal((n, 2))
    assert np.linalg.norm(ob.apply(fs, c) - Phi @ c) <= 1e-10 * np.linalg.norm(Phi @ c)
    assert np.linalg.norm(ob.apply_transpose(fs, f) - Phi.T @ f) <= 1e-10 * np.linalg.norm(Phi.T @ f)


@pytest.mark.parametrize("tol", [1e-4, 1e-8])
def test_factorization_of_fourier_matrix(tol):
    # 2-D Fourier matrix at sorted random points on the torus: points split by
    # coordinate so that space nodes are compact, modes in eigenvalue order
    rng = np.random.default_rng(7)
    n, m, L = 256, 96, 3
    pts = rng.uniform(-np.pi, np.pi, (n, 2))
    modes = om.fourier_modes(m)
    Phi = om.phi(pts, modes)
    perm = np.lexsort((pts[:, 1], np.floor(pts[:, 0] / (2 * np.pi / 8)))).astype(np.int32)
    xoff = np.linspace(0, n, 2 ** L + 1).astype(np.int64)
    koff = np.linspace(0, m, 2 ** L + 1).astype(np.int64)
    fs = ofz.butterfly_factorization(Phi, perm, xoff, koff, L, tol)
    assert (fs["rank"][1:] < 2 * fs["rank"][:-1].max()).any() and fs["ident"].sum() < fs["ident"].size
    c = rng.standard_normal(m)
    err = np.linalg.norm(ob.apply(fs, c) - Phi @ c) / np.linalg.norm(Phi @ c)
    assert err <= 50 * (L + 1) * tol
    g = np.linalg.norm(ob.apply_transpose(fs, Phi @ c) - Phi.T @ (Phi @ c)) / np.linalg.norm(Phi.T @ Phi @ c)
    assert g <= 50 * (L + 1) * tol


def test_planted_child_order_swap_is_caught(monkeypatch):
    """Concatenating the children's skeletons in the wrong order mismatches the
    previous level's P rows: the exact-rank pin fails."""
    rng = np.random.default_rng(11)
    n, m, L, r = 64, 48, 2, 5
    Phi = rng.standard_normal((n, r)) @ rng.standard_normal((r, m))
    perm, xoff, koff = _trees(rng, n, m, L)
    real_concat = np.concatenate

    def swapped(parts, *a, **kw):
        if isinstance(parts, list) and len(parts) == 2 and all(np.asarray(p).dtype.kind == "i" for p in parts):
            parts = parts[::-1]
        return real_concat(parts, *a, **kw)

    monkeypatch.setattr(ofz.np, "concatenate", swapped)
    fs = ofz.butterfly_factorization(Phi, perm, xoff, koff, L, 1e-11)
    monkeypatch.undo()
    c = rng.standard_normal(m)
    assert np.linalg.norm(ob.apply(fs, c) - Phi @ c) > 1e-3 * np.linalg.norm(Phi @ c)


def test_planted_unpivoted_skeleton_is_caught(monkeypatch):
    """Taking the first k columns instead of the pivots breaks the ID."""
    rng = np.random.default_rng(12)
    A = _spectrum(rng, 40, 20, np.geomspace(1.0, 1e-12, 20))
    real = oi.sla.qr

    def no_pivot(a, **kw):
        R, piv = real(a, **kw)
        return R, np.arange(len(piv))

    monkeypatch.setattr(oi.sla, "qr", no_pivot)
    J, P, _ = oi.column_id(A, 1e-6)
    monkeypatch.undo()
    assert np.linalg.norm(A - A[:, J] @ P) > 1e-3 * np.linalg.norm(A)
