"""Pins of the oracle's LSQR (CPU only): a library routine and the normal equations."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.lsqr import lsqr


@pytest.mark.parametrize("seed,k", [(0, 5), (1, 20)])
def test_iterates_equal_library_lsqr(seed, k):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((80, 30))
    b = rng.standard_normal(80)
    x, res = lsqr(lambda v: A @ v, lambda u: A.T @ u, b, k)
    ref = spla.lsqr(A, b, atol=0, btol=0, conlim=0, iter_lim=k)
    assert np.allclose(x, ref[0], rtol=1e-10, atol=1e-12)
    assert abs(res[-1] - ref[3]) <= 1e-10 * max(1.0, ref[3])


def test_converges_to_least_squares_solution():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((120, 25)) @ np.diag(np.linspace(1, 3, 25))
    b = rng.standard_normal(120)
    x, res = lsqr(lambda v: A @ v, lambda u: A.T @ u, b, 60)
    xs = np.linalg.lstsq(A, b, rcond=None)[0]
    assert np.allclose(x, xs, rtol=1e-10, atol=1e-10)
    assert abs(res[-1] - np.linalg.norm(A @ xs - b)) <= 1e-9 * np.linalg.norm(b)
    assert np.all(np.diff(res) <= 1e-12)   # the residual never grows


def test_consistent_system_is_solved_exactly():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((50, 10))
    xt = rng.standard_normal(10)
    x, res = lsqr(lambda v: A @ v, lambda u: A.T @ u, A @ xt, 40)
    assert np.allclose(x, xt, rtol=1e-10, atol=1e-10) and res[-1] < 1e-9


def test_right_hand_side_orthogonal_to_the_range():
    # A^T b = 0: x = 0 is the least-squares solution and the residual is ||b||
    # at every step (the recurrence ends at once; the library routine agrees)
    rng = np.random.default_rng(4)
    Q = np.linalg.qr(rng.standard_normal((40, 12)))[0]
    A = Q[:, :8] @ rng.standard_normal((8, 8))
    b = Q[:, 8:] @ rng.standard_normal(4)
    assert np.abs(A.T @ b).max() < 1e-12
    x, res = lsqr(lambda v: A @ v, lambda u: A.T @ u, b, 6)
    assert np.abs(x).max() < 1e-12
    assert np.allclose(res, np.linalg.norm(b), rtol=1e-12)
    ref = spla.lsqr(A, b, atol=0, btol=0, conlim=0, iter_lim=6)
    assert np.abs(ref[0]).max() < 1e-12 and abs(ref[3] - np.linalg.norm(b)) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("rows,cols", [(6, 0), (0, 5)])
def test_empty_operator(rows, cols):
    # no unknowns: the residual is b; no equations: x = 0 and nothing is left
    b = np.arange(1.0, rows + 1.0)
    A = np.zeros((rows, cols))
    x, res = lsqr(lambda v: A @ v, lambda u: A.T @ u, b, 3)
    assert x.shape == (cols,) and not np.any(x)
    assert np.allclose(res, np.linalg.norm(b), rtol=1e-15)
