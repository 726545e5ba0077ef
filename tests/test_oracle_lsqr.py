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
