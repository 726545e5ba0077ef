"""Pins of the oracle's butterfly apply O2 (CPU).

O2 is pinned by: (1) exactness at tolerance 0, where the factor set reproduces
Phi and O2 must equal the dense product; (2) the independent sparse-product
formulation (Sec. 2, Remark on the sparse-factor view) on random factor sets
with uneven ranks, identity blocks and empty leaves; (3) the adjoint identity;
(4) the error tracking the ID tolerance (Sec. 6.1, the matvec error follows
the requested tolerance).  Mutation tests plant plausible mistakes in the
oracle and show that a pin fails.
"""
import numpy as np
import pytest

from factor_gen import random_factor_set
from oracle import butterfly as ob
from oracle import dense as od
from oracle import modes as om
from oracle import sparse as osp
from paper_2605_21828_amd.factor import io as fio


def _grid_factors(N, m, leaf, tol):
    pts = om.uniform_grid(N)
    fs, _ = fio.fourier_factors(pts, m, leaf, tol, workers=1, cache=False)
    return fs, pts


@pytest.fixture(scope="module")
def exact_small():
    # 16 x 16 grid, 64 modes, leaf 16 -> L = 4; tol 0 keeps every column the
    # blocks can hold, so the last levels carry non-trivial P (|tau| < r_in)
    fs, pts = _grid_factors(16, 64, 16, 0.0)
    return fs, pts, om.phi(pts, om.fourier_modes(64))


def test_exact_factors_have_nontrivial_transfers(exact_small):
    fs, _, _ = exact_small
    assert fs["ident"].sum() < fs["ident"].size
    assert fs["P"].size > 0


def test_tol0_apply_equals_dense(exact_small):
    fs, _, Phi = exact_small
    rng = np.random.default_rng(0)
    c = rng.standard_normal((Phi.shape[1], 3))
    f = rng.standard_normal((Phi.shape[0], 3))
    assert np.linalg.norm(ob.apply(fs, c) - Phi @ c) <= 1e-12 * np.linalg.norm(Phi @ c)
    assert np.linalg.norm(ob.apply_transpose(fs, f) - Phi.T @ f) <= 1e-12 * np.linalg.norm(Phi.T @ f)


def test_tol0_apply_equals_inverse_dft():
    fs, pts = _grid_factors(32, 256, 16, 0.0)
    c = np.random.default_rng(4).standard_normal(256)
    ref = om.grid_synthesis_ifft2(32, om.fourier_modes(256), c)
    assert np.linalg.norm(ob.apply(fs, c) - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("seed,n,m,L", [(0, 40, 24, 2), (1, 64, 64, 3), (2, 33, 70, 3), (3, 17, 5, 2), (4, 90, 50, 4)])
def test_apply_equals_sparse_product(seed, n, m, L):
    fs = random_factor_set(seed, n, m, L, max_rank=12)
    A = osp.dense_operator(fs)
    eye_m = np.eye(m)
    assert np.allclose(ob.apply(fs, eye_m), A, atol=1e-12, rtol=1e-12)
    assert np.allclose(ob.apply_transpose(fs, np.eye(n)), A.T, atol=1e-12, rtol=1e-12)


@pytest.mark.parametrize("seed", [5, 6, 7])
def test_adjoint_identity(seed):
    fs = random_factor_set(seed, 120, 80, 4, max_rank=16)
    rng = np.random.default_rng(seed)
    c, f = rng.standard_normal((80, 2)), rng.standard_normal((120, 2))
    lhs = np.sum(ob.apply(fs, c) * f)
    rhs = np.sum(c * ob.apply_transpose(fs, f))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


def test_permutation_factor_set_is_exact_scatter():
    fs = random_factor_set(11, 50, 50, 3, identity_values=True)
    c = np.arange(50, dtype=float)
    f = ob.apply(fs, c)
    assert np.array_equal(f[fs["perm_x"]], c)
    assert np.array_equal(ob.apply_transpose(fs, f), c)


@pytest.mark.parametrize("tol", [1e-4, 1e-6, 1e-8])
def test_error_tracks_tolerance(tol):
    rng = np.random.default_rng(9)
    pts = rng.uniform(-np.pi, np.pi, (4096, 2))
    fs, _ = fio.fourier_factors(pts, 512, 32, tol, workers=1, cache=False)
    Phi = om.phi(pts, om.fourier_modes(512))
    c = rng.standard_normal(512)
    err = np.linalg.norm(ob.apply(fs, c) - Phi @ c) / np.linalg.norm(Phi @ c)
    assert 1e-3 * tol < err < 30 * tol


def test_stored_entries_counts_blocks(exact_small):
    fs, _, _ = exact_small
    assert ob.stored_entries(fs) == fs["P"].size + fs["U"].size


# ---- mutation tests: plausible mistakes planted in the oracle must fail a pin ----

def _planted(monkeypatch, name, fn):
    monkeypatch.setattr(ob, name, fn)


def test_mutant_transposed_block_fails(monkeypatch, exact_small):
    fs, _, Phi = exact_small
    orig = ob._P

    def bad(f, lvl, q):
        P = orig(f, lvl, q)
        if P.shape[0] == P.shape[1] and P.shape[0] > 1 and not np.allclose(P, np.eye(P.shape[0])):
            return P.T
        # reverse the rows: the wrong output ordering of a block
        return P[::-1] if P.shape[0] > 1 else P
    _planted(monkeypatch, "_P", bad)
    c = np.random.default_rng(0).standard_normal(Phi.shape[1])
    assert np.linalg.norm(ob.apply(fs, c) - Phi @ c) > 1e-3 * np.linalg.norm(Phi @ c)


def test_mutant_swapped_children_fails(monkeypatch):
    fs = random_factor_set(21, 64, 64, 3, max_rank=10, p_ident=0.0)
    A = osp.dense_operator(fs)
    orig = ob._children
    _planted(monkeypatch, "_children", lambda L, lvl, i, j, k=2: orig(L, lvl, i, j, k)[::-1])
    try:
        got = ob.apply(fs, np.eye(64))
    except ValueError:
        return   # shapes no longer fit: the mistake is caught
    assert not np.allclose(got, A, atol=1e-9)


def test_mutant_wrong_parent_fails(monkeypatch):
    fs = random_factor_set(22, 64, 64, 3, max_rank=10, p_ident=0.0)
    A = osp.dense_operator(fs)
    orig = ob._children
    _planted(monkeypatch, "_children", lambda L, lvl, i, j, k=2: orig(L, lvl, i ^ 2 if i >= 2 else i, j, k))
    try:
        got = ob.apply(fs, np.eye(64))
    except ValueError:
        return
    assert not np.allclose(got, A, atol=1e-9)


def test_mutant_dropped_leaf_permutation_fails(monkeypatch, exact_small):
    fs, _, Phi = exact_small
    fs2 = dict(fs)
    fs2["perm_x"] = np.arange(fs["n"], dtype=np.int32)   # forget the space-tree ordering
    c = np.random.default_rng(1).standard_normal(Phi.shape[1])
    assert np.linalg.norm(ob.apply(fs2, c) - Phi @ c) > 1e-3 * np.linalg.norm(Phi @ c)


def test_mutant_dropped_transfer_term_fails(monkeypatch, exact_small):
    fs, _, Phi = exact_small
    orig = ob._P

    def bad(f, lvl, q):
        P = orig(f, lvl, q).copy()
        if lvl == int(f["L"]) and P.shape[1] > 1:
            P[:, -1] = 0.0   # drop the last input's contribution
        return P
    _planted(monkeypatch, "_P", bad)
    c = np.random.default_rng(2).standard_normal(Phi.shape[1])
    assert np.linalg.norm(ob.apply(fs, c) - Phi @ c) > 1e-6 * np.linalg.norm(Phi @ c)


# ---- k-ary trees (Sec. 2: the construction generalizes to k-ary trees; Sec. 5:
# quadtree in space, 4-ary tree on the eigenvalues) ----

def test_quadtree_tol0_apply_equals_dense_and_dft():
    """A 4-ary factor set built at tolerance 0 reproduces the transform: the
    dense product and, on the grid, the inverse DFT."""
    pts = om.uniform_grid(32)
    fs, _ = fio.fourier_factors(pts, 256, 16, 0.0, workers=1, cache=False, arity=4)
    assert int(fs["arity"]) == 4 and int(fs["L"]) == 3
    assert fs["ident"].sum() < fs["ident"].size and fs["P"].size > 0
    Phi = om.phi(pts, om.fourier_modes(256))
    rng = np.random.default_rng(21)
    c = rng.standard_normal((256, 3))
    f = rng.standard_normal((1024, 3))
    assert np.linalg.norm(ob.apply(fs, c) - Phi @ c) <= 1e-12 * np.linalg.norm(Phi @ c)
    assert np.linalg.norm(ob.apply_transpose(fs, f) - Phi.T @ f) <= 1e-12 * np.linalg.norm(Phi.T @ f)
    ref = om.grid_synthesis_ifft2(32, om.fourier_modes(256), c)
    assert np.linalg.norm(ob.apply(fs, c) - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("seed,n,m,L", [(30, 40, 24, 1), (31, 70, 64, 2), (32, 200, 90, 2), (33, 17, 5, 2)])
def test_quadtree_apply_equals_sparse_product(seed, n, m, L):
    fs = random_factor_set(seed, n, m, L, max_rank=12, arity=4)
    A = osp.dense_operator(fs)
    assert np.allclose(ob.apply(fs, np.eye(m)), A, atol=1e-12, rtol=1e-12)
    assert np.allclose(ob.apply_transpose(fs, np.eye(n)), A.T, atol=1e-12, rtol=1e-12)


def test_quadtree_adjoint_identity_and_error_tracks_tolerance():
    fs = random_factor_set(34, 300, 120, 2, max_rank=16, arity=4)
    rng = np.random.default_rng(34)
    c, f = rng.standard_normal((120, 2)), rng.standard_normal((300, 2))
    lhs, rhs = np.sum(ob.apply(fs, c) * f), np.sum(c * ob.apply_transpose(fs, f))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)
    pts = rng.uniform(-np.pi, np.pi, (4096, 2))
    fq, _ = fio.fourier_factors(pts, 512, 32, 1e-8, workers=1, cache=False, arity=4)
    Phi = om.phi(pts, om.fourier_modes(512))
    c1 = rng.standard_normal(512)
    err = np.linalg.norm(ob.apply(fq, c1) - Phi @ c1) / np.linalg.norm(Phi @ c1)
    assert 1e-5 * 1e-8 < err < 30 * 1e-8


def test_quadtree_mutant_swapped_children_fails(monkeypatch):
    """Reversing the order of a block's four inputs is caught by the sparse product."""
    fs = random_factor_set(35, 70, 64, 2, max_rank=12, arity=4)
    A = osp.dense_operator(fs)
    orig = ob._children
    _planted(monkeypatch, "_children", lambda L, lvl, i, j, k=2: orig(L, lvl, i, j, k)[::-1])
    assert not np.allclose(ob.apply(fs, np.eye(64)), A, atol=1e-9)
