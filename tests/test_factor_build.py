"""Host factor builder (CPU): the full-rank shortcut of the column ID.

A block whose smallest singular value is far above tol times its largest keeps
every column under the pivoted-QR rule, so the builder may flag it as the
identity from the Gram matrix's eigenvalues instead of running the QR.  These
tests show that the shortcut is taken only where the QR gives the same answer,
and that a whole factor set comes out bit for bit the same with it.
"""
import numpy as np
import pytest

from paper_2605_21828_amd.factor import build as fb
from paper_2605_21828_amd.factor import interp
from paper_2605_21828_amd.factor import io as fio


def _with_spectrum(rng, rows, cols, sv):
    U = np.linalg.qr(rng.standard_normal((rows, cols)))[0]
    V = np.linalg.qr(rng.standard_normal((cols, cols)))[0]
    return (U * sv) @ V.T


@pytest.mark.parametrize("rows,cols,lo,tol", [
    (300, 20, 0.5, 1e-8),      # well conditioned: identity both ways
    (300, 20, 1e-6, 1e-8),     # full rank at tol, shortcut may or may not fire
    (300, 20, 1e-9, 1e-8),     # numerically rank deficient: pivoted QR
    (64, 40, 1e-12, 1e-10),
    (40, 40, 1e-3, 1e-4),      # square
    (30, 50, 1.0, 1e-8),       # wide: never the shortcut
])
def test_shortcut_gives_the_pivoted_qr_result(rows, cols, lo, tol):
    rng = np.random.default_rng(rows + cols)
    k = min(rows, cols)
    A = _with_spectrum(rng, rows, k, np.geomspace(1.0, lo, k))
    if cols > k:
        A = np.hstack([A, A[:, : cols - k] @ rng.standard_normal((cols - k, cols - k))])
    J1, P1, id1 = interp.column_id(A, tol)
    J2, P2, id2 = interp.column_id(A, tol, gram_check=False)
    assert id1 == id2 and np.array_equal(J1, J2)
    assert (P1 is None and P2 is None) or np.array_equal(P1, P2)


def test_shortcut_declines_near_the_tolerance():
    rng = np.random.default_rng(1)
    tol = 1e-6
    A = _with_spectrum(rng, 500, 30, np.geomspace(1.0, 5 * tol, 30))
    assert not interp.surely_full_rank(A, tol)          # needs a factor 10 of margin
    assert interp.column_id(A, tol, gram_check=False)[2]   # the QR still keeps every column
    B = _with_spectrum(rng, 500, 30, np.geomspace(1.0, 1e-2, 30))
    assert interp.surely_full_rank(B, tol)
    assert not interp.surely_full_rank(np.zeros((10, 3)), tol)
    assert not interp.surely_full_rank(rng.standard_normal((3, 10)), tol)


def test_factor_set_is_unchanged_by_the_shortcut(monkeypatch):
    rng = np.random.default_rng(5)
    pts = rng.uniform(-np.pi, np.pi, (4096, 2))
    taken = []
    real = interp.surely_full_rank

    def counting(A, tol):
        r = real(A, tol)
        taken.append(r)
        return r
    monkeypatch.setattr(interp, "surely_full_rank", counting)
    fs1, _ = fio.fourier_factors(pts, 512, 32, 1e-8, workers=1, cache=False)
    assert any(taken)                                    # the shortcut ran on some blocks
    monkeypatch.setattr(fb, "column_id", lambda A, tol: interp.column_id(A, tol, gram_check=False))
    fs2, _ = fio.fourier_factors(pts, 512, 32, 1e-8, workers=1, cache=False)
    for key in ("rank", "ident", "P", "P_off", "U", "U_off", "skel_L", "perm_x", "xoff", "koff"):
        assert np.array_equal(fs1[key], fs2[key]), key
    assert fs1["ident"].sum() > 0


def test_parallel_build_equals_serial_build():
    # blocks of a level are independent; the process pool returns them out of
    # order and the builder must place each by its id
    rng = np.random.default_rng(6)
    pts = rng.uniform(-np.pi, np.pi, (2048, 2))
    fs1, _ = fio.fourier_factors(pts, 256, 32, 1e-8, workers=1, cache=False)
    fs2, _ = fio.fourier_factors(pts, 256, 32, 1e-8, workers=3, cache=False)
    for key in ("rank", "ident", "P", "P_off", "U", "U_off", "skel_L"):
        assert np.array_equal(fs1[key], fs2[key]), key


def test_quadtree_is_a_partition_into_quadrants():
    """Quadtree on the 16 x 16 grid: a permutation, 4^2 leaves of 16 points each,
    every leaf inside its quadrant box, and its leaves are the binary Neumann-box
    tree's leaves at twice the depth (square boxes alternate the split axis)."""
    import numpy as np
    from paper_2605_21828_amd import workloads as wl
    from paper_2605_21828_amd.factor.trees import box_bisection_tree, frequency_tree, quadtree
    pts = wl.grid_points(16)
    perm, xoff = quadtree(pts, 2)
    assert sorted(perm.tolist()) == list(range(256))
    assert np.array_equal(np.diff(xoff), np.full(16, 16))
    perm2, xoff2 = box_bisection_tree(pts, 4)
    assert np.array_equal(xoff, xoff2)
    for i in range(16):
        assert set(perm[xoff[i]:xoff[i + 1]].tolist()) == set(perm2[xoff2[i]:xoff2[i + 1]].tolist())
    rng = np.random.default_rng(3)
    iid = rng.uniform(-np.pi, np.pi, (1000, 2))
    p3, x3 = quadtree(iid, 3)
    assert sorted(p3.tolist()) == list(range(1000)) and x3[-1] == 1000 and len(x3) == 65
    # 4-ary frequency leaves are the binary index tree's leaves at twice the depth
    assert np.array_equal(frequency_tree(1000, 3, 4), frequency_tree(1000, 6))


@pytest.mark.parametrize("seed", range(6))
def test_device_build_chunks_cover_the_level_within_the_budget(seed):
    """The device build processes a level's blocks in chunks: consecutive ranges
    that cover every block once, in order, each within the memory budget unless
    it is a single block larger than the budget, and each as long as the budget
    allows (the next block would not fit)."""
    from paper_2605_21828_amd.factor.device_build import _chunks
    rng = np.random.default_rng(seed)
    sizes = [int(x) for x in rng.integers(0, 100, size=int(rng.integers(0, 40)))]
    if seed == 5 and sizes:
        sizes[len(sizes) // 2] = 1000   # one block above the budget
    budget = 250
    ch = _chunks(sizes, budget)
    assert [i for a, b in ch for i in range(a, b)] == list(range(len(sizes)))
    for a, b in ch:
        assert b > a
        total = sum(sizes[a:b])
        assert total <= budget or b - a == 1
        if b < len(sizes):
            assert total + sizes[b] > budget
