"""Pins of the oracle's Fourier modes and dense transform (CPU).

Each check ties the oracle to something other than itself: a hand-written mode
list, lattice-point counts, Weyl's law, numpy's FFT, and the closed-form
discrete orthogonality of trigonometric functions on a uniform grid.
"""
import os

import numpy as np
import pytest

from oracle import dense as od
from oracle import modes as om

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fourier_modes_first21.txt")


def test_first_modes_match_hand_written_list():
    rows = np.loadtxt(GOLDEN, dtype=np.int64, comments="#")
    got = om.fourier_modes(len(rows))
    assert np.array_equal(got, rows[:, :4])
    assert np.array_equal(om.eigenvalues(got), rows[:, 4].astype(float))


@pytest.mark.parametrize("R2", [1, 2, 5, 10, 25, 50, 97, 130])
def test_one_mode_per_lattice_point(R2):
    # the number of modes with lambda <= R^2 equals the lattice points in the disk
    cnt = om.lattice_count_in_disk(R2)
    md = om.fourier_modes(cnt + 1)
    lam = om.eigenvalues(md)
    assert np.all(lam[:cnt] <= R2) and lam[cnt] > R2


def test_eigenvalues_sorted_and_weyl():
    for m in (1024, 16384):
        lam = om.eigenvalues(om.fourier_modes(m))
        assert np.all(np.diff(lam) >= 0)
        # Weyl's law on the torus of area 4 pi^2: lambda_m ~ m / pi
        assert abs(lam[-1] - m / np.pi) / (m / np.pi) < 0.05


@pytest.mark.parametrize("N,m", [(16, 40), (32, 200), (64, 1024)])
def test_grid_synthesis_equals_inverse_fft(N, m):
    md = om.fourier_modes(m)
    pts = om.uniform_grid(N)
    c = np.random.default_rng(1).standard_normal((m, 3))
    f_dense = od.synthesis(om.phi(pts, md), c)
    f_fft = om.grid_synthesis_ifft2(N, md, c)
    assert np.linalg.norm(f_dense - f_fft) <= 1e-13 * np.linalg.norm(f_fft)


@pytest.mark.parametrize("N,m", [(16, 40), (64, 1024)])
def test_grid_analysis_equals_forward_fft(N, m):
    md = om.fourier_modes(m)
    pts = om.uniform_grid(N)
    f = np.random.default_rng(2).standard_normal((N * N, 2))
    g_dense = od.analysis(om.phi(pts, md), f)
    g_fft = om.grid_analysis_fft2(N, md, f)
    assert np.linalg.norm(g_dense - g_fft) <= 1e-13 * np.linalg.norm(g_fft)


def test_grid_gram_is_closed_form_diagonal():
    N, m = 32, 300   # all |k_i| < N / 2
    md = om.fourier_modes(m)
    assert md[:, :2].max() < N // 2
    Phi = om.phi(om.uniform_grid(N), md)
    G = Phi.T @ Phi
    assert np.allclose(G, np.diag(N * N * om.grid_gram_weights(md)), atol=1e-9)


def test_point_indexing_of_grid():
    pts = om.uniform_grid(8)
    # point id = N * j1 + j2
    assert np.allclose(pts[8 * 3 + 5], [-np.pi + 2 * np.pi * 3 / 8, -np.pi + 2 * np.pi * 5 / 8])


def test_sampled_rows_and_columns_match_dense():
    rng = np.random.default_rng(3)
    pts = rng.uniform(-np.pi, np.pi, (500, 2))
    md = om.fourier_modes(120)
    Phi = om.phi(pts, md)
    c = rng.standard_normal((120, 2))
    f = rng.standard_normal((500, 2))
    rows = np.array([0, 7, 99, 499])
    cols = np.array([1, 5, 119])
    assert np.allclose(od.fourier_synthesis_rows(pts, md, rows, c), (Phi @ c)[rows], rtol=1e-13, atol=1e-12)
    assert np.allclose(od.fourier_analysis_cols(pts, md, cols, f, chunk=64), (Phi.T @ f)[cols], rtol=1e-13, atol=1e-11)


def test_full_synthesis_regrouping_equals_definition():
    rng = np.random.default_rng(4)
    pts = rng.uniform(-np.pi, np.pi, (700, 2))
    md = om.fourier_modes(300)
    c = rng.standard_normal((300, 3))
    ref = om.phi(pts, md) @ c
    assert np.allclose(od.fourier_synthesis_all(pts, md, c, chunk=128), ref, rtol=1e-12, atol=1e-11)
    assert np.allclose(od.fourier_synthesis_all(pts, md, c[:, 1]), ref[:, 1], rtol=1e-12, atol=1e-11)
    # a planted mistake (the sin/cos roles of the x2 factor swapped) is caught
    bad = md.copy()
    bad[:, 3] = 1 - bad[:, 3]
    bad[:, 1] = np.maximum(bad[:, 1], 1)
    assert not np.allclose(od.fourier_synthesis_all(pts, bad, c), ref, rtol=1e-6, atol=1e-6)


def test_rel_err_cols_is_max_over_columns():
    ref = np.array([[1.0, 2.0], [0.0, 0.0]])
    x = np.array([[1.1, 2.0], [0.0, 0.0]])
    mx, fro = od.rel_err_cols(x, ref)
    assert abs(mx - 0.1) < 1e-12 and 0 < fro < 0.1


def test_builder_exact_synthesis_matches_definition():
    from paper_2605_21828_amd.factor.fourier import FourierBlocks, real_modes
    rng = np.random.default_rng(5)
    pts = rng.uniform(-np.pi, np.pi, (900, 2))
    c = rng.standard_normal((400, 2))
    got = FourierBlocks(pts, real_modes(400)).synthesis(c, chunk=100)
    assert np.allclose(got, om.phi(pts, om.fourier_modes(400)) @ c, rtol=1e-12, atol=1e-11)
