"""Perturbed-sphere workload pins (CPU): the discrete Laplace-Beltrami problem and its trees."""
import numpy as np
import pytest

from oracle import butterfly as ob
from oracle import dense as od
from oracle import fem as ofem
from paper_2605_21828_amd import sphere as S
from paper_2605_21828_amd.factor import io as fio
from paper_2605_21828_amd.factor.mesh_tree import mesh_fiedler_tree


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_icosphere_counts(level):
    v, f = S.icosphere(level)
    assert len(v) == 10 * 4 ** level + 2 and len(f) == 20 * 4 ** level
    edges = np.unique(np.sort(np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]]), axis=1), axis=0)
    assert len(v) - len(edges) + len(f) == 2        # Euler characteristic of the sphere
    assert np.allclose(np.linalg.norm(v, axis=1), 1.0)


def test_unperturbed_sphere_has_spherical_harmonic_spectrum():
    """Textbook fact: on the unit sphere the Laplace-Beltrami eigenvalues are l(l+1)
    with multiplicity 2l+1; linear elements on a level-4 icosphere (h ~ 0.05)
    reproduce the first 25 to about 1%."""
    v, f = S.icosphere(4)
    K, M = S.cotangent_fem(v, f)
    lam, _ = S.eigenpairs(K, M, 25, workers=1)
    expect = np.concatenate([[l * (l + 1)] * (2 * l + 1) for l in range(5)]).astype(float)
    assert abs(lam[0]) < 1e-10
    assert np.all(np.abs(lam[1:] - expect[1:]) <= 0.012 * expect[1:])
    assert abs(M.sum() - 4 * np.pi) < 0.01 * 4 * np.pi


def test_cotangent_stiffness_matches_elementwise_fem():
    v, f = S.perturbed_sphere(2, 7)
    K, M = S.cotangent_fem(v, f)
    Kd, Md = ofem.stiffness_and_mass(v, f)
    assert np.max(np.abs(K.toarray() - Kd)) <= 1e-12 * np.max(np.abs(Kd))
    assert np.allclose(M, Md, rtol=1e-13)


def test_real_harmonics_are_orthonormal():
    v, f = S.icosphere(5)
    _, M = S.cotangent_fem(v, f)
    Y = S.real_sph_harm(4, v)
    G = Y.T @ (M[:, None] * Y)
    assert np.max(np.abs(G - np.eye(25))) < 5e-3


def test_perturbed_eigenpairs_are_m_orthonormal():
    v, f = S.perturbed_sphere(3, 3)
    K, M = S.cotangent_fem(v, f)
    lam, Phi = S.eigenpairs(K, M, 300, slice_size=64, workers=2)
    assert np.all(np.diff(lam) >= 0)
    assert np.max(np.abs(Phi.T @ (M[:, None] * Phi) - np.eye(300))) < 1e-10
    assert np.max(np.abs(K @ Phi - (M[:, None] * Phi) * lam)) < 1e-9 * max(1.0, lam[-1])
    r = np.abs(np.linalg.norm(v, axis=1) - 1.0)
    assert 0.05 < r.max() <= 0.1 + 1e-12


def test_mesh_fiedler_tree_partition():
    v, f = S.perturbed_sphere(4, 3)
    K, M = S.cotangent_fem(v, f)
    perm, xoff = mesh_fiedler_tree(K, M, 6)
    assert np.array_equal(np.sort(perm), np.arange(len(v)))
    sizes = np.diff(xoff)
    assert len(sizes) == 64 and sizes.min() > 0 and sizes.max() < 3 * len(v) / 64
    # the first split is the sign of the whole mesh's Fiedler vector
    from paper_2605_21828_amd.factor.mesh_tree import fiedler_vector
    phi = fiedler_vector(K, M)
    first = set(np.nonzero(phi <= 0)[0].tolist())
    assert set(perm[:xoff[32]].tolist()) == first


def test_small_sphere_factors_reproduce_dense_transform():
    fs, prob = fio.sphere_factors(3, 3, 200, 16, 1e-10, workers=2, cache=False)
    c = np.random.default_rng(0).standard_normal((200, 3))
    f = np.random.default_rng(1).standard_normal((len(prob["v"]), 3))
    Phi = prob["Phi"]
    assert od.rel_err_cols(ob.apply(fs, c), Phi @ c)[0] < 1e-8
    assert od.rel_err_cols(ob.apply_transpose(fs, f), Phi.T @ f)[0] < 1e-8
