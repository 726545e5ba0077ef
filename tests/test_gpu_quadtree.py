"""4-ary trees on the GPU (Sec. 2: the construction generalizes to k-ary trees;
Sec. 5 analyses the quadtree in space with a 4-ary tree on the eigenvalues),
through the C ABI, against the oracle's butterfly apply of the same factor set
and against the dense transform.  A transposed 4-ary job has four consumers:
the library runs two of them per launch, the second launch adding to the rows
the first one wrote."""
import numpy as np
import pytest

from factor_gen import random_factor_set
from oracle import butterfly as ob
from oracle import dense as od
from oracle import modes as om
from paper_2605_21828_amd import workloads as wl
from paper_2605_21828_amd.factor import io as fio

pytestmark = pytest.mark.gpu

CASES = [  # seed, n, m, L, max_rank, p_id_form, ident_levels
    (50, 700, 256, 3, 40, 0.0, 0),
    (51, 3000, 1024, 3, 60, 0.7, 0),
    (52, 900, 300, 2, 50, 0.5, 1),
    (53, 2000, 512, 3, 30, 0.5, 2),
    (54, 40, 30, 2, 8, 0.3, 0),      # empty leaves
]


def _dt(prec):
    import torch
    return torch.float64 if prec == "f64" else torch.float32


def _t(x, dt):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")


def _np(x):
    import torch
    torch.cuda.synchronize()
    return x.double().cpu().numpy()


@pytest.fixture(scope="module")
def sets():
    return [random_factor_set(s, n, m, L, max_rank=r, p_id_form=p, ident_levels=k, arity=4)
            for s, n, m, L, r, p, k in CASES]


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
@pytest.mark.parametrize("nrhs", [1, 3, 16, 70])   # few-RHS kernel and MFMA tiles
def test_quadtree_random_factors_vs_oracle(gpu, sets, prec, tol, nrhs):
    from paper_2605_21828_amd.bfmht import Plan
    rng = np.random.default_rng(nrhs)
    for fs, case in zip(sets, CASES):
        assert int(fs["arity"]) == 4
        p = Plan(fs, prec, max_nrhs=nrhs)
        c = rng.standard_normal((int(fs["m"]), nrhs))
        f = rng.standard_normal((int(fs["n"]), nrhs))
        assert od.rel_err_cols(_np(p.apply(_t(c, _dt(prec)))), ob.apply(fs, c))[0] <= tol, case
        assert od.rel_err_cols(_np(p.apply_t(_t(f, _dt(prec)))), ob.apply_transpose(fs, f))[0] <= tol, case


@pytest.mark.parametrize("prec", ["bf16x2", "bf16x3"])
def test_quadtree_bf16_splits_within_bound(gpu, sets, prec):
    """The split products on 4-ary sets: every output within (L+2) gamma of the
    same apply with absolute factors and inputs (gamma 2^-14 for two terms,
    2^-21 for three), as for binary trees."""
    from paper_2605_21828_amd.bfmht import Plan
    gamma = 2.0 ** -14 if prec == "bf16x2" else 2.0 ** -21
    rng = np.random.default_rng(5)
    for fs in sets[:4]:
        fa = dict(fs, P=np.abs(fs["P"]), U=np.abs(fs["U"]))
        k = (int(fs["L"]) + 2) * gamma
        p = Plan(fs, prec, max_nrhs=20)
        c = rng.standard_normal((int(fs["m"]), 20))
        f = rng.standard_normal((int(fs["n"]), 20))
        y = _np(p.apply(_t(c, _dt(prec))))
        assert np.all(np.abs(y - ob.apply(fs, c)) <= k * ob.apply(fa, np.abs(c)) + 1e-30)
        g = _np(p.apply_t(_t(f, _dt(prec))))
        assert np.all(np.abs(g - ob.apply_transpose(fs, f)) <= k * ob.apply_transpose(fa, np.abs(f)) + 1e-30)


def test_quadtree_folded_identity_levels_match_unfolded_bitwise(gpu, sets):
    """Two leading all-identity 4-ary levels: the single transposed apply sums
    the 16 copies of each row of c with one gather-sum, the batched apply runs
    the identity stages (two launches each); the sums come in the same order."""
    from paper_2605_21828_amd.bfmht import Batch, Plan
    fs = sets[3]
    assert fs["ident"][0].all() and fs["ident"][1].all()
    rng = np.random.default_rng(11)
    for prec in ("f64", "f32"):
        for nrhs in (3, 16):
            p = Plan(fs, prec, max_nrhs=nrhs)
            f = _t(rng.standard_normal((int(fs["n"]), nrhs)), _dt(prec))
            g_single = _np(p.apply_t(f))
            g_batch = _np(Batch([p]).run([f], transpose=True)[0])
            assert np.array_equal(g_single, g_batch), (prec, nrhs)


def test_quadtree_batched_matches_oracle(gpu, sets):
    from paper_2605_21828_amd.bfmht import Batch, Plan
    rng = np.random.default_rng(12)
    rhs = [5, 1, 33, 17, 2]
    plans = [Plan(fs, "f32", max_nrhs=b) for fs, b in zip(sets, rhs)]
    xs = [rng.standard_normal((int(fs["m"]), b)) for fs, b in zip(sets, rhs)]
    fv = [rng.standard_normal((int(fs["n"]), b)) for fs, b in zip(sets, rhs)]
    ys = Batch(plans).run([_t(x, _dt("f32")) for x in xs])
    gs = Batch(plans).run([_t(f, _dt("f32")) for f in fv], transpose=True)
    for fs, x, f, y, g in zip(sets, xs, fv, ys, gs):
        assert od.rel_err_cols(_np(y), ob.apply(fs, x))[0] <= 1e-5
        assert od.rel_err_cols(_np(g), ob.apply_transpose(fs, f))[0] <= 1e-5


def test_quadtree_fourier_transform_vs_dense(gpu):
    """A 4-ary factor set of the Fourier transform on 4096 nonuniform points
    (quadtree in space, 4-ary index tree on the modes, tol 1e-8): FP64 against
    the oracle's apply of the same set, FP32 and BF16X3 against the dense Phi."""
    from paper_2605_21828_amd.bfmht import Plan
    pts = wl.iid_points(55, 4096)
    fs, _ = fio.fourier_factors(pts, 1024, 16, 1e-8, workers=8, cache=False, arity=4)
    assert int(fs["arity"]) == 4 and int(fs["L"]) == 4
    Phi = om.phi(pts, om.fourier_modes(1024))
    rng = np.random.default_rng(56)
    c = rng.standard_normal((1024, 8))
    f = rng.standard_normal((4096, 8))
    p64 = Plan(fs, "f64", max_nrhs=8)
    assert od.rel_err_cols(_np(p64.apply(_t(c, _dt("f64")))), ob.apply(fs, c))[0] <= 1e-12
    assert od.rel_err_cols(_np(p64.apply_t(_t(f, _dt("f64")))), ob.apply_transpose(fs, f))[0] <= 1e-12
    for prec in ("f32", "bf16x3"):
        p = Plan(fs, prec, max_nrhs=8)
        assert od.rel_err_cols(_np(p.apply(_t(c, _dt(prec)))), Phi @ c)[0] <= 1e-5, prec
        assert od.rel_err_cols(_np(p.apply_t(_t(f, _dt(prec)))), Phi.T @ f)[0] <= 1e-5, prec
