"""Scaled applies on the GPU (Sec. 7.2: Karhunen-Loeve samples and covariance
matrix-vector products of a Gaussian random field), through the C ABI, against
the oracle."""
import numpy as np
import pytest

from oracle import butterfly as ob
from oracle import dense as od
from oracle import modes as om
from paper_2605_21828_amd import workloads as wl
from paper_2605_21828_amd.factor import io as fio

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def grid():
    w = wl.WORKLOADS["grid64"]
    pts = wl.points_for(w)
    fs, _ = fio.fourier_factors(pts, w["m"], w["leaf"], w["tol"], workers=8, cache=False)
    md = om.fourier_modes(w["m"])
    from paper_2605_21828_amd.grf import matern_density
    s = matern_density(om.eigenvalues(md), nu=1.5, kappa=0.5)
    return w, pts, fs, md, s


def _t(x, dtype):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _np(x):
    import torch
    torch.cuda.synchronize()
    return x.detach().double().cpu().numpy()


def test_scaled_apply_f64_vs_oracle(gpu, grid):
    import torch
    from paper_2605_21828_amd.bfmht import Plan
    w, pts, fs, md, s = grid
    p = Plan(fs, "f64", max_nrhs=8)
    z = wl.coefficients(w["wid"], w["m"], 8, stream=5)
    y = _np(p.apply_scaled(_t(np.sqrt(s), torch.float64), _t(z, torch.float64)))
    assert od.rel_err_cols(y, ob.apply(fs, np.sqrt(s)[:, None] * z))[0] <= 1e-12
    fv = wl.values(w["wid"], w["n"], 8)
    g = _np(p.apply_t_scaled(_t(s, torch.float64), _t(fv, torch.float64)))
    assert od.rel_err_cols(g, s[:, None] * ob.apply_transpose(fs, fv))[0] <= 1e-12


@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("bf16x3", 1e-5)])
def test_kl_sample_and_covariance_vs_dense(gpu, grid, prec, tol):
    import torch
    from paper_2605_21828_amd.bfmht import Plan
    w, pts, fs, md, s = grid
    Phi = om.phi(pts, md)
    p = Plan(fs, prec, max_nrhs=16)
    z = wl.coefficients(w["wid"], w["m"], 16, stream=5)
    y = _np(p.apply_scaled(_t(np.sqrt(s), torch.float32), _t(z, torch.float32)))
    assert od.rel_err_cols(y, od.kl_sample(Phi, s, z))[0] <= tol
    v = wl.values(w["wid"], w["n"], 4)
    cv = _np(p.covariance_matvec(_t(s, torch.float32), _t(v, torch.float32)))
    assert od.rel_err_cols(cv, od.covariance(Phi, s) @ v)[0] <= tol


def test_scaled_apply_leaves_input_and_rejects_null_scale(gpu, grid):
    import torch
    from paper_2605_21828_amd import bfmht as B
    w, pts, fs, md, s = grid
    p = B.Plan(fs, "f32", max_nrhs=2)
    z = _t(wl.coefficients(w["wid"], w["m"], 2, stream=5), torch.float32)
    z0 = z.clone()
    p.apply_scaled(_t(s, torch.float32), z)
    torch.cuda.synchronize()
    assert torch.equal(z, z0)
    f = torch.empty((p.n, 2), dtype=torch.float32, device="cuda")
    ws, wsb = p.workspace(2)
    with pytest.raises(B.BfmhtError) as e:
        B.bfmht_apply_scaled(p.handle, None, z.data_ptr(), 2, f.data_ptr(), 2, 2, ws, wsb, 0)
    assert e.value.status == B.EINVAL


def _leading_identity_levels(fs):
    L = int(fs["L"])
    k = 0
    while k <= L and fs["ident"][k].all():
        k += 1
    return k


@pytest.fixture(scope="module")
def odd_fold():
    """A nonuniform factor set whose first three levels are all identities, so
    the first forward stage that runs is level 3 (an odd level)."""
    pts = wl.iid_points(13, 4096)
    fs, _ = fio.fourier_factors(pts, 1024, 64, 1e-8, workers=8, cache=False)
    return pts, fs, om.fourier_modes(1024)


@pytest.mark.parametrize("nrhs", [3, 8])   # few-RHS kernel and MFMA tiles
def test_scaled_applies_after_odd_fold_f64_vs_oracle(gpu, odd_fold, nrhs):
    import torch
    from paper_2605_21828_amd.bfmht import Plan
    from paper_2605_21828_amd.grf import matern_density
    pts, fs, md = odd_fold
    assert _leading_identity_levels(fs) == 3
    s = matern_density(om.eigenvalues(md), nu=1.5, kappa=0.5)
    p = Plan(fs, "f64", max_nrhs=nrhs)
    z = wl.coefficients(13, 1024, nrhs, stream=5)
    y = _np(p.apply_scaled(_t(np.sqrt(s), torch.float64), _t(z, torch.float64)))
    assert od.rel_err_cols(y, ob.apply(fs, np.sqrt(s)[:, None] * z))[0] <= 1e-12
    v = wl.values(13, 4096, nrhs)
    cv = _np(p.covariance_matvec(_t(s, torch.float64), _t(v, torch.float64)))
    assert od.rel_err_cols(cv, ob.apply(fs, s[:, None] * ob.apply_transpose(fs, v)))[0] <= 1e-12


@pytest.mark.parametrize("nrhs", [3, 8])
def test_scaled_applies_after_odd_fold_f32_vs_dense(gpu, odd_fold, nrhs):
    import torch
    from paper_2605_21828_amd.bfmht import Plan
    from paper_2605_21828_amd.grf import matern_density
    pts, fs, md = odd_fold
    s = matern_density(om.eigenvalues(md), nu=1.5, kappa=0.5)
    Phi = om.phi(pts, md)
    p = Plan(fs, "f32", max_nrhs=nrhs)
    z = wl.coefficients(13, 1024, nrhs, stream=5)
    y = _np(p.apply_scaled(_t(np.sqrt(s), torch.float32), _t(z, torch.float32)))
    assert od.rel_err_cols(y, od.kl_sample(Phi, s, z))[0] <= 1e-5
    v = wl.values(13, 4096, nrhs)
    cv = _np(p.covariance_matvec(_t(s, torch.float32), _t(v, torch.float32)))
    assert od.rel_err_cols(cv, od.covariance(Phi, s) @ v)[0] <= 1e-5


@pytest.mark.parametrize("ident_levels", [1, 2, 3])
def test_scaled_apply_random_factors_any_fold_depth(gpu, ident_levels):
    import torch
    from factor_gen import random_factor_set
    from paper_2605_21828_amd.bfmht import Plan
    fs = random_factor_set(70 + ident_levels, 700, 300, 5, max_rank=40, p_ident=0.1, ident_levels=ident_levels,
                           p_id_form=0.5)
    assert _leading_identity_levels(fs) == ident_levels
    s = np.random.default_rng(ident_levels).uniform(0.5, 2.0, 300)
    for b in (2, 16):
        z = wl.coefficients(71, 300, b, stream=5)
        p = Plan(fs, "f64", max_nrhs=b)
        y = _np(p.apply_scaled(_t(s, torch.float64), _t(z, torch.float64)))
        assert od.rel_err_cols(y, ob.apply(fs, s[:, None] * z))[0] <= 1e-12
