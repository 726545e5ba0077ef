"""Inverse transform by LSQR on the GPU (Sec. 7.1, eq. inverse-MHT), through the
C ABI, against the oracle's LSQR over the oracle's butterfly apply and against
dense least squares."""
import numpy as np
import pytest

from oracle import butterfly as ob
from oracle import dense as od
from oracle import modes as om
from oracle.lsqr import lsqr as oracle_lsqr
from paper_2605_21828_amd import workloads as wl
from paper_2605_21828_amd.factor import io as fio

pytestmark = pytest.mark.gpu


def _t(x, dtype):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _np(x):
    import torch
    torch.cuda.synchronize()
    return x.detach().double().cpu().numpy()


@pytest.fixture(scope="module")
def grid():
    w = wl.WORKLOADS["grid64"]
    pts = wl.points_for(w)
    fs, _ = fio.fourier_factors(pts, w["m"], w["leaf"], w["tol"], workers=8, cache=False)
    md = om.fourier_modes(w["m"])
    c_star = wl.coefficients(w["wid"], w["m"], 3, stream=5)
    f = om.grid_synthesis_ifft2(w["N"], md, c_star)      # exact transform of known coefficients
    return w, fs, md, c_star, f


def test_lsqr_f64_matches_oracle_lsqr_and_recovers_coefficients(gpu, grid):
    import torch
    from paper_2605_21828_amd.bfmht import Plan
    w, fs, md, c_star, f = grid
    p = Plan(fs, "f64", max_nrhs=3)
    x, rn = p.lsqr(_t(f, torch.float64), 25)
    x, rn = _np(x), _np(rn)
    for j in range(3):
        xo, res = oracle_lsqr(lambda v: ob.apply(fs, v[:, None])[:, 0],
                              lambda u: ob.apply_transpose(fs, u[:, None])[:, 0], f[:, j], 25)
        assert np.linalg.norm(x[:, j] - xo) <= 1e-10 * np.linalg.norm(xo)
        assert abs(rn[j] - res[-1]) <= 1e-8 * np.linalg.norm(f[:, j])
    # the grid transform has orthogonal columns (condition number 2): 25 steps reach the exact coefficients
    assert od.rel_err_cols(x, c_star)[0] <= 1e-8


def test_lsqr_f32_vs_oracle(gpu):
    import torch
    from paper_2605_21828_amd.bfmht import Plan
    wid = 12
    pts = wl.iid_points(wid, 8192)
    fs, _ = fio.fourier_factors(pts, 2048, 64, 1e-8, workers=8, cache=False)
    f = wl.values(wid, 8192, 2)
    p = Plan(fs, "f32", max_nrhs=2)
    x, rn = p.lsqr(_t(f, torch.float32), 30)
    x = _np(x)
    for j in range(2):
        xo, res = oracle_lsqr(lambda v: ob.apply(fs, v[:, None])[:, 0],
                              lambda u: ob.apply_transpose(fs, u[:, None])[:, 0], f[:, j], 30)
        assert np.linalg.norm(x[:, j] - xo) <= 1e-4 * np.linalg.norm(xo)
    # the residual estimate agrees with the residual of the returned iterate
    r = _np(p.apply(_t(x, torch.float32))) - f
    assert np.allclose(np.linalg.norm(r, axis=0), _np(rn), rtol=1e-3)


def test_inverse_transform_of_sphere_coordinates(gpu):
    """The mesh-processing use of Sec. 7.1: the coordinates of a perturbed
    sphere's vertices are solved for in the eigenbasis, as dense least squares would."""
    import torch
    from paper_2605_21828_amd.bfmht import Plan
    fs, prob = fio.sphere_factors(3, 3, 200, 16, 1e-10, workers=2, cache=False)
    X = np.asarray(prob["v"], dtype=np.float64)          # n x 3 vertex coordinates
    p = Plan(fs, "f64", max_nrhs=3)
    c, _ = p.lsqr(_t(X, torch.float64), 200)
    c = _np(c)
    ref = np.linalg.lstsq(prob["Phi"], X, rcond=None)[0]
    assert od.rel_err_cols(c, ref)[0] <= 1e-6
    # a filtered mesh is one synthesis of the filtered coefficients
    F = (prob["lam"] < prob["lam"][40]).astype(np.float64)
    Xf = _np(p.apply(_t(F[:, None] * c, torch.float64)))
    assert od.rel_err_cols(Xf, prob["Phi"] @ (F[:, None] * ref))[0] <= 1e-6


def test_lsqr_argument_errors(gpu, grid):
    import torch
    from paper_2605_21828_amd import bfmht as B
    w, fs, md, c_star, f = grid
    p = B.Plan(fs, "f32", max_nrhs=1)
    ft = _t(f[:, :1], torch.float32)
    x = torch.empty((p.m, 1), dtype=torch.float32, device="cuda")
    need = B.bfmht_lsqr_workspace_bytes(p.handle, 1)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    wp = (ws.data_ptr() + 255) // 256 * 256
    with pytest.raises(B.BfmhtError) as e:
        B.bfmht_lsqr(p.handle, ft.data_ptr(), 1, x.data_ptr(), 1, 1, -1, None, wp, need, 0)
    assert e.value.status == B.EINVAL
    with pytest.raises(B.BfmhtError) as e:
        B.bfmht_lsqr(p.handle, ft.data_ptr(), 1, x.data_ptr(), 1, 1, 3, None, wp, need - 256, 0)
    assert e.value.status == B.ENOSPACE
    B.bfmht_lsqr(p.handle, ft.data_ptr(), 1, x.data_ptr(), 1, 1, 0, None, wp, need, 0)
    assert not _np(x).any()       # zero steps leave the zero iterate


def test_lsqr_zero_steps_reports_the_norm_of_f(gpu, grid):
    """With no step the iterate is zero and the residual estimate is ||f|| per column."""
    import torch
    from paper_2605_21828_amd.bfmht import Plan
    w, fs, md, c_star, f = grid
    for prec, dt, tol in (("f64", torch.float64, 1e-13), ("f32", torch.float32, 1e-6)):
        p = Plan(fs, prec, max_nrhs=3)
        x, rn = p.lsqr(_t(f, dt), 0)
        assert not _np(x).any()
        assert np.allclose(_np(rn), np.linalg.norm(f, axis=0), rtol=tol, atol=0)
