"""Autograd through the butterfly transform (GPU, through the C ABI).

The loss ||Phi~ c - f||^2 is quadratic in c, so a central finite difference is
exact for any step up to rounding; evaluated with the oracle's FP64 butterfly
apply it pins the autograd gradient independently of the GPU path.  The
gradient is also compared with the dense FP64 2 Phi^T (Phi c - f) of the exact
transform on sampled columns.
"""
import numpy as np
import pytest

from oracle import butterfly as ob
from oracle import dense as od
from oracle import modes as om
from paper_2605_21828_amd import workloads as wl
from paper_2605_21828_amd.factor import io as fio

pytestmark = pytest.mark.gpu

WID = 50


@pytest.fixture(scope="module")
def problem():
    n, m = 16384, 4096
    pts = wl.iid_points(WID, n)
    fs, _ = fio.fourier_factors(pts, m, 128, 1e-8, workers=8, cache=False)
    md = om.fourier_modes(m)
    lam = om.eigenvalues(md)
    c_star = wl.coefficients(WID, m, 1, lam=lam, kind="decay")[:, 0]
    f = om.phi(pts, md) @ c_star + 1e-3 * wl.values(WID, n, 1, stream=2)[:, 0]
    return pts, fs, md, c_star, f


def _grad(plan, c, f, dtype):
    import torch
    from paper_2605_21828_amd.autograd import BFApply
    ct = torch.tensor(c, dtype=dtype, device="cuda", requires_grad=True)
    ft = torch.tensor(f, dtype=dtype, device="cuda")
    r = BFApply.apply(ct, plan) - ft
    loss = (r * r).sum()
    loss.backward()
    return ct.grad.double().cpu().numpy(), float(loss)


def _fd(fs, c, f, coords, h=1.0):
    E = np.zeros((c.size, len(coords)))
    E[coords, np.arange(len(coords))] = h
    Cp, Cm = c[:, None] + E, c[:, None] - E
    Lp = np.sum((ob.apply(fs, Cp) - f[:, None]) ** 2, axis=0)
    Lm = np.sum((ob.apply(fs, Cm) - f[:, None]) ** 2, axis=0)
    return (Lp - Lm) / (2 * h)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-5), ("bf16x3", 1e-5)])
def test_gradient_matches_central_differences(gpu, problem, prec, tol):
    import torch
    from paper_2605_21828_amd.bfmht import Plan
    pts, fs, md, c_star, f = problem
    c = wl.coefficients(WID, fs["m"], 1, stream=5)[:, 0]
    coords = wl.sample_indices(WID, int(fs["m"]), 64, stream=4)
    plan = Plan(fs, prec, max_nrhs=1)
    g, _ = _grad(plan, c, f, torch.float64 if prec == "f64" else torch.float32)
    fd = _fd(fs, c, f, coords)
    assert np.linalg.norm(g[coords] - fd) <= tol * np.linalg.norm(fd)


def test_gradient_matches_dense_fp64_on_sampled_columns(gpu, problem):
    import torch
    from paper_2605_21828_amd.bfmht import Plan
    pts, fs, md, c_star, f = problem
    c = wl.coefficients(WID, fs["m"], 1, stream=5)[:, 0]
    cols = wl.sample_indices(WID, int(fs["m"]), 256, stream=3)
    plan = Plan(fs, "f32", max_nrhs=1)
    g, _ = _grad(plan, c, f, torch.float32)
    Phi = om.phi(pts, md)
    ref = 2.0 * od.fourier_analysis_cols(pts, md, cols, Phi @ c - f)
    assert np.linalg.norm(g[cols] - ref) <= 1e-5 * np.linalg.norm(ref)


def test_backward_of_analysis_is_synthesis(gpu, problem):
    import torch
    from paper_2605_21828_amd.autograd import BFApplyT
    from paper_2605_21828_amd.bfmht import Plan
    pts, fs, md, c_star, f = problem
    plan = Plan(fs, "f64", max_nrhs=2)
    fv = torch.tensor(wl.values(WID, int(fs["n"]), 2), dtype=torch.float64, device="cuda", requires_grad=True)
    w = torch.tensor(wl.coefficients(WID, int(fs["m"]), 2, stream=5), dtype=torch.float64, device="cuda")
    (BFApplyT.apply(fv, plan) * w).sum().backward()
    ref = ob.apply(fs, w.cpu().numpy())
    assert od.rel_err_cols(fv.grad.cpu().numpy(), ref)[0] <= 1e-12


def test_gradient_descent_decreases_loss(gpu, problem):
    import torch
    from paper_2605_21828_amd.autograd import least_squares_step
    from paper_2605_21828_amd.bfmht import Plan
    pts, fs, md, c_star, f = problem
    plan = Plan(fs, "f32", max_nrhs=1)
    ft = torch.tensor(f, dtype=torch.float32, device="cuda")
    c = torch.zeros(int(fs["m"]), dtype=torch.float32, device="cuda")
    # step size from the largest singular value of Phi~ (power iteration on Phi~^T Phi~)
    v = torch.tensor(wl.values(WID, int(fs["m"]), 1, stream=5)[:, 0], dtype=torch.float32, device="cuda")
    for _ in range(20):
        v = plan.apply_t(plan.apply(v))
        s2 = torch.linalg.norm(v)
        v = v / s2
    lr = 0.5 / float(s2)
    losses = []
    for _ in range(30):
        c, loss = least_squares_step(plan, c, ft, lr)
        losses.append(float(loss))
    assert all(b <= a * (1 + 1e-6) for a, b in zip(losses, losses[1:]))
    assert losses[-1] < 0.5 * losses[0]
