"""GPU parity of the HIP butterfly apply against the CPU oracle (through the C ABI).

Bars: FP64 GPU vs the oracle's butterfly apply O2 within 1e-12 relative; FP32
and BF16-split GPU vs the dense FP64 product O1 within 1e-5 relative 2-norm,
max over right-hand-side columns; pure permutation factor sets bit-exact.
"""
import numpy as np
import pytest

from factor_gen import random_factor_set
from oracle import butterfly as ob
from oracle import dense as od
from oracle import modes as om
from paper_2605_21828_amd import workloads as wl
from paper_2605_21828_amd.factor import io as fio

pytestmark = pytest.mark.gpu


def _plan(fs, prec, max_nrhs=64):
    from paper_2605_21828_amd.bfmht import Plan
    return Plan(fs, prec, max_nrhs=max_nrhs)


def _t(x, dtype):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _np(x):
    import torch
    torch.cuda.synchronize()
    return x.detach().double().cpu().numpy()


def _rel(x, ref):
    return od.rel_err_cols(x, ref)[0]


@pytest.fixture(scope="module")
def grid64():
    w = wl.WORKLOADS["grid64"]
    pts = wl.points_for(w)
    fs, _ = fio.fourier_factors(pts, w["m"], w["leaf"], w["tol"], workers=8, cache=False)
    return w, pts, fs


def test_grid64_f64_matches_oracle(gpu, grid64):
    import torch
    w, pts, fs = grid64
    md = om.fourier_modes(w["m"])
    c = wl.coefficients(w["wid"], w["m"], 1)
    p = _plan(fs, "f64", 1)
    f = _np(p.apply(_t(c, torch.float64)))
    assert _rel(f, ob.apply(fs, c)) <= 1e-12
    # end to end against the exact transform (inverse DFT) at the factor tolerance
    assert _rel(f, om.grid_synthesis_ifft2(w["N"], md, c)) <= 1e-9
    fv = wl.values(w["wid"], w["n"], 1)
    g = _np(p.apply_t(_t(fv, torch.float64)))
    assert _rel(g, ob.apply_transpose(fs, fv)) <= 1e-12
    assert _rel(g, om.grid_analysis_fft2(w["N"], md, fv)) <= 1e-9


RANDOM_CASES = [
    # seed, n, m, L, max_rank
    (0, 300, 200, 4, 40),
    (1, 1000, 333, 5, 90),
    (2, 77, 500, 3, 130),    # ranks above one tile, ragged tails
    (3, 257, 129, 7, 20),    # many empty leaves
    (4, 5, 3, 2, 4),         # tiny
]


@pytest.mark.parametrize("case", RANDOM_CASES)
@pytest.mark.parametrize("nrhs", [1, 3, 17, 64, 100])
def test_random_factors_f64_vs_oracle(gpu, case, nrhs):
    import torch
    seed, n, m, L, mr = case
    fs = random_factor_set(seed, n, m, L, max_rank=mr)
    rng = np.random.default_rng(seed + 100)
    c, f = rng.standard_normal((m, nrhs)), rng.standard_normal((n, nrhs))
    p = _plan(fs, "f64", nrhs)
    assert _rel(_np(p.apply(_t(c, torch.float64))), ob.apply(fs, c)) <= 1e-12
    assert _rel(_np(p.apply_t(_t(f, torch.float64))), ob.apply_transpose(fs, f)) <= 1e-12


@pytest.mark.parametrize("case", RANDOM_CASES)
@pytest.mark.parametrize("nrhs", [1, 33, 64])
def test_random_factors_f32_vs_oracle(gpu, case, nrhs):
    import torch
    seed, n, m, L, mr = case
    fs = random_factor_set(seed, n, m, L, max_rank=mr)
    rng = np.random.default_rng(seed + 200)
    c, f = rng.standard_normal((m, nrhs)), rng.standard_normal((n, nrhs))
    p = _plan(fs, "f32", nrhs)
    assert _rel(_np(p.apply(_t(c, torch.float32))), ob.apply(fs, c)) <= 1e-5
    assert _rel(_np(p.apply_t(_t(f, torch.float32))), ob.apply_transpose(fs, f)) <= 1e-5


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("L", [0, 3, 6])
def test_permutation_is_bit_exact(gpu, prec, L):
    import torch
    n = 1000
    fs = random_factor_set(30 + L, n, n, L, identity_values=True)
    dt = torch.float64 if prec == "f64" else torch.float32
    c = np.arange(n * 5, dtype=np.float64).reshape(n, 5)   # integers < 2^24: exact in FP32
    p = _plan(fs, prec, 5)
    f = _np(p.apply(_t(c, dt)))
    assert np.array_equal(f[fs["perm_x"]], c)
    g = _np(p.apply_t(_t(f, dt)))
    assert np.array_equal(g, c)


@pytest.fixture(scope="module")
def iid_medium():
    wid = 12
    pts = wl.iid_points(wid, 8192)
    fs, _ = fio.fourier_factors(pts, 2048, 64, 1e-8, workers=8, cache=False)
    return wid, pts, fs, om.fourier_modes(2048)


def test_iid_f32_apply_and_transpose_vs_dense(gpu, iid_medium):
    import torch
    wid, pts, fs, md = iid_medium
    Phi = om.phi(pts, md)
    c = wl.coefficients(wid, 2048, 64, lam=om.eigenvalues(md), kind="decay")
    fv = wl.values(wid, 8192, 64)
    p = _plan(fs, "f32", 64)
    assert _rel(_np(p.apply(_t(c, torch.float32))), Phi @ c) <= 1e-5
    assert _rel(_np(p.apply_t(_t(fv, torch.float32))), Phi.T @ fv) <= 1e-5


def test_iid_f64_vs_oracle_and_dense(gpu, iid_medium):
    import torch
    wid, pts, fs, md = iid_medium
    c = wl.coefficients(wid, 2048, 16)
    p = _plan(fs, "f64", 16)
    f = _np(p.apply(_t(c, torch.float64)))
    assert _rel(f, ob.apply(fs, c)) <= 1e-12
    assert _rel(f, om.phi(pts, md) @ c) <= 1e-6


def test_strided_rows_and_nrhs_zero(gpu):
    import torch
    fs = random_factor_set(40, 200, 150, 4, max_rank=30)
    rng = np.random.default_rng(40)
    c = rng.standard_normal((150, 7))
    p = _plan(fs, "f32", 7)
    wide_c = torch.zeros((150, 12), dtype=torch.float32, device="cuda")
    wide_c[:, 2:9] = _t(c, torch.float32)
    wide_f = torch.full((200, 11), 7.0, dtype=torch.float32, device="cuda")
    p.apply(wide_c[:, 2:9], out=wide_f[:, 1:8])
    out = _np(wide_f)
    assert _rel(out[:, 1:8], ob.apply(fs, c)) <= 1e-5
    assert np.all(out[:, 0] == 7.0) and np.all(out[:, 8:] == 7.0)
    # nrhs = 0 is a no-op returning OK
    from paper_2605_21828_amd import bfmht as B
    B.bfmht_apply(p.handle, wide_c.data_ptr(), 12, wide_f.data_ptr(), 11, 0, 0, 0, 0)


def test_repeat_is_bitwise_deterministic(gpu, iid_medium):
    import torch
    wid, pts, fs, md = iid_medium
    c = _t(wl.coefficients(wid, 2048, 64), torch.float32)
    p = _plan(fs, "f32", 64)
    a = _np(p.apply(c))
    b = _np(p.apply(c))
    assert np.array_equal(a, b)


def test_workspace_too_small_is_rejected(gpu):
    import torch
    from paper_2605_21828_amd import bfmht as B
    fs = random_factor_set(41, 100, 80, 3, max_rank=20)
    p = _plan(fs, "f32", 4)
    c = torch.zeros((80, 4), dtype=torch.float32, device="cuda")
    f = torch.zeros((100, 4), dtype=torch.float32, device="cuda")
    ws, wsb = p.workspace(4)
    with pytest.raises(B.BfmhtError) as e:
        B.bfmht_apply(p.handle, c.data_ptr(), 4, f.data_ptr(), 4, 4, ws, wsb - 256, 0)
    assert e.value.status == B.ENOSPACE
    with pytest.raises(B.BfmhtError) as e:
        B.bfmht_apply(p.handle, c.data_ptr(), 3, f.data_ptr(), 4, 4, ws, wsb, 0)
    assert e.value.status == B.EINVAL
    with pytest.raises(B.BfmhtError) as e:
        B.bfmht_plan_upload(p.handle, p._dev_ptr, p.device_bytes, 0)
    assert e.value.status == B.ESTATE


# ---- BF16 split products ----
# A value split into t bfloat16 terms (8 significand bits each, round to
# nearest) is represented to 2^-8t relative.  BF16X2 keeps hi*hi + hi*lo +
# lo*hi, so one product differs from the exact one by at most about 3 * 2^-16
# of |w||x|; BF16X3 keeps the six products with term-index sum <= 2 and is good
# to a few 2^-24.  Over the L+2 stages of an apply the error of every output is
# then bounded by (L+2) * gamma * (|Phi~| |c|), where |Phi~| multiplies the
# absolute values of the factors; gamma below adds headroom for FP32
# accumulation (2^-14 for X2, 2^-21 for X3).  Relative bars are also asserted on
# realistic (non-cancelling) inputs: 1e-5 for X3, 1e-4 for X2.
BF16_GAMMA = {"bf16x2": 2.0 ** -14, "bf16x3": 2.0 ** -21}
BF16_TOL = {"bf16x3": 1e-5, "bf16x2": 1e-4}


def _abs_factors(fs):
    return dict(fs, P=np.abs(fs["P"]), U=np.abs(fs["U"]))


@pytest.mark.parametrize("prec", ["bf16x2", "bf16x3"])
@pytest.mark.parametrize("case", RANDOM_CASES)
@pytest.mark.parametrize("nrhs", [1, 40, 64])
def test_random_factors_bf16_within_error_bound(gpu, prec, case, nrhs):
    import torch
    seed, n, m, L, mr = case
    fs = random_factor_set(seed, n, m, L, max_rank=mr)
    fa = _abs_factors(fs)
    rng = np.random.default_rng(seed + 300)
    c, f = rng.standard_normal((m, nrhs)), rng.standard_normal((n, nrhs))
    p = _plan(fs, prec, nrhs)
    k = (L + 2) * BF16_GAMMA[prec]
    y = _np(p.apply(_t(c, torch.float32)))
    assert np.all(np.abs(y - ob.apply(fs, c)) <= k * ob.apply(fa, np.abs(c)) + 1e-30)
    g = _np(p.apply_t(_t(f, torch.float32)))
    assert np.all(np.abs(g - ob.apply_transpose(fs, f)) <= k * ob.apply_transpose(fa, np.abs(f)) + 1e-30)
    if prec == "bf16x3" and n >= 64:
        assert _rel(y, ob.apply(fs, c)) <= 1e-5


@pytest.mark.parametrize("prec", ["bf16x2", "bf16x3"])
def test_bf16_permutation_is_bit_exact(gpu, prec):
    import torch
    n = 1000
    fs = random_factor_set(37, n, n, 4, identity_values=True)
    c = np.arange(n * 5, dtype=np.float64).reshape(n, 5)   # integers < 2^16: exact in two bf16 terms
    p = _plan(fs, prec, 5)
    f = _np(p.apply(_t(c, torch.float32)))
    assert np.array_equal(f[fs["perm_x"]], c)
    assert np.array_equal(_np(p.apply_t(_t(f, torch.float32))), c)


@pytest.mark.parametrize("prec", ["bf16x2", "bf16x3"])
def test_iid_bf16_vs_dense(gpu, iid_medium, prec):
    import torch
    wid, pts, fs, md = iid_medium
    Phi = om.phi(pts, md)
    c = wl.coefficients(wid, 2048, 64, lam=om.eigenvalues(md), kind="decay")
    fv = wl.values(wid, 8192, 64)
    p = _plan(fs, prec, 64)
    e1 = _rel(_np(p.apply(_t(c, torch.float32))), Phi @ c)
    e2 = _rel(_np(p.apply_t(_t(fv, torch.float32))), Phi.T @ fv)
    print("%s synthesis %.2e analysis %.2e" % (prec, e1, e2))
    assert e1 <= BF16_TOL[prec] and e2 <= BF16_TOL[prec]


@pytest.fixture(scope="module")
def small_sphere():
    return fio.sphere_factors(3, 3, 200, 16, 1e-8, workers=4, cache=False)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-7), ("f32", 1e-5), ("bf16x3", 1e-5), ("bf16x2", 1e-4)])
def test_sphere_vs_dense(gpu, small_sphere, prec, tol):
    """Perturbed icosphere (642 vertices, 200 eigenvectors, Fiedler tree) against the dense Phi."""
    import torch
    fs, prob = small_sphere
    Phi = prob["Phi"]
    c = np.random.default_rng(20).standard_normal((200, 256))
    f = np.random.default_rng(21).standard_normal((Phi.shape[0], 256))
    p = _plan(fs, prec, 256)
    dt = torch.float64 if prec == "f64" else torch.float32
    assert _rel(_np(p.apply(_t(c, dt))), Phi @ c) <= tol
    assert _rel(_np(p.apply_t(_t(f, dt))), Phi.T @ f) <= tol


def test_binding_rejects_bad_out_tensors(gpu):
    """out= tensors are checked before the library writes into them."""
    import torch
    from factor_gen import random_factor_set
    from paper_2605_21828_amd.bfmht import Batch, Plan
    fs = random_factor_set(31, 300, 200, 4, max_rank=40)
    p = Plan(fs, "f32", max_nrhs=4)
    c = torch.zeros((200, 4), dtype=torch.float32, device="cuda")
    f = torch.zeros((300, 4), dtype=torch.float32, device="cuda")
    bad = [torch.empty((299, 4), dtype=torch.float32, device="cuda"),      # too few rows
           torch.empty((300, 3), dtype=torch.float32, device="cuda"),      # too few columns
           torch.empty((300, 4), dtype=torch.float64, device="cuda"),      # wrong element type
           torch.empty((300, 4), dtype=torch.float32),                     # host memory
           torch.empty((4, 300), dtype=torch.float32, device="cuda").t()]  # column stride 300
    for out in bad:
        with pytest.raises(ValueError):
            p.apply(c, out=out)
    with pytest.raises(ValueError):
        p.apply_t(f, out=torch.empty((201, 4), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        p.apply_scaled(torch.ones(200, device="cuda"), c, out=bad[0])
    with pytest.raises(ValueError):
        p.apply_t_scaled(torch.ones(200, device="cuda"), f, out=bad[2])
    with pytest.raises(ValueError):
        Batch([p, p]).launch([c], [f])                                     # fewer inputs than plans
    with pytest.raises(ValueError):
        Batch([p]).launch([c], [bad[1]])
    # a 1-D out takes a single column; a wider row stride is fine
    y1 = torch.empty(300, dtype=torch.float32, device="cuda")
    p.apply(c[:, 0], out=y1)
    wide = torch.zeros((300, 6), dtype=torch.float32, device="cuda")
    p.apply(c, out=wide[:, 1:5])
    torch.cuda.synchronize()
    assert torch.equal(wide[:, 1:5], p.apply(c))
