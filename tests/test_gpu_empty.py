"""Degenerate transforms through the C ABI: no points (n = 0), no modes (m = 0)
or neither, with and without positive ranks in the levels between.

Phi is then an empty matrix: the synthesis of m = 0 modes is the zero field, the
analysis of n = 0 points gives zero coefficients, and operands with no rows may
be NULL (torch hands out a null pointer for an empty tensor).  Outputs start as
NaN so that every element the call must write is checked.
"""
import numpy as np
import pytest

from factor_gen import random_factor_set
from oracle import butterfly as ob

pytestmark = pytest.mark.gpu

CASES = [
    # seed, n, m, L
    (60, 0, 7, 0),
    (61, 0, 7, 2),      # positive ranks in the levels, empty leaf bases
    (62, 0, 300, 3),
    (63, 9, 0, 2),
    (64, 40, 0, 0),
    (65, 0, 0, 1),
]


def _t(x, dtype):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _np(x):
    import torch
    torch.cuda.synchronize()
    return x.detach().double().cpu().numpy()


def _nan(rows, cols, dtype):
    import torch
    return torch.full((rows, cols), float("nan"), dtype=dtype, device="cuda")


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x2"])
@pytest.mark.parametrize("nrhs", [3, 20])
def test_empty_transform_apply_and_transpose(gpu, case, prec, nrhs):
    from paper_2605_21828_amd.bfmht import Plan
    seed, n, m, L = case
    fs = random_factor_set(seed, n, m, L, max_rank=6)
    print("case", case, prec, nrhs, "ranks", fs["rank"].tolist(), flush=True)
    p = Plan(fs, prec, max_nrhs=nrhs)
    rng = np.random.default_rng(seed)
    c, fv = rng.standard_normal((m, nrhs)), rng.standard_normal((n, nrhs))
    f = p.apply(_t(c, p.dtype), out=_nan(n, nrhs, p.dtype))
    g = p.apply_t(_t(fv, p.dtype), out=_nan(m, nrhs, p.dtype))
    fo, go = ob.apply(fs, c), ob.apply_transpose(fs, fv)
    assert fo.shape == (n, nrhs) and go.shape == (m, nrhs)
    assert np.array_equal(_np(f), fo) and np.array_equal(_np(g), go)   # all zeros or empty
    assert not np.any(fo) and not np.any(go)


@pytest.mark.parametrize("case", [CASES[1], CASES[3]])
def test_empty_transform_scaled_and_batched(gpu, case):
    import torch
    from paper_2605_21828_amd.bfmht import Batch, Plan
    seed, n, m, L = case
    fs = random_factor_set(seed, n, m, L, max_rank=6)
    other = random_factor_set(66, 50, 30, 2, max_rank=10)
    p, q = Plan(fs, "f32", max_nrhs=5), Plan(other, "f32", max_nrhs=5)
    s = torch.ones(m, dtype=torch.float32, device="cuda")
    f = p.apply_scaled(s, torch.zeros((m, 5), dtype=torch.float32, device="cuda"), out=_nan(n, 5, torch.float32))
    g = p.apply_t_scaled(s, torch.ones((n, 5), dtype=torch.float32, device="cuda"), out=_nan(m, 5, torch.float32))
    assert not np.any(_np(f)) and not np.any(_np(g))
    rng = np.random.default_rng(seed)
    cs = [rng.standard_normal((m, 5)), rng.standard_normal((30, 4))]
    fs_in = [rng.standard_normal((n, 5)), rng.standard_normal((50, 4))]
    bt = Batch([p, q])
    outs = bt.launch([_t(x, torch.float32) for x in cs], [_nan(n, 5, torch.float32), _nan(50, 4, torch.float32)])
    outs_t = bt.launch([_t(x, torch.float32) for x in fs_in], [_nan(m, 5, torch.float32), _nan(30, 4, torch.float32)],
                       transpose=True)
    assert not np.any(_np(outs[0])) and not np.any(_np(outs_t[0]))
    ref, ref_t = ob.apply(other, cs[1]), ob.apply_transpose(other, fs_in[1])
    assert np.linalg.norm(_np(outs[1]) - ref) <= 1e-5 * np.linalg.norm(ref)
    assert np.linalg.norm(_np(outs_t[1]) - ref_t) <= 1e-5 * np.linalg.norm(ref_t)


@pytest.mark.parametrize("case", [CASES[1], CASES[3]])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_empty_transform_lsqr(gpu, case, prec):
    # no points: x = 0 and nothing is left over; no modes: x is empty and the
    # residual is f itself (Phi~^T f = 0 ends the recurrence at once)
    from paper_2605_21828_amd.bfmht import Plan
    seed, n, m, L = case
    fs = random_factor_set(seed, n, m, L, max_rank=6)
    p = Plan(fs, prec, max_nrhs=3)
    fv = np.random.default_rng(seed).standard_normal((n, 3))
    x, rnorm = p.lsqr(_t(fv, p.dtype), 4, out=_nan(m, 3, p.dtype))
    assert not np.any(_np(x))
    assert np.allclose(_np(rnorm), np.linalg.norm(fv, axis=0), rtol=1e-6, atol=0)
