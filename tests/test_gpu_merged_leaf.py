"""GPU parity of plans whose leaf bases are merged into the last transfer level
(the default when the last level's blocks are full rank over their leaves, as
in the builder's factor sets): the last stage applies U_i P_{L,i} in one pass.

Bars: FP64 against the oracle's butterfly apply O2 within 1e-12 relative, FP32
and the BF16 three-term split within 1e-5 (max over right-hand-side columns),
both directions, through the MFMA stage kernel and the few-RHS kernel; merged
and separate leaf stages agree to the same bars; batched applies of merged
plans equal their single applies bitwise.
"""
import numpy as np
import pytest

from factor_gen import random_factor_set
from oracle import butterfly as ob
from oracle import dense as od

pytestmark = pytest.mark.gpu

CASES = [
    # seed, n, m, L, max_rank, arity, ident_levels, p_id_form
    (200, 900, 300, 4, 60, 2, 0, 0.7),     # ragged leaves (some empty), ID-form blocks
    (201, 3000, 700, 5, 150, 2, 0, 1.0),   # jobs of several tiles, ragged tails
    (202, 600, 256, 3, 40, 2, 3, 0.5),     # levels 0-2 identities: the merged stage runs first
    (203, 500, 300, 2, 40, 4, 0, 0.7),     # 4-ary trees: two transposed job parts
    (204, 800, 200, 4, 50, 2, 1, 0.5),     # one folded level
]
TOL = {"f64": 1e-12, "f32": 1e-5, "bf16x3": 1e-5}


def _fs(case):
    seed, n, m, L, mr, a, il, pid = case
    return random_factor_set(seed, n, m, L, max_rank=mr, arity=a, ident_levels=il, p_id_form=pid,
                             full_rank_leaves=True)


def _dt(prec):
    import torch
    return torch.float64 if prec == "f64" else torch.float32


def _t(x, dtype):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _np(x):
    import torch
    torch.cuda.synchronize()
    return x.detach().double().cpu().numpy()


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_merged_plan_matches_oracle(gpu, case, prec):
    from paper_2605_21828_amd.bfmht import Plan
    fs = _fs(case)
    L = int(fs["L"])
    rng = np.random.default_rng(case[0] + 1)
    for nrhs in (1, 5, 64):   # few-RHS kernel (f32, f64), narrow and full MFMA tiles
        p = Plan(fs, prec, max_nrhs=nrhs)
        assert p.leaf_merged and not Plan(fs, prec, max_nrhs=nrhs, leaf_stage=True).leaf_merged
        c = rng.standard_normal((int(fs["m"]), nrhs))
        f = rng.standard_normal((int(fs["n"]), nrhs))
        y = _np(p.apply(_t(c, _dt(prec))))
        g = _np(p.apply_t(_t(f, _dt(prec))))
        assert od.rel_err_cols(y, ob.apply(fs, c))[0] <= TOL[prec], (case, nrhs, L)
        assert od.rel_err_cols(g, ob.apply_transpose(fs, f))[0] <= TOL[prec], (case, nrhs, L)


@pytest.mark.parametrize("case", CASES[:3])
def test_merged_and_separate_leaf_stages_agree(gpu, case):
    from paper_2605_21828_amd.bfmht import Plan
    fs = _fs(case)
    rng = np.random.default_rng(case[0] + 2)
    c = rng.standard_normal((int(fs["m"]), 17))
    f = rng.standard_normal((int(fs["n"]), 17))
    pm = Plan(fs, "f64", max_nrhs=17)
    ps = Plan(fs, "f64", max_nrhs=17, leaf_stage=True)
    assert pm.leaf_merged and not ps.leaf_merged
    ym, ys = _np(pm.apply(_t(c, _dt("f64")))), _np(ps.apply(_t(c, _dt("f64"))))
    gm, gs = _np(pm.apply_t(_t(f, _dt("f64")))), _np(ps.apply_t(_t(f, _dt("f64"))))
    assert od.rel_err_cols(ym, ys)[0] <= 1e-12
    assert od.rel_err_cols(gm, gs)[0] <= 1e-12


@pytest.mark.parametrize("case", [CASES[2], CASES[4]])
def test_merged_plan_scaled_applies(gpu, case):
    """Scaled synthesis and the covariance product: the scaled coefficients sit
    in the level buffer the first running stage does not write, also when that
    stage is the merged last level."""
    from paper_2605_21828_amd.bfmht import Plan
    fs = _fs(case)
    m, n = int(fs["m"]), int(fs["n"])
    s = np.random.default_rng(case[0] + 3).uniform(0.5, 2.0, m)
    for b in (2, 16):
        p = Plan(fs, "f64", max_nrhs=b)
        assert p.leaf_merged
        z = np.random.default_rng(case[0] + b).standard_normal((m, b))
        y = _np(p.apply_scaled(_t(s, _dt("f64")), _t(z, _dt("f64"))))
        assert od.rel_err_cols(y, ob.apply(fs, s[:, None] * z))[0] <= 1e-12
        v = np.random.default_rng(case[0] + 10 + b).standard_normal((n, b))
        cv = _np(p.covariance_matvec(_t(s, _dt("f64")), _t(v, _dt("f64"))))
        assert od.rel_err_cols(cv, ob.apply(fs, s[:, None] * ob.apply_transpose(fs, v)))[0] <= 1e-12


def test_batched_merged_plans_match_single_applies(gpu):
    from paper_2605_21828_amd.bfmht import Batch, Plan
    sets = [_fs(c) for c in CASES]
    rhs = [3, 40, 0, 9, 64]
    plans = [Plan(fs, "f32", max_nrhs=max(1, b)) for fs, b in zip(sets, rhs)]
    assert all(p.leaf_merged for p in plans)
    rng = np.random.default_rng(5)
    xs = [_t(rng.standard_normal((int(fs["m"]), b)), _dt("f32")) for fs, b in zip(sets, rhs)]
    fv = [_t(rng.standard_normal((int(fs["n"]), b)), _dt("f32")) for fs, b in zip(sets, rhs)]
    batch = Batch(plans)
    ys = batch.run(xs)
    gs = batch.run(fv, transpose=True)
    for fs, p, x, f, y, g, b in zip(sets, plans, xs, fv, ys, gs, rhs):
        if b == 0:
            continue
        assert np.array_equal(_np(p.apply(x)), _np(y)), b
        assert od.rel_err_cols(_np(y), ob.apply(fs, _np(x)))[0] <= 1e-5, b
        assert od.rel_err_cols(_np(g), ob.apply_transpose(fs, _np(f)))[0] <= 1e-5, b
