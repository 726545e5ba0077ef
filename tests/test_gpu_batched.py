"""Batched multi-instance apply and per-stage tile widths (GPU, through the C ABI)."""
import numpy as np
import pytest

from factor_gen import random_factor_set
from oracle import butterfly as ob
from oracle import dense as od
from oracle import modes as om
from paper_2605_21828_amd import workloads as wl
from paper_2605_21828_amd.factor import io as fio

pytestmark = pytest.mark.gpu

CASES = [  # seed, n, m, L, max_rank, nrhs
    (60, 300, 200, 4, 40, 1),
    (61, 1000, 333, 5, 90, 5),
    (62, 77, 500, 3, 130, 17),
    (63, 257, 129, 7, 20, 33),
    (64, 5, 3, 2, 4, 64),
    (65, 640, 640, 6, 70, 100),
    (66, 90, 60, 3, 30, 0),      # skipped instance
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
def instances():
    return [random_factor_set(s, n, m, L, max_rank=r) for s, n, m, L, r, _ in CASES]


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5), ("bf16x3", 1e-5)])
def test_batched_matches_oracle(gpu, instances, prec, tol):
    from paper_2605_21828_amd.bfmht import Batch, Plan
    plans = [Plan(fs, prec, max_nrhs=max(1, c[5])) for fs, c in zip(instances, CASES)]
    rng = np.random.default_rng(7)
    cs = [rng.standard_normal((int(fs["m"]), c[5])) for fs, c in zip(instances, CASES)]
    fv = [rng.standard_normal((int(fs["n"]), c[5])) for fs, c in zip(instances, CASES)]
    batch = Batch(plans)
    ys = batch.run([_t(c, _dt(prec)) for c in cs])
    gs = batch.run([_t(f, _dt(prec)) for f in fv], transpose=True)
    for fs, c, f, y, g, case in zip(instances, cs, fv, ys, gs, CASES):
        if case[5] == 0:
            continue
        assert od.rel_err_cols(_np(y), ob.apply(fs, c))[0] <= tol, case
        assert od.rel_err_cols(_np(g), ob.apply_transpose(fs, f))[0] <= tol, case


def test_batched_equals_single_applies_bitwise(gpu, instances):
    from paper_2605_21828_amd.bfmht import Batch, Plan
    plans = [Plan(fs, "f32", max_nrhs=max(1, c[5])) for fs, c in zip(instances, CASES)]
    rng = np.random.default_rng(8)
    xs = [_t(rng.standard_normal((int(fs["m"]), c[5])), _dt("f32")) for fs, c in zip(instances, CASES)]
    ys = Batch(plans).run(xs)
    for p, x, y, c in zip(plans, xs, ys, CASES):
        if c[5]:
            assert np.array_equal(_np(p.apply(x)), _np(y))


def test_grid_instances_vs_inverse_dft(gpu):
    """Uniform-grid instances of uneven size in one launch, each against its inverse DFT."""
    from paper_2605_21828_amd.bfmht import Batch, Plan
    rng = wl.rng(40, 5)
    sides = [16, 24, 32, 48, 32, 16, 64, 24]
    plans, cs, refs = [], [], []
    for i, N in enumerate(sides):
        n, m = N * N, N * N // 4
        fs, _ = fio.fourier_factors(wl.grid_points(N), m, 64, 1e-8, workers=4, cache=False)
        b = int(rng.integers(1, 129))
        c = wl.coefficients(400 + i, m, b)
        plans.append(Plan(fs, "f32", max_nrhs=b))
        cs.append(c)
        refs.append(om.grid_synthesis_ifft2(N, om.fourier_modes(m), c))
    ys = Batch(plans).run([_t(c, _dt("f32")) for c in cs])
    for y, ref in zip(ys, refs):
        assert od.rel_err_cols(_np(y), ref)[0] <= 1e-5


def test_tile_shape_does_not_change_results(gpu, instances):
    from paper_2605_21828_amd import bfmht as B
    from paper_2605_21828_amd.bfmht import Plan
    fs = instances[5]
    p = Plan(fs, "f32", max_nrhs=100)
    x = _t(np.random.default_rng(9).standard_normal((int(fs["m"]), 100)), _dt("f32"))
    f = _t(np.random.default_rng(10).standard_normal((int(fs["n"]), 100)), _dt("f32"))
    base_y, base_g = _np(p.apply(x)), _np(p.apply_t(f))
    S = B.bfmht_plan_num_stages(p.handle)
    assert S == int(fs["L"]) + (1 if p.leaf_merged else 2)
    for k in range(S):
        B.bfmht_plan_set_tile(p.handle, 0, k, (64, 128)[k % 2], (16, 32, 64)[k % 3])
        B.bfmht_plan_set_tile(p.handle, 1, k, (128, 64)[k % 2], (64, 16, 32)[k % 3])
    assert B.bfmht_plan_get_tile(p.handle, 0, 1) == (128, 32)
    assert np.array_equal(_np(p.apply(x)), base_y)
    assert np.array_equal(_np(p.apply_t(f)), base_g)
    with pytest.raises(B.BfmhtError):
        B.bfmht_plan_set_tile(p.handle, 0, 0, 64, 48)
    with pytest.raises(B.BfmhtError):
        B.bfmht_plan_set_tile(p.handle, 0, 0, 96, 16)
    with pytest.raises(B.BfmhtError):
        B.bfmht_plan_set_tile(p.handle, 0, S, 64, 16)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x2", "bf16x3"])
def test_tall_tiles_match_oracle(gpu, instances, prec):
    """128-row tiles (two 16-row blocks per wave) in every stage, all precisions."""
    from paper_2605_21828_amd import bfmht as B
    from paper_2605_21828_amd.bfmht import Plan
    tol = {"f64": 1e-12, "f32": 1e-5, "bf16x3": 1e-5, "bf16x2": 2e-4}[prec]
    for fs, case in zip(instances[:6], CASES[:6]):
        b = max(1, case[5])
        p = Plan(fs, prec, max_nrhs=b)
        for k in range(B.bfmht_plan_num_stages(p.handle)):
            B.bfmht_plan_set_tile(p.handle, 0, k, 128, 0)
            B.bfmht_plan_set_tile(p.handle, 1, k, 128, 0)
        rng = np.random.default_rng(case[0])
        c, f = rng.standard_normal((p.m, b)), rng.standard_normal((p.n, b))
        assert od.rel_err_cols(_np(p.apply(_t(c, _dt(prec)))), ob.apply(fs, c))[0] <= tol, case
        assert od.rel_err_cols(_np(p.apply_t(_t(f, _dt(prec)))), ob.apply_transpose(fs, f))[0] <= tol, case


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5), ("bf16x2", 1e-4)])
def test_batched_compact_mixed_shapes_match_oracle(gpu, prec, tol):
    """ID-form blocks (compact applies) in every instance, and a different tile
    shape per instance, so one stage position runs several per-shape launches."""
    from paper_2605_21828_amd import bfmht as B
    from paper_2605_21828_amd.bfmht import Batch, Plan
    sets = [random_factor_set(s + 100, n, m, L, max_rank=r, p_id_form=0.8) for s, n, m, L, r, _ in CASES]
    shapes = [(64, 16), (128, 32), (64, 64), (128, 16), (64, 32), (128, 64), (64, 16)]
    plans = []
    for fs, c, sh in zip(sets, CASES, shapes):
        p = Plan(fs, prec, max_nrhs=max(1, c[5]))
        for k in range(B.bfmht_plan_num_stages(p.handle)):
            B.bfmht_plan_set_tile(p.handle, 0, k, *sh)
            B.bfmht_plan_set_tile(p.handle, 1, k, *sh)
        plans.append(p)
    rng = np.random.default_rng(8)
    cs = [rng.standard_normal((int(fs["m"]), c[5])) for fs, c in zip(sets, CASES)]
    fv = [rng.standard_normal((int(fs["n"]), c[5])) for fs, c in zip(sets, CASES)]
    batch = Batch(plans)
    ys = batch.run([_t(c, _dt(prec)) for c in cs])
    gs = batch.run([_t(f, _dt(prec)) for f in fv], transpose=True)
    for fs, c, f, y, g, case in zip(sets, cs, fv, ys, gs, CASES):
        if case[5] == 0:
            continue
        assert od.rel_err_cols(_np(y), ob.apply(fs, c))[0] <= tol, case
        assert od.rel_err_cols(_np(g), ob.apply_transpose(fs, f))[0] <= tol, case


@pytest.mark.skip(reason="persistent single launch is switched off in the library: its one GPU run (this test, "
                         "FP64 case) wrote nothing for 180 s and was killed (no fault); every wait is bounded, so "
                         "the likely cause is cache thrashing by agent-scope acquire polls and per-tile L2 "
                         "write-backs, not a deadlock (the work order is replayed on the CPU in "
                         "test_persistent_order.py)")
@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_persistent_single_launch_matches_oracle(gpu, instances, prec, tol):
    """Every stage of every instance in one persistent launch (work items taken
    from per-XCD ticket queues in stage order; tests/test_persistent_order.py
    replays that order on the CPU), forward and transposed, every tile width,
    against the oracle; a second call on the same workspace repeats the first."""
    from paper_2605_21828_amd import bfmht as B
    from paper_2605_21828_amd.bfmht import Batch, Plan
    w = wl.WORKLOADS["grid64"]
    grid_fs, _ = fio.fourier_factors(wl.points_for(w), w["m"], w["leaf"], w["tol"], workers=8, cache=False)
    sets = list(instances) + [grid_fs]
    rhs = [c[5] for c in CASES] + [7]
    plans = [Plan(fs, prec, max_nrhs=max(1, b)) for fs, b in zip(sets, rhs)]
    rng = np.random.default_rng(17)
    xs = [rng.standard_normal((int(fs["m"]), b)) for fs, b in zip(sets, rhs)]
    fvs = [rng.standard_normal((int(fs["n"]), b)) for fs, b in zip(sets, rhs)]
    batch = Batch(plans)
    for width in (16, 32, 64):
        ys = batch.run([_t(x, _dt(prec)) for x in xs], persistent=True, width=width)
        gs = batch.run([_t(f, _dt(prec)) for f in fvs], transpose=True, persistent=True, width=width)
        for fs, x, f, y, g, b in zip(sets, xs, fvs, ys, gs, rhs):
            if b == 0:
                continue
            assert od.rel_err_cols(_np(y), ob.apply(fs, x))[0] <= tol, (width, b)
            assert od.rel_err_cols(_np(g), ob.apply_transpose(fs, f))[0] <= tol, (width, b)
        again = batch.run([_t(x, _dt(prec)) for x in xs], persistent=True, width=width)
        for y, y2 in zip(ys, again):
            assert np.array_equal(_np(y), _np(y2))
    with pytest.raises(B.BfmhtError) as e:
        batch.run([_t(x, _dt(prec)) for x in xs], persistent=True, width=48)
    assert e.value.status == B.EINVAL


def test_persistent_launch_is_switched_off(gpu, instances):
    from paper_2605_21828_amd import bfmht as B
    from paper_2605_21828_amd.bfmht import Batch, Plan
    fs = instances[1]
    p = Plan(fs, "f32", max_nrhs=5)
    x = _t(np.ones((int(fs["m"]), 5)), _dt("f32"))
    with pytest.raises(B.BfmhtError) as e:
        Batch([p]).run([x], persistent=True)
    assert e.value.status == B.EINVAL and "switched off" in str(e.value)


def test_autotune_sets_widths_and_keeps_results(gpu, instances, tmp_path):
    from paper_2605_21828_amd import autotune
    from paper_2605_21828_amd import bfmht as B
    from paper_2605_21828_amd.bfmht import Batch, Plan
    fs = instances[5]
    p = Plan(fs, "f32", max_nrhs=100)
    x = _t(np.random.default_rng(12).standard_normal((int(fs["m"]), 100)), _dt("f32"))
    base = _np(p.apply(x))
    cfg = autotune.tune_plan(p, fs, 100, reps=3, cache_path=str(tmp_path / "t.json"))
    S = B.bfmht_plan_num_stages(p.handle)
    assert len(cfg["fwd"]) == S and len(cfg["bwd"]) == S
    assert all(tuple(s) in autotune.SHAPES + [(64, 0)] for s in cfg["fwd"] + cfg["bwd"])
    q_cfg = None
    assert [B.bfmht_plan_get_tile(p.handle, 0, k) for k in range(S)] == [tuple(s) for s in cfg["fwd"]]
    assert np.array_equal(_np(p.apply(x)), base)
    # a second plan of the same shape picks the cached choice up
    q = Plan(fs, "f32", max_nrhs=100)
    assert autotune.tune_plan(q, fs, 100, cache_path=str(tmp_path / "t.json")) == cfg
    plans = [Plan(f, "f32", max_nrhs=max(1, c[5])) for f, c in zip(instances, CASES)]
    xs = [_t(np.random.default_rng(13).standard_normal((pl.m, max(1, c[5]))), _dt("f32")) for pl, c in zip(plans, CASES)]
    choice, ms = autotune.tune_batch(Batch(plans), xs, reps=2)
    assert len(choice) == len(plans) and ms > 0


@pytest.mark.parametrize("nrhs", [3, 16])
def test_folded_identity_levels_match_unfolded_bitwise(gpu, nrhs):
    """The single apply folds leading all-identity levels (forward: rows read
    through the composed map; transposed: one pairwise gather-sum of the row
    copies); the batched apply runs those stages transposed one by one.  The
    sums happen in the same order, so results agree bitwise."""
    import torch
    from paper_2605_21828_amd.bfmht import Batch, Plan
    w = wl.WORKLOADS["grid64"]
    fs, _ = fio.fourier_factors(wl.points_for(w), w["m"], w["leaf"], w["tol"], workers=8, cache=False)
    assert fs["ident"][0].all() and fs["ident"][1].all()
    rng = np.random.default_rng(9)
    for prec in ("f64", "f32"):
        p = Plan(fs, prec, max_nrhs=nrhs)
        f = _t(rng.standard_normal((int(fs["n"]), nrhs)), _dt(prec))
        c = _t(rng.standard_normal((int(fs["m"]), nrhs)), _dt(prec))
        g_single, y_single = _np(p.apply_t(f)), _np(p.apply(c))
        g_batch = _np(Batch([p]).run([f], transpose=True)[0])
        assert np.array_equal(g_single, g_batch), prec
        tol = 1e-12 if prec == "f64" else 1e-5
        assert od.rel_err_cols(g_single, ob.apply_transpose(fs, f.double().cpu().numpy()))[0] <= tol
        assert od.rel_err_cols(y_single, ob.apply(fs, c.double().cpu().numpy()))[0] <= tol


@pytest.fixture(scope="module")
def deep_identity():
    """Depth 16, one point per space leaf, a single mode: every level is all
    identities, so folding them would need 2^16 copies per row of c (beyond the
    gather-sum's 2^15); the transposed apply then runs those stages one by one."""
    fs = random_factor_set(80, 1 << 16, 1, 16, ident_levels=17, allow_empty=True)
    assert fs["ident"].all()
    rng = np.random.default_rng(81)
    c = rng.standard_normal((1, 16))
    f = rng.standard_normal((1 << 16, 16))
    return fs, c, f, ob.apply(fs, c), ob.apply_transpose(fs, f)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_deep_identity_levels_beyond_fold_limit(gpu, deep_identity, prec, tol):
    from paper_2605_21828_amd.bfmht import Plan
    fs, c, f, y_ref, g_ref = deep_identity
    for b in (1, 16):
        p = Plan(fs, prec, max_nrhs=b)
        assert od.rel_err_cols(_np(p.apply(_t(c[:, :b], _dt(prec)))), y_ref[:, :b])[0] <= tol
        assert od.rel_err_cols(_np(p.apply_t(_t(f[:, :b], _dt(prec)))), g_ref[:, :b])[0] <= tol


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_shared_plan_instances_are_packed_into_one_apply(gpu, instances, prec, tol):
    """Instances that share a plan are applied as one block of columns (inputs
    packed, outputs unpacked): every output matches the oracle, and a member
    with more than four columns equals its own single apply bit for bit (the
    same MFMA sums per column)."""
    from paper_2605_21828_amd.bfmht import Batch, Plan
    fs_a, fs_b = instances[1], instances[5]
    pa = Plan(fs_a, prec, max_nrhs=64)
    pb = Plan(fs_b, prec, max_nrhs=64)
    plans = [pa, pb, pa, pa, pb]
    rhs = [7, 3, 2, 40, 19]
    rng = np.random.default_rng(31)
    sets = {id(pa): fs_a, id(pb): fs_b}
    for transpose in (False, True):
        xs = [rng.standard_normal(((p.n if transpose else p.m), b)) for p, b in zip(plans, rhs)]
        outs = Batch(plans).run([_t(x, _dt(prec)) for x in xs], transpose=transpose)
        for p, x, y, b in zip(plans, xs, outs, rhs):
            fs = sets[id(p)]
            ref = ob.apply_transpose(fs, x) if transpose else ob.apply(fs, x)
            assert od.rel_err_cols(_np(y), ref)[0] <= tol, (transpose, b)
            if b > 4:
                single = p.apply_t(_t(x, _dt(prec))) if transpose else p.apply(_t(x, _dt(prec)))
                assert np.array_equal(_np(single), _np(y)), (transpose, b)
