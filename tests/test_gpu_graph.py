"""HIP graph capture of the applies (GPU, through the C ABI).

The applies enqueue only kernels on the caller's stream (no allocation, copy,
memset or synchronization), so a torch CUDA graph can capture them.  Each graph
is replayed several times with eager work and synchronizations in between, and
every replay must reproduce the eager result bitwise (same kernels, same
inputs) and the oracle within the precision's bar.
"""
import numpy as np
import pytest

from factor_gen import random_factor_set
from oracle import butterfly as ob
from oracle import dense as od

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
@pytest.mark.parametrize("nrhs", [1, 16])
def test_graph_replays_match_eager(gpu, prec, tol, nrhs):
    import torch
    from paper_2605_21828_amd.bfmht import Plan
    fs = random_factor_set(70, 500, 300, 5, max_rank=60, p_id_form=0.5)
    dt = torch.float64 if prec == "f64" else torch.float32
    rng = np.random.default_rng(71)
    c, f = rng.standard_normal((300, nrhs)), rng.standard_normal((500, nrhs))
    p = Plan(fs, prec, max_nrhs=nrhs)
    x = torch.tensor(c, dtype=dt, device="cuda")
    fv = torch.tensor(f, dtype=dt, device="cuda")
    y = torch.empty((500, nrhs), dtype=dt, device="cuda")
    g = torch.empty((300, nrhs), dtype=dt, device="cuda")
    p.apply(x, out=y)
    p.apply_t(fv, out=g)
    torch.cuda.synchronize()
    y0, g0 = y.clone(), g.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):   # warm-up on a side stream before capture
        p.apply(x, out=y)
        p.apply_t(fv, out=g)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        p.apply(x, out=y)
        p.apply_t(fv, out=g)
    for rep in range(3):
        y.zero_()
        g.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, y0) and torch.equal(g, g0), rep
    yn, gn = y.double().cpu().numpy(), g.double().cpu().numpy()
    assert od.rel_err_cols(yn, ob.apply(fs, c))[0] <= tol
    assert od.rel_err_cols(gn, ob.apply_transpose(fs, f))[0] <= tol
