"""The apply that allocates nothing (bfmht_apply_noalloc: level buffers in the
library's fixed device array), through the C ABI, against bfmht_apply with a
caller workspace and against the oracle."""
import numpy as np
import pytest

from factor_gen import random_factor_set
from oracle import butterfly as ob
from oracle import dense as od
from paper_2605_21828_amd import workloads as wl
from paper_2605_21828_amd.factor import io as fio

pytestmark = pytest.mark.gpu


def _np(x):
    import torch
    torch.cuda.synchronize()
    return x.double().cpu().numpy()


@pytest.fixture(scope="module")
def cases():
    pts = wl.iid_points(21, 8192)
    big, _ = fio.fourier_factors(pts, 2048, 64, 1e-8, workers=8, cache=False)
    small = random_factor_set(22, 700, 300, 5, max_rank=40, p_id_form=0.5)
    return big, small


def _noalloc(p, c, stream):
    import torch
    from paper_2605_21828_amd import bfmht as B
    f = torch.empty((p.n, c.shape[1]), dtype=p.dtype, device=p.device)
    B.bfmht_apply_noalloc(p.handle, c.data_ptr(), c.stride(0), f.data_ptr(), f.stride(0), c.shape[1], stream)
    return f


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_noalloc_matches_workspace_apply_twice(gpu, cases, prec, tol):
    """Two calls in a row, the second on a smaller input, on the default stream
    and on a stream of its own; each equals bfmht_apply bitwise and the oracle
    within the precision's bar."""
    import torch
    from paper_2605_21828_amd.bfmht import Plan
    big, small = cases
    dt = torch.float64 if prec == "f64" else torch.float32
    rng = np.random.default_rng(23)
    side = torch.cuda.Stream()
    for stream_obj in (None, side):
        stream = 0 if stream_obj is None else stream_obj.cuda_stream
        for fs, b in ((big, 24), (small, 5)):     # the second call is smaller in rows and columns
            p = Plan(fs, prec, max_nrhs=b)
            c_np = rng.standard_normal((int(fs["m"]), b))
            c = torch.tensor(c_np, dtype=dt, device="cuda")
            if stream_obj is None:
                y = _noalloc(p, c, stream)
            else:
                side.wait_stream(torch.cuda.current_stream())
                with torch.cuda.stream(side):
                    y = _noalloc(p, c, stream)
                torch.cuda.current_stream().wait_stream(side)
            ref = p.apply(c)
            y_np, ref_np = _np(y), _np(ref)
            assert np.array_equal(y_np, ref_np), (prec, b)
            assert od.rel_err_cols(y_np, ob.apply(fs, c_np))[0] <= tol, (prec, b)


def test_noalloc_rejects_more_columns_than_the_array_holds(gpu, cases):
    import torch
    from paper_2605_21828_amd import bfmht as B
    from paper_2605_21828_amd.bfmht import Plan
    big, _ = cases
    p = Plan(big, "f32", max_nrhs=1)
    b = 1
    while B.bfmht_workspace_bytes(p.handle, b) <= B.NOALLOC_WORKSPACE_BYTES:
        b *= 2
    c = torch.zeros((p.m, b), dtype=torch.float32, device="cuda")
    f = torch.zeros((p.n, b), dtype=torch.float32, device="cuda")
    with pytest.raises(B.BfmhtError) as e:
        B.bfmht_apply_noalloc(p.handle, c.data_ptr(), b, f.data_ptr(), b, b, 0)
    assert e.value.status == B.ENOSPACE
    assert "fixed device array" in str(e.value)
