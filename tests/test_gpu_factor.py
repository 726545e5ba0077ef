"""The factorization on the GPU (bfmht_form_blocks, bfmht_column_id,
bfmht_id_coefficients, factor/device_build.py) against the oracle.

- Column IDs of uneven blocks (tall, wide, exact low rank, decaying spectra,
  all-zero, one column) against oracle/interp.column_id: the same rank and
  skeleton in the same pivot order, P within rounding of the triangular solve,
  and the residual bound of the ID.
- Formed blocks against the oracle's Fourier matrix entries.
- Whole factor sets (binary and 4-ary trees, Fourier and a dense eigenvector
  matrix) against oracle/factorize on the same trees: ranks, identity flags and
  skeletons equal, P and U within rounding, and the applied factor set against
  the dense transform.
- The full-size Fourier set (n = 65536, m = 16384, leaf 128, tol 1e-8): sampled
  blocks of every level re-decomposed by the oracle from the device's own
  previous-level skeletons, and the synthesis on sampled rows.
"""
import numpy as np
import pytest

from oracle import butterfly as ob
from oracle import dense as od
from oracle import factorize as ofz
from oracle import interp as oi
from oracle import modes as om

pytestmark = pytest.mark.gpu


def _device_ids(blocks, tol):
    """Column IDs of host blocks through the C ABI; per block (J, P, ident)."""
    import torch
    from paper_2605_21828_amd.factor.device_build import _Runner

    class _NoTables:
        pass

    run = _Runner(_NoTables(), torch.device("cuda:0"), torch.cuda.current_stream().cuda_stream)
    rows = np.array([b.shape[0] for b in blocks], np.int64)
    K = np.array([b.shape[1] for b in blocks], np.int64)
    col_off = np.concatenate([[0], np.cumsum(K)]).astype(np.int64)
    a_off = np.concatenate([[0], np.cumsum(rows * K)[:-1]]).astype(np.int64)
    flat = np.concatenate([np.asarray(b, np.float64).T.ravel() for b in blocks])
    run.a = torch.tensor(flat, dtype=torch.float64, device="cuda")
    lay = dict(rows=rows, col_off=col_off, a_off=a_off, a_len=int(flat.size), K=K)
    return run.column_ids(lay, tol)


def _p_bound(tol):
    """Allowed max difference of two computed interpolation matrices, relative
    to their size: 1000 rounding units amplified by the condition bound 1 / tol."""
    return 1e3 * np.finfo(np.float64).eps / max(tol, 1e-15)


def _blocks(seed):
    rng = np.random.default_rng(seed)
    out = []

    def spectrum(M, K, lo):
        r = min(M, K)
        U = np.linalg.qr(rng.standard_normal((M, r)))[0]
        V = np.linalg.qr(rng.standard_normal((K, r)))[0]
        return (U * np.geomspace(1.0, lo, r)) @ V.T

    out.append(spectrum(300, 40, 1e-14))          # tall, numerically low rank
    out.append(spectrum(50, 120, 1e-12))          # wide
    out.append(rng.standard_normal((700, 9)) @ rng.standard_normal((9, 64)))   # exact rank 9
    out.append(np.zeros((40, 7)))                 # all zero
    out.append(rng.standard_normal((33, 1)))      # one column
    out.append(rng.standard_normal((90, 30)))     # full rank
    out.append(spectrum(30000, 40, 1e-15))        # reflector longer than its copy in local memory
    out.append(spectrum(128, 300, 1e-13) * 1e-3)  # scale does not matter
    for _ in range(20):                           # ragged random
        M, K = int(rng.integers(1, 400)), int(rng.integers(1, 150))
        out.append(spectrum(M, K, 10.0 ** -rng.uniform(2, 15)))
    out.append(spectrum(900, 45, 1e-10))          # a tall reduced block whose last panel is partial ...
    out.append(spectrum(200, 3, 1e-3))            # ... and one narrower than a panel, last in the buffer
    return out


@pytest.mark.parametrize("tol", [1e-8, 1e-4, 1e-11])
def test_column_id_matches_oracle(gpu, tol):
    blocks = _blocks(int(-np.log10(tol)))
    got = _device_ids(blocks, tol)
    for t, (A, (J, P, idf)) in enumerate(zip(blocks, got)):
        Jo, Po, ido = oi.column_id(A, tol)
        assert idf == ido and np.array_equal(J, Jo), (t, A.shape, len(J), len(Jo))
        if P is not None and P.size:
            assert np.array_equal(P[:, J], np.eye(len(J)))
            # T = R11^-1 R12 carries rounding times the condition of R11, at most
            # about |R_00| / |R_k-1,k-1| < 1 / tol for a pivoted QR
            assert np.abs(P - Po).max() <= _p_bound(tol) * max(1.0, np.abs(Po).max()), t
            k, K = P.shape
            res = np.linalg.norm(A - A[:, J] @ P, 2)
            assert res <= 1.01 * np.sqrt(K - k) * tol * np.linalg.norm(A, 2) + 1e-13 * np.linalg.norm(A, 2), t


def test_form_blocks_fourier(gpu):
    import torch
    from paper_2605_21828_amd.factor.device_build import _Runner, fourier_tables
    rng = np.random.default_rng(5)
    n, m = 3000, 500
    pts = rng.uniform(-np.pi, np.pi, (n, 2))
    modes = om.fourier_modes(m)
    perm = rng.permutation(n)
    tabs = fourier_tables(pts, modes, perm, torch.device("cuda:0"))
    run = _Runner(tabs, torch.device("cuda:0"), torch.cuda.current_stream().cuda_stream)
    specs = [(0, n, np.arange(m)), (17, 400, rng.choice(m, 90, replace=False)), (2999, 1, np.array([3, 0, 499])),
             (1000, 1500, rng.choice(m, 7, replace=False))]
    lay = run.form([s[0] for s in specs], [s[1] for s in specs], [s[2] for s in specs])
    got = run.blocks_to_host(lay)
    for (r0, M, cols), G in zip(specs, got):
        ref = om.phi(pts[perm[r0:r0 + M]], modes[cols])
        assert G.shape == ref.shape
        assert np.abs(G - ref).max() <= 1e-14


def _fourier_problem(n, m, leaf, arity, seed=0):
    from paper_2605_21828_amd.factor import trees
    rng = np.random.default_rng(seed)
    pts = rng.uniform(-np.pi, np.pi, (n, 2))
    L = trees.depth_for(n, leaf, arity)
    perm, xoff = trees.box_bisection_tree(pts, L) if arity == 2 else trees.quadtree(pts, L)
    koff = trees.frequency_tree(m, L, arity)
    return pts, om.fourier_modes(m), perm, xoff, koff, L


def _compare_sets(fd, fo, tol):
    assert np.array_equal(fd["rank"], fo["rank"])
    assert np.array_equal(fd["ident"], fo["ident"])
    assert np.array_equal(fd["skel_L"], fo["skel_L"])
    assert np.array_equal(fd["P_off"], fo["P_off"])
    assert fd["P"].size == fo["P"].size and fd["U"].size == fo["U"].size
    if fd["P"].size:
        assert np.abs(fd["P"] - fo["P"]).max() <= _p_bound(tol) * max(1.0, np.abs(fo["P"]).max())
    assert np.abs(fd["U"] - fo["U"]).max() <= 1e-15   # the same Phi entries


@pytest.mark.parametrize("n,m,leaf,arity,tol", [(4096, 1024, 64, 2, 1e-8), (2048, 512, 32, 2, 1e-4),
                                                  (4096, 1024, 64, 4, 1e-8), (1000, 300, 40, 2, 1e-10)])
def test_device_build_matches_oracle_factorization(gpu, n, m, leaf, arity, tol):
    import torch
    from paper_2605_21828_amd.factor.device_build import build_factors_device, fourier_tables
    pts, modes, perm, xoff, koff, L = _fourier_problem(n, m, leaf, arity)
    tabs = fourier_tables(pts, modes, perm, torch.device("cuda:0"))
    fd = build_factors_device(tabs, n, m, perm, xoff, koff, L, tol, arity=arity, budget_bytes=8 << 20)
    Phi = om.phi(pts, modes)
    fo = ofz.butterfly_factorization(Phi, perm, xoff, koff, L, tol, arity=arity)
    _compare_sets(fd, fo, tol)
    c = np.random.default_rng(1).standard_normal((m, 2))
    err = od.rel_err_cols(ob.apply(fd, c), Phi @ c)[0]
    assert err <= 50 * (L + 1) * tol


def test_device_build_dense_eigenvectors(gpu):
    """A dense Phi (eigenvectors of the perturbed sphere) through the ones-row tables."""
    import torch
    from paper_2605_21828_amd import sphere
    from paper_2605_21828_amd.factor import trees
    from paper_2605_21828_amd.factor.device_build import build_factors_device, dense_tables
    from paper_2605_21828_amd.factor.mesh_tree import mesh_fiedler_tree
    v, f, K, M, lam, Phi = sphere.sphere_problem(3, 0, 200)
    n, m = Phi.shape
    L = trees.depth_for(n, 40)
    perm, xoff = mesh_fiedler_tree(K, M, L)
    koff = trees.frequency_tree(m, L)
    fd = build_factors_device(dense_tables(Phi, perm, torch.device("cuda:0")), n, m, perm, xoff, koff, L, 1e-8)
    fo = ofz.butterfly_factorization(Phi, perm, xoff, koff, L, 1e-8)
    _compare_sets(fd, fo, 1e-8)


def test_device_build_empty_nodes(gpu):
    """Empty space leaves and empty frequency leaves: blocks without rows or columns stay on the host."""
    import torch
    from paper_2605_21828_amd.factor.device_build import build_factors_device, fourier_tables
    rng = np.random.default_rng(3)
    n, m, L = 60, 24, 3
    pts = rng.uniform(-np.pi, np.pi, (n, 2))
    modes = om.fourier_modes(m)
    perm = rng.permutation(n).astype(np.int32)
    xoff = np.array([0, 0, 10, 10, 30, 31, 60, 60, 60], np.int64)
    koff = np.array([0, 5, 5, 5, 12, 20, 20, 24, 24], np.int64)
    tabs = fourier_tables(pts, modes, perm, torch.device("cuda:0"))
    fd = build_factors_device(tabs, n, m, perm, xoff, koff, L, 1e-9)
    fo = ofz.butterfly_factorization(om.phi(pts, modes), perm, xoff, koff, L, 1e-9)
    _compare_sets(fd, fo, 1e-9)


@pytest.mark.slow
def test_device_build_full_size_sampled():
    """n = 65536, m = 16384 (leaf 128, tol 1e-8, i.i.d. points): every level's
    sampled blocks re-decomposed by the oracle from the device's skeletons."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2605_21828_amd import workloads as wl
    from paper_2605_21828_amd.factor import trees
    from paper_2605_21828_amd.factor.device_build import build_factors_device, fourier_tables
    w = wl.WORKLOADS["iid65536"]
    pts = wl.points_for(w)
    n, m, leaf, tol = pts.shape[0], w["m"], w["leaf"], w["tol"]
    L = trees.depth_for(n, leaf)
    perm, xoff = trees.box_bisection_tree(pts, L)
    koff = trees.frequency_tree(m, L)
    modes = om.fourier_modes(m)
    import time
    t0 = time.time()
    fd = build_factors_device(fourier_tables(pts, modes, perm, torch.device("cuda:0")), n, m, perm, xoff, koff, L,
                              tol, log=lambda d: print(d, flush=True))
    print(dict(device_build_seconds=round(time.time() - t0, 2)), flush=True)
    rng = np.random.default_rng(0)
    nb = 2 ** L
    # skeletons of every level, rebuilt from the stored P blocks: J = cols[pivot columns],
    # i.e. the columns whose P column is a unit vector in row order
    skel = [None] * nb
    for lvl in range(L + 1):
        nf = 2 ** (L - lvl)
        new = [None] * nb
        sample = set(rng.choice(nb, 3, replace=False).tolist())
        for q in range(nb):
            i, j = divmod(q, nf)
            cols = np.arange(koff[j], koff[j + 1]) if lvl == 0 else \
                np.concatenate([skel[(i // 2) * 2 * nf + 2 * j], skel[(i // 2) * 2 * nf + 2 * j + 1]])
            r = int(fd["rank"][lvl, q])
            if fd["ident"][lvl, q]:
                new[q] = cols
                Jl = np.arange(cols.size)
                P = None
            else:
                o = int(fd["P_off"][lvl, q])
                P = fd["P"][o:o + r * cols.size].reshape(r, cols.size)
                unit = (P == 1.0) & (np.abs(P).sum(axis=0) == 1.0)[None, :]   # unit columns e_t
                Jl = np.array([int(np.flatnonzero(unit[t])[0]) for t in range(r)], np.int64)
                new[q] = cols[Jl]
            if q in sample and cols.size:
                rows = perm[xoff[i * nf]:xoff[(i + 1) * nf]]
                A = om.phi(pts[rows], modes[cols])
                Jo, Po, ido = oi.column_id(A, tol)
                assert bool(fd["ident"][lvl, q]) == ido and np.array_equal(Jl, Jo), (lvl, q)
                if P is not None and P.size:
                    assert np.abs(P - Po).max() <= _p_bound(tol) * max(1.0, np.abs(Po).max()), (lvl, q)
        skel = new
    from paper_2605_21828_amd.bfmht import Plan
    p = Plan(fd, "f64", max_nrhs=2)
    c = wl.coefficients(w["wid"], m, 2)   # standard normal
    f = p.apply(torch.tensor(c, dtype=torch.float64, device="cuda")).cpu().numpy()
    rows = wl.sample_indices(w["wid"], n, 256)
    ref = od.fourier_synthesis_rows(pts, modes, rows, c)
    assert od.rel_err_cols(f[rows], ref)[0] <= 1e-6
