"""Factor-set files and the Fourier factor-set recipe.

A factor set is a dict of NumPy arrays (the schema the C ABI documents for
bfmht_factors_host):
  n, m, L, tol, arity (children per tree node, 2 or 4; k below)
  perm_x [n] int32, xoff [k^L+1] int64, koff [k^L+1] int64
  rank [L+1, k^L] int32, ident [L+1, k^L] uint8
  P float64, P_off [L+1, 2^L] int64 (-1 for identity blocks)
  U float64, U_off [2^L] int64
  skel_L (the final skeleton columns, for reference) and build_stats.
Files are .npz written with allow_pickle off; the cache key is a hash of the
recipe parameters, so a cached file is reused only for the same inputs.
"""
import hashlib
import json
import os
import time

import numpy as np

from .build import build_factors
from .fourier import FourierBlocks, real_modes
from .trees import box_bisection_tree, depth_for, frequency_tree, quadtree

CACHE_DIR = os.environ.get("BFMHT_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "bfmht"))


def save(path, fs):
    tmp = path + ".tmp.npz"
    np.savez(tmp, **fs)
    os.replace(tmp, path)


def load(path):
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def stored_entries(fs):
    """Stored factor entries F (identity blocks store nothing)."""
    return int(fs["P"].size + fs["U"].size)


def fourier_factors(points, m, leaf, tol, workers=None, log=None, cache=True, tag="", arity=2, device=None):
    """Build (or load from the cache) the factor set of the Fourier transform at `points`.

    Returns (fs, modes).  Trees: Neumann-box bisection on the points and index
    halving on the sorted modes, both of depth L = ceil(log2(n / leaf)); with
    arity 4 a quadtree on the points and a 4-ary index tree on the modes, of
    depth ceil(log4(n / leaf)).  device: a torch CUDA device to compute the
    column IDs there (device_build.py), else the host builder.
    """
    points = np.ascontiguousarray(points, dtype=np.float64)
    n = points.shape[0]
    modes = real_modes(m)
    ver = "fourier-v1" if arity == 2 else "fourier-v1-arity%d" % arity
    if device is not None:
        ver += "-dev"
    key = hashlib.sha1(points.tobytes() + json.dumps([m, leaf, float(tol), ver]).encode()).hexdigest()[:16]
    path = os.path.join(CACHE_DIR, "fourier_%s_%d_%d_%s.npz" % (tag or "x", n, m, key))
    if cache and os.path.exists(path):
        return load(path), modes
    L = depth_for(n, leaf, arity)
    perm, xoff = box_bisection_tree(points, L) if arity == 2 else quadtree(points, L)
    koff = frequency_tree(m, L, arity)
    t0 = time.time()
    if device is not None:
        from .device_build import build_factors_device, fourier_tables
        fs = build_factors_device(fourier_tables(points, modes, perm, device), n, m, perm, xoff, koff, L, tol,
                                  arity=arity, log=log, device=device)
    else:
        fs = build_factors(FourierBlocks(points, modes), n, m, perm, xoff, koff, L, tol, workers=workers, log=log,
                           arity=arity)
    if log:
        log(dict(build_seconds=round(time.time() - t0, 2), stored=stored_entries(fs)))
    if cache:
        os.makedirs(CACHE_DIR, exist_ok=True)
        save(path, fs)
    return fs, modes


def sphere_factors(level, wid, m, leaf, tol, workers=None, log=None, cache=True, device=None):
    """Build (or load from the cache) the perturbed-sphere problem and its factor set.

    Returns (fs, problem) with problem = dict(v, f, M, lam, Phi).  Space tree:
    Neumann Fiedler tree on the mesh; frequency tree: index halving on the
    eigenvalue-sorted columns; both of depth L = ceil(log2(n / leaf)).  device:
    a torch CUDA device to compute the column IDs there, else the host builder.
    """
    from .. import sphere
    from .mesh_tree import mesh_fiedler_tree
    tag = "sphere_l%d_w%d_m%d_leaf%d_tol%g_v1" % (level, wid, m, leaf, tol) + ("_dev" if device is not None else "")
    path = os.path.join(CACHE_DIR, tag + ".npz")
    ppath = os.path.join(CACHE_DIR, tag + "_problem.npz")
    if cache and os.path.exists(path) and os.path.exists(ppath):
        return load(path), load(ppath)
    t0 = time.time()
    v, f = sphere.perturbed_sphere(level, wid)
    K, M = sphere.cotangent_fem(v, f)
    lam, Phi = sphere.eigenpairs(K, M, m, workers=workers, log=log)
    if log:
        log(dict(eigenpairs_seconds=round(time.time() - t0, 1)))
    n = len(v)
    L = depth_for(n, leaf)
    perm, xoff = mesh_fiedler_tree(K, M, L)
    koff = frequency_tree(m, L)
    Phi = np.ascontiguousarray(Phi)

    def blocks(rows, cols):
        return Phi[:, cols] if rows is None else Phi[np.ix_(rows, cols)]

    if device is not None:
        from .device_build import build_factors_device, dense_tables
        fs = build_factors_device(dense_tables(Phi, perm, device), n, m, perm, xoff, koff, L, tol, log=log,
                                  device=device)
    else:
        fs = build_factors(blocks, n, m, perm, xoff, koff, L, tol, workers=workers, log=log)
    problem = dict(v=v, f=f, M=M, lam=lam, Phi=Phi)
    if cache:
        os.makedirs(CACHE_DIR, exist_ok=True)
        save(path, fs)
        save(ppath, problem)
    return fs, problem
