"""Factor-set files and the Fourier factor-set recipe.

A factor set is a dict of NumPy arrays (the schema the C ABI documents for
bfmht_factors_host):
  n, m, L, tol
  perm_x [n] int32, xoff [2^L+1] int64, koff [2^L+1] int64
  rank [L+1, 2^L] int32, ident [L+1, 2^L] uint8
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
from .trees import box_bisection_tree, depth_for, frequency_tree

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


def fourier_factors(points, m, leaf, tol, workers=None, log=None, cache=True, tag=""):
    """Build (or load from the cache) the factor set of the Fourier transform at `points`.

    Returns (fs, modes).  Trees: Neumann-box bisection on the points and index
    halving on the sorted modes, both of depth L = ceil(log2(n / leaf)).
    """
    points = np.ascontiguousarray(points, dtype=np.float64)
    n = points.shape[0]
    modes = real_modes(m)
    key = hashlib.sha1(points.tobytes() + json.dumps([m, leaf, float(tol), "fourier-v1"]).encode()).hexdigest()[:16]
    path = os.path.join(CACHE_DIR, "fourier_%s_%d_%d_%s.npz" % (tag or "x", n, m, key))
    if cache and os.path.exists(path):
        return load(path), modes
    L = depth_for(n, leaf)
    perm, xoff = box_bisection_tree(points, L)
    koff = frequency_tree(m, L)
    t0 = time.time()
    fs = build_factors(FourierBlocks(points, modes), n, m, perm, xoff, koff, L, tol, workers=workers, log=log)
    if log:
        log(dict(build_seconds=round(time.time() - t0, 2), stored=stored_entries(fs)))
    if cache:
        os.makedirs(CACHE_DIR, exist_ok=True)
        save(path, fs)
    return fs, modes
