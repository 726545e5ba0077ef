"""Seeded synthetic inputs: point sets, coefficient blocks and the named workloads.

This module holds no arithmetic of the transform; it only draws inputs.  Seeds
are numpy Generators keyed by (workload id, stream): stream 0 = geometry,
1 = coefficients, 2 = noise, 3 = row/column sampling, 4 = finite-difference
coordinates, 5 = anything else.

The paper's own meshes and datasets are not available; these workloads stand
in for them with the sizes and structure of its experiments on the flat
periodic square (Sec. 6.1: uniform and nonuniform points on [-pi, pi]^2, modes
ordered by eigenvalue).
"""
import numpy as np

WORKLOADS = {
    # Plain FP64 synthesis on a uniform 64 x 64 grid, 1024 modes, one RHS.
    "grid64": dict(wid=1, kind="grid", N=64, n=4096, m=1024, leaf=64, tol=1e-10, nrhs=1,
                   precision="f64", coef="normal"),
    # Nonuniform square: 65536 iid points, 16384 modes, 64 RHS with decaying spectrum.
    "iid65536": dict(wid=2, kind="iid", n=65536, m=16384, leaf=128, tol=1e-8, nrhs=64,
                     precision="f32", coef="decay"),
    # Differentiable least-squares fit: 262144 iid points, 65536 modes, one RHS.
    "iid262144": dict(wid=5, kind="iid", n=262144, m=65536, leaf=128, tol=1e-8, nrhs=1,
                      precision="f32", coef="decay"),
    # The same fit at half the linear size (131072 points, 32768 modes).
    "iid131072": dict(wid=5, kind="iid", n=131072, m=32768, leaf=128, tol=1e-8, nrhs=1,
                      precision="f32", coef="decay"),
}


# Perturbed sphere: icosphere level 6 (40962 vertices), r = 1 + 0.1 g, first 4096
# generalized eigenvectors of the cotangent Laplacian, Fiedler tree, leaf 64.
SPHERE = dict(wid=3, level=6, n=40962, m=4096, leaf=64, tol=1e-8, nrhs=256)

# Many uneven instances in one call: 32 uniform-grid problems on the periodic
# square, side drawn from SIDES, m = n / 4 modes, leaf 64, tol 1e-8, 1..128 RHS.
BATCHED = dict(wid=4, count=32, sides=(32, 48, 64, 96, 128, 192, 256), leaf=64, tol=1e-8, max_nrhs=128)


def batched_instances(spec=BATCHED):
    """[(side, nrhs)] of the multi-instance workload, drawn from its seed."""
    r = rng(spec["wid"], 0)
    sides = r.choice(np.array(spec["sides"]), size=spec["count"])
    nrhs = rng(spec["wid"], 1).integers(1, spec["max_nrhs"] + 1, size=spec["count"])
    return [(int(a), int(b)) for a, b in zip(sides, nrhs)]


def rng(wid, stream):
    return np.random.default_rng([int(wid), int(stream)])


def grid_points(N):
    """x = -pi + 2 pi j / N on an N x N grid; point id = N * j1 + j2."""
    t = -np.pi + 2.0 * np.pi * np.arange(N) / N
    a, b = np.meshgrid(t, t, indexing="ij")
    return np.stack([a.ravel(), b.ravel()], axis=1)


def iid_points(wid, n):
    """n points i.i.d. uniform on [-pi, pi)^2."""
    return rng(wid, 0).uniform(-np.pi, np.pi, size=(n, 2))


def points_for(w):
    return grid_points(w["N"]) if w["kind"] == "grid" else iid_points(w["wid"], w["n"])


def coefficients(wid, m, nrhs, lam=None, kind="normal", stream=1):
    """m x nrhs coefficient block; kind "decay" scales row k by 1 / (1 + lam_k)."""
    c = rng(wid, stream).standard_normal((m, nrhs))
    if kind == "decay":
        if lam is None:
            raise ValueError("decaying coefficients need the eigenvalues")
        c /= (1.0 + np.asarray(lam, dtype=np.float64))[:, None]
    return c


def values(wid, n, nrhs, stream=2):
    """n x nrhs standard normal point values (inputs of the analysis direction)."""
    return rng(wid, stream).standard_normal((n, nrhs))


def sample_indices(wid, total, count, stream=3):
    """`count` distinct sorted indices in [0, total)."""
    count = min(count, total)
    return np.sort(rng(wid, stream).choice(total, size=count, replace=False))
