"""Perturbed-sphere workload: mesh, linear finite elements and the eigenvector matrix Phi.

This module draws the problem, not the transform: a seeded surface, its
cotangent stiffness matrix K and lumped mass matrix M, and the first m
generalized eigenpairs K phi = lambda M phi (the discrete Laplace-Beltrami
eigenproblem of Sec. 1, eq. eigenproblem; columns sorted by eigenvalue).
Phi[j, k] = phi_k(x_j) is then the matrix the factorization compresses.

Surface: icosphere (icosahedron refined `level` times, new vertices pushed to
the unit sphere), radius scaled to r = 1 + 0.1 g, with g a combination of real
spherical harmonics of degree <= 4 with N(0, 1) coefficients, scaled so that
max |g| over the vertices is 1.

Eigenpairs: shift-invert Lanczos on overlapping spectrum slices solved in
parallel (see `eigenpairs`), then one M-orthonormalisation (Cholesky in the M
inner product).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .workloads import rng


def icosphere(level):
    """(vertices (V, 3) on the unit sphere, faces (F, 3) int64), V = 10 * 4^level + 2."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0], [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11], [1, 5, 9], [5, 11, 4], [11, 10, 2],
                  [10, 7, 6], [7, 1, 8], [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9], [4, 9, 5], [2, 4, 11],
                  [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    verts = [v]
    nv = len(v)
    for _ in range(level):
        edges = np.sort(np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]]), axis=1)
        uniq, inv = np.unique(edges, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        allv = np.concatenate(verts)
        mid = allv[uniq[:, 0]] + allv[uniq[:, 1]]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        verts.append(mid)
        nf = len(f)
        a, b, c = inv[:nf] + nv, inv[nf:2 * nf] + nv, inv[2 * nf:] + nv
        f = np.concatenate([np.stack([f[:, 0], a, c], 1), np.stack([f[:, 1], b, a], 1),
                            np.stack([f[:, 2], c, b], 1), np.stack([a, b, c], 1)])
        nv += len(uniq)
    return np.concatenate(verts), f


def real_sph_harm(lmax, xyz):
    """(V, (lmax+1)^2) real spherical harmonics at unit vectors, ordered (l, m), m = -l..l."""
    from scipy.special import sph_harm_y
    theta = np.arccos(np.clip(xyz[:, 2], -1.0, 1.0))   # polar angle
    phi = np.arctan2(xyz[:, 1], xyz[:, 0])              # azimuth
    cols = []
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            y = sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                cols.append(np.sqrt(2.0) * (-1) ** m * y.real)
            elif m < 0:
                cols.append(np.sqrt(2.0) * (-1) ** m * y.imag)
            else:
                cols.append(y.real)
    return np.stack(cols, axis=1)


def perturbed_sphere(level, wid, amplitude=0.1, lmax=4):
    """Icosphere scaled radially by 1 + amplitude * g (g: seeded real SH of degree <= lmax)."""
    v, f = icosphere(level)
    if amplitude == 0.0:
        return v, f
    Y = real_sph_harm(lmax, v)
    a = rng(wid, 0).standard_normal(Y.shape[1])
    g = Y @ a
    g /= np.max(np.abs(g))
    return v * (1.0 + amplitude * g)[:, None], f


def cotangent_fem(v, f):
    """Cotangent stiffness K (CSR, symmetric PSD) and lumped mass diagonal M (1/3 of incident areas)."""
    n = len(v)
    p0, p1, p2 = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    cr = np.cross(p1 - p0, p2 - p0)
    area2 = np.linalg.norm(cr, axis=1)          # twice the triangle area
    rows, cols, vals = [], [], []
    # the angle at vertex k is opposite edge (i, j); its cotangent weights that edge
    for (i, j, k) in ((1, 2, 0), (2, 0, 1), (0, 1, 2)):
        u = v[f[:, i]] - v[f[:, k]]
        w = v[f[:, j]] - v[f[:, k]]
        cot = np.einsum("ij,ij->i", u, w) / area2
        rows += [f[:, i], f[:, j]]
        cols += [f[:, j], f[:, i]]
        vals += [-0.5 * cot, -0.5 * cot]
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n)).tocsr()
    K = K - sp.diags(np.asarray(K.sum(axis=1)).ravel())
    M = np.zeros(n)
    np.add.at(M, f.ravel(), np.repeat(area2 / 6.0, 3))
    return K.tocsr(), M


_EIG = {}


def _solve_slice(sigma):
    K, Mmat, k, tol = _EIG["K"], _EIG["M"], _EIG["k"], _EIG["tol"]
    w, V = spla.eigsh(K, k=k, M=Mmat, sigma=sigma, which="LM", tol=tol)
    order = np.argsort(w)
    return sigma, w[order], V[:, order]


def _init_worker():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass


def _solve_all(sigmas, workers):
    if workers <= 1 or len(sigmas) == 1:
        return [_solve_slice(s) for s in sigmas]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(min(workers, len(sigmas)), initializer=_init_worker) as pool:
        return pool.map(_solve_slice, sigmas)


def eigenpairs(K, M, m, slice_size=160, tol=1e-12, workers=None, log=None):
    """First m generalized eigenpairs (lambda ascending, Phi^T M Phi = I) by spectrum slicing.

    A shift-invert solve returns the k eigenvalues nearest its shift sigma: all
    eigenvalues within a distance d of sigma, an interval of the spectrum.  The
    shifts are spread by Weyl's law, N(lambda) ~ area lambda / (4 pi), so that
    neighbouring intervals overlap, and solved in parallel.  Consecutive
    intervals are cut at the widest gap between eigenvalues inside their
    overlap (a cluster is never split); where two intervals do not overlap, a
    shift is added in the gap and solved.  The first shift lies below the
    spectrum, so its interval starts at the smallest eigenvalue.
    """
    import os
    n = K.shape[0]
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    k = min(slice_size, n - 2)
    _EIG.update(K=K, M=sp.diags(M).tocsr(), k=k, tol=tol)
    area = M.sum()
    step = 0.6 * k * 4.0 * np.pi / area          # spacing of shifts: about 0.6 k eigenvalues apart
    lam_need = 4.0 * np.pi * (1.1 * m + k) / area
    sigmas = [-1e-3] + list(np.arange(0.5 * step + 0.3 * step, lam_need + step, step))
    slices = sorted(_solve_all(sigmas, workers), key=lambda t: t[0])
    for _ in range(20):
        gaps = [0.5 * (slices[i][1][-1] + slices[i + 1][1][0]) for i in range(len(slices) - 1)
                if slices[i][1][-1] < slices[i + 1][1][0]]
        low = sum(int(np.sum(s[1] < slices[-1][1][-1])) for s in slices)
        extra = list(gaps)
        if low < m + k:   # not enough yet: extend upward
            extra.append(slices[-1][0] + step)
        if not extra:
            break
        slices = sorted(slices + _solve_all(extra, workers), key=lambda t: t[0])
        if log:
            log(dict(extra_shifts=len(extra)))
    # cut points: the widest gap inside each overlap
    cuts = []
    for i in range(len(slices) - 1):
        a, b = slices[i][1], slices[i + 1][1]
        lo, hi = b[0], a[-1]
        inside = np.unique(np.concatenate([a[(a >= lo) & (a <= hi)], b[(b >= lo) & (b <= hi)]]))
        if len(inside) < 2:
            raise RuntimeError("spectrum slices do not overlap enough near %g" % lo)
        j = int(np.argmax(np.diff(inside)))
        cuts.append(0.5 * (inside[j] + inside[j + 1]))
    ws, Vs = [], []
    for i, (sigma, w, V) in enumerate(slices):
        lo = -np.inf if i == 0 else cuts[i - 1]
        hi = np.inf if i == len(slices) - 1 else cuts[i]
        if hi <= lo:
            continue
        sel = (w >= lo) & (w < hi)
        if i == len(slices) - 1:
            sel &= w < w[-1]   # the last interval's far end may be incomplete
        ws.append(w[sel])
        Vs.append(V[:, sel])
    w = np.concatenate(ws)
    V = np.concatenate(Vs, axis=1)
    if log:
        log(dict(slices=len(slices), eigenpairs=len(w)))
    if len(w) < m:
        raise RuntimeError("found only %d of %d eigenpairs" % (len(w), m))
    order = np.argsort(w, kind="stable")[:m]
    w, V = w[order], V[:, order]
    # one M-orthonormalisation: V <- V R^{-1} with R^T R = V^T M V
    G = V.T @ (M[:, None] * V)
    R = sla.cholesky(G, lower=False)
    V = sla.solve_triangular(R, V.T, trans="T", lower=False).T
    return w, V


def sphere_problem(level, wid, m, amplitude=0.1, log=None):
    """(vertices, faces, K, M, lambda[m], Phi[n, m]) of the perturbed-sphere workload."""
    v, f = perturbed_sphere(level, wid, amplitude)
    K, M = cotangent_fem(v, f)
    lam, Phi = eigenpairs(K, M, m, log=log)
    return v, f, K, M, lam, Phi
