"""O1: the dense manifold harmonic transform and its adjoint (oracle, test infrastructure).

Synthesis is f = Phi c with Phi[j, k] = phi_k(x_j) (Sec. 1, eq. MHT-sum); the
analysis map sends point values back to coefficients through the adjoint, which
for a real Phi is Phi^T (Sec. 1, the remark on the adjoint transform that maps
function values to expansion coefficients).  A library matmul is the only step.

Functions take either an explicit Phi or (points, modes) for the closed-form
Fourier case, in which case rows/columns are evaluated on demand so that a
sampled subset of a large transform can be checked without forming Phi.
"""
import numpy as np

from . import modes as _modes


def synthesis(Phi, c):
    """f = Phi c (float64)."""
    return np.asarray(Phi, dtype=np.float64) @ np.asarray(c, dtype=np.float64)


def analysis(Phi, f):
    """g = Phi^T f (float64)."""
    return np.asarray(Phi, dtype=np.float64).T @ np.asarray(f, dtype=np.float64)


def fourier_synthesis_rows(points, modes, rows, c):
    """(Phi c)[rows] for the Fourier transform, evaluating only the rows needed."""
    P = _modes.phi(np.asarray(points)[np.asarray(rows)], modes)
    return P @ np.asarray(c, dtype=np.float64)


def fourier_synthesis_all(points, modes, c, chunk=16384):
    """Phi c at every point, for transforms too large to form.

    The sum over modes of c_k s1(k1 x1) s2(k2 x2) is regrouped by distributivity:
    for each point, sum over the (k1, s1) factors of s1(k1 x1) times the inner
    sum over the modes sharing that factor, which is one matmul of the x2 factor
    table with the coefficients laid out on the (k1, s1) x (k2, s2) grid (each
    mode owns one grid cell).  Nothing else is reordered.
    """
    points = np.asarray(points, dtype=np.float64)
    modes = np.asarray(modes)
    c = np.asarray(c, dtype=np.float64)
    vec = c.ndim == 1
    if vec:
        c = c[:, None]
    a = 2 * modes[:, 0] + modes[:, 2]          # index of the x1 factor
    b = 2 * modes[:, 1] + modes[:, 3]          # index of the x2 factor
    A, B = int(a.max()) + 1, int(b.max()) + 1
    out = np.zeros((points.shape[0], c.shape[1]), dtype=np.float64)
    for s in range(0, points.shape[0], chunk):
        x1, x2 = points[s:s + chunk, 0], points[s:s + chunk, 1]
        t1 = np.empty((len(x1), A))
        t2 = np.empty((len(x2), B))
        for i in range(A):
            t1[:, i] = _modes._trig(i % 2, (i // 2) * x1)
        for i in range(B):
            t2[:, i] = _modes._trig(i % 2, (i // 2) * x2)
        for r in range(c.shape[1]):
            C = np.zeros((A, B))
            C[a, b] = c[:, r]
            out[s:s + chunk, r] = np.sum(t1 * (t2 @ C.T), axis=1)
    return out[:, 0] if vec else out


def fourier_analysis_cols(points, modes, cols, f, chunk=8192):
    """(Phi^T f)[cols] for the Fourier transform, streaming over point chunks."""
    points = np.asarray(points)
    f = np.asarray(f, dtype=np.float64)
    sel = np.asarray(modes)[np.asarray(cols)]
    out = np.zeros((len(cols),) + f.shape[1:], dtype=np.float64)
    for s in range(0, points.shape[0], chunk):
        P = _modes.phi(points[s:s + chunk], sel)
        out += P.T @ f[s:s + chunk]
    return out


def rel_err_cols(x, ref):
    """Relative 2-norm error per right-hand-side column; returns (max over columns, frobenius)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if x.ndim == 1:
        x, ref = x[:, None], ref[:, None]
    num = np.linalg.norm(x - ref, axis=0)
    den = np.linalg.norm(ref, axis=0)
    den = np.where(den == 0, 1.0, den)
    fro = np.linalg.norm(x - ref) / max(np.linalg.norm(ref), 1e-300)
    return float(np.max(num / den)), float(fro)


def covariance(Phi, s):
    """The truncated kernel matrix Sigma = Phi diag(s) Phi^T (Sec. 7.2, eq.
    kernel-representation truncated after the columns of Phi)."""
    Phi = np.asarray(Phi, dtype=np.float64)
    return Phi @ np.diag(np.asarray(s, dtype=np.float64)) @ Phi.T


def kl_sample(Phi, s, z):
    """y = Phi diag(sqrt(s)) z: the truncated Karhunen-Loeve expansion (Sec. 7.2,
    eq. KL-expansion) for standard normal coefficients z."""
    return np.asarray(Phi, dtype=np.float64) @ (np.sqrt(np.asarray(s, dtype=np.float64))[:, None] *
                                                np.asarray(z, dtype=np.float64).reshape(len(s), -1))
