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
