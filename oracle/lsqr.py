"""LSQR for min ||A x - b||_2 (oracle, test infrastructure).

The inverse transform of Sec. 7.1 (eq. inverse-MHT) is solved with LSQR, which
the paper cites (Paige and Saunders, 1982) without restating.  This is the
published recurrence written out plainly, one right-hand side at a time:
Golub-Kahan bidiagonalization of A started from b, then a plane rotation per
step that updates the iterate along the search direction w.  The matrix enters
only through the two callables matvec(v) = A v and rmatvec(u) = A^T u.
"""
import numpy as np


def lsqr(matvec, rmatvec, b, iters):
    """Returns (x_iters, ||r|| estimates after every step) for a 1-D b."""
    b = np.asarray(b, dtype=np.float64)
    beta = np.linalg.norm(b)
    u = b / beta if beta > 0 else np.zeros_like(b)
    v = np.asarray(rmatvec(u), dtype=np.float64)
    alpha = np.linalg.norm(v)
    v = v / alpha if alpha > 0 else np.zeros_like(v)
    w = v.copy()
    x = np.zeros_like(v)
    phibar, rhobar = beta, alpha
    res = []
    for _ in range(iters):
        # bidiagonalization: beta u = A v - alpha u, alpha v = A^T u - beta v
        u = np.asarray(matvec(v), dtype=np.float64) - alpha * u
        beta = np.linalg.norm(u)
        u = u / beta if beta > 0 else np.zeros_like(u)
        v = np.asarray(rmatvec(u), dtype=np.float64) - beta * v
        alpha = np.linalg.norm(v)
        v = v / alpha if alpha > 0 else np.zeros_like(v)
        # plane rotation eliminating the subdiagonal beta
        rho = np.hypot(rhobar, beta)
        if rho > 0:
            c, s = rhobar / rho, beta / rho
            theta = s * alpha
            rhobar = -c * alpha
            phi = c * phibar
            phibar = s * phibar
            x = x + (phi / rho) * w
            w = v - (theta / rho) * w
        # else: rhobar = beta = 0, so A^T r = 0 and u = v = 0: the recurrence has
        # ended, x is a least-squares solution and its residual norm stays phibar
        res.append(abs(phibar))
    return x, np.array(res)
