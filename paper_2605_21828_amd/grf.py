"""Gaussian random fields through the butterfly transform (Sec. 7.2).

A covariance on the manifold is built from a positive spectral density S of
the Laplace-Beltrami eigenvalues (eq. kernel-representation); truncated after
m terms its matrix is Phi S Phi^T, and samples come from the truncated
Karhunen-Loeve expansion y = Phi S^(1/2) z with z ~ N(0, I) (eq. KL-expansion).
Both are one scaled apply each on the GPU (`Plan.apply_scaled`,
`Plan.covariance_matvec`); this module holds the host-side spectral density.
"""
import numpy as np


def matern_density(lam, nu, kappa, sigma2=1.0, dim=2):
    """Matern-type spectral density sigma2 * (2 nu / kappa^2 + lambda)^-(nu + dim/2),
    unnormalised (the paper leaves the parametric family open)."""
    lam = np.asarray(lam, dtype=np.float64)
    return sigma2 * (2.0 * nu / kappa ** 2 + lam) ** (-(nu + dim / 2.0))


def sample(plan, s_sqrt, count, generator=None):
    """`count` field samples at the plan's points: Phi~ diag(s_sqrt) z, z ~ N(0, I)."""
    torch = plan.torch
    z = torch.randn((plan.m, count), dtype=plan.dtype, device=plan.device, generator=generator)
    return plan.apply_scaled(s_sqrt, z)
