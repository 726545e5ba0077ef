"""Pins of the oracle's covariance and Karhunen-Loeve sampling (Sec. 7.2), CPU only."""
import numpy as np

from oracle import dense as od
from oracle import modes as om


def _small(seed=0, n=300, m=60):
    rng = np.random.default_rng(seed)
    pts = rng.uniform(-np.pi, np.pi, (n, 2))
    md = om.fourier_modes(m)
    s = 1.0 / (1.0 + om.eigenvalues(md)) ** 2
    return pts, md, om.phi(pts, md), s


def test_covariance_entries_follow_the_kernel_expansion():
    pts, md, Phi, s = _small()
    Sig = od.covariance(Phi, s)
    for j, k in [(0, 0), (3, 17), (120, 5), (299, 298)]:
        kjk = 0.0
        for l in range(len(s)):   # K(x_j, x_k) = sum_l S(lambda_l) phi_l(x_j) phi_l(x_k)
            k1, k2, s1, s2 = (int(v) for v in md[l])
            fj = om._trig(s1, k1 * pts[j, 0]) * om._trig(s2, k2 * pts[j, 1])
            fk = om._trig(s1, k1 * pts[k, 0]) * om._trig(s2, k2 * pts[k, 1])
            kjk += s[l] * fj * fk
        assert abs(Sig[j, k] - kjk) <= 1e-12 * max(1.0, abs(kjk))
    assert np.allclose(Sig, Sig.T)
    assert np.linalg.eigvalsh(Sig).min() > -1e-10


def test_grid_covariance_matvec_equals_fft_form():
    N, m = 16, 60
    md = om.fourier_modes(m)
    s = np.exp(-0.1 * om.eigenvalues(md))
    Phi = om.phi(om.uniform_grid(N), md)
    v = np.random.default_rng(1).standard_normal((N * N, 2))
    ref = om.grid_synthesis_ifft2(N, md, s[:, None] * om.grid_analysis_fft2(N, md, v))
    assert np.allclose(od.covariance(Phi, s) @ v, ref, rtol=1e-11, atol=1e-11)


def test_kl_samples_have_the_covariance():
    pts, md, Phi, s = _small(2, n=40, m=12)
    z = np.random.default_rng(3).standard_normal((12, 40000))
    y = od.kl_sample(Phi, s, z)
    emp = y @ y.T / z.shape[1]
    Sig = od.covariance(Phi, s)
    assert np.linalg.norm(emp - Sig) <= 0.03 * np.linalg.norm(Sig)
    # one coefficient at a time gives sqrt(S_l) phi_l
    e = np.zeros((12, 1))
    e[5] = 1.0
    assert np.allclose(od.kl_sample(Phi, s, e)[:, 0], np.sqrt(s[5]) * Phi[:, 5])
