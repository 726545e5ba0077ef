"""Real Fourier modes on the flat periodic square [-pi, pi]^2 (oracle, test infrastructure).

On the periodic square the Laplace-Beltrami eigenfunctions are the complex
exponentials exp(i k.x) with eigenvalue |k|^2 (Sec. 1, eq. 2D-DFT; Sec. 5,
opening of the rank analysis).  The transform matrix of the paper has entries
Phi[j, k] = phi_k(x_j) with the columns ordered by eigenvalue (Sec. 1, eq.
MHT-sum; Sec. 6.1 orders the modes by k1^2 + k2^2).

Reading used here (the paper works with complex modes; the real basis, its
tie-break and its normalisation are not fixed by the paper):
  * one real mode per point of Z^2: a mode is (k1, k2, s1, s2) with k1, k2 >= 0,
    s in {0 = cos, 1 = sin}, and sin only allowed for k > 0;
  * phi(x) = s1(k1 x1) * s2(k2 x2), amplitude one (Phi[j, k] = phi_k(x_j) as is);
  * order by (k1^2 + k2^2, k1, k2, s1, s2), cos before sin.

Everything is brute force and float64.
"""
import numpy as np


def fourier_modes(m):
    """The first m real modes, as an int64 array of rows (k1, k2, s1, s2).

    Brute force: list every mode in a box [0, K]^2 large enough that the m
    smallest eigenvalues all fall inside the disk of radius K, then sort by the
    key (lambda, k1, k2, s1, s2).
    """
    if m < 0:
        raise ValueError("m must be non-negative")
    K = 1
    while True:
        # all modes with k1^2 + k2^2 <= K^2 lie inside the box [0, K]^2
        rows = []
        for k1 in range(K + 1):
            for k2 in range(K + 1):
                for s1 in (0, 1):
                    if s1 == 1 and k1 == 0:
                        continue
                    for s2 in (0, 1):
                        if s2 == 1 and k2 == 0:
                            continue
                        rows.append((k1 * k1 + k2 * k2, k1, k2, s1, s2))
        inside = [r for r in rows if r[0] <= K * K]
        if len(inside) >= m:
            inside.sort()
            sel = inside[:m]
            return np.array([r[1:] for r in sel], dtype=np.int64).reshape(m, 4)
        K *= 2


def eigenvalues(modes):
    """lambda_k = k1^2 + k2^2 for each mode row."""
    modes = np.asarray(modes)
    return (modes[:, 0] ** 2 + modes[:, 1] ** 2).astype(np.float64)


def _trig(s, arg):
    return np.sin(arg) if s == 1 else np.cos(arg)


def phi(points, modes):
    """Dense Phi[j, k] = phi_k(x_j), evaluated entry by entry from the closed form.

    points: (n, 2) float64; modes: (m, 4) int64.  Column by column, so it is
    slow but obviously the definition.
    """
    points = np.asarray(points, dtype=np.float64)
    modes = np.asarray(modes)
    n, m = points.shape[0], modes.shape[0]
    out = np.empty((n, m), dtype=np.float64)
    x1, x2 = points[:, 0], points[:, 1]
    for k in range(m):
        k1, k2, s1, s2 = (int(v) for v in modes[k])
        out[:, k] = _trig(s1, k1 * x1) * _trig(s2, k2 * x2)
    return out


def uniform_grid(N):
    """Points x = -pi + 2 pi j / N on an N x N grid, point id = N*j1 + j2."""
    t = -np.pi + 2.0 * np.pi * np.arange(N) / N
    g1, g2 = np.meshgrid(t, t, indexing="ij")
    return np.stack([g1.ravel(), g2.ravel()], axis=1)


def grid_synthesis_ifft2(N, modes, c):
    """f = Phi c on the uniform N x N grid, computed with numpy's inverse FFT.

    Each real mode is expanded into complex exponentials:
      cos(a) = (e^{ia} + e^{-ia}) / 2,  sin(a) = (e^{ia} - e^{-ia}) / (2i).
    On the grid x = -pi + 2 pi j / N one has e^{i kappa x} = (-1)^kappa
    e^{2 pi i kappa j / N}, so f[j1, j2] = N^2 * ifft2(H)[j1, j2] with
    H[kappa mod N] accumulating G_kappa (-1)^(kappa1 + kappa2).  Exact for any
    kappa because the exponential is N-periodic in kappa.
    c: (m,) or (m, b).  Returns (N*N,) or (N*N, b) in point-id order.
    """
    c = np.asarray(c, dtype=np.float64)
    squeeze = c.ndim == 1
    if squeeze:
        c = c[:, None]
    b = c.shape[1]
    H = np.zeros((N, N, b), dtype=np.complex128)
    for k in range(modes.shape[0]):
        k1, k2, s1, s2 = (int(v) for v in modes[k])
        # coefficient pairs for one factor: list of (frequency, complex weight)
        f1 = [(k1, 0.5), (-k1, 0.5)] if s1 == 0 else [(k1, -0.5j), (-k1, 0.5j)]
        f2 = [(k2, 0.5), (-k2, 0.5)] if s2 == 0 else [(k2, -0.5j), (-k2, 0.5j)]
        for a, wa in f1:
            for bb, wb in f2:
                sign = -1.0 if (a + bb) % 2 else 1.0
                H[a % N, bb % N, :] += wa * wb * sign * c[k, :]
    f = np.fft.ifft2(H, axes=(0, 1)) * (N * N)
    f = f.real.reshape(N * N, b)
    return f[:, 0] if squeeze else f


def grid_analysis_fft2(N, modes, f):
    """g = Phi^T f on the uniform N x N grid, computed with numpy's forward FFT.

    g_k = sum_j phi_k(x_j) f_j = Re/Im parts of F[kappa] = sum_j f_j e^{i kappa x_j},
    and sum_j f_j e^{i kappa x_j} = (-1)^(kappa1+kappa2) * conj(fft2(f))[kappa mod N]
    for real f.  Each real mode is the matching real combination.
    """
    f = np.asarray(f, dtype=np.float64)
    squeeze = f.ndim == 1
    if squeeze:
        f = f[:, None]
    b = f.shape[1]
    F = np.conj(np.fft.fft2(f.reshape(N, N, b), axes=(0, 1)))  # sum_j f_j e^{+2 pi i kappa j / N}

    def E(a, bb):
        sign = -1.0 if (a + bb) % 2 else 1.0
        return sign * F[a % N, bb % N, :]

    m = modes.shape[0]
    g = np.empty((m, b), dtype=np.float64)
    for k in range(m):
        k1, k2, s1, s2 = (int(v) for v in modes[k])
        # phi = s1(k1 x1) s2(k2 x2) written through e^{+-i k x}; sum_j f_j phi(x_j)
        f1 = [(k1, 0.5), (-k1, 0.5)] if s1 == 0 else [(k1, -0.5j), (-k1, 0.5j)]
        f2 = [(k2, 0.5), (-k2, 0.5)] if s2 == 0 else [(k2, -0.5j), (-k2, 0.5j)]
        acc = np.zeros(b, dtype=np.complex128)
        for a, wa in f1:
            for bb, wb in f2:
                acc += wa * wb * E(a, bb)
        g[k] = acc.real
    return g[:, 0] if squeeze else g


def grid_gram_weights(modes):
    """Closed-form diagonal of Phi^T Phi / n on a uniform grid (modes with |k_i| < N/2).

    w = 1 for k = (0, 0); 1/2 if exactly one of k1, k2 is zero; 1/4 otherwise.
    """
    modes = np.asarray(modes)
    z = (modes[:, 0] == 0).astype(int) + (modes[:, 1] == 0).astype(int)
    return np.where(z == 2, 1.0, np.where(z == 1, 0.5, 0.25))


def lattice_count_in_disk(R2):
    """Number of points of Z^2 with k1^2 + k2^2 <= R2 (brute force)."""
    K = int(np.floor(np.sqrt(R2))) + 1
    k = np.arange(-K, K + 1)
    a, b = np.meshgrid(k, k, indexing="ij")
    return int(np.count_nonzero(a * a + b * b <= R2))
