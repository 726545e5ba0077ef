"""Closed-form entries of the Fourier transform matrix for the factor builder (host, FP64).

On the flat periodic square the Laplacian eigenfunctions are Fourier modes with
eigenvalue k1^2 + k2^2 (Sec. 1, eq. 2D-DFT; Sec. 5).  The build uses one real
mode per point of Z^2: (k1, k2, s1, s2) with k >= 0, s = 0 for cos and 1 for
sin (sin only for k > 0), phi = s1(k1 x1) s2(k2 x2), columns sorted by
(k1^2 + k2^2, k1, k2, s1, s2).  Entries are evaluated lazily, so the builder
never holds Phi: per point it keeps cos/sin tables of k x for k up to the
largest wavenumber and forms a block as a product of two table lookups.
"""
import numpy as np


def real_modes(m):
    """First m real Fourier modes, int64 rows (k1, k2, s1, s2), vectorised."""
    K = max(1, int(np.ceil(np.sqrt(m / np.pi))) + 2)
    while True:
        k = np.arange(K + 1)
        k1, k2 = np.meshgrid(k, k, indexing="ij")
        k1, k2 = k1.ravel(), k2.ravel()
        rows = []
        for s1 in (0, 1):
            for s2 in (0, 1):
                ok = np.ones_like(k1, dtype=bool)
                if s1:
                    ok &= k1 > 0
                if s2:
                    ok &= k2 > 0
                rows.append(np.stack([k1[ok], k2[ok], np.full(ok.sum(), s1),
                                      np.full(ok.sum(), s2)], axis=1))
        allm = np.concatenate(rows)
        lam = allm[:, 0] ** 2 + allm[:, 1] ** 2
        inside = lam <= K * K
        if inside.sum() >= m:
            allm, lam = allm[inside], lam[inside]
            order = np.lexsort((allm[:, 3], allm[:, 2], allm[:, 1], allm[:, 0], lam))
            return allm[order[:m]].astype(np.int64)
        K *= 2


class FourierBlocks:
    """Phi(rows, cols) for real Fourier modes at fixed points, from trig tables."""

    def __init__(self, points, modes):
        pts = np.asarray(points, dtype=np.float64)
        self.modes = np.asarray(modes, dtype=np.int64)
        kmax = int(self.modes[:, :2].max()) if len(self.modes) else 0
        k = np.arange(kmax + 1, dtype=np.float64)
        # tab[a][j, 2*k + s] = cos(k x_a) (s = 0) or sin(k x_a) (s = 1)
        self.tab = []
        for a in range(2):
            arg = pts[:, a:a + 1] * k[None, :]
            t = np.empty((pts.shape[0], 2 * (kmax + 1)), dtype=np.float64)
            t[:, 0::2] = np.cos(arg)
            t[:, 1::2] = np.sin(arg)
            self.tab.append(t)
        self.c1 = 2 * self.modes[:, 0] + self.modes[:, 2]
        self.c2 = 2 * self.modes[:, 1] + self.modes[:, 3]

    @property
    def shape(self):
        return (self.tab[0].shape[0], self.modes.shape[0])

    def synthesis(self, c, chunk=16384):
        """Exact Phi c at every point (used to build workload data, e.g. the
        right-hand side of a least-squares fit).  Each mode's coefficient goes
        to the cell (x1 factor, x2 factor) of a coefficient grid G; then
        (Phi c)_j = sum_a tab0[j, a] (tab1 G^T)[j, a]."""
        c = np.asarray(c, dtype=np.float64)
        vec = c.ndim == 1
        if vec:
            c = c[:, None]
        A, B = self.tab[0].shape[1], self.tab[1].shape[1]
        n = self.tab[0].shape[0]
        out = np.empty((n, c.shape[1]))
        for r in range(c.shape[1]):
            G = np.zeros((A, B))
            G[self.c1, self.c2] = c[:, r]
            for s in range(0, n, chunk):
                out[s:s + chunk, r] = np.einsum("ja,ja->j", self.tab[0][s:s + chunk], self.tab[1][s:s + chunk] @ G.T)
        return out[:, 0] if vec else out

    def tree_ordered(self, perm):
        """(a, b, cols) -> Phi[perm[a:b]][:, cols], from copies of the tables with
        their rows in the order perm, so a range of positions is a row slice."""
        perm = np.asarray(perm)
        t0, t1 = self.tab[0][perm], self.tab[1][perm]
        c1, c2 = self.c1, self.c2

        def block(a, b, cols):
            cols = np.asarray(cols)
            return t0[a:b][:, c1[cols]] * t1[a:b][:, c2[cols]]
        return block

    def __call__(self, rows, cols):
        """Phi[rows][:, cols]; rows=None selects every point."""
        cols = np.asarray(cols)
        if rows is None:
            return self.tab[0][:, self.c1[cols]] * self.tab[1][:, self.c2[cols]]
        rows = np.asarray(rows)
        return (self.tab[0][np.ix_(rows, self.c1[cols])] *
                self.tab[1][np.ix_(rows, self.c2[cols])])
