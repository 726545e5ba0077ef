"""The butterfly factorization on the GPU: FP64 column IDs in HIP kernels.

Same blocks, order and factor-set schema as the host builder (build.py):
level 0 factors each frequency-leaf column block, level l the concatenated
skeleton columns of a frequency node's children restricted to a space node,
and the leaf bases come last (Sec. 2, Alg. "Butterfly factorization").  Every
block is a submatrix of Phi, the property Sec. 4's streaming variant rests on,
so no dense basis is ever carried between levels: the host keeps only the
skeleton index lists.  Per level, the blocks are formed on the GPU from tables
held there (bfmht_form_blocks), decomposed there (bfmht_column_id: pivoted
QR, rank, pivots; bfmht_id_coefficients: P = [I R11^-1 R12] Pi^T), and ranks,
pivot lists and the P blocks come back.  A level runs in chunks whose dense
blocks fit `budget_bytes` of device memory, so the memory held stays bounded
whatever n and m are; the level order and Sec. 4's post-order compute the same
blocks (each depends only on its children), and the level order gives each
launch every block of a level.

Blocks without columns keep nothing (identity of size 0) and blocks without
rows keep no column, as in the host builder; neither goes to the GPU.
"""
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

from .. import bfmht as B


class Tables:
    """Phi[perm_x[r], c] = tab0[ta[c], r] * tab1[tb[c], r] at tree position r,
    with both tables held on the GPU (rows of a table are its columns in the
    C call's terms: one row per table column, points in tree order)."""

    def __init__(self, tab0, ta, tab1, tb, device):
        tab0 = np.ascontiguousarray(tab0, dtype=np.float64)
        tab1 = np.ascontiguousarray(tab1, dtype=np.float64)
        if tab0.shape[1] != tab1.shape[1]:
            raise ValueError("tables must cover the same points")
        self.n = tab0.shape[1]
        self.w0, self.w1 = tab0.shape[0], tab1.shape[0]
        self.ta = np.ascontiguousarray(ta, dtype=np.int32)
        self.tb = np.ascontiguousarray(tb, dtype=np.int32)
        self.tab0 = torch.from_numpy(tab0).to(device)
        self.tab1 = torch.from_numpy(tab1).to(device)


def fourier_tables(points, modes, perm_x, device):
    """Tables of the real Fourier matrix (Sec. 1, eq. 2D-DFT): row 2k + s of
    table a holds cos (s = 0) or sin (s = 1) of k x_a at every point."""
    pts = np.asarray(points, dtype=np.float64)[np.asarray(perm_x)]
    modes = np.asarray(modes, dtype=np.int64)
    kmax = int(modes[:, :2].max()) if len(modes) else 0
    k = np.arange(kmax + 1, dtype=np.float64)
    tabs = []
    for a in range(2):
        arg = k[:, None] * pts[None, :, a]
        t = np.empty((2 * (kmax + 1), pts.shape[0]))
        t[0::2] = np.cos(arg)
        t[1::2] = np.sin(arg)
        tabs.append(t)
    return Tables(tabs[0], 2 * modes[:, 0] + modes[:, 2], tabs[1], 2 * modes[:, 1] + modes[:, 3], device)


def dense_tables(Phi, perm_x, device):
    """Tables of a dense Phi (eigenvectors, Sec. 7): Phi^T in tree order times a row of ones."""
    Phi = np.asarray(Phi, dtype=np.float64)
    n, m = Phi.shape
    return Tables(Phi[np.asarray(perm_x)].T, np.arange(m), np.ones((1, n)), np.zeros(m), device)


class _Runner:
    """One GPU's buffers for the chunks of a build: the dense blocks, the staged
    metadata and the outputs, grown as needed."""

    def __init__(self, tables, device, stream, events=None):
        self.t, self.dev, self.stream = tables, device, stream
        self.a = torch.empty(0, dtype=torch.float64, device=device)
        self.ws = torch.empty(0, dtype=torch.uint8, device=device)
        self.events = events   # list: (start, end) event pairs around each bfmht_column_id call

    def _grow(self, name, n, dtype):
        buf = getattr(self, name)
        if buf.numel() < n:
            buf = torch.empty(int(n), dtype=dtype, device=self.dev)
            setattr(self, name, buf)
        return buf

    def form(self, row0, rows, cols_list):
        """Form the blocks Phi(rows [row0, row0 + rows), cols) column-major; returns the layout."""
        count = len(rows)
        K = np.array([c.size for c in cols_list], dtype=np.int64)
        col_off = np.concatenate([[0], np.cumsum(K)]).astype(np.int64)
        sizes = np.asarray(rows, dtype=np.int64) * K
        a_off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64) if count else np.zeros(0, np.int64)
        a_len = int(sizes.sum())
        cols = np.concatenate(cols_list).astype(np.int64) if count else np.zeros(0, np.int64)
        a = self._grow("a", max(a_len, 1), torch.float64)
        ws_bytes = B.bfmht_factor_meta_bytes(count, int(col_off[-1]))
        ws = self._grow("ws", ws_bytes, torch.uint8)
        t = self.t
        B.bfmht_form_blocks(row0, rows, col_off, t.ta[cols], t.tb[cols], a_off, t.tab0.data_ptr(), t.n, t.w0,
                            t.tab1.data_ptr(), t.n, t.w1, a.data_ptr(), a_len, ws.data_ptr(), ws_bytes, self.stream)
        return dict(rows=np.asarray(rows, np.int64), col_off=col_off, a_off=a_off, a_len=a_len, K=K)

    def column_ids_device(self, lay, tol):
        """Column IDs of the formed blocks, P left on the device: returns
        (rank, piv, p_off, p) with rank and piv on the host, p_off[b] the offset of
        block b's P in the device tensor p (-1 when the block keeps all or none
        of its columns; p is None when no block has a P)."""
        count = len(lay["rows"])
        tc = int(lay["col_off"][-1])
        rank_d = torch.empty(max(count, 1), dtype=torch.int32, device=self.dev)
        piv_d = torch.empty(max(tc, 1), dtype=torch.int32, device=self.dev)
        ws_bytes = B.bfmht_factor_meta_bytes(count, tc)
        ws = self._grow("ws", ws_bytes, torch.uint8)
        ev = None
        if self.events is not None:
            ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            ev[0].record(torch.cuda.current_stream(self.dev))
        B.bfmht_column_id(lay["rows"], lay["col_off"], lay["a_off"], self.a.data_ptr(), lay["a_len"], tol,
                          rank_d.data_ptr(), piv_d.data_ptr(), ws.data_ptr(), ws_bytes, self.stream)
        if ev is not None:
            ev[1].record(torch.cuda.current_stream(self.dev))
            self.events.append(ev)
        rank = rank_d[:count].cpu().numpy()
        piv = piv_d[:tc].cpu().numpy()
        K = lay["K"]
        need = (rank > 0) & (rank < K)
        p_off = np.full(count, -1, dtype=np.int64)
        sz = np.where(need, rank.astype(np.int64) * K, 0)
        p_off[need] = np.concatenate([[0], np.cumsum(sz)[:-1]])[need]
        p_len = int(sz.sum())
        p_d = None
        if p_len:
            p_d = torch.empty(p_len, dtype=torch.float64, device=self.dev)
            B.bfmht_id_coefficients(lay["rows"], lay["col_off"], lay["a_off"], self.a.data_ptr(), lay["a_len"], rank,
                                    piv_d.data_ptr(), p_off, p_d.data_ptr(), p_len, ws.data_ptr(), ws_bytes,
                                    self.stream)
        return rank, piv, p_off, p_d

    def column_ids(self, lay, tol):
        """Column IDs of the formed blocks: per block (local J, P or None, ident) on the host."""
        rank, piv, p_off, p_d = self.column_ids_device(lay, tol)
        P_h = p_d.cpu().numpy() if p_d is not None else None
        out = []
        for b in range(len(rank)):
            k, Kb, c0 = int(rank[b]), int(lay["K"][b]), int(lay["col_off"][b])
            if k == Kb:
                out.append((np.arange(Kb, dtype=np.int64), None, True))
            elif k == 0:
                out.append((np.zeros(0, np.int64), np.zeros((0, Kb)), False))
            else:
                o = int(p_off[b])
                out.append((piv[c0:c0 + k].astype(np.int64), P_h[o:o + k * Kb].reshape(k, Kb).copy(), False))
        return out

    def blocks_to_host(self, lay):
        """The formed blocks, row-major (rows x K) on the host."""
        a = self.a[:max(lay["a_len"], 1)].cpu().numpy()
        out = []
        for b in range(len(lay["rows"])):
            M, Kb, o = int(lay["rows"][b]), int(lay["K"][b]), int(lay["a_off"][b])
            out.append(np.ascontiguousarray(a[o:o + M * Kb].reshape(Kb, M).T))
        return out


def _chunks(sizes, budget):
    """Consecutive index ranges whose summed sizes stay within budget (a block
    larger than the budget forms its own chunk)."""
    out, start, acc = [], 0, 0
    for i, s in enumerate(sizes):
        if i > start and acc + s > budget:
            out.append((start, i))
            start, acc = i, 0
        acc += s
    if start < len(sizes):
        out.append((start, len(sizes)))
    return out


def build_factors_device(tables, n, m, perm_x, xoff, koff, L, tol, arity=2, log=None, budget_bytes=16 << 30,
                         device=None, events=None):
    """Build the factor set dict (schema in io.py) with the column IDs on the GPU.
    tables: a Tables on `device` (default: the current CUDA device), its points
    in the tree order of perm_x.  events: optional list that receives a pair of
    timing events around every bfmht_column_id launch (the stream is the current
    torch stream of the device)."""
    device = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    stream = torch.cuda.current_stream(device).cuda_stream
    run = _Runner(tables, device, stream, events)
    a_ = int(arity)
    nb = a_ ** L
    perm_x = np.asarray(perm_x, dtype=np.int32)
    xoff = np.asarray(xoff, dtype=np.int64)
    koff = np.asarray(koff, dtype=np.int64)
    if tables.n != n:
        raise ValueError("tables cover %d points, the factor set %d" % (tables.n, n))
    rank = np.zeros((L + 1, nb), dtype=np.int32)
    ident = np.zeros((L + 1, nb), dtype=np.uint8)
    P_off = np.full((L + 1, nb), -1, dtype=np.int64)
    # P of every chunk goes to the host while later levels compute (a copy stream
    # driven by one worker thread); the parts are joined into one array at the end
    copy_stream = torch.cuda.Stream(device=device)
    copier = ThreadPoolExecutor(1)
    copies, parts, futs = [], {}, []   # (offset, part index); part index -> host array
    p_total = 0

    def _download(i, p_d, ev):
        h = np.empty(p_d.numel(), dtype=np.float64)
        with torch.cuda.stream(copy_stream):
            copy_stream.wait_event(ev)
            torch.from_numpy(h).copy_(p_d)
        parts[i] = h

    J_prev = None
    stats = []
    budget_el = max(1, int(budget_bytes) // 8)
    try:
        for lvl in range(L + 1):
            t0 = time.time()
            tasks = []   # (q, first row, rows, global columns)
            if lvl == 0:
                for j in range(nb):
                    tasks.append((j, 0, n, np.arange(koff[j], koff[j + 1], dtype=np.int64)))
            else:
                nf = a_ ** (L - lvl)
                for i in range(a_ ** lvl):
                    r0, r1 = int(xoff[i * nf]), int(xoff[(i + 1) * nf])
                    p = i // a_
                    for j in range(nf):
                        q1 = p * (a_ * nf) + a_ * j
                        cols = np.concatenate([J_prev[q1 + t] for t in range(a_)])
                        tasks.append((i * nf + j, r0, r1 - r0, cols))
            J_cur = [None] * nb
            dev_tasks = []
            for q, r0, M, cols in tasks:
                if cols.size == 0:
                    J_cur[q], rank[lvl, q], ident[lvl, q] = cols, 0, 1
                elif M == 0:
                    J_cur[q], rank[lvl, q] = cols[:0], 0
                else:
                    dev_tasks.append((q, r0, M, cols))
            sizes = [M * cols.size for _, _, M, cols in dev_tasks]
            for s0, s1 in _chunks(sizes, budget_el):
                part = dev_tasks[s0:s1]
                lay = run.form([t[1] for t in part], [t[2] for t in part], [t[3] for t in part])
                rk, piv, p_off, p_d = run.column_ids_device(lay, tol)
                for b, (q, _, _, cols) in enumerate(part):
                    k, Kb, c0 = int(rk[b]), cols.size, int(lay["col_off"][b])
                    rank[lvl, q] = k
                    if k == Kb:
                        ident[lvl, q] = 1
                        J_cur[q] = cols
                    else:
                        J_cur[q] = cols[piv[c0:c0 + k]]
                        if k > 0:
                            P_off[lvl, q] = p_total + p_off[b]
                if p_d is not None:
                    ev = torch.cuda.Event()
                    ev.record(torch.cuda.current_stream(device))
                    futs.append(copier.submit(_download, len(copies), p_d, ev))
                    copies.append((p_total, len(copies)))
                    p_total += p_d.numel()
            # blocks that keep no column have an empty P at the running offset
            for q in range(nb):
                if not ident[lvl, q] and rank[lvl, q] == 0:
                    later = P_off[lvl, q + 1:][P_off[lvl, q + 1:] >= 0]
                    P_off[lvl, q] = later[0] if later.size else p_total
            J_prev = J_cur
            st = dict(level=lvl, seconds=round(time.time() - t0, 3),
                      rank_min=int(rank[lvl].min()), rank_max=int(rank[lvl].max()),
                      rank_mean=float(rank[lvl].mean()), ident=int(ident[lvl].sum()))
            stats.append(st)
            if log:
                log(st)
    except BaseException:
        copier.shutdown(wait=True)   # no download is left running behind the error
        raise
    t0 = time.time()
    copier.shutdown(wait=True)
    for f in futs:
        f.result()   # re-raises a failed download
    P_all = np.empty(p_total, dtype=np.float64)

    def _place(item):
        off, i = item
        h = parts.pop(i)
        P_all[off:off + h.size] = h

    with ThreadPoolExecutor(16) as pool:
        list(pool.map(_place, copies))
    if log:
        log(dict(p_download_wait_seconds=round(time.time() - t0, 3), p_entries=int(P_all.size)))
    t0 = time.time()
    # leaf column bases U_i = Phi(tau_i, J_{L,i}), formed on the GPU
    U_off = np.zeros(nb, dtype=np.int64)
    U_off[1:] = np.cumsum([(xoff[i + 1] - xoff[i]) * J_prev[i].size for i in range(nb - 1)])
    U_all = np.zeros(int(U_off[-1] + (xoff[nb] - xoff[nb - 1]) * J_prev[nb - 1].size))
    leaf = [i for i in range(nb) if xoff[i + 1] > xoff[i] and J_prev[i].size]
    sizes = [int(xoff[i + 1] - xoff[i]) * J_prev[i].size for i in leaf]
    for s0, s1 in _chunks(sizes, budget_el):
        part = leaf[s0:s1]
        lay = run.form([int(xoff[i]) for i in part], [int(xoff[i + 1] - xoff[i]) for i in part],
                       [J_prev[i] for i in part])
        for i, U in zip(part, run.blocks_to_host(lay)):
            U_all[U_off[i]:U_off[i] + U.size] = U.ravel()
    if log:
        log(dict(leaf_bases_seconds=round(time.time() - t0, 3)))
    return dict(
        n=np.int64(n), m=np.int64(m), L=np.int64(L), tol=np.float64(tol), arity=np.int64(a_),
        perm_x=perm_x, xoff=xoff, koff=koff, rank=rank, ident=ident, P=P_all, P_off=P_off,
        U=U_all, U_off=U_off, skel_L=np.concatenate([J_prev[i] for i in range(nb)]).astype(np.int64),
        build_stats=np.array([[s["level"], s["seconds"], s["rank_min"], s["rank_max"],
                               s["rank_mean"], s["ident"]] for s in stats]),
    )
