"""Level-by-level butterfly factorization with column IDs (host, FP64).

Follows the butterfly factorization (Sec. 2, Alg. "Butterfly factorization"):
level 0 factors each frequency-leaf column block, levels 1..L re-factor the
concatenated previous-level bases restricted to the current space node, and the
leaf column bases are kept at the end.  With column IDs the previous level's
column basis restricted to tau is Phi(tau, J) for the previous skeleton J, so a
block at level l is simply Phi(tau_i, [J_{l-1,p,2j}, J_{l-1,p,2j+1}]) and only
entries of Phi are needed (the property that makes the streaming variant of
Sec. 4 possible).  Blocks of one level are independent and run in a process
pool; skeletons of the previous level are the only state passed on.

`blocks(rows, cols)` must return Phi[rows][:, cols] in float64; rows=None means
all points.  A blocks object that also has `tree_ordered(perm_x)` hands back a
callable `(a, b, cols) -> Phi[perm_x[a:b]][:, cols]`, used instead, which can
read the rows of a space node as one contiguous range.
"""
import os
import time

import numpy as np

from .interp import column_id

_CTX = {}


def _id_task(task):
    lvl, q, a, b, cols = task
    blocks, perm, tol, tree = _CTX["blocks"], _CTX["perm"], _CTX["tol"], _CTX["tree"]
    if cols.size == 0:
        return lvl, q, cols, None, True
    if tree is not None:
        A = tree(a, b, cols)
    else:
        A = blocks(None if lvl == 0 else perm[a:b], cols)
    J, P, ident = column_id(A, tol)
    return lvl, q, cols[J], P, ident


def _init_worker():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass


def _cost(task):
    """Rough flop count of a task's ID (the QR of a rows x cols block)."""
    _, _, a, b, cols = task
    k = cols.size
    return (b - a) * k * k + k ** 3


def _run(tasks, workers):
    """Yield the ID of every task (in completion order when parallel).  A
    parallel level hands the tasks out one at a time, most expensive first, so
    the level does not wait on a long task started last."""
    if workers <= 1:
        for t in tasks:
            yield _id_task(t)
        return
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    order = sorted(tasks, key=_cost, reverse=True)
    with ctx.Pool(workers, initializer=_init_worker) as pool:
        yield from pool.imap_unordered(_id_task, order, chunksize=1)


def build_factors(blocks, n, m, perm_x, xoff, koff, L, tol, workers=None, log=None, arity=2):
    """Build the factor set dict (schema documented in `io.py`).  arity: children
    per tree node (2, or 4 for a quadtree in space with a 4-ary frequency tree);
    a block at level l concatenates the skeletons of its `arity` inputs."""
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    a_ = int(arity)
    nb = a_ ** L
    perm_x = np.asarray(perm_x, dtype=np.int32)
    xoff = np.asarray(xoff, dtype=np.int64)
    koff = np.asarray(koff, dtype=np.int64)
    tree = blocks.tree_ordered(perm_x) if hasattr(blocks, "tree_ordered") else None
    _CTX.update(blocks=blocks, perm=perm_x, tol=float(tol), tree=tree)
    rank = np.zeros((L + 1, nb), dtype=np.int32)
    ident = np.zeros((L + 1, nb), dtype=np.uint8)
    P_blocks = [[None] * nb for _ in range(L + 1)]
    J_prev = None
    stats = []
    for lvl in range(L + 1):
        t0 = time.time()
        tasks = []
        if lvl == 0:
            for j in range(nb):
                tasks.append((0, j, 0, n, np.arange(koff[j], koff[j + 1], dtype=np.int64)))
        else:
            nf = a_ ** (L - lvl)
            w = a_ ** (L - lvl)   # leaves per space node at depth lvl
            for i in range(a_ ** lvl):
                a, b = int(xoff[i * w]), int(xoff[(i + 1) * w])
                p = i // a_
                for j in range(nf):
                    q1 = p * (a_ * nf) + a_ * j
                    cols = np.concatenate([J_prev[q1 + t] for t in range(a_)])
                    tasks.append((lvl, i * nf + j, a, b, cols))
        J_cur = [None] * nb
        t_note = time.time()
        for done, (_, q, J, P, idf) in enumerate(_run(tasks, workers), 1):
            J_cur[q] = J
            rank[lvl, q] = len(J)
            ident[lvl, q] = 1 if idf else 0
            P_blocks[lvl][q] = P
            if log and time.time() - t_note > 30.0:   # progress on long levels
                log(dict(level=lvl, blocks_done=done, blocks=len(tasks), seconds=round(time.time() - t0, 1)))
                t_note = time.time()
        J_prev = J_cur
        st = dict(level=lvl, seconds=round(time.time() - t0, 3),
                  rank_min=int(rank[lvl].min()), rank_max=int(rank[lvl].max()),
                  rank_mean=float(rank[lvl].mean()), ident=int(ident[lvl].sum()))
        stats.append(st)
        if log:
            log(st)
    # leaf column bases U_i = Phi(tau_i, J_{L,i})
    U_list = []
    for i in range(nb):
        rows = perm_x[xoff[i]:xoff[i + 1]]
        cols = J_prev[i]
        if rows.size and cols.size:
            U = tree(int(xoff[i]), int(xoff[i + 1]), cols) if tree is not None else blocks(rows, cols)
            U_list.append(np.ascontiguousarray(U))
        else:
            U_list.append(np.zeros((rows.size, cols.size)))
    return pack_factor_set(n, m, L, tol, a_, perm_x, xoff, koff, rank, ident, P_blocks, U_list, J_prev, stats)


def pack_factor_set(n, m, L, tol, a_, perm_x, xoff, koff, rank, ident, P_blocks, U_list, J_last, stats):
    """Pack per-block P and leaf U arrays into the factor-set dict (schema in
    io.py), releasing every block once it is copied, so the peak host memory
    stays near one copy of the factors."""
    nb = a_ ** L
    P_off = np.full((L + 1, nb), -1, dtype=np.int64)
    off = 0
    for lvl in range(L + 1):
        for q in range(nb):
            P = P_blocks[lvl][q]
            if P is not None and not ident[lvl, q]:
                P_off[lvl, q] = off
                off += P.size
    P_all = np.empty(off, dtype=np.float64)
    for lvl in range(L + 1):
        for q in range(nb):
            if P_off[lvl, q] >= 0:
                P = P_blocks[lvl][q]
                P_all[P_off[lvl, q]:P_off[lvl, q] + P.size] = np.asarray(P, dtype=np.float64).ravel()
            P_blocks[lvl][q] = None
    U_off = np.zeros(nb, dtype=np.int64)
    uo = 0
    for i in range(nb):
        U_off[i] = uo
        uo += U_list[i].size
    U_all = np.empty(uo, dtype=np.float64)
    for i in range(nb):
        U_all[U_off[i]:U_off[i] + U_list[i].size] = U_list[i].ravel()
        U_list[i] = None
    return dict(
        n=np.int64(n), m=np.int64(m), L=np.int64(L), tol=np.float64(tol), arity=np.int64(a_),
        perm_x=perm_x, xoff=xoff, koff=koff, rank=rank, ident=ident,
        P=P_all,
        P_off=P_off,
        U=U_all,
        U_off=U_off,
        skel_L=np.concatenate([J_last[i] for i in range(nb)]).astype(np.int64),
        build_stats=np.array([[s["level"], s["seconds"], s["rank_min"], s["rank_max"],
                               s["rank_mean"], s["ident"]] for s in stats]),
    )
