"""C ABI checks that need no GPU: the library loads, exports every declared
symbol, and rejects bad factor sets and calls with the documented status."""
import ctypes
import os
import re

import numpy as np
import pytest

from factor_gen import random_factor_set
from paper_2605_21828_amd import bfmht as B

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "bfmht.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bfmht_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    syms = declared_symbols()
    assert "bfmht_apply" in syms and "bfmht_apply_transpose" in syms
    lib = ctypes.CDLL(B.LIB_PATH)
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) <= set(B.EXPORTED)


def _dynamic_c_symbols(path):
    """Names of the functions an ELF shared library exports with C linkage
    (defined, global, not C++-mangled), read from its .dynsym table."""
    import struct
    data = open(path, "rb").read()
    assert data[:4] == b"\x7fELF" and data[4] == 2 and data[5] == 1   # 64-bit little-endian
    shoff, = struct.unpack_from("<Q", data, 0x28)
    shentsize, shnum = struct.unpack_from("<HH", data, 0x3A)
    secs = [struct.unpack_from("<IIQQQQIIQQ", data, shoff + i * shentsize) for i in range(shnum)]
    out = set()
    for name, typ, flags, addr, off, size, link, info, align, entsize in secs:
        if typ != 11:   # SHT_DYNSYM
            continue
        stroff = secs[link][4]
        for k in range(size // entsize):
            st_name, st_info, st_other, st_shndx, st_value, st_size = struct.unpack_from(
                "<IBBHQQ", data, off + k * entsize)
            bind, kind = st_info >> 4, st_info & 15
            if st_shndx == 0 or bind != 1 or kind != 2:   # undefined, not global, not a function
                continue
            end = data.index(b"\0", stroff + st_name)
            sym = data[stroff + st_name:end].decode()
            if not sym.startswith("_Z"):
                out.add(sym)
    return out


def test_library_exports_only_declared_c_symbols():
    assert _dynamic_c_symbols(B.LIB_PATH) == set(declared_symbols())


def test_struct_layout_matches_header_order():
    names = [f[0] for f in B.bfmht_factors_host._fields_]
    text = open(HEADER).read()
    body = text[text.index("typedef struct {"):text.index("} bfmht_factors_host;")]
    hdr = re.findall(r"\*?\s*(\w+)(?:,\s*(\w+))?;", body)
    flat = []
    for a, b in hdr:
        flat.append(a)
        if b:
            flat.append(b)
    assert flat == names


@pytest.fixture(scope="module")
def good():
    return random_factor_set(3, 60, 40, 3, max_rank=8)


def test_plan_create_sizes(good):
    for prec in (B.F64, B.F32, B.BF16X2, B.BF16X3):
        h = B.bfmht_plan_create(good, prec, 4)
        assert B.bfmht_plan_device_bytes(h) > 0
        w1, w8 = B.bfmht_workspace_bytes(h, 1), B.bfmht_workspace_bytes(h, 8)
        assert 0 < w1 <= w8
        assert B.bfmht_workspace_bytes(h, -1) == -1
        B.bfmht_plan_destroy(h)


def _expect(fs, status, prec=B.F32, max_nrhs=1):
    with pytest.raises(B.BfmhtError) as e:
        B.bfmht_plan_create(fs, prec, max_nrhs)
    assert e.value.status == status


def test_rejects_bad_permutation(good):
    bad = dict(good, perm_x=good["perm_x"].copy())
    bad["perm_x"][0] = bad["perm_x"][1]
    _expect(bad, B.EINVAL)


def test_rejects_bad_offsets(good):
    bad = dict(good, xoff=good["xoff"].copy())
    bad["xoff"][-1] += 1
    _expect(bad, B.EINVAL)
    bad = dict(good, koff=good["koff"][::-1].copy())
    _expect(bad, B.EINVAL)


def test_rejects_rank_above_inputs(good):
    bad = dict(good, rank=good["rank"].copy())
    bad["rank"][0, 0] = good["koff"][1] - good["koff"][0] + 1
    _expect(bad, B.EINVAL)


def test_rejects_out_of_bounds_block(good):
    bad = dict(good, P_off=good["P_off"].copy())
    q = np.argwhere((good["ident"] == 0) & (good["rank"] > 0))[0]
    bad["P_off"][q[0], q[1]] = good["P"].size
    _expect(bad, B.EINVAL)
    bad = dict(good, U=good["U"][:-1].copy())
    if good["U"].size:
        _expect(bad, B.EINVAL)


def test_rejects_bad_arguments(good):
    _expect(good, B.EINVAL, prec=7)
    _expect(good, B.EINVAL, max_nrhs=0)
    h = ctypes.c_void_p()
    assert B.lib.bfmht_plan_create(None, 0, 1, ctypes.byref(h)) == B.EINVAL
    assert h.value is None
    # every failed create leaves *plan NULL, whatever it held before
    st, keep = B.factors_struct(good)
    for prec, flags in ((B.F32, 1 << 5), (7, 0)):
        h = ctypes.c_void_p(0x1234)
        assert B.lib.bfmht_plan_create_ex(ctypes.byref(st), prec, 1, flags, ctypes.byref(h)) == B.EINVAL
        assert h.value is None
    bad = dict(good, perm_x=good["perm_x"].copy())
    bad["perm_x"][0] = bad["perm_x"][1]
    st, keep = B.factors_struct(bad)
    h = ctypes.c_void_p(0x1234)
    assert B.lib.bfmht_plan_create(ctypes.byref(st), B.F32, 1, ctypes.byref(h)) == B.EINVAL
    assert h.value is None


def test_apply_before_upload_is_state_error(good):
    h = B.bfmht_plan_create(good, B.F32, 1)
    try:
        st = B.lib.bfmht_apply(h, 1 << 20, 1, 1 << 21, 1, 1, 1 << 22, 1 << 20, None)
        assert st == B.ESTATE
        st = B.lib.bfmht_apply_transpose(h, 1 << 20, 1, 1 << 21, 1, 1, 1 << 22, 1 << 20, None)
        assert st == B.ESTATE
        assert b"not uploaded" in B.lib.bfmht_last_error()
    finally:
        B.bfmht_plan_destroy(h)


def test_destroy_null_is_noop():
    B.lib.bfmht_plan_destroy(None)
    assert B.lib.bfmht_version().startswith(b"bfmht")


def _inputs(fs, lvl, q):
    """Input rows of block (lvl, q): its frequency leaf's modes at level 0, else the
    ranks of its arity consecutive input blocks of level lvl-1."""
    a = int(fs.get("arity", 2)) or 2
    L = int(fs["L"])
    if lvl == 0:
        return int(fs["koff"][q + 1] - fs["koff"][q])
    nf = a ** (L - lvl)
    i, j = divmod(q, nf)
    q1 = (i // a) * a * nf + a * j
    return int(fs["rank"][lvl - 1, q1:q1 + a].sum())


def _is_id_form(P, r, k):
    unit = [np.flatnonzero((P[:, j] == 1.0) & (np.count_nonzero(P[:, j]) == 1)) for j in range(k)]
    return 0 < r < k and len({int(u[0]) for u in unit if u.size}) == r


def _id_saving(fs):
    """Entries the compact form drops: r^2 per ID-form block (read from the
    blocks directly)."""
    L = int(fs["L"])
    nb = (int(fs.get("arity", 2)) or 2) ** L
    save = 0
    for lvl in range(L + 1):
        for q in range(nb):
            if fs["ident"][lvl, q] or fs["P_off"][lvl, q] < 0:
                continue
            r, k = int(fs["rank"][lvl, q]), _inputs(fs, lvl, q)
            if not 0 < r < k:
                continue
            P = fs["P"][fs["P_off"][lvl, q]:fs["P_off"][lvl, q] + r * k].reshape(r, k)
            if _is_id_form(P, r, k):
                save += r * r
    return save


def _leaf_merge(fs):
    """(whether a default plan merges the leaf bases into the last level, the
    entries U_i and the stored P_{L,i} take apart, the entries of the merged
    blocks U_i P_{L,i}), counted from the factor set."""
    L = int(fs["L"])
    nb = (int(fs.get("arity", 2)) or 2) ** L
    if L < 1 or all(fs["ident"][: L + 1].reshape(-1)):
        return False, 0, 0
    sep = mrg = 0
    for q in range(nb):
        r, n_i, k = int(fs["rank"][L, q]), int(fs["xoff"][q + 1] - fs["xoff"][q]), _inputs(fs, L, q)
        pe = 0
        if not fs["ident"][L, q] and r * k > 0:
            P = fs["P"][fs["P_off"][L, q]:fs["P_off"][L, q] + r * k].reshape(r, k)
            pe = r * (k - r) if _is_id_form(P, r, k) else r * k
        sep += n_i * r + pe
        mrg += n_i * k
    return 32 * mrg <= 33 * sep, sep, mrg


@pytest.mark.parametrize("p_id_form", [0.0, 0.5, 1.0])
@pytest.mark.parametrize("full_rank_leaves", [False, True])
@pytest.mark.parametrize("arity", [2, 4])
def test_stored_entries_compact_and_full(p_id_form, full_rank_leaves, arity):
    """Compact blocks drop their identity part in both directions; a default
    plan merges the leaf bases into the last level exactly when the merged
    blocks are at most 1/32 larger, and then stores n_i K_i for each leaf
    instead of U_i and P_{L,i}."""
    fs = random_factor_set(7, 400, 300, 4 if arity == 2 else 2, max_rank=40, p_id_form=p_id_form,
                           full_rank_leaves=full_rank_leaves, arity=arity)
    full = int(fs["P"].size + fs["U"].size)
    merge, sep, mrg = _leaf_merge(fs)
    assert merge or not full_rank_leaves   # full-rank leaf blocks always pay for the merge
    hs = B.bfmht_plan_create_ex(fs, B.F32, 4, B.PLAN_LEAF_STAGE)
    try:
        assert B.bfmht_plan_num_stages(hs) == int(fs["L"]) + 2
        assert B.bfmht_plan_stored_entries(hs, False) == full - _id_saving(fs)
        assert B.bfmht_plan_stored_entries(hs, True) == full - _id_saving(fs)
    finally:
        B.bfmht_plan_destroy(hs)
    hm = B.bfmht_plan_create_ex(fs, B.F32, 4, 0)
    try:
        assert B.bfmht_plan_num_stages(hm) == int(fs["L"]) + (1 if merge else 2)
        expect = full - _id_saving(fs) - (sep - mrg if merge else 0)
        assert B.bfmht_plan_stored_entries(hm, False) == expect
        assert B.bfmht_plan_stored_entries(hm, True) == expect
    finally:
        B.bfmht_plan_destroy(hm)
    h = B.bfmht_plan_create_ex(fs, B.F32, 4, B.PLAN_LEAF_STAGE)
    hf = B.bfmht_plan_create_ex(fs, B.F32, 4, B.PLAN_FULL_BLOCKS)
    try:
        assert B.bfmht_plan_stored_entries(hf, True) == full
        assert B.bfmht_plan_stored_entries(hf, False) == full
        save = _id_saving(fs)
        assert (save > 0) == (p_id_form > 0)
        # both directions drop the identity part of every ID-form block
        assert B.bfmht_plan_stored_entries(h, False) == full - save
        assert B.bfmht_plan_stored_entries(h, True) == full - save
    finally:
        B.bfmht_plan_destroy(h)
        B.bfmht_plan_destroy(hf)


def test_id_block_with_a_perturbed_skeleton_stays_full():
    fs = random_factor_set(8, 200, 150, 3, max_rank=30, p_id_form=1.0)
    base = _id_saving(fs)
    assert base > 0
    P = fs["P"].copy()
    P[np.flatnonzero(P == 1.0)[0]] = 1.0 + 2.0 ** -40   # one skeleton entry no longer exactly 1
    bad = dict(fs, P=P)
    h = B.bfmht_plan_create_ex(bad, B.F64, 1, B.PLAN_LEAF_STAGE)
    try:
        assert B.bfmht_plan_stored_entries(h, False) == int(P.size + fs["U"].size) - _id_saving(bad)
        assert B.bfmht_plan_stored_entries(h, True) == int(P.size + fs["U"].size) - _id_saving(bad)
        assert _id_saving(bad) < base
    finally:
        B.bfmht_plan_destroy(h)


def test_plan_create_ex_rejects_unknown_flags(good):
    with pytest.raises(B.BfmhtError) as e:
        B.bfmht_plan_create_ex(good, B.F32, 1, 4)
    assert e.value.status == B.EINVAL
    assert B.bfmht_plan_stored_entries(None, 0) == -1


def test_fourier_factor_set_is_applied_in_compact_form():
    """Factor sets from the builder keep exact unit skeleton columns, so every
    non-identity transfer and level-0 block is compact in both directions."""
    from paper_2605_21828_amd import workloads as wl
    from paper_2605_21828_amd.factor import io as fio
    w = wl.WORKLOADS["grid64"]
    fs, _ = fio.fourier_factors(wl.points_for(w), w["m"], w["leaf"], w["tol"], workers=1, cache=False)
    full = int(fs["P"].size + fs["U"].size)
    save = _id_saving(fs)
    h = B.bfmht_plan_create_ex(fs, B.F64, 1, B.PLAN_LEAF_STAGE)
    try:
        assert save > 0
        assert B.bfmht_plan_stored_entries(h, False) == B.bfmht_plan_stored_entries(h, True) == full - save
    finally:
        B.bfmht_plan_destroy(h)
    # its last level has full-rank leaf blocks, so a default plan merges the
    # leaf bases into it, at no more entries than the blocks apart
    merge, sep, mrg = _leaf_merge(fs)
    assert merge and mrg <= sep
    h = B.bfmht_plan_create_ex(fs, B.F64, 1, 0)
    try:
        assert B.bfmht_plan_num_stages(h) == int(fs["L"]) + 1
        assert B.bfmht_plan_stored_entries(h, False) == full - save - sep + mrg
    finally:
        B.bfmht_plan_destroy(h)
    # every stored transfer/level-0 block with 0 < rank < inputs has the ID form:
    # its saving is rank^2, so the total saving is the sum of rank^2 over them
    L, nb = int(fs["L"]), 1 << int(fs["L"])
    expect = 0
    for lvl in range(L + 1):
        nf = 1 << (L - lvl)
        for q in range(nb):
            if fs["ident"][lvl, q] or fs["P_off"][lvl, q] < 0:
                continue
            r = int(fs["rank"][lvl, q])
            if lvl == 0:
                k = int(fs["koff"][q + 1] - fs["koff"][q])
            else:
                i, j = divmod(q, nf)
                q1 = (i >> 1) * 2 * nf + 2 * j
                k = int(fs["rank"][lvl - 1, q1] + fs["rank"][lvl - 1, q1 + 1])
            if 0 < r < k:
                expect += r * r
    assert save == expect


def test_tile_shapes_are_host_state(good):
    # stage count L + 2 (separate leaf stage), default 64 x 0 (smallest width
    # covering nrhs), the six legal shapes accepted per direction and stage,
    # anything else rejected
    h = B.bfmht_plan_create_ex(good, B.F32, 4, B.PLAN_LEAF_STAGE)
    try:
        S = B.bfmht_plan_num_stages(h)
        assert S == int(good["L"]) + 2
        assert all(B.bfmht_plan_get_tile(h, d, k) == (64, 0) for d in (0, 1) for k in range(S))
        for k in range(S):
            B.bfmht_plan_set_tile(h, 1, k, (64, 128)[k % 2], (0, 16, 32, 64)[k % 4])
        assert [B.bfmht_plan_get_tile(h, 1, k) for k in range(S)] == \
            [((64, 128)[k % 2], (0, 16, 32, 64)[k % 4]) for k in range(S)]
        assert all(B.bfmht_plan_get_tile(h, 0, k) == (64, 0) for k in range(S))   # directions are separate
        for bad in ((1, S, 64, 16), (1, -1, 64, 16), (0, 0, 96, 16), (0, 0, 64, 48), (0, 0, 0, 16)):
            with pytest.raises(B.BfmhtError) as e:
                B.bfmht_plan_set_tile(h, *bad)
            assert e.value.status == B.EINVAL
    finally:
        B.bfmht_plan_destroy(h)
    assert B.lib.bfmht_plan_num_stages(None) == -1


def test_deep_all_identity_factor_set_creates_a_plan():
    """17 levels of identity blocks (more row copies than the transposed
    gather-sum takes): the plan keeps those transposed stages instead of folding
    them, and creation, sizes and stage counts are unaffected."""
    fs = random_factor_set(80, 1 << 16, 1, 16, ident_levels=17, allow_empty=True)
    assert fs["ident"].all()
    h = B.bfmht_plan_create(fs, B.F32, 1)
    try:
        assert B.bfmht_plan_num_stages(h) == 18
        assert B.bfmht_plan_stored_entries(h, False) == fs["U"].size
        assert B.bfmht_workspace_bytes(h, 1) >= 2 * (1 << 16) * 4
    finally:
        B.bfmht_plan_destroy(h)


def test_batched_mode_bits_are_checked_before_any_device_work(good):
    """Unknown mode bits and the (switched-off) persistent launch are refused
    on the host (the plans here are never uploaded)."""
    import ctypes
    h = B.bfmht_plan_create(good, B.F32, 4)
    try:
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        plans = (vp * 1)(h)
        one = (vp * 1)(None)
        lds = (i64 * 1)(4)
        nr = (i32 * 1)(4)
        for mode, msg in ((4, "unknown batch mode"), (1 << 20, "unknown batch mode"),
                          (B.BATCH_PERSISTENT, "switched off"),
                          (B.BATCH_PERSISTENT | B.BATCH_WIDTH(48), "tile width")):
            st = B.lib.bfmht_apply_batched(plans, 1, one, lds, one, lds, nr, mode, None, 0, None)
            assert st == B.EINVAL, mode
            assert msg in B.lib.bfmht_last_error().decode(), mode
    finally:
        B.bfmht_plan_destroy(h)


@pytest.mark.parametrize("seed,n,m,L,p_id", [(40, 300, 200, 2, 0.0), (41, 700, 256, 3, 0.7), (42, 64, 40, 1, 0.5)])
def test_quadtree_factor_sets_create_plans(seed, n, m, L, p_id):
    """4-ary factor sets (arity 4): validated, laid out, and counted like the
    binary ones; the transposed direction has a second job part per transfer level."""
    fs = random_factor_set(seed, n, m, L, max_rank=20, p_id_form=p_id, arity=4)
    full = fs["P"].size + fs["U"].size
    h = B.bfmht_plan_create_ex(fs, B.F32, 4, B.PLAN_FULL_BLOCKS)
    try:
        assert B.bfmht_plan_stored_entries(h, False) == full
        assert B.bfmht_plan_num_stages(h) == L + 2
        assert B.bfmht_workspace_bytes(h, 4) > 0
    finally:
        B.bfmht_plan_destroy(h)
    h = B.bfmht_plan_create(fs, B.BF16X3, 4)
    B.bfmht_plan_destroy(h)


def test_arity_other_than_two_or_four_is_rejected(good):
    bad = dict(good, arity=np.int64(3))
    with pytest.raises(B.BfmhtError) as e:
        B.bfmht_plan_create(bad, B.F32, 1)
    assert e.value.status == B.EINVAL and "arity" in str(e.value)
    # a 4-ary set whose arrays are sized for a binary tree is refused by the
    # binding (the library reads arity^L + 1 offsets and cannot see the lengths)
    bad4 = dict(good, arity=np.int64(4))
    with pytest.raises(ValueError):
        B.bfmht_plan_create(bad4, B.F32, 1)


def test_factor_calls_check_their_metadata_before_any_device_work():
    """The device-factorization calls reject bad host metadata with EINVAL and
    touch no device memory doing so (fake device addresses, no GPU needed)."""
    fake = ctypes.c_void_p(1 << 20)
    assert B.bfmht_factor_meta_bytes(-1, 0) == -1
    assert B.bfmht_factor_meta_bytes(0, 0) == 256
    assert B.bfmht_factor_meta_bytes(2, 10) % 256 == 0
    rows, col_off, a_off = [5, 3], [0, 2, 4], [0, 10]

    def cid(rows=rows, col_off=col_off, a_off=a_off, a_len=19, tol=1e-8):
        B.bfmht_column_id(rows, col_off, a_off, fake, a_len, tol, fake, fake, fake, 1 << 20)

    for kw, msg in [(dict(tol=-1.0), "tol"), (dict(col_off=[1, 2, 4]), "col_off"), (dict(col_off=[0, 3, 2]), "decreases"),
                    (dict(a_len=15), "outside a"), (dict(rows=[-1, 3]), "row count")]:
        with pytest.raises(B.BfmhtError, match=msg) as e:
            cid(**kw)
        assert e.value.status == B.EINVAL
    with pytest.raises(ValueError):
        cid(col_off=[0, 2])                      # binding: wrong length
    B.bfmht_column_id([], [0], [], None, 0, 1e-8, None, None, None, 0)   # count 0: no-op

    def form(ta=(0, 1, 2, 0), row0=(0, 4), ld=8, w0=3):
        B.bfmht_form_blocks(list(row0), rows, col_off, list(ta), [0, 0, 0, 0], a_off, fake, ld, w0, fake, ld, 1,
                            fake, 19, fake, 1 << 20)

    with pytest.raises(B.BfmhtError, match="table column") as e:
        form(ta=(0, 1, 3, 0))
    assert e.value.status == B.EINVAL
    with pytest.raises(B.BfmhtError, match="outside the tables"):
        form(row0=(0, 6))
    with pytest.raises(B.BfmhtError, match="negative"):
        form(ld=-1)

    def coef(rank=(1, 2), p_off=(0, 2), p_len=6):
        B.bfmht_id_coefficients(rows, col_off, a_off, fake, 19, list(rank), fake, list(p_off), fake, p_len, fake, 1 << 20)

    with pytest.raises(B.BfmhtError, match="bad rank"):
        coef(rank=(3, 1))
    with pytest.raises(B.BfmhtError, match="outside p"):
        coef(p_len=5)
