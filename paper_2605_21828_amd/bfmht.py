"""ctypes binding of libbfmht.so (the C ABI declared in include/bfmht.h).

Argument marshalling only: every step of the apply runs in the HIP library.
The raw entry points keep the C names (bfmht_plan_create, bfmht_apply, ...);
`Plan` wraps them with PyTorch tensors for device memory and streams.  The
library must have been built (python -m paper_2605_21828_amd.build); importing
this module on a machine without it raises immediately, and a Plan refuses to
run without a HIP device.  There is no CPU fallback.
"""
import ctypes
import os

import numpy as np
# PyTorch carries its own HIP runtime (soname libamdhip64.so.7).  Importing it
# before the library is loaded makes the library's libamdhip64 dependency
# resolve to that same runtime, so one HIP runtime owns the device, the
# streams and the memory in the process.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
# BFMHT_LIB selects another build of the library (the AddressSanitizer build of
# the host code, for instance); by default the in-tree libbfmht.so.
LIB_PATH = os.environ.get("BFMHT_LIB") or os.path.join(_HERE, "libbfmht.so")

F64, F32, BF16X2, BF16X3 = 0, 1, 2, 3
PRECISIONS = {"f64": F64, "f32": F32, "bf16x2": BF16X2, "bf16x3": BF16X3}
OK, EINVAL, ESTATE, ENOSPACE, EHIP = 0, 1, 2, 3, 4
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ESTATE", 3: "ENOSPACE", 4: "EHIP"}


class bfmht_factors_host(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("m", ctypes.c_int64), ("L", ctypes.c_int32), ("arity", ctypes.c_int32),
        ("perm_x", ctypes.c_void_p), ("xoff", ctypes.c_void_p), ("koff", ctypes.c_void_p),
        ("rank", ctypes.c_void_p), ("ident", ctypes.c_void_p),
        ("P", ctypes.c_void_p), ("P_off", ctypes.c_void_p), ("P_len", ctypes.c_int64),
        ("U", ctypes.c_void_p), ("U_off", ctypes.c_void_p), ("U_len", ctypes.c_int64),
    ]


EXPORTED = [
    "bfmht_plan_create", "bfmht_plan_device_bytes", "bfmht_workspace_bytes", "bfmht_plan_upload",
    "bfmht_apply", "bfmht_apply_transpose", "bfmht_plan_destroy", "bfmht_last_error", "bfmht_version",
    "bfmht_plan_num_stages", "bfmht_plan_set_tile", "bfmht_plan_get_tile",
    "bfmht_batched_workspace_bytes", "bfmht_apply_batched",
    "bfmht_apply_scaled", "bfmht_apply_transpose_scaled", "bfmht_lsqr", "bfmht_lsqr_workspace_bytes",
    "bfmht_plan_create_ex", "bfmht_plan_stored_entries", "bfmht_apply_noalloc",
    "bfmht_factor_meta_bytes", "bfmht_form_blocks", "bfmht_column_id", "bfmht_id_coefficients",
]

NOALLOC_WORKSPACE_BYTES = 256 << 20  # BFMHT_NOALLOC_WORKSPACE_BYTES

PLAN_FULL_BLOCKS = 1  # plan flag: keep every ID block as the full P (no compact form, no merged leaf blocks)
PLAN_LEAF_STAGE = 2   # plan flag: keep the leaf bases as a stage of their own
# mode bits of bfmht_apply_batched
BATCH_TRANSPOSE, BATCH_PERSISTENT = 1, 2


def BATCH_WIDTH(w):
    return int(w) << 8


def load_library(path=LIB_PATH):
    if not os.path.exists(path):
        raise RuntimeError("libbfmht.so not built: run `python -m paper_2605_21828_amd.build` (%s)" % path)
    lib = ctypes.CDLL(path)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.bfmht_plan_create.argtypes = [ctypes.POINTER(bfmht_factors_host), ctypes.c_int, i32, ctypes.POINTER(vp)]
    lib.bfmht_plan_create.restype = ctypes.c_int
    lib.bfmht_plan_create_ex.argtypes = [ctypes.POINTER(bfmht_factors_host), ctypes.c_int, i32, i32,
                                         ctypes.POINTER(vp)]
    lib.bfmht_plan_create_ex.restype = ctypes.c_int
    lib.bfmht_plan_stored_entries.argtypes = [vp, i32]
    lib.bfmht_plan_stored_entries.restype = i64
    lib.bfmht_plan_device_bytes.argtypes = [vp]
    lib.bfmht_plan_device_bytes.restype = i64
    lib.bfmht_workspace_bytes.argtypes = [vp, i32]
    lib.bfmht_workspace_bytes.restype = i64
    lib.bfmht_plan_upload.argtypes = [vp, vp, i64, vp]
    lib.bfmht_plan_upload.restype = ctypes.c_int
    lib.bfmht_apply.argtypes = [vp, vp, i64, vp, i64, i32, vp, i64, vp]
    lib.bfmht_apply.restype = ctypes.c_int
    lib.bfmht_apply_transpose.argtypes = [vp, vp, i64, vp, i64, i32, vp, i64, vp]
    lib.bfmht_apply_transpose.restype = ctypes.c_int
    lib.bfmht_apply_noalloc.argtypes = [vp, vp, i64, vp, i64, i32, vp]
    lib.bfmht_apply_noalloc.restype = ctypes.c_int
    lib.bfmht_apply_scaled.argtypes = [vp, vp, vp, i64, vp, i64, i32, vp, i64, vp]
    lib.bfmht_apply_scaled.restype = ctypes.c_int
    lib.bfmht_apply_transpose_scaled.argtypes = [vp, vp, vp, i64, vp, i64, i32, vp, i64, vp]
    lib.bfmht_apply_transpose_scaled.restype = ctypes.c_int
    lib.bfmht_lsqr.argtypes = [vp, vp, i64, vp, i64, i32, i32, vp, vp, i64, vp]
    lib.bfmht_lsqr.restype = ctypes.c_int
    lib.bfmht_lsqr_workspace_bytes.argtypes = [vp, i32]
    lib.bfmht_lsqr_workspace_bytes.restype = i64
    lib.bfmht_plan_destroy.argtypes = [vp]
    lib.bfmht_plan_destroy.restype = None
    lib.bfmht_last_error.argtypes = []
    lib.bfmht_last_error.restype = ctypes.c_char_p
    lib.bfmht_version.argtypes = []
    lib.bfmht_version.restype = ctypes.c_char_p
    lib.bfmht_plan_num_stages.argtypes = [vp]
    lib.bfmht_plan_num_stages.restype = i32
    lib.bfmht_plan_set_tile.argtypes = [vp, i32, i32, i32, i32]
    lib.bfmht_plan_set_tile.restype = ctypes.c_int
    lib.bfmht_plan_get_tile.argtypes = [vp, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.bfmht_plan_get_tile.restype = ctypes.c_int
    pp = ctypes.POINTER(vp)
    lib.bfmht_batched_workspace_bytes.argtypes = [pp, i32, ctypes.POINTER(i32)]
    lib.bfmht_batched_workspace_bytes.restype = i64
    lib.bfmht_apply_batched.argtypes = [pp, i32, pp, ctypes.POINTER(i64), pp, ctypes.POINTER(i64),
                                        ctypes.POINTER(i32), i32, vp, i64, vp]
    lib.bfmht_apply_batched.restype = ctypes.c_int
    I64P, I32P, DP = ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)
    lib.bfmht_factor_meta_bytes.argtypes = [i32, i64]
    lib.bfmht_factor_meta_bytes.restype = i64
    lib.bfmht_form_blocks.argtypes = [i32, I64P, I64P, I64P, I32P, I32P, I64P, vp, i64, i64, vp, i64, i64, vp, i64,
                                      vp, i64, vp]
    lib.bfmht_form_blocks.restype = ctypes.c_int
    lib.bfmht_column_id.argtypes = [i32, I64P, I64P, I64P, vp, i64, ctypes.c_double, vp, vp, vp, i64, vp]
    lib.bfmht_column_id.restype = ctypes.c_int
    lib.bfmht_id_coefficients.argtypes = [i32, I64P, I64P, I64P, vp, i64, I32P, vp, I64P, vp, i64, vp, i64, vp]
    lib.bfmht_id_coefficients.restype = ctypes.c_int
    return lib


lib = load_library()


class BfmhtError(RuntimeError):
    def __init__(self, status, where):
        msg = lib.bfmht_last_error().decode()
        super().__init__("%s failed: %s (%s)" % (where, STATUS_NAMES.get(status, status), msg))
        self.status = status


def _check(status, where):
    if status != OK:
        raise BfmhtError(status, where)


def _c(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def factors_struct(fs):
    """Build the C struct from a factor-set dict; returns (struct, keepalive list).
    The C side reads every array to the length the tree implies (arity^L + 1
    offsets, (L+1) arity^L ranks, ...); those lengths are checked here first,
    since the library cannot see them."""
    arity = int(fs["arity"]) if "arity" in fs else 2
    L = int(fs["L"])
    if arity in (2, 4) and 0 <= L and arity ** L <= (1 << 24):
        nb = arity ** L
        need = dict(perm_x=int(fs["n"]), xoff=nb + 1, koff=nb + 1, rank=(L + 1) * nb, ident=(L + 1) * nb,
                    P_off=(L + 1) * nb, U_off=nb)
        for k, ln in need.items():
            if np.asarray(fs[k]).size != ln:
                raise ValueError("factor set field %s has %d entries, the tree needs %d" % (k, np.asarray(fs[k]).size, ln))
    keep = dict(
        perm_x=_c(fs["perm_x"], np.int32), xoff=_c(fs["xoff"], np.int64), koff=_c(fs["koff"], np.int64),
        rank=_c(fs["rank"], np.int32).ravel(), ident=_c(fs["ident"], np.uint8).ravel(),
        P=_c(fs["P"], np.float64), P_off=_c(fs["P_off"], np.int64).ravel(),
        U=_c(fs["U"], np.float64), U_off=_c(fs["U_off"], np.int64),
    )
    st = bfmht_factors_host()
    st.n, st.m, st.L = int(fs["n"]), int(fs["m"]), int(fs["L"])
    st.arity = int(fs["arity"]) if "arity" in fs else 2
    for k in ("perm_x", "xoff", "koff", "rank", "ident", "P", "P_off", "U", "U_off"):
        setattr(st, k, keep[k].ctypes.data if keep[k].size else None)
    st.P_len, st.U_len = keep["P"].size, keep["U"].size
    return st, keep


def bfmht_plan_create(fs, precision, max_nrhs=1):
    """Returns an opaque plan handle (int) or raises BfmhtError."""
    st, keep = factors_struct(fs)
    h = ctypes.c_void_p()
    _check(lib.bfmht_plan_create(ctypes.byref(st), int(precision), int(max_nrhs), ctypes.byref(h)),
           "bfmht_plan_create")
    del keep
    return h.value


def bfmht_plan_create_ex(fs, precision, max_nrhs=1, flags=0):
    """bfmht_plan_create with plan flags (PLAN_FULL_BLOCKS, PLAN_LEAF_STAGE); returns the handle."""
    st, keep = factors_struct(fs)
    h = ctypes.c_void_p()
    _check(lib.bfmht_plan_create_ex(ctypes.byref(st), int(precision), int(max_nrhs), int(flags), ctypes.byref(h)),
           "bfmht_plan_create_ex")
    del keep
    return h.value


def bfmht_plan_stored_entries(plan, transpose=False):
    return lib.bfmht_plan_stored_entries(plan, 1 if transpose else 0)


def bfmht_plan_device_bytes(plan):
    return lib.bfmht_plan_device_bytes(plan)


def bfmht_workspace_bytes(plan, nrhs):
    return lib.bfmht_workspace_bytes(plan, int(nrhs))


def bfmht_plan_upload(plan, dev_ptr, dev_bytes, stream=0):
    _check(lib.bfmht_plan_upload(plan, dev_ptr, int(dev_bytes), stream), "bfmht_plan_upload")


def bfmht_apply(plan, c_ptr, ldc, f_ptr, ldf, nrhs, ws_ptr, ws_bytes, stream=0):
    _check(lib.bfmht_apply(plan, c_ptr, ldc, f_ptr, ldf, nrhs, ws_ptr, ws_bytes, stream), "bfmht_apply")


def bfmht_apply_noalloc(plan, c_ptr, ldc, f_ptr, ldf, nrhs, stream=0):
    _check(lib.bfmht_apply_noalloc(plan, c_ptr, ldc, f_ptr, ldf, nrhs, stream), "bfmht_apply_noalloc")


def bfmht_apply_transpose(plan, f_ptr, ldf, g_ptr, ldg, nrhs, ws_ptr, ws_bytes, stream=0):
    _check(lib.bfmht_apply_transpose(plan, f_ptr, ldf, g_ptr, ldg, nrhs, ws_ptr, ws_bytes, stream),
           "bfmht_apply_transpose")


def bfmht_apply_scaled(plan, s_ptr, c_ptr, ldc, f_ptr, ldf, nrhs, ws_ptr, ws_bytes, stream=0):
    _check(lib.bfmht_apply_scaled(plan, s_ptr, c_ptr, ldc, f_ptr, ldf, nrhs, ws_ptr, ws_bytes, stream),
           "bfmht_apply_scaled")


def bfmht_apply_transpose_scaled(plan, s_ptr, f_ptr, ldf, g_ptr, ldg, nrhs, ws_ptr, ws_bytes, stream=0):
    _check(lib.bfmht_apply_transpose_scaled(plan, s_ptr, f_ptr, ldf, g_ptr, ldg, nrhs, ws_ptr, ws_bytes, stream),
           "bfmht_apply_transpose_scaled")


def bfmht_lsqr(plan, f_ptr, ldf, x_ptr, ldx, nrhs, iters, rnorm_ptr, ws_ptr, ws_bytes, stream=0):
    _check(lib.bfmht_lsqr(plan, f_ptr, ldf, x_ptr, ldx, nrhs, iters, rnorm_ptr, ws_ptr, ws_bytes, stream),
           "bfmht_lsqr")


def bfmht_lsqr_workspace_bytes(plan, nrhs):
    return lib.bfmht_lsqr_workspace_bytes(plan, int(nrhs))


def bfmht_plan_destroy(plan):
    lib.bfmht_plan_destroy(plan)


def bfmht_plan_num_stages(plan):
    return lib.bfmht_plan_num_stages(plan)


def bfmht_plan_set_tile(plan, transpose, stage, rows, cols):
    _check(lib.bfmht_plan_set_tile(plan, int(transpose), int(stage), int(rows), int(cols)), "bfmht_plan_set_tile")


def bfmht_plan_get_tile(plan, transpose, stage):
    r, c = ctypes.c_int32(), ctypes.c_int32()
    _check(lib.bfmht_plan_get_tile(plan, int(transpose), int(stage), ctypes.byref(r), ctypes.byref(c)),
           "bfmht_plan_get_tile")
    return r.value, c.value


def _arr(ctype, vals):
    return (ctype * max(1, len(vals)))(*vals)


def bfmht_batched_workspace_bytes(plans, nrhs):
    return lib.bfmht_batched_workspace_bytes(_arr(ctypes.c_void_p, plans), len(plans), _arr(ctypes.c_int32, nrhs))


def bfmht_apply_batched(plans, ins, ldin, outs, ldout, nrhs, mode, ws_ptr, ws_bytes, stream=0):
    """mode: BATCH_TRANSPOSE | BATCH_PERSISTENT | BATCH_WIDTH(w) bits (0 = forward, per-stage launches)."""
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    _check(lib.bfmht_apply_batched(_arr(vp, plans), len(plans), _arr(vp, ins), _arr(i64, ldin), _arr(vp, outs),
                                   _arr(i64, ldout), _arr(i32, nrhs), int(mode), ws_ptr, int(ws_bytes),
                                   stream), "bfmht_apply_batched")


def _host(a, dtype, n, name):
    """Contiguous host copy of a metadata array, checked to hold n entries."""
    a = np.ascontiguousarray(np.asarray(a), dtype=dtype)
    if a.ndim != 1 or a.size != n:
        raise ValueError("%s: expected %d entries, got shape %s" % (name, n, a.shape))
    return a


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def bfmht_factor_meta_bytes(count, total_cols):
    return lib.bfmht_factor_meta_bytes(int(count), int(total_cols))


def bfmht_form_blocks(row0, rows, col_off, ta, tb, a_off, tab0_ptr, ld0, w0, tab1_ptr, ld1, w1, a_ptr, a_len,
                      ws_ptr, ws_bytes, stream=0):
    """Host metadata arrays (numpy), device tables, blocks and workspace (addresses)."""
    count = len(rows)
    col_off = _host(col_off, np.int64, count + 1, "col_off")
    tc = int(col_off[-1]) if count else 0
    row0, rows, a_off = (_host(x, np.int64, count, nm) for x, nm in ((row0, "row0"), (rows, "rows"), (a_off, "a_off")))
    ta, tb = _host(ta, np.int32, tc, "ta"), _host(tb, np.int32, tc, "tb")
    I64, I32 = ctypes.c_int64, ctypes.c_int32
    _check(lib.bfmht_form_blocks(count, _ptr(row0, I64), _ptr(rows, I64), _ptr(col_off, I64), _ptr(ta, I32),
                                 _ptr(tb, I32), _ptr(a_off, I64), tab0_ptr, int(ld0), int(w0), tab1_ptr, int(ld1),
                                 int(w1), a_ptr, int(a_len), ws_ptr, int(ws_bytes), stream), "bfmht_form_blocks")


def bfmht_column_id(rows, col_off, a_off, a_ptr, a_len, tol, rank_ptr, piv_ptr, ws_ptr, ws_bytes, stream=0):
    count = len(rows)
    col_off = _host(col_off, np.int64, count + 1, "col_off")
    rows, a_off = _host(rows, np.int64, count, "rows"), _host(a_off, np.int64, count, "a_off")
    I64 = ctypes.c_int64
    _check(lib.bfmht_column_id(count, _ptr(rows, I64), _ptr(col_off, I64), _ptr(a_off, I64), a_ptr, int(a_len),
                               float(tol), rank_ptr, piv_ptr, ws_ptr, int(ws_bytes), stream), "bfmht_column_id")


def bfmht_id_coefficients(rows, col_off, a_off, a_ptr, a_len, rank, piv_ptr, p_off, p_ptr, p_len, ws_ptr, ws_bytes,
                          stream=0):
    count = len(rows)
    col_off = _host(col_off, np.int64, count + 1, "col_off")
    rows, a_off = _host(rows, np.int64, count, "rows"), _host(a_off, np.int64, count, "a_off")
    rank, p_off = _host(rank, np.int32, count, "rank"), _host(p_off, np.int64, count, "p_off")
    I64, I32 = ctypes.c_int64, ctypes.c_int32
    _check(lib.bfmht_id_coefficients(count, _ptr(rows, I64), _ptr(col_off, I64), _ptr(a_off, I64), a_ptr, int(a_len),
                                     _ptr(rank, I32), piv_ptr, _ptr(p_off, I64), p_ptr, int(p_len), ws_ptr,
                                     int(ws_bytes), stream), "bfmht_id_coefficients")


class Plan:
    """A factor set uploaded to one GPU in one precision.

    apply(c)   -> f = Phi~ c      c: (m,) or (m, b) tensor on the plan's device
    apply_t(f) -> g = Phi~^T f    f: (n,) or (n, b)
    full_blocks: store every ID block as the full P (by default blocks with the
    column-ID structure keep only T, and the leaf bases are merged into the last
    transfer level when that stores about as many entries).
    leaf_stage: keep the leaf bases as a stage of their own (no merged blocks).
    leaf_merged (attribute): whether the plan merged them.
    Element type: float64 for precision "f64", float32 otherwise.
    Calls run on the current torch stream of the plan's device.
    """

    def __init__(self, fs, precision="f32", max_nrhs=64, device="cuda", full_blocks=False, leaf_stage=False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("bfmht.Plan needs a HIP device; there is no CPU path")
        self.torch = torch
        dev = torch.device(device)
        if dev.index is None:
            dev = torch.device(dev.type, torch.cuda.current_device())
        self.device = dev
        self.prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.precision = precision
        self.dtype = torch.float64 if self.prec == F64 else torch.float32
        self.n, self.m, self.L = int(fs["n"]), int(fs["m"]), int(fs["L"])
        flags = (PLAN_FULL_BLOCKS if full_blocks else 0) | (PLAN_LEAF_STAGE if leaf_stage else 0)
        self.handle = bfmht_plan_create_ex(fs, self.prec, max_nrhs, flags)
        self.leaf_merged = bfmht_plan_num_stages(self.handle) == self.L + 1
        self.stored_fwd = bfmht_plan_stored_entries(self.handle, False)
        self.stored_t = bfmht_plan_stored_entries(self.handle, True)
        nbytes = bfmht_plan_device_bytes(self.handle)
        self._dev = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._dev.data_ptr()
        self._dev_ptr = (base + 255) // 256 * 256
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream().cuda_stream
            bfmht_plan_upload(self.handle, self._dev_ptr, nbytes, stream)
        self.device_bytes = nbytes
        self._ws = None
        self._ws_ptr = 0
        self._ws_bytes = 0

    def workspace(self, nrhs):
        need = bfmht_workspace_bytes(self.handle, nrhs)
        if self._ws is None or self._ws_bytes < need:
            self._ws = self.torch.empty(need + 256, dtype=self.torch.uint8, device=self.device)
            self._ws_ptr = (self._ws.data_ptr() + 255) // 256 * 256
            self._ws_bytes = need
        return self._ws_ptr, self._ws_bytes

    def _prep(self, x, rows):
        torch = self.torch
        if x.device != self.device or x.dtype != self.dtype:
            raise ValueError("expected a %s tensor on %s, got %s on %s" % (self.dtype, self.device, x.dtype, x.device))
        squeeze = x.dim() == 1
        if squeeze:
            x = x.unsqueeze(1)
        if x.dim() != 2 or x.shape[0] != rows:
            raise ValueError("expected %d rows, got shape %s" % (rows, tuple(x.shape)))
        if x.stride(1) != 1:
            x = x.contiguous()
        return x, squeeze

    def _out(self, out, rows, b):
        """The output block: a new (rows, b) tensor, or `out` after checking that
        the library may write rows x b elements into it (its device, element
        type, shape, unit column stride and row stride >= b); a 1-D out of
        `rows` elements is accepted for b = 1."""
        torch = self.torch
        if out is None:
            return torch.empty((rows, b), dtype=self.dtype, device=self.device)
        if out.device != self.device or out.dtype != self.dtype:
            raise ValueError("out must be a %s tensor on %s, got %s on %s"
                             % (self.dtype, self.device, out.dtype, out.device))
        if out.dim() == 1 and b == 1:
            out = out.unsqueeze(1)
        if out.dim() != 2 or tuple(out.shape) != (rows, b):
            raise ValueError("out must have shape (%d, %d), got %s" % (rows, b, tuple(out.shape)))
        if rows > 0 and b > 0 and ((b > 1 and out.stride(1) != 1) or out.stride(0) < b):
            raise ValueError("out must have unit column stride and row stride >= %d, got strides %s"
                             % (b, tuple(out.stride())))
        return out

    def apply(self, c, out=None):
        torch = self.torch
        c, squeeze = self._prep(c, self.m)
        b = c.shape[1]
        f = self._out(out, self.n, b)
        ws, wsb = self.workspace(b)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        bfmht_apply(self.handle, c.data_ptr(), c.stride(0), f.data_ptr(), f.stride(0), b, ws, wsb, stream)
        return f[:, 0] if squeeze else f

    def apply_t(self, f, out=None):
        torch = self.torch
        f, squeeze = self._prep(f, self.n)
        b = f.shape[1]
        g = self._out(out, self.m, b)
        ws, wsb = self.workspace(b)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        bfmht_apply_transpose(self.handle, f.data_ptr(), f.stride(0), g.data_ptr(), g.stride(0), b, ws, wsb, stream)
        return g[:, 0] if squeeze else g

    def _scale(self, s):
        if s.device != self.device or s.dtype != self.dtype or s.dim() != 1 or s.shape[0] != self.m:
            raise ValueError("expected a (%d,) %s tensor on %s" % (self.m, self.dtype, self.device))
        return s.contiguous()

    def apply_scaled(self, s, c, out=None):
        """f = Phi~ diag(s) c (a Karhunen-Loeve sample when s = sqrt(S) and c ~ N(0, I))."""
        torch = self.torch
        s = self._scale(s)
        c, squeeze = self._prep(c, self.m)
        b = c.shape[1]
        f = self._out(out, self.n, b)
        ws, wsb = self.workspace(b)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        bfmht_apply_scaled(self.handle, s.data_ptr(), c.data_ptr(), c.stride(0), f.data_ptr(), f.stride(0), b, ws,
                           wsb, stream)
        return f[:, 0] if squeeze else f

    def apply_t_scaled(self, s, f, out=None):
        """g = diag(s) Phi~^T f."""
        torch = self.torch
        s = self._scale(s)
        f, squeeze = self._prep(f, self.n)
        b = f.shape[1]
        g = self._out(out, self.m, b)
        ws, wsb = self.workspace(b)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        bfmht_apply_transpose_scaled(self.handle, s.data_ptr(), f.data_ptr(), f.stride(0), g.data_ptr(),
                                     g.stride(0), b, ws, wsb, stream)
        return g[:, 0] if squeeze else g

    def lsqr(self, f, iters, out=None):
        """Least squares min ||Phi~ x - f|| per column by `iters` LSQR steps on the GPU
        (the inverse transform); returns (x, rnorm estimate per column)."""
        torch = self.torch
        f, squeeze = self._prep(f, self.n)
        b = f.shape[1]
        x = self._out(out, self.m, b)
        rnorm = torch.empty(b, dtype=self.dtype, device=self.device)
        need = bfmht_lsqr_workspace_bytes(self.handle, b)
        ws = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        ws_ptr = (ws.data_ptr() + 255) // 256 * 256
        stream = torch.cuda.current_stream(self.device).cuda_stream
        bfmht_lsqr(self.handle, f.data_ptr(), f.stride(0), x.data_ptr(), x.stride(0), b, int(iters),
                   rnorm.data_ptr(), ws_ptr, need, stream)
        self._lsqr_ws = ws   # kept alive until the enqueued solve has run
        return (x[:, 0] if squeeze else x), rnorm

    def covariance_matvec(self, s, v):
        """Phi~ diag(s) Phi~^T v: the truncated kernel expansion with spectral weights s."""
        return self.apply(self.apply_t_scaled(s, v))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            bfmht_plan_destroy(h)
            self.handle = None


class Batch:
    """Several uploaded plans of one precision applied together.

    run(inputs, transpose=False) takes one (rows, nrhs_i) tensor per plan and
    returns the outputs; launch k runs the k-th stage of every instance.
    """

    def __init__(self, plans):
        if not plans:
            raise ValueError("empty batch")
        dt = {p.dtype for p in plans}
        if len(dt) != 1:
            raise ValueError("plans of a batch must share one precision")
        self.plans = list(plans)
        self.torch = plans[0].torch
        self.device = plans[0].device
        self._ws = None
        self._ws_bytes = 0

    def workspace(self, nrhs):
        need = bfmht_batched_workspace_bytes([p.handle for p in self.plans], nrhs)
        if need < 0:
            raise ValueError("bad batch arguments")
        if self._ws is None or self._ws_bytes < need:
            self._ws = self.torch.empty(need + 256, dtype=self.torch.uint8, device=self.device)
            self._ws_bytes = need
        return (self._ws.data_ptr() + 255) // 256 * 256, need

    def launch(self, inputs, outputs, transpose=False, persistent=False, width=0):
        """Apply every plan to its input into its output.  persistent=True asks
        for all stages of all instances in one launch (tile width `width`: 16,
        32, 64, or 0 for 32); that mode is switched off in the library and
        raises BfmhtError (EINVAL)."""
        torch = self.torch
        if len(inputs) != len(self.plans) or len(outputs) != len(self.plans):
            raise ValueError("a batch of %d plans needs %d inputs and %d outputs, got %d and %d"
                             % (len(self.plans), len(self.plans), len(self.plans), len(inputs), len(outputs)))
        xs, ys = [], []
        for p, x, y in zip(self.plans, inputs, outputs):
            x, _ = p._prep(x, p.n if transpose else p.m)
            xs.append(x)
            ys.append(p._out(y, p.m if transpose else p.n, int(x.shape[1])))
        outputs = ys
        nrhs = [int(x.shape[1]) for x in xs]
        ws, wsb = self.workspace(nrhs)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        mode = (BATCH_TRANSPOSE if transpose else 0) | (BATCH_PERSISTENT | BATCH_WIDTH(width) if persistent else 0)
        bfmht_apply_batched([p.handle for p in self.plans], [x.data_ptr() for x in xs], [x.stride(0) for x in xs],
                            [y.data_ptr() for y in outputs], [y.stride(0) for y in outputs], nrhs,
                            mode, ws, wsb, stream)
        return outputs

    def run(self, inputs, transpose=False, persistent=False, width=0):
        torch = self.torch
        outs = [torch.empty(((p.m if transpose else p.n), int(x.shape[1] if x.dim() == 2 else 1)),
                            dtype=p.dtype, device=self.device) for p, x in zip(self.plans, inputs)]
        return self.launch(inputs, outs, transpose, persistent, width)
