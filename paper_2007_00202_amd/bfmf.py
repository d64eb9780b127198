"""ctypes binding of libbfmf (include/bfmf.h), argument marshalling only.

The module-level functions carry the names of the C entry points; the
``Solver`` class strings them together.  Every numerical step runs inside
the library; when the library is not built this module raises on import.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libbfmf.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libbfmf.so is not built ({LIB_PATH}); run __graft_entry__.build()")
# One HIP runtime per process.  torch bundles its own libamdhip64 (same
# SONAME as the system one) and loads it by file name; if this library were
# loaded first it would bring the system runtime and torch would then add a
# second one beside it, and the two cannot share the device.  Loading torch
# first makes the library bind to torch's runtime.
import torch  # noqa: E402,F401  (imported for its HIP runtime)

_lib = C.CDLL(LIB_PATH)

# --------------------------------------------------------------- constants
BFMF_OK, BFMF_E_INVAL, BFMF_E_NOMEM, BFMF_E_STATE = 0, -1, -2, -3
BFMF_E_SINGULAR, BFMF_E_NOCONV, BFMF_E_DEVICE = -4, -5, -6
BFMF_ORD_GRID, BFMF_ORD_YEE, BFMF_ORD_USER = 0, 1, 2
BFMF_C128, BFMF_C64_MIXED = 0, 1
BFMF_HOST, BFMF_DEVICE = 0, 1


class bfmf_ordering(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("coords", C.POINTER(C.c_int32)), ("leaf_max", C.c_int32), ("sep_leaf", C.c_int32),
                ("parallel_levels", C.c_int32), ("nfronts", C.c_int32), ("perm", C.POINTER(C.c_int64)),
                ("front_ptr", C.POINTER(C.c_int64)), ("front_parent", C.POINTER(C.c_int32))]


class bfmf_factor_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("n_min", C.c_int64), ("precision", C.c_int32),
                ("batched", C.c_int32), ("samples", C.c_int32), ("knn", C.c_int32),
                ("alpha", C.c_double), ("seed", C.c_uint64), ("hbm_budget", C.c_uint64),
                ("keep_fronts", C.c_int32), ("timing", C.c_int32), ("smw_dense", C.c_int32),
                ("id_max_cols", C.c_int32), ("compress_cb", C.c_int32), ("reserved", C.c_int32 * 3)]


class bfmf_kernel_stat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("seconds", C.c_double),
                ("flops", C.c_double), ("bytes", C.c_double), ("launches_all", C.c_int64)]


BFMF_KERNEL_CLASSES = 12


class bfmf_solve_opts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("max_iter", C.c_int32), ("rtol", C.c_double),
                ("atol", C.c_double), ("true_rtol", C.c_double), ("iters_max", C.c_int32),
                ("graphs", C.c_int32), ("relres_max", C.c_double), ("seconds", C.c_double)]


class bfmf_symbolic_view(C.Structure):
    _fields_ = [("n", C.c_int64), ("nfronts", C.c_int32), ("nlevels", C.c_int32),
                ("perm", C.POINTER(C.c_int64)), ("sbeg", C.POINTER(C.c_int64)),
                ("send", C.POINTER(C.c_int64)), ("parent", C.POINTER(C.c_int32)),
                ("level", C.POINTER(C.c_int32)), ("child_ptr", C.POINTER(C.c_int32)),
                ("child_list", C.POINTER(C.c_int32)), ("iu_ptr", C.POINTER(C.c_int64)),
                ("iu", C.POINTER(C.c_int64)), ("map", C.POINTER(C.c_int32)),
                ("sep_ptr", C.POINTER(C.c_int32)), ("sep_nodes", C.POINTER(C.c_int32))]


class bfmf_stats(C.Structure):
    _fields_ = [("nfronts", C.c_int32), ("compressed_fronts", C.c_int32), ("dense_fronts", C.c_int32),
                ("nlevels", C.c_int32), ("analyze_seconds", C.c_double), ("factor_seconds", C.c_double),
                ("factor_flops", C.c_double), ("factor_bytes", C.c_double),
                ("dense_factor_bytes", C.c_double), ("max_rank", C.c_int32),
                ("singular_front", C.c_int32), ("singular_index", C.c_int32), ("id_chunked", C.c_int32),
                ("solve_flops_per_rhs", C.c_double), ("device_bytes_peak", C.c_uint64),
                ("cb_bytes", C.c_double), ("cb_dense_bytes", C.c_double), ("cb_compressed", C.c_int32),
                ("pad0", C.c_int32), ("workspace_bytes", C.c_double), ("reserved", C.c_double * 4)]


class bfmf_server_opts(C.Structure):
    _fields_ = [("max_batch_rhs", C.c_int32), ("reserved0", C.c_int32), ("hbm_budget", C.c_uint64),
                ("result_bytes", C.c_uint64), ("solve", bfmf_solve_opts)]


class bfmf_request_info(C.Structure):
    _fields_ = [("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double),
                ("model", C.c_int32), ("nrhs", C.c_int32), ("batch_rhs", C.c_int32),
                ("batch_requests", C.c_int32), ("iters", C.c_int32), ("status", C.c_int32),
                ("relres", C.c_double)]


_h = C.c_void_p
_P = C.c_void_p
_SIGS = {
    "bfmf_create": (C.c_int, [C.POINTER(_h), C.c_int32, _P]),
    "bfmf_analyze": (C.c_int, [_h, C.c_int64, _P, _P, _P, C.POINTER(bfmf_ordering)]),
    "bfmf_set_values": (C.c_int, [_h, _P]),
    "bfmf_default_factor_opts": (None, [C.POINTER(bfmf_factor_opts)]),
    "bfmf_default_solve_opts": (None, [C.POINTER(bfmf_solve_opts)]),
    "bfmf_factor": (C.c_int, [_h, C.POINTER(bfmf_factor_opts)]),
    "bfmf_solve": (C.c_int, [_h, C.c_int64, _P, C.c_int64, _P, C.c_int64, C.c_int32,
                             C.POINTER(bfmf_solve_opts)]),
    "bfmf_solve_async": (C.c_int, [_h, C.c_int64, _P, C.c_int64, _P, C.c_int64, _P, C.POINTER(bfmf_solve_opts)]),
    "bfmf_apply_preconditioner": (C.c_int, [_h, C.c_int64, _P, C.c_int64, _P, C.c_int64, C.c_int32]),
    "bfmf_get_symbolic": (C.c_int, [_h, C.POINTER(bfmf_symbolic_view)]),
    "bfmf_get_stats": (C.c_int, [_h, C.POINTER(bfmf_stats)]),
    "bfmf_get_front": (C.c_int, [_h, C.c_int32, C.c_int32, _P, C.c_int64]),
    "bfmf_extract_front": (C.c_int, [_h, C.c_int32, C.c_int32, _P, C.c_int32, _P, _P, C.c_int64]),
    "bfmf_apply_front_block": (C.c_int, [_h, C.c_int32, C.c_int32, C.c_int32, _P, C.c_int64, _P, C.c_int64]),
    "bfmf_get_kernel_stats": (C.c_int, [_h, C.c_int32, C.POINTER(bfmf_kernel_stat)]),
    "bfmf_reset_kernel_stats": (C.c_int, [_h]),
    "bfmf_set_gemm_tile": (C.c_int, [C.c_int32]),
    "bfmf_device_allocation_count": (C.c_int64, []),
    "bfmf_get_gemm_tile_launches": (C.c_int, [_h, C.POINTER(C.c_int64), C.c_int32]),
    "bfmf_bf_compress_dense": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, _P, C.c_int64, C.c_int32, C.c_double,
                                         C.c_int32, C.c_int32, C.c_uint64, C.POINTER(_P)]),
    "bfmf_bf_apply": (C.c_int, [_P, C.c_int32, C.c_int32, _P, C.c_int64, _P, C.c_int64]),
    "bfmf_bf_apply_noalloc": (C.c_int, [_P, C.c_int32, C.c_int32, _P, C.c_int64, _P, C.c_int64, _P]),
    "bfmf_bf_import": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, _P, _P, _P, C.c_int64,
                                 C.POINTER(_P)]),
    "bfmf_bf_extract": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P, _P]),
    "bfmf_bf_info": (C.c_int, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    "bfmf_bf_destroy": (None, [_P]),
    "bfmf_default_server_opts": (None, [C.POINTER(bfmf_server_opts)]),
    "bfmf_server_create": (C.c_int, [C.c_int32, C.POINTER(bfmf_server_opts), C.POINTER(_P)]),
    "bfmf_server_attach": (C.c_int, [_P, _h, C.POINTER(C.c_int32)]),
    "bfmf_server_submit": (C.c_int, [_P, C.c_int32, C.c_int32, _P, _P, _P, C.POINTER(C.c_uint64)]),
    "bfmf_server_wait": (C.c_int, [_P, C.c_uint64, C.POINTER(bfmf_request_info), _P, C.c_int64, C.c_int32]),
    "bfmf_server_clock": (C.c_double, [_P]),
    "bfmf_server_last_error": (C.c_char_p, [_P]),
    "bfmf_server_destroy": (None, [_P]),
    "bfmf_status_str": (C.c_char_p, [C.c_int]),
    "bfmf_last_error": (C.c_char_p, [_h]),
    "bfmf_destroy": (None, [_h]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


class BfmfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_lib.bfmf_status_str(status).decode()} ({status}): {msg}")
        self.status = status


def _check(h, st):
    if st != BFMF_OK:
        msg = _lib.bfmf_last_error(h).decode() if h else ""
        raise BfmfError(st, msg)


def _ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


# ------------------------------------------------------- entry-point wrappers
def bfmf_create(device=0, stream=None):
    h = _h()
    st = _lib.bfmf_create(C.byref(h), int(device), C.c_void_p(stream) if stream else None)
    if st != BFMF_OK:
        raise BfmfError(st, "create")
    return h


def bfmf_analyze(h, rowptr, colind, values, kind=BFMF_ORD_GRID, dims=(0, 0, 0), coords=None,
                 leaf_max=512, sep_leaf=64, parallel_levels=0, perm=None, front_ptr=None, front_parent=None):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    colind = np.ascontiguousarray(colind, dtype=np.int32)
    vals = None if values is None else np.ascontiguousarray(values, dtype=np.complex128)
    cc = None if coords is None else np.ascontiguousarray(coords, dtype=np.int32)
    pm = None if perm is None else np.ascontiguousarray(perm, dtype=np.int64)
    fp = None if front_ptr is None else np.ascontiguousarray(front_ptr, dtype=np.int64)
    fpar = None if front_parent is None else np.ascontiguousarray(front_parent, dtype=np.int32)
    o = bfmf_ordering(kind, dims[0], dims[1], dims[2],
                      cc.ctypes.data_as(C.POINTER(C.c_int32)) if cc is not None else None,
                      leaf_max, sep_leaf, parallel_levels,
                      0 if fpar is None else fpar.shape[0],
                      pm.ctypes.data_as(C.POINTER(C.c_int64)) if pm is not None else None,
                      fp.ctypes.data_as(C.POINTER(C.c_int64)) if fp is not None else None,
                      fpar.ctypes.data_as(C.POINTER(C.c_int32)) if fpar is not None else None)
    _check(h, _lib.bfmf_analyze(h, rowptr.shape[0] - 1, _ptr(rowptr), _ptr(colind), _ptr(vals), C.byref(o)))


def bfmf_set_values(h, values):
    vals = np.ascontiguousarray(values, dtype=np.complex128)
    _check(h, _lib.bfmf_set_values(h, _ptr(vals)))


def bfmf_default_factor_opts():
    o = bfmf_factor_opts()
    _lib.bfmf_default_factor_opts(C.byref(o))
    return o


def bfmf_default_solve_opts():
    o = bfmf_solve_opts()
    _lib.bfmf_default_solve_opts(C.byref(o))
    return o


def bfmf_factor(h, opts=None):
    opts = opts or bfmf_default_factor_opts()
    _check(h, _lib.bfmf_factor(h, C.byref(opts)))


def bfmf_solve(h, B, opts=None, X=None):
    """Host arrays: B (n, nrhs) complex128.  Returns (X, opts) with the outputs filled."""
    B = np.asfortranarray(B, dtype=np.complex128)
    if B.ndim == 1:
        B = B[:, None]
    n, nrhs = B.shape
    if X is None:
        X = np.zeros((n, nrhs), dtype=np.complex128, order="F")
    opts = opts or bfmf_default_solve_opts()
    st = _lib.bfmf_solve(h, nrhs, _ptr(B), n, _ptr(X), n, BFMF_HOST, C.byref(opts))
    if st not in (BFMF_OK, BFMF_E_NOCONV):
        _check(h, st)
    return X, opts, st


def bfmf_solve_device(h, dB, ldb, dX, ldx, nrhs, opts=None):
    """Device pointers (e.g. torch tensors' data_ptr()) of interleaved complex128."""
    opts = opts or bfmf_default_solve_opts()
    st = _lib.bfmf_solve(h, nrhs, C.c_void_p(dB), ldb, C.c_void_p(dX), ldx, BFMF_DEVICE, C.byref(opts))
    if st not in (BFMF_OK, BFMF_E_NOCONV):
        _check(h, st)
    return opts, st


def bfmf_solve_async(h, dB, ldb, dX, ldx, nrhs, stream=None):
    """Direct solve X = M^-1 B queued on `stream` (a hipStream_t as an int, e.g. torch's
    cuda_stream); device pointers of interleaved complex128."""
    o = bfmf_default_solve_opts()
    o.max_iter = -1
    _check(h, _lib.bfmf_solve_async(h, nrhs, C.c_void_p(dB), ldb, C.c_void_p(dX), ldx,
                                    C.c_void_p(stream) if stream else None, C.byref(o)))
    return o


def bfmf_apply_preconditioner(h, B):
    B = np.asfortranarray(B, dtype=np.complex128)
    if B.ndim == 1:
        B = B[:, None]
    n, nrhs = B.shape
    X = np.zeros((n, nrhs), dtype=np.complex128, order="F")
    _check(h, _lib.bfmf_apply_preconditioner(h, nrhs, _ptr(B), n, _ptr(X), n, BFMF_HOST))
    return X


def bfmf_get_symbolic(h):
    v = bfmf_symbolic_view()
    _check(h, _lib.bfmf_get_symbolic(h, C.byref(v)))
    nf = v.nfronts

    def arr(p, cnt, dt):
        return np.ctypeslib.as_array(p, shape=(cnt,)).astype(dt, copy=True) if cnt else np.zeros(0, dt)

    out = {"n": v.n, "nfronts": nf, "nlevels": v.nlevels}
    out["perm"] = arr(v.perm, v.n, np.int64)
    out["sbeg"] = arr(v.sbeg, nf, np.int64)
    out["send"] = arr(v.send, nf, np.int64)
    out["parent"] = arr(v.parent, nf, np.int32)
    out["level"] = arr(v.level, nf, np.int32)
    out["child_ptr"] = arr(v.child_ptr, nf + 1, np.int32)
    out["child_list"] = arr(v.child_list, int(out["child_ptr"][-1]), np.int32)
    out["iu_ptr"] = arr(v.iu_ptr, nf + 1, np.int64)
    out["iu"] = arr(v.iu, int(out["iu_ptr"][-1]), np.int64)
    out["map"] = arr(v.map, int(out["iu_ptr"][-1]), np.int32)
    out["sep_ptr"] = arr(v.sep_ptr, nf + 1, np.int32)
    out["sep_nodes"] = arr(v.sep_nodes, 4 * int(out["sep_ptr"][-1]), np.int32).reshape(-1, 4)
    return out


def bfmf_get_stats(h):
    s = bfmf_stats()
    _check(h, _lib.bfmf_get_stats(h, C.byref(s)))
    return {name: getattr(s, name) for name, _ in bfmf_stats._fields_ if not name.startswith("reserved")}


def bfmf_get_front(h, front, what, n):
    if what == 2:
        out = np.zeros(max(n, 1), dtype=np.int32)
        _check(h, _lib.bfmf_get_front(h, front, what, _ptr(out), 1))
        return out[:n]
    out = np.zeros((n, n), dtype=np.complex128, order="F")
    _check(h, _lib.bfmf_get_front(h, front, what, _ptr(out), n))
    return out


def bfmf_apply_front_block(h, front, what, X, rows):
    """Y = B X for a block of a compressed front (0 F11, 1 F11^-1, 2 F12, 3 F21, 4 S); rows of B given."""
    X = np.asfortranarray(X, dtype=np.complex128)
    if X.ndim == 1:
        X = X[:, None]
    Y = np.zeros((rows, X.shape[1]), dtype=np.complex128, order="F")
    _check(h, _lib.bfmf_apply_front_block(h, front, what, X.shape[1], _ptr(X), max(X.shape[0], 1), _ptr(Y),
                                          max(rows, 1)))
    return Y


def bfmf_extract_front(h, front, rows, cols):
    """F(rows, cols) of a front (front-local indices) through the GPU's list routing."""
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    out = np.zeros((rows.shape[0], cols.shape[0]), dtype=np.complex128, order="F")
    _check(h, _lib.bfmf_extract_front(h, front, rows.shape[0], _ptr(rows), cols.shape[0], _ptr(cols), _ptr(out),
                                      max(rows.shape[0], 1)))
    return out


def bfmf_get_kernel_stats(h):
    out = {}
    for k in range(BFMF_KERNEL_CLASSES):
        st = bfmf_kernel_stat()
        _check(h, _lib.bfmf_get_kernel_stats(h, k, C.byref(st)))
        out[st.name.decode()] = {"launches": st.launches, "seconds": st.seconds, "flops": st.flops,
                                 "bytes": st.bytes, "launches_all": st.launches_all}
    return out


def bfmf_reset_kernel_stats(h):
    _check(h, _lib.bfmf_reset_kernel_stats(h))


BFMF_GEMM_TILES = 8
GEMM_TILE_SHAPES = ["64x64", "32x128", "128x32", "16x256", "256x16", "256x16 streaming", "48x128", "96x64"]


def bfmf_device_allocation_count():
    return int(_lib.bfmf_device_allocation_count())


def bfmf_set_gemm_tile(cfg):
    """Force one grouped-GEMM tile shape for the process (-1: the autotuned choice)."""
    _check(None, _lib.bfmf_set_gemm_tile(cfg))


def bfmf_get_gemm_tile_launches(h):
    out = (C.c_int64 * BFMF_GEMM_TILES)()
    _check(h, _lib.bfmf_get_gemm_tile_launches(h, out, BFMF_GEMM_TILES))
    return {GEMM_TILE_SHAPES[i]: int(out[i]) for i in range(BFMF_GEMM_TILES)}


def bfmf_status_str(st):
    return _lib.bfmf_status_str(st).decode()


def bfmf_last_error(h):
    return _lib.bfmf_last_error(h).decode()


def bfmf_destroy(h):
    _lib.bfmf_destroy(h)


def bfmf_bf_compress_dense(K, L, tol, method=0, samples=64, seed=0, device=0):
    K = np.asfortranarray(K, dtype=np.complex128)
    m, n = K.shape
    out = _P()
    st = _lib.bfmf_bf_compress_dense(device, m, n, _ptr(K), m, L, tol, method, samples, seed, C.byref(out))
    if st != BFMF_OK:
        raise BfmfError(st, "bf_compress_dense: " + _lib.bfmf_last_error(None).decode())
    return out, (m, n)


def bfmf_bf_apply(b, shape, X, adjoint=False):
    m, n = shape
    X = np.asfortranarray(X, dtype=np.complex128)
    if X.ndim == 1:
        X = X[:, None]
    rows_out = n if adjoint else m
    Y = np.zeros((rows_out, X.shape[1]), dtype=np.complex128, order="F")
    st = _lib.bfmf_bf_apply(b, int(adjoint), X.shape[1], _ptr(X), X.shape[0], _ptr(Y), rows_out)
    if st != BFMF_OK:
        raise BfmfError(st, "bf_apply")
    return Y


def bfmf_bf_apply_noalloc(b, adjoint, nrhs, dX, ldx, dY, ldy, stream=None):
    """Device pointers (e.g. torch tensors' data_ptr()); returns the status (0 on success)."""
    return _lib.bfmf_bf_apply_noalloc(b, int(adjoint), nrhs, C.c_void_p(dX), ldx, C.c_void_p(dY), ldy,
                                      C.c_void_p(stream) if stream else None)


def bfmf_bf_import(m, n, L, ranks_left, ranks_right, factors, device=0):
    """ranks_left: (L - L//2 + 1, 2^L) int, ranks_right: (L//2 + 1, 2^L) int, factors: complex128
    entries in the order bfmf_bf_import documents."""
    rl = np.ascontiguousarray(ranks_left, dtype=np.int32)
    rr = np.ascontiguousarray(ranks_right, dtype=np.int32)
    f = np.ascontiguousarray(factors, dtype=np.complex128)
    if rl.shape != (L - L // 2 + 1, 1 << L) or rr.shape != (L // 2 + 1, 1 << L):
        raise BfmfError(BFMF_E_INVAL, "bf_import: rank arrays of the wrong shape")
    out = _P()
    st = _lib.bfmf_bf_import(device, m, n, L, _ptr(rl), _ptr(rr), _ptr(f) if f.size else None, f.size,
                             C.byref(out))
    if st != BFMF_OK:
        raise BfmfError(st, "bf_import: " + _lib.bfmf_last_error(None).decode())
    return out, (m, n)


def bfmf_bf_extract(b, requests):
    """requests: list of (rows, cols); returns the list of submatrices K(rows, cols)."""
    rows = [np.asarray(r, dtype=np.int32).ravel() for r, _ in requests]
    cols = [np.asarray(c, dtype=np.int32).ravel() for _, c in requests]
    rp = np.zeros(len(requests) + 1, dtype=np.int64)
    cp = np.zeros(len(requests) + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    cp[1:] = np.cumsum([len(c) for c in cols])
    R = np.concatenate(rows) if rows else np.zeros(0, np.int32)
    Cc = np.concatenate(cols) if cols else np.zeros(0, np.int32)
    sizes = [len(r) * len(c) for r, c in zip(rows, cols)]
    out = np.zeros(max(sum(sizes), 1), dtype=np.complex128)
    st = _lib.bfmf_bf_extract(b, len(requests), _ptr(rp), _ptr(R) if R.size else None, _ptr(cp),
                              _ptr(Cc) if Cc.size else None, _ptr(out))
    if st != BFMF_OK:
        raise BfmfError(st, "bf_extract")
    res, pos = [], 0
    for r, c, sz in zip(rows, cols, sizes):
        res.append(out[pos:pos + sz].reshape((len(c), len(r))).T.copy())
        pos += sz
    return res


def bfmf_bf_info(b):
    L, r, e = C.c_int32(), C.c_int32(), C.c_int64()
    _lib.bfmf_bf_info(b, C.byref(L), C.byref(r), C.byref(e))
    return {"L": L.value, "max_rank": r.value, "entries": e.value}


def bfmf_bf_destroy(b):
    _lib.bfmf_bf_destroy(b)


# ------------------------------------------------------------ convenience
class Solver:
    """analyze(A, ordering) -> factor(tol) -> solve(B) on one device."""

    def __init__(self, device=0, stream=None):
        self.h = bfmf_create(device, stream)
        self.n = None

    def analyze(self, rowptr, colind, values, dims=None, coords=None, cells=None, leaf_max=512, sep_leaf=64,
                parallel_levels=0, perm=None, front_ptr=None, front_parent=None):
        if perm is not None:  # the caller's ordering and assembly tree
            bfmf_analyze(self.h, rowptr, colind, values, BFMF_ORD_USER, (0, 0, 0), None, leaf_max, sep_leaf,
                         parallel_levels, perm, front_ptr, front_parent)
        elif coords is not None:
            bfmf_analyze(self.h, rowptr, colind, values, BFMF_ORD_YEE, (cells, 0, 0), coords, leaf_max, sep_leaf,
                         parallel_levels)
        else:
            bfmf_analyze(self.h, rowptr, colind, values, BFMF_ORD_GRID, dims, None, leaf_max, sep_leaf,
                         parallel_levels)
        self.n = rowptr.shape[0] - 1
        return self

    def factor(self, tol=1e-3, n_min=1024, precision=BFMF_C128, batched=False, samples=64, knn=8,
               alpha=2.0, seed=0, hbm_budget=0, keep_fronts=False, timing=False, smw_dense=0, id_max_cols=0,
               compress_cb=False):
        o = bfmf_default_factor_opts()
        o.smw_dense, o.id_max_cols = smw_dense, id_max_cols
        o.compress_cb = int(bool(compress_cb))
        o.timing = int(bool(timing))
        o.tol, o.n_min, o.precision, o.batched = tol, n_min, precision, int(bool(batched))
        o.samples, o.knn, o.alpha, o.seed = samples, knn, alpha, seed
        o.hbm_budget, o.keep_fronts = hbm_budget, int(bool(keep_fronts))
        bfmf_factor(self.h, o)
        return self

    def solve(self, B, restart=30, max_iter=300, rtol=1e-6, atol=1e-10, true_rtol=0.0, graphs=True):
        o = bfmf_default_solve_opts()
        o.restart, o.max_iter, o.rtol, o.atol, o.true_rtol = restart, max_iter, rtol, atol, true_rtol
        o.graphs = int(bool(graphs))
        X, o, st = bfmf_solve(self.h, B, o)
        return X, {"iters": o.iters_max, "relres": o.relres_max, "seconds": o.seconds, "status": st}

    def precondition(self, B):
        return bfmf_apply_preconditioner(self.h, B)

    def symbolic(self):
        return bfmf_get_symbolic(self.h)

    def stats(self):
        return bfmf_get_stats(self.h)

    def kernel_stats(self):
        return bfmf_get_kernel_stats(self.h)

    def gemm_tile_launches(self):
        return bfmf_get_gemm_tile_launches(self.h)

    def front(self, f, what):
        sym = self.symbolic()
        n = int(sym["send"][f] - sym["sbeg"][f] + sym["iu_ptr"][f + 1] - sym["iu_ptr"][f])
        if what == 2:
            n = int(sym["send"][f] - sym["sbeg"][f])
        return bfmf_get_front(self.h, f, what, n)

    def front_block(self, f, what, X):
        """Y = B X for block `what` of compressed front f (0 F11, 1 F11^-1, 2 F12, 3 F21, 4 S, 5 the
        contribution block in HOD-BF form)."""
        sym = self.symbolic()
        ns = int(sym["send"][f] - sym["sbeg"][f])
        nu = int(sym["iu_ptr"][f + 1] - sym["iu_ptr"][f])
        return bfmf_apply_front_block(self.h, f, what, X, ns if what <= 2 else nu)

    def close(self):
        if self.h:
            bfmf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ serving
def bfmf_default_server_opts():
    o = bfmf_server_opts()
    _lib.bfmf_default_server_opts(C.byref(o))
    return o


class Server:
    """Resident factorizations answering right-hand-side requests (continuous
    batching per model, models concurrent); see bfmf_server_* in bfmf.h."""

    def __init__(self, device=0, max_batch_rhs=64, hbm_budget=0, result_bytes=4 << 30, restart=30, max_iter=300,
                 rtol=1e-6, atol=1e-10, true_rtol=1e-3):
        o = bfmf_default_server_opts()
        o.max_batch_rhs, o.hbm_budget, o.result_bytes = max_batch_rhs, hbm_budget, result_bytes
        o.solve.restart, o.solve.max_iter, o.solve.rtol = restart, max_iter, rtol
        o.solve.atol, o.solve.true_rtol = atol, true_rtol
        self.s = _P()
        st = _lib.bfmf_server_create(device, C.byref(o), C.byref(self.s))
        if st != BFMF_OK:
            raise BfmfError(st, "server_create: " + _lib.bfmf_last_error(None).decode())
        self.n = {}

    def _err(self, st, what):
        raise BfmfError(st, what + ": " + _lib.bfmf_server_last_error(self.s).decode())

    def attach(self, solver):
        m = C.c_int32()
        st = _lib.bfmf_server_attach(self.s, solver.h, C.byref(m))
        if st != BFMF_OK:
            self._err(st, "server_attach")
        self.n[m.value] = solver.n
        return m.value

    def submit(self, model, colptr, rowind, values):
        """colptr (nrhs+1), rowind, complex values: the request's right-hand sides as sparse columns."""
        colptr = np.ascontiguousarray(colptr, dtype=np.int64)
        rowind = np.ascontiguousarray(rowind, dtype=np.int64)
        values = np.ascontiguousarray(values, dtype=np.complex128)
        t = C.c_uint64()
        st = _lib.bfmf_server_submit(self.s, model, colptr.shape[0] - 1, _ptr(colptr), _ptr(rowind), _ptr(values),
                                     C.byref(t))
        if st != BFMF_OK:
            self._err(st, "server_submit")
        return t.value

    def submit_points(self, model, rows, values=None):
        """One point source per column: column q is values[q] (default 1) at row rows[q]."""
        rows = np.asarray(rows, dtype=np.int64)
        vals = np.ones(rows.shape[0], dtype=np.complex128) if values is None else np.asarray(values)
        return self.submit(model, np.arange(rows.shape[0] + 1, dtype=np.int64), rows, vals)

    def wait(self, ticket, out=None, device_ptr=None, ld=None):
        """Waits for a request; its solution goes to the host array `out`
        (n x nrhs, column-major), to device memory at device_ptr (leading
        dimension ld), or is discarded.  Returns the request's info dict."""
        info = bfmf_request_info()
        if out is not None:
            st = _lib.bfmf_server_wait(self.s, ticket, C.byref(info), _ptr(out), out.shape[0], BFMF_HOST)
        elif device_ptr is not None:
            st = _lib.bfmf_server_wait(self.s, ticket, C.byref(info), C.c_void_p(device_ptr), ld, BFMF_DEVICE)
        else:
            st = _lib.bfmf_server_wait(self.s, ticket, C.byref(info), None, 0, BFMF_HOST)
        d = {k: getattr(info, k) for k, _ in bfmf_request_info._fields_}
        d["status"] = st
        return d

    def clock(self):
        return _lib.bfmf_server_clock(self.s)

    def close(self):
        if self.s:
            _lib.bfmf_server_destroy(self.s)
            self.s = None
