"""Thin Python binding of the C ABI declared in ``include/parac.h``.

Argument marshalling only: every step of the factorisation and the solves
runs in the library's HIP kernels.  PyTorch supplies device memory and the
stream.  The library must be built (``paper_2505_02977_amd/build.py``); if it
is missing this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libparac.so")

OK, EINVAL, ENOTLAP, EPOOL, ENOMEM, ETIMEOUT, EDEVICE, EINCONSISTENT, ENOCONV, EINTERNAL = (
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9)
MODE_AUTO, MODE_LAPLACIAN, MODE_SDDM = 0, 1, 2
ORDER_RANDOM, ORDER_NNZ, ORDER_MIS = 0, 1, 2
PREC_FP64, PREC_MIXED = 0, 1


class ParacError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (status %d)" % (msg, status))
        self.status = status


class parac_csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p), ("on_device", C.c_int32)]


class parac_factor_opts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("perm", C.c_void_p), ("mode", C.c_int32),
                ("pool_factor", C.c_double), ("workers", C.c_int32), ("keep_fp32", C.c_int32),
                ("timeout_s", C.c_double), ("tail_fraction", C.c_double), ("samples", C.c_int32)]


class parac_factor_stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("ntot", C.c_int64), ("mode", C.c_int32),
                ("nnz_off", C.c_int64), ("n_input_edges", C.c_int64), ("n_fill", C.c_int64),
                ("max_gather", C.c_int64), ("max_deg", C.c_int64), ("depth", C.c_int64),
                ("n_zero_pivots", C.c_int64), ("workers", C.c_int32), ("retries", C.c_int32),
                ("pool_factor", C.c_double), ("ms_setup", C.c_double),
                ("ms_eliminate", C.c_double), ("ms_finalize", C.c_double),
                ("ms_total", C.c_double), ("narrow_levels", C.c_int64)]


class parac_pcg_opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("maxit", C.c_int32), ("precision", C.c_int32),
                ("check_every", C.c_int32), ("timing", C.c_int32)]


class parac_pcg_stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("relres", C.c_double),
                ("true_relres", C.c_double), ("ms_total", C.c_double), ("ms_apply", C.c_double),
                ("applies", C.c_int32), ("ms_fwd", C.c_double)]


class parac_block_shape(C.Structure):
    _fields_ = [("cols_per_sweep", C.c_int32), ("workgroups", C.c_int32), ("source", C.c_int32),
                ("ms", C.c_float)]


class parac_request(C.Structure):
    _fields_ = [("A", parac_csr), ("perm", C.c_void_p), ("b", C.c_void_p), ("x", C.c_void_p),
                ("seed", C.c_uint64), ("rtol", C.c_double), ("arrival_s", C.c_double)]


class parac_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("true_relres", C.c_double),
                ("t_arrive", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("bytes_resident", C.c_int64)]


class parac_host_factor(C.Structure):
    _fields_ = [("n", C.c_int64), ("ntot", C.c_int64), ("mode", C.c_int32), ("threads", C.c_int32),
                ("nnz_off", C.c_int64), ("n_fill", C.c_int64), ("depth", C.c_int64),
                ("colptr", C.POINTER(C.c_int64)), ("rowind", C.POINTER(C.c_int32)),
                ("val", C.POINTER(C.c_double)), ("D", C.POINTER(C.c_double)),
                ("level", C.POINTER(C.c_int32)), ("ms_total", C.c_double)]


class parac_serve_opts(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("max_slots", C.c_int32), ("precision", C.c_int32),
                ("maxit", C.c_int32), ("check_every", C.c_int32)]


_lib = None


def lib():
    """Load libparac.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (loads the HIP runtime the library binds to)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libparac.so is not built: run paper_2505_02977_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.parac_factor.argtypes = [C.POINTER(parac_csr), C.POINTER(parac_factor_opts), P,
                                   C.POINTER(P)]
        L.parac_factor_info.argtypes = [P, C.POINTER(parac_factor_stats)]
        L.parac_debug_factor_forced.argtypes = [C.POINTER(parac_csr), C.POINTER(parac_factor_opts),
                                                P, C.c_int32, C.c_int64, P, C.POINTER(P)]
        L.parac_debug_factor_forced.restype = C.c_int
        L.parac_factor_export.argtypes = [P, P, P, P, P, P]
        L.parac_apply.argtypes = [P, P, P, C.c_int64, C.c_int32, P]
        L.parac_pcg.argtypes = [C.POINTER(parac_csr), P, P, P, C.c_int64,
                                C.POINTER(parac_pcg_opts), C.POINTER(parac_pcg_stats), P]
        L.parac_pcg_static.argtypes = [C.POINTER(parac_csr), P, P, P, C.POINTER(parac_pcg_opts),
                                       C.POINTER(parac_pcg_stats), P]
        L.parac_order.argtypes = [C.POINTER(parac_csr), C.c_int32, C.c_uint64, P,
                                  C.POINTER(C.c_int32), P]
        L.parac_order.restype = C.c_int
        L.parac_device_bytes.argtypes = [C.c_int32]
        L.parac_device_bytes.restype = C.c_int64
        L.parac_pcg_static_max_rows.argtypes = []
        L.parac_pcg_static_max_rows.restype = C.c_int64
        L.parac_serve.argtypes = [C.POINTER(parac_request), C.c_int64,
                                  C.POINTER(parac_serve_opts), C.POINTER(parac_result)]
        L.parac_block_shape_set.argtypes = [P, C.c_int32, C.c_int32, C.POINTER(parac_block_shape)]
        L.parac_block_shape_get.argtypes = [P, C.c_int32, C.c_int32, C.POINTER(parac_block_shape)]
        L.parac_factor_host.argtypes = [C.POINTER(parac_csr), C.POINTER(parac_factor_opts),
                                        C.c_int32, C.POINTER(parac_host_factor)]
        L.parac_factor_host.restype = C.c_int
        L.parac_host_factor_free.argtypes = [C.POINTER(parac_host_factor)]
        L.parac_host_factor_free.restype = None
        L.parac_host_last_error.restype = C.c_char_p
        L.parac_factor_free.argtypes = [P]
        L.parac_status_str.restype = C.c_char_p
        L.parac_status_str.argtypes = [C.c_int]
        L.parac_last_error.restype = C.c_char_p
        for name in ("parac_factor", "parac_factor_info", "parac_factor_export", "parac_apply",
                     "parac_pcg", "parac_pcg_static", "parac_serve", "parac_block_shape_set",
                     "parac_block_shape_get"):
            getattr(L, name).restype = C.c_int
        L.parac_factor_free.restype = None
        _lib = L
    return _lib


def _raise(st):
    if st != OK:
        raise ParacError(st, lib().parac_last_error().decode())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class DeviceCSR:
    """A CSR matrix resident on the device (torch tensors) and its ABI view."""

    def __init__(self, A, device="cuda"):
        import torch
        self.n = int(A.n)
        self.rowptr = torch.as_tensor(np.ascontiguousarray(A.rowptr, np.int64), device=device)
        self.col = torch.as_tensor(np.ascontiguousarray(A.col, np.int32), device=device)
        self.val = torch.as_tensor(np.ascontiguousarray(A.val, np.float64), device=device)
        self.c = parac_csr(self.n, int(self.col.numel()), self.rowptr.data_ptr(),
                           self.col.data_ptr(), self.val.data_ptr(), 1)


class Factor:
    """Owns a parac_factor_t."""

    def __init__(self, handle):
        self.h = handle

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.parac_factor_free(self.h)
            self.h = None

    def info(self) -> dict:
        s = parac_factor_stats()
        _raise(lib().parac_factor_info(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in parac_factor_stats._fields_}

    def export(self):
        """(colptr, rowind, val, D, level) as numpy arrays (label space)."""
        s = self.info()
        ntot, nnz = s["ntot"], s["nnz_off"]
        colptr = np.zeros(ntot + 1, np.int64)
        rowind = np.zeros(max(nnz, 1), np.int32)
        val = np.zeros(max(nnz, 1), np.float64)
        D = np.zeros(max(ntot, 1), np.float64)
        lev = np.zeros(max(ntot, 1), np.int32)
        p = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
        _raise(lib().parac_factor_export(self.h, p(colptr), p(rowind), p(val), p(D), p(lev)))
        return colptr, rowind[:nnz], val[:nnz], D[:ntot], lev[:ntot]


def parac_factor(A: DeviceCSR, perm=None, seed=0, mode=MODE_AUTO, pool_factor=4.0, workers=0,
                 keep_fp32=False, timeout_s=30.0, tail_fraction=0.0, samples=1,
                 stream=None, forced=None) -> Factor:
    """samples = k > 1 builds the AC(k) factor (k sampling slots per entry).
    forced (test hook): a 2-D int array, forced[k, s] the partner offset of
    slot s of pivot label k (-1: drawn), passed to parac_debug_factor_forced."""
    import torch
    pt = None
    if perm is not None:
        pt = torch.as_tensor(np.ascontiguousarray(perm, np.int32), device=A.rowptr.device)
    o = parac_factor_opts(int(seed) & (2**64 - 1), pt.data_ptr() if pt is not None else None,
                          mode, pool_factor, workers, 1 if keep_fp32 else 0, timeout_s,
                          tail_fraction, samples)
    h = C.c_void_p()
    if forced is None:
        _raise(lib().parac_factor(C.byref(A.c), C.byref(o), _stream(stream), C.byref(h)))
    else:
        fa = np.ascontiguousarray(forced, np.int32)
        assert fa.ndim == 2
        _raise(lib().parac_debug_factor_forced(
            C.byref(A.c), C.byref(o), fa.ctypes.data_as(C.c_void_p), int(fa.shape[1]),
            int(fa.size), _stream(stream), C.byref(h)))
    return Factor(h)


def parac_apply(f: Factor, r, z, precision=PREC_FP64, stream=None):
    """z = M^+ r for contiguous float64 device tensors r, z of shape (n,)
    or (n, nrhs)."""
    nrhs = 1 if r.dim() == 1 else int(r.shape[1])
    _raise(lib().parac_apply(f.h, C.c_void_p(r.data_ptr()), C.c_void_p(z.data_ptr()), nrhs,
                             precision, _stream(stream)))
    return z


def parac_block_shape_set(f: Factor, cols, precision=PREC_FP64, cols_per_sweep=None,
                          workgroups=0):
    """Fix the block-apply shape for chunks of `cols` columns: sweep slots of
    `cols_per_sweep` columns (1, 2, 4; 8 with the FP32 apply), at most
    `workgroups` sweep workgroups per slot (0 = as its units need).
    cols_per_sweep=None forgets it (the next use takes the cache file's shape
    or times the candidates)."""
    sh = None if cols_per_sweep is None else C.byref(
        parac_block_shape(cols_per_sweep, workgroups, 0, 0.0))
    _raise(lib().parac_block_shape_set(f.h, cols, precision, sh))


SHAPE_SOURCES = {0: "fixed", 1: "timed", 2: "cache"}


def parac_block_shape_get(f: Factor, cols, precision=PREC_FP64):
    """The shape in use for (cols, precision): dict with cols_per_sweep,
    workgroups, source ('fixed', 'timed' or 'cache') and ms (time of one
    block apply when it was timed)."""
    sh = parac_block_shape()
    _raise(lib().parac_block_shape_get(f.h, cols, precision, C.byref(sh)))
    return dict(cols_per_sweep=sh.cols_per_sweep, workgroups=sh.workgroups,
                source=SHAPE_SOURCES.get(sh.source, str(sh.source)), ms=float(sh.ms))


def parac_pcg(A: DeviceCSR, f: Factor, b, x, nrhs=None, rtol=1e-6, maxit=10000,
              precision=PREC_FP64, check_every=8, timing=False, stream=None):
    """PCG (x0 = 0) on contiguous device tensors b, x of shape (n,) or
    (n, nrhs).  Returns a list of per-column stat dicts; raises on
    EINVAL/EINCONSISTENT."""
    if nrhs is None:
        nrhs = 1 if b.dim() == 1 else int(b.shape[1])
    o = parac_pcg_opts(rtol, maxit, precision, check_every, 1 if timing else 0)
    st = (parac_pcg_stats * nrhs)()
    rc = lib().parac_pcg(C.byref(A.c), f.h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                         nrhs, C.byref(o), st, _stream(stream))
    if rc not in (OK, ENOCONV):
        _raise(rc)
    return [dict(status=s.status, iterations=s.iterations, relres=s.relres,
                 true_relres=s.true_relres, ms_total=s.ms_total, ms_apply=s.ms_apply,
                 applies=s.applies, ms_fwd=s.ms_fwd) for s in st]


def parac_pcg_static(A: DeviceCSR, f: Factor, b, x, rtol=1e-6, maxit=10000,
                     precision=PREC_FP64, check_every=8, stream=None):
    """parac_pcg_static: single right-hand-side PCG whose per-call buffers
    live in the library's fixed device array (no device allocation).
    Returns one stat dict; raises on EINVAL/EINCONSISTENT."""
    o = parac_pcg_opts(rtol, maxit, precision, check_every, 0)
    st = parac_pcg_stats()
    rc = lib().parac_pcg_static(C.byref(A.c), f.h, C.c_void_p(b.data_ptr()),
                                C.c_void_p(x.data_ptr()), C.byref(o), C.byref(st),
                                _stream(stream))
    if rc not in (OK, ENOCONV):
        _raise(rc)
    return dict(status=st.status, iterations=st.iterations, relres=st.relres,
                true_relres=st.true_relres, applies=st.applies)


def parac_order(A, kind, seed=0, stream=None):
    """An elimination order computed on the device (parac_order): A is a
    DeviceCSR (the result is computed from its device arrays) or a host CSR
    with n, rowptr, col.  Returns (perm as an int32 numpy array, MIS rounds)."""
    rounds = C.c_int32(0)
    if isinstance(A, DeviceCSR):
        import torch
        perm = torch.empty(max(A.n, 1), dtype=torch.int32, device=A.rowptr.device)
        rc = lib().parac_order(C.byref(A.c), kind, int(seed) & (2**64 - 1),
                               C.c_void_p(perm.data_ptr()), C.byref(rounds), _stream(stream))
        _raise(rc)
        return perm.cpu().numpy()[:A.n], rounds.value
    n = int(A.n)
    rowptr = np.ascontiguousarray(A.rowptr, np.int64)
    col = np.ascontiguousarray(A.col, np.int32)
    csr = parac_csr(n, int(col.size), rowptr.ctypes.data, col.ctypes.data, None, 0)
    perm = np.empty(max(n, 1), np.int32)
    _raise(lib().parac_order(C.byref(csr), kind, int(seed) & (2**64 - 1), perm.ctypes.data,
                             C.byref(rounds), _stream(stream)))
    return perm[:n], rounds.value


def device_bytes(what=0):
    """Device bytes the library holds: 0 now, 1 the peak since the last
    reset, 2 reset the peak to now (parac_device_bytes)."""
    return int(lib().parac_device_bytes(what))


def pcg_static_max_rows():
    """Largest system (rows, ground vertex included) parac_pcg_static takes."""
    return int(lib().parac_pcg_static_max_rows())


def parac_factor_host(A, perm=None, seed=0, mode=MODE_AUTO, pool_factor=4.0, threads=0):
    """The CPU factorisation on the host's cores (parac_factor_host): A is a
    host CSR (n, rowptr, col, val).  Returns a dict with the canonical CSC
    (colptr, rowind, val), D, level (numpy copies) and statistics."""
    n = int(A.n)
    rowptr = np.ascontiguousarray(A.rowptr, np.int64)
    col = np.ascontiguousarray(A.col, np.int32)
    val = np.ascontiguousarray(A.val, np.float64)
    pm = None if perm is None else np.ascontiguousarray(perm, np.int32)
    csr = parac_csr(n, int(col.size), rowptr.ctypes.data, col.ctypes.data, val.ctypes.data, 0)
    o = parac_factor_opts(int(seed) & (2**64 - 1), None if pm is None else pm.ctypes.data, mode,
                          pool_factor, 0, 0, 0.0, 0.0, 1)
    out = parac_host_factor()
    rc = lib().parac_factor_host(C.byref(csr), C.byref(o), threads, C.byref(out))
    if rc != OK:
        raise ParacError(rc, lib().parac_host_last_error().decode())
    try:
        nt, m = out.ntot, out.nnz_off

        def arr(ptr, count, dtype):
            if count == 0:
                return np.zeros(0, dtype)
            return np.ctypeslib.as_array(ptr, shape=(count,)).astype(dtype, copy=True)
        res = dict(colptr=arr(out.colptr, nt + 1, np.int64), rowind=arr(out.rowind, m, np.int32),
                   val=arr(out.val, m, np.float64), D=arr(out.D, nt, np.float64),
                   level=arr(out.level, nt, np.int32), n=out.n, ntot=nt, mode=out.mode,
                   nnz_off=m, n_fill=out.n_fill, depth=out.depth, threads=out.threads,
                   ms_total=out.ms_total)
    finally:
        lib().parac_host_factor_free(C.byref(out))
    return res


def parac_serve(requests, hbm_budget=0, max_slots=0, precision=PREC_FP64, maxit=0,
                check_every=0):
    """Serve a stream of systems.  Each request is a dict with A (host CSR
    with n, rowptr, col, val), b, and optionally perm, seed, rtol and
    arrival_s.  Returns (results, xs): per-request result dicts and solution
    arrays (host float64)."""
    keep, xs = [], []
    reqs = (parac_request * len(requests))()
    for k, rq in enumerate(requests):
        A = rq["A"]
        n = int(A.n)
        rowptr = np.ascontiguousarray(A.rowptr, np.int64)
        col = np.ascontiguousarray(A.col, np.int32)
        val = np.ascontiguousarray(A.val, np.float64)
        b = np.ascontiguousarray(rq["b"], np.float64)
        perm = rq.get("perm")
        perm = None if perm is None else np.ascontiguousarray(perm, np.int32)
        x = np.zeros(max(n, 1), np.float64)
        keep.append((rowptr, col, val, b, perm))
        xs.append(x)
        p = lambda a: a.ctypes.data if a is not None else None  # noqa: E731
        reqs[k] = parac_request(parac_csr(n, int(col.size), p(rowptr), p(col), p(val), 0),
                                p(perm), p(b), p(x), int(rq.get("seed", 0)) & (2**64 - 1),
                                float(rq.get("rtol", 1e-6)), float(rq.get("arrival_s", 0.0)))
    out = (parac_result * len(requests))()
    o = parac_serve_opts(int(hbm_budget), max_slots, precision, maxit, check_every)
    _raise(lib().parac_serve(reqs, len(requests), C.byref(o), out))
    res = [{k: getattr(r, k) for k, _ in parac_result._fields_} for r in out]
    return res, [x[:int(rq["A"].n)] for x, rq in zip(xs, requests)]


def status_str(st):
    return lib().parac_status_str(st).decode()
