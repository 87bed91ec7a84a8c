"""Sequential CPU oracle for ParAC (ctypes binding over ``parac_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is the reference the GPU library is
checked against: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import it.  No product path calls it, and it
imports nothing from the GPU package.

What it computes follows the paper: the rchol elimination (Alg. 1, Alg. 2)
scheduled by the dependency counters of §III, in the scaled form
``L ~= F D F^T`` of §IV, and PCG as in §V's methodology.  The readings of
points the paper leaves open are listed at the top of ``parac_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "parac_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MODE_AUTO, MODE_LAPLACIAN, MODE_SDDM = 0, 1, 2
SCHED_LABEL, SCHED_ASYNC = 0, 1
DBG_DELETE_FIRST = 1
EV_CLAIM, EV_INSERT, EV_DEC, EV_ENQ, EV_INIT_DP, EV_INIT_Q = 1, 2, 3, 4, 5, 6
OK, EINVAL, ENOTLAP, ENOMEM, EINCONSISTENT, ENOCONV, EINTERNAL = 0, -1, -2, -4, -7, -8, -9


def build(force: bool = False) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` (gcc, C11, FP64,
    -O2 -ffp-contract=off, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
        os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "parac_oracle.h"))
    ):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-std=gnu11", "-O2", "-ffp-contract=off", "-fno-fast-math",
             "-Wall", "-Wextra", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


class _Res(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("mode", C.c_int32),
        ("n", C.c_int64), ("ntot", C.c_int64), ("nnz_off", C.c_int64),
        ("colptr", C.POINTER(C.c_int64)), ("rowind", C.POINTER(C.c_int32)),
        ("val", C.POINTER(C.c_double)), ("D", C.POINTER(C.c_double)),
        ("level", C.POINTER(C.c_int32)),
        ("rowptr_f", C.POINTER(C.c_int64)), ("colind_f", C.POINTER(C.c_int32)),
        ("val_f", C.POINTER(C.c_double)),
        ("n_input_edges", C.c_int64), ("n_fill", C.c_int64),
        ("max_gather", C.c_int64), ("max_deg", C.c_int64), ("depth", C.c_int64),
        ("n_zero_pivots", C.c_int64),
        ("n_choice", C.c_int64), ("choice_nopt", C.POINTER(C.c_int32)),
        ("choice_pick", C.POINTER(C.c_int32)), ("choice_prob", C.POINTER(C.c_double)),
        ("n_trace", C.c_int64), ("trace", C.POINTER(C.c_int64)),
        ("fill_count", C.POINTER(C.c_int32)),
    ]


class _PcgStats(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32),
                ("relres", C.c_double), ("true_relres", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _LIB if os.path.exists(_LIB) else build()
        L = C.CDLL(path)
        P = C.c_void_p
        L.orc_philox4x64_10.argtypes = [P, P, P]
        L.orc_classify.argtypes = [C.c_int64, P, P, P, C.c_int32, P, P]
        L.orc_factor.argtypes = [C.c_int64, P, P, P, P, C.c_uint64, C.c_int32, C.c_int32,
                                 C.c_uint64, C.c_int32, P, C.c_int64, C.c_int32, C.c_int32,
                                 C.c_int32, C.c_int32, C.POINTER(C.POINTER(_Res))]
        L.orc_factor_free.argtypes = [C.POINTER(_Res)]
        L.orc_apply.argtypes = [C.POINTER(_Res), P, P, P]
        L.orc_apply32.argtypes = [C.POINTER(_Res), P, P, P]
        L.orc_check_consistent.argtypes = [C.c_int64, P, P, P, C.c_int32, P]
        L.orc_pcg.argtypes = [C.c_int64, P, P, P, C.POINTER(_Res), P, P, C.c_double,
                              C.c_int32, C.c_int32, P, C.POINTER(_PcgStats)]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _csr(A):
    """(n, rowptr int64, col int32, val f64) from a scipy CSR matrix or any
    object with ``n, rowptr, col, val`` attributes."""
    if hasattr(A, "indptr"):
        return (A.shape[0], np.ascontiguousarray(A.indptr, np.int64),
                np.ascontiguousarray(A.indices, np.int32), np.ascontiguousarray(A.data, np.float64))
    return (int(A.n), np.ascontiguousarray(A.rowptr, np.int64),
            np.ascontiguousarray(A.col, np.int32), np.ascontiguousarray(A.val, np.float64))


def philox4x64_10(ctr, key):
    c = np.array(ctr, dtype=np.uint64)
    k = np.array(key, dtype=np.uint64)
    out = np.zeros(4, np.uint64)
    lib().orc_philox4x64_10(_p(c), _p(k), _p(out))
    return out


def classify(A, mode=MODE_AUTO):
    n, rp, ci, v = _csr(A)
    m = np.zeros(1, np.int32)
    ex = np.zeros(max(n, 1), np.float64)
    st = lib().orc_classify(n, _p(rp), _p(ci), _p(v), mode, _p(m), _p(ex))
    return st, int(m[0]), ex[:n]


def _arr(ptr, count, dtype):
    if count == 0 or not ptr:
        return np.zeros(0, dtype)
    return np.ctypeslib.as_array(ptr, shape=(count,)).astype(dtype, copy=True)


class Factor:
    """Result of :func:`factor`: canonical CSC of ``F`` (label space) and ``D``,
    with statistics.  Keeps the C result alive for :func:`apply`/:func:`pcg`."""

    def __init__(self, res_ptr, perm):
        self._ptr = res_ptr
        r = res_ptr.contents
        self.status = r.status
        self.perm = perm
        self.mode = r.mode
        self.n, self.ntot, self.nnz_off = r.n, r.ntot, r.nnz_off
        self.n_trace = r.n_trace
        self.trace = _arr(r.trace, 4 * r.n_trace, np.int64).reshape(-1, 4)
        if r.status == 0:
            self.colptr = _arr(r.colptr, r.ntot + 1, np.int64)
            self.rowind = _arr(r.rowind, r.nnz_off, np.int32)
            self.val = _arr(r.val, r.nnz_off, np.float64)
            self.D = _arr(r.D, r.ntot, np.float64)
            self.level = _arr(r.level, r.ntot, np.int32)
            self.rowptr_f = _arr(r.rowptr_f, r.ntot + 1, np.int64)
            self.colind_f = _arr(r.colind_f, r.nnz_off, np.int32)
            self.val_f = _arr(r.val_f, r.nnz_off, np.float64)
            self.fill_count = _arr(r.fill_count, r.ntot, np.int32)
            self.choice_nopt = _arr(r.choice_nopt, r.n_choice, np.int32)
            self.choice_pick = _arr(r.choice_pick, r.n_choice, np.int32)
            self.choice_prob = _arr(r.choice_prob, r.n_choice, np.float64)
            self.stats = dict(n_input_edges=r.n_input_edges, n_fill=r.n_fill,
                              max_gather=r.max_gather, max_deg=r.max_deg, depth=r.depth,
                              n_zero_pivots=r.n_zero_pivots, nnz_off=r.nnz_off)

    def __del__(self):
        if getattr(self, "_ptr", None) is not None and _lib is not None:
            _lib.orc_factor_free(self._ptr)
            self._ptr = None

    def dense_F(self):
        """Unit lower-triangular F (label space) as a dense array (tiny cases)."""
        F = np.eye(self.ntot)
        for k in range(self.ntot):
            for e in range(self.colptr[k], self.colptr[k + 1]):
                F[self.rowind[e], k] = self.val[e]
        return F


def factor(A, perm=None, seed=0, mode=MODE_AUTO, schedule=SCHED_LABEL, sched_seed=0,
           nworkers=1, forced=None, trace=False, debug_flags=0, samples=1):
    """The sequential elimination; samples > 1 is AC(k) with k = samples
    (R18).  forced: a 1-D sequence of offsets, one per draw in this
    schedule's order, or a 2-D table forced[k, s] keyed by pivot label and
    slot (-1: the draw)."""
    n, rp, ci, v = _csr(A)
    pm = None if perm is None else np.ascontiguousarray(perm, np.int32)
    fc = None if forced is None else np.ascontiguousarray(forced, np.int32)
    stride = 0
    if fc is not None and fc.ndim == 2:
        stride = int(fc.shape[1])
        fc = fc.reshape(-1)
    if fc is not None and fc.size == 0:
        fc = np.zeros(1, np.int32)
        nf = 0
    else:
        nf = 0 if fc is None else fc.size
    out = C.POINTER(_Res)()
    lib().orc_factor(n, _p(rp), _p(ci), _p(v), _p(pm), C.c_uint64(int(seed) & (2**64 - 1)),
                     mode, schedule, C.c_uint64(int(sched_seed) & (2**64 - 1)), nworkers,
                     _p(fc), nf, stride, 1 if trace else 0, debug_flags, int(samples),
                     C.byref(out))
    return Factor(out, pm)


def apply(fac: Factor, r, precision=0):
    r = np.ascontiguousarray(r, np.float64)
    z = np.zeros_like(r)
    fn = lib().orc_apply32 if precision else lib().orc_apply
    st = fn(fac._ptr, _p(fac.perm), _p(r), _p(z))
    if st:
        raise RuntimeError("oracle apply failed: %d" % st)
    return z


def check_consistent(A, mode, b):
    n, rp, ci, v = _csr(A)
    b = np.ascontiguousarray(b, np.float64)
    return lib().orc_check_consistent(n, _p(rp), _p(ci), _p(v), mode, _p(b))


def pcg(A, fac: Factor, b, rtol=1e-6, maxit=10000, precision=0):
    """PCG with x0 = 0 (returns x and a stats dict)."""
    n, rp, ci, v = _csr(A)
    b = np.ascontiguousarray(b, np.float64)
    x = np.zeros(n, np.float64)
    st = _PcgStats()
    lib().orc_pcg(n, _p(rp), _p(ci), _p(v), fac._ptr, _p(fac.perm), _p(b), rtol, maxit,
                  precision, _p(x), C.byref(st))
    return x, dict(status=st.status, iterations=st.iterations, relres=st.relres,
                   true_relres=st.true_relres)
