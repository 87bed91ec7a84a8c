"""Per-element rounding bound of the preconditioner apply.

Two implementations of z = P^T F^-T D^+ F^-1 P r that differ only in the
order in which each row's products are summed agree to within the bound
computed here.  A row value s - (p_1 + ... + p_m), summed in any order,
is within gamma_(m+1) (|s| + sum |p_j|) of its exact value (gamma_k =
k u / (1 - k u), u the unit roundoff), so two orders differ by at most
twice that.  A difference made at row i then travels through the rest of
the solve exactly as a change of the right-hand side does: through F^-1
forward, D^+, and F^-T backward.  F is unit lower triangular with
non-positive off-diagonal entries, so F^-1 and F^-T are entrywise
non-negative and the propagated bound is one more solve of each kind on the
(non-negative) local bounds.  The result is first order in u; the caller
multiplies it by a safety factor.
"""
import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import spsolve_triangular


def _gamma(k, u):
    k = np.asarray(k, dtype=np.float64)
    return k * u / (1.0 - k * u)


def apply_bound(fac, r, precision=0):
    """Bound on |z_a - z_b| for two applies of the oracle factor ``fac`` to
    ``r`` (original ordering) in FP64 (precision 0) or FP32 (precision 1)."""
    u = 2.0 ** -53 if precision == 0 else 2.0 ** -24
    n = fac.n
    ntot = fac.ntot
    F = sp.csc_matrix((fac.val, fac.rowind, fac.colptr), shape=(ntot, ntot))
    F = F[:n, :n].tocsr()  # SDDM: the ground row and column are not part of the apply
    if precision:
        F = sp.csr_matrix((F.data.astype(np.float32).astype(np.float64), F.indices, F.indptr),
                          shape=F.shape)
    L = (sp.identity(n, format="csr") + F).tocsr()
    Fa = abs(F).tocsr()
    D = fac.D[:n]
    Dp = np.where(D > 0, 1.0 / np.where(D > 0, D, 1.0), 0.0)
    if precision:
        Dp = Dp.astype(np.float32).astype(np.float64)
    perm = fac.perm if fac.perm is not None else np.arange(n, dtype=np.int32)
    pr = np.empty(n)
    pr[perm] = r
    if precision:
        pr = pr.astype(np.float32).astype(np.float64)
    if n == 0:
        return np.zeros(0)
    y = spsolve_triangular(L, pr, lower=True, unit_diagonal=True)
    mrow = np.diff(F.indptr)
    e = 2.0 * _gamma(mrow + 1, u) * (np.abs(pr) + Fa @ np.abs(y))
    dy = spsolve_triangular(L, e, lower=True, unit_diagonal=True)
    s = Dp * y
    LT = L.T.tocsr()
    x = spsolve_triangular(LT, s, lower=False, unit_diagonal=True)
    mcol = np.diff(F.tocsc().indptr)
    e2 = 2.0 * _gamma(mcol + 2, u) * (np.abs(s) + Fa.T @ np.abs(x)) + Dp * dy
    dx = spsolve_triangular(LT, e2, lower=False, unit_diagonal=True)
    return dx[perm]


def within_apply_bound(z, zr, fac, r, precision=0, safety=4.0):
    """True when every |z_i - zr_i| is within ``safety`` times the bound (an
    absolute floor of a few smallest normals covers zeros)."""
    tiny = 4.0 * (np.finfo(np.float64).tiny if precision == 0 else float(np.finfo(np.float32).tiny))
    bnd = safety * apply_bound(fac, r, precision) + tiny
    diff = np.abs(np.asarray(z) - np.asarray(zr))
    return bool(np.all(diff <= bnd)), float(np.max(diff / bnd)) if diff.size else 0.0
