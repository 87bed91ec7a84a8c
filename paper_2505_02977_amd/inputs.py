"""Seeded synthetic inputs: graphs, edge weights, elimination orders and
right-hand sides.

This module holds none of the method's arithmetic.  It builds the matrices
the solver is given (graph Laplacians in the sign convention of §V: positive
diagonal, non-positive off-diagonals, full symmetric CSR with the diagonal;
SDDM matrices with a non-negative diagonal excess) and the data both the GPU
library and the CPU oracle consume: the permutation ``perm[v] = label`` and
the right-hand side.

The paper measures SuiteSparse, Laplacians.jl, SPE10 and SDDM2023 matrices
(Table I, §V-C); none is available here, so these generators stand in for them
with the same shapes: 2D/3D grid stencils (the 3D Poisson family of Table I is
a 7-point stencil), power-law networks (Chung-Lu expected-degree model), and
random geometric graphs, with seeded weights.

Seeds: workload ``c`` uses ``seed_c = 2505029770 + c``; its sub-streams are
graph / weights / order / rhs / factor = ``splitmix64(seed_c + j)``, j = 0..4.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 2505029770
_M64 = (1 << 64) - 1

# optional progress callback (a function of one string) for the stages of
# the large generators
PROGRESS = None


def _note(msg):
    if PROGRESS is not None:
        PROGRESS(msg)


def splitmix64(x: int) -> int:
    """One SplitMix64 output for state ``x`` (Steele, Lea, Flood 2014)."""
    z = (int(x) + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def substream(seed_c: int, j: int) -> np.random.Generator:
    return np.random.default_rng(splitmix64(seed_c + j))


@dataclasses.dataclass
class CSR:
    """Full symmetric CSR (diagonal included), columns strictly increasing."""
    n: int
    rowptr: np.ndarray  # int64[n+1]
    col: np.ndarray     # int32[nnz]
    val: np.ndarray     # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))

    def to_dense(self):
        return self.to_scipy().toarray()


# --------------------------------------------------------------------------
# matrix assembly from an undirected weighted edge list
# --------------------------------------------------------------------------
def laplacian_from_edges(n, i, j, w, excess=None) -> CSR:
    """L = sum_e w_e (e_i - e_j)(e_i - e_j)^T (+ diag(excess)).

    ``i, j`` are edge endpoints (i != j, each undirected edge once), ``w > 0``.
    """
    i = np.asarray(i, np.int64)
    j = np.asarray(j, np.int64)
    w = np.asarray(w, np.float64)
    diag = np.bincount(i, weights=w, minlength=n) + np.bincount(j, weights=w, minlength=n)
    if excess is not None:
        diag = diag + np.asarray(excess, np.float64)
    ar = np.arange(n, dtype=np.int64)
    rows = np.concatenate([i, j, ar])
    cols = np.concatenate([j, i, ar])
    vals = np.concatenate([-w, -w, diag])
    # sort by (row, column): a stable counting sort by row after a stable
    # sort by column (scipy's compressed-format conversion does both)
    import scipy.sparse as sp
    _note("assembling %d x %d CSR from %d entries" % (n, n, len(rows)))
    m = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    if m.nnz != len(rows):
        raise ValueError("duplicate edge")
    m.sort_indices()
    return CSR(n, m.indptr.astype(np.int64), m.indices.astype(np.int32),
               m.data.astype(np.float64))


def dedupe_edges(i, j):
    """Undirected simple edge set (self-loops dropped, duplicates merged)."""
    i = np.asarray(i, np.int64)
    j = np.asarray(j, np.int64)
    keep = i != j
    a = np.minimum(i[keep], j[keep])
    b = np.maximum(i[keep], j[keep])
    nmax = int(max(a.max(initial=0), b.max(initial=0))) + 1
    key = np.unique(a * nmax + b)
    return key // nmax, key % nmax


def largest_component(n, i, j):
    """Vertices of the largest connected component, relabelled compactly in
    their original order: returns (n_lcc, i', j', keep_mask)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    _note("largest component of %d vertices, %d edges" % (n, len(i)))
    g = sp.coo_matrix((np.ones(len(i), np.int8), (i, j)), shape=(n, n))
    ncomp, lab = connected_components(g, directed=False)
    if ncomp == 1:
        return n, np.asarray(i), np.asarray(j), np.ones(n, bool)
    big = np.argmax(np.bincount(lab))
    keep = lab == big
    newid = np.full(n, -1, np.int64)
    newid[keep] = np.arange(int(keep.sum()))
    ek = keep[i]  # both ends share a component
    return int(keep.sum()), newid[i[ek]], newid[j[ek]], keep


# --------------------------------------------------------------------------
# graph families
# --------------------------------------------------------------------------
def grid2d_edges(nx, ny):
    """5-point stencil on an nx-by-ny grid (vertex id = x + nx*y)."""
    idx = np.arange(nx * ny, dtype=np.int64).reshape(ny, nx)
    h = (idx[:, :-1].ravel(), idx[:, 1:].ravel())
    v = (idx[:-1, :].ravel(), idx[1:, :].ravel())
    return np.concatenate([h[0], v[0]]), np.concatenate([h[1], v[1]])


def grid3d_edges(nx, ny, nz):
    """7-point stencil on an nx-by-ny-by-nz grid (id = x + nx*(y + ny*z))."""
    idx = np.arange(nx * ny * nz, dtype=np.int64).reshape(nz, ny, nx)
    parts = [(idx[:, :, :-1].ravel(), idx[:, :, 1:].ravel()),
             (idx[:, :-1, :].ravel(), idx[:, 1:, :].ravel()),
             (idx[:-1, :, :].ravel(), idx[1:, :, :].ravel())]
    return (np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts]))


def chung_lu_weights(N, dbar, beta):
    """Expected degrees w_i = w_max (i0/(i+i0))^(1/(beta-1)) with the
    structural cutoff w_max = sqrt(N dbar) and i0 set so mean(w) = dbar."""
    wmax = math.sqrt(N * dbar)
    gam = 1.0 / (beta - 1.0)
    ii = np.arange(N, dtype=np.float64)

    def mean_w(i0):
        return float(np.mean(wmax * (i0 / (ii + i0)) ** gam))

    lo, hi = 1e-6, float(N)
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if mean_w(mid) < dbar:
            lo = mid
        else:
            hi = mid
        if hi / lo < 1 + 1e-12:
            break
    i0 = math.sqrt(lo * hi)
    return wmax * (i0 / (ii + i0)) ** gam


def _draw(cdf, r):
    """searchsorted(cdf, r, side="right"), with the queries visited in sorted
    order (the same result; far fewer cache misses on a large cdf)."""
    o = np.argsort(r)
    out = np.empty(len(r), np.int64)
    out[o] = np.searchsorted(cdf, r[o], side="right")
    return out


def chung_lu_edges(N, dbar, beta, rng):
    """Expected-degree random graph: round(N dbar / 2) endpoint pairs drawn
    i.i.d. with probability proportional to w, self-loops dropped and
    duplicates merged."""
    w = chung_lu_weights(N, dbar, beta)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    M = int(round(N * dbar / 2))
    out_i, out_j = [], []
    chunk = 1 << 24
    for s in range(0, M, chunk):
        _note("Chung-Lu endpoints %d of %d" % (s, M))
        m = min(chunk, M - s)
        a = _draw(cdf, rng.random(m))
        b = _draw(cdf, rng.random(m))
        out_i.append(np.minimum(a, N - 1))
        out_j.append(np.minimum(b, N - 1))
    _note("deduplicating %d edges" % M)
    return dedupe_edges(np.concatenate(out_i), np.concatenate(out_j))


def rgg_edges(N, dbar, rng):
    """Random geometric graph: N uniform points in the unit square joined
    when closer than r = sqrt(dbar / (pi N))."""
    from scipy.spatial import cKDTree
    pts = rng.random((N, 2))
    r = math.sqrt(dbar / (math.pi * N))
    pairs = cKDTree(pts).query_pairs(r, output_type="ndarray")
    return pairs[:, 0].astype(np.int64), pairs[:, 1].astype(np.int64)


# --------------------------------------------------------------------------
# orders and right-hand sides
# --------------------------------------------------------------------------
def perm_random(n, rng) -> np.ndarray:
    """Uniformly random elimination order, perm[v] = label of vertex v."""
    return rng.permutation(n).astype(np.int32)


def perm_nnz_sorted(A: CSR, rng) -> np.ndarray:
    """NNZ-sorted order (§V orderings): ascending row nonzero count, ties
    broken randomly; perm[v] = label."""
    deg = np.diff(A.rowptr)
    tie = rng.random(A.n)
    order = np.lexsort((tie, deg))          # vertices in elimination order
    perm = np.empty(A.n, np.int32)
    perm[order] = np.arange(A.n, dtype=np.int32)
    return perm


def rhs(n, rng, nrhs=1, center=True) -> np.ndarray:
    """N(0,1) right-hand side(s), each column centred in FP64 (b orthogonal
    to the all-ones null vector of a connected Laplacian).  Shape (n,) or
    (n, nrhs) row-major."""
    b = rng.standard_normal((n, nrhs)) if nrhs > 1 else rng.standard_normal(n)
    if center:
        b = b - b.mean(axis=0)
    return np.ascontiguousarray(b)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    A: CSR
    perm: np.ndarray
    b: np.ndarray
    seed: int            # factor (Philox) seed
    meta: dict


def _finish(name, c, n, i, j, w, excess=None, nrhs=1, center=True, meta=None):
    seed_c = BASE_SEED + c
    A = laplacian_from_edges(n, i, j, w, excess)
    _note("order and right-hand side")
    perm = perm_random(n, substream(seed_c, 2))
    b = rhs(n, substream(seed_c, 3), nrhs=nrhs, center=center)
    m = dict(n=n, edges=int(len(i)), nnz=A.nnz, seed_c=seed_c)
    m.update(meta or {})
    return Workload(name, A, perm, b, splitmix64(seed_c + 4), m)


def with_nnz_order(W: Workload) -> Workload:
    """The workload with its random order replaced by the NNZ-sorted one
    (ties broken by sub-stream 5 of the workload's seed)."""
    perm = perm_nnz_sorted(W.A, substream(W.meta["seed_c"], 5))
    return dataclasses.replace(W, perm=perm)


def grid2d_workload(side=64, c=1):
    """2D 5-point grid Laplacian side x side, weights U[1,2], random order,
    one centred N(0,1) right-hand side."""
    seed_c = BASE_SEED + c
    i, j = grid2d_edges(side, side)
    w = 1.0 + substream(seed_c, 1).random(len(i))
    return _finish("grid2d_%d" % side, c, side * side, i, j, w, meta=dict(side=side))


def grid3d_workload(side=128, c=2):
    """3D 7-point grid Laplacian side^3, weights log-uniform in [1e-2, 1e2]
    (a high-contrast coefficient field), random order, one RHS."""
    seed_c = BASE_SEED + c
    i, j = grid3d_edges(side, side, side)
    w = 10.0 ** substream(seed_c, 1).uniform(-2.0, 2.0, len(i))
    return _finish("grid3d_%d" % side, c, side ** 3, i, j, w, meta=dict(side=side))


def chung_lu_workload(log2n=22, dbar=16.0, beta=2.1, nrhs=1, c=3):
    """Chung-Lu power-law Laplacian on the largest component, weights in
    (0, 1], random order, nrhs centred N(0,1) right-hand sides."""
    seed_c = BASE_SEED + c
    N = 1 << log2n
    i, j = chung_lu_edges(N, dbar, beta, substream(seed_c, 0))
    n, i, j, _ = largest_component(N, i, j)
    w = 1.0 - substream(seed_c, 1).random(len(i))
    return _finish("chunglu_2^%d_d%g" % (log2n, dbar), c, n, i, j, w, nrhs=nrhs,
                   meta=dict(N_generated=N, dbar=dbar, beta=beta, nrhs=nrhs))


SDDM_FAMILIES = ("grid2d", "grid3d", "chunglu", "rgg")


def _sddm_draws(k, nmin, nmax, c):
    seed_c = BASE_SEED + c
    rng = np.random.default_rng(splitmix64(seed_c * 1000003 + k))
    N = int(round(10 ** rng.uniform(math.log10(nmin), math.log10(nmax))))
    fam = int(rng.integers(0, 4))
    dbar = float(rng.integers(8, 17))
    return rng, N, fam, dbar


def sddm_system_plan(k, nmin=1e3, nmax=1e6, c=4):
    """Requested size and family of system ``k`` of the serving stream,
    without building it."""
    _, N, fam, dbar = _sddm_draws(k, nmin, nmax, c)
    return N, SDDM_FAMILIES[fam], dbar


def sddm_system(k, nmin=1e3, nmax=1e6, c=4):
    """System ``k`` of the serving stream: size log-uniform in [nmin, nmax],
    family uniform over {2D grid, 3D grid, Chung-Lu (beta 2.1), RGG}, average
    degree uniform in {8..16} for the random families, largest component,
    excess U[0,1] on ceil(0.1 n) random vertices, weights U(0,1] on even k and
    unit on odd k, one N(0,1) right-hand side (SDDM: nonsingular)."""
    rng, N, fam, dbar = _sddm_draws(k, nmin, nmax, c)
    seed_c = BASE_SEED + c
    if fam == 0:
        s = max(2, int(round(math.sqrt(N))))
        n, (i, j) = s * s, grid2d_edges(s, s)
        fname = "grid2d"
    elif fam == 1:
        s = max(2, int(round(N ** (1.0 / 3.0))))
        n, (i, j) = s ** 3, grid3d_edges(s, s, s)
        fname = "grid3d"
    elif fam == 2:
        i, j = chung_lu_edges(N, dbar, 2.1, rng)
        n, i, j, _ = largest_component(N, i, j)
        fname = "chunglu"
    else:
        i, j = rgg_edges(N, dbar, rng)
        n, i, j, _ = largest_component(N, i, j)
        fname = "rgg"
    w = (1.0 - rng.random(len(i))) if k % 2 == 0 else np.ones(len(i))
    excess = np.zeros(n)
    hot = rng.choice(n, size=int(math.ceil(0.1 * n)), replace=False)
    excess[hot] = rng.random(len(hot))
    A = laplacian_from_edges(n, i, j, w, excess)
    perm = perm_random(n, rng)
    b = rng.standard_normal(n)
    return Workload("sddm_%03d_%s" % (k, fname), A, perm, b,
                    splitmix64(seed_c * 7919 + k),
                    dict(n=n, edges=int(len(i)), nnz=A.nnz, family=fname, dbar=dbar,
                         weighted=(k % 2 == 0)))


def poisson_arrivals(count, rate, c=4):
    """Arrival times of a Poisson process with the given rate (per second)."""
    rng = np.random.default_rng(splitmix64((BASE_SEED + c) * 31 + 7))
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


# --------------------------------------------------------------------------
# tiny graphs for pins
# --------------------------------------------------------------------------
def path_edges(n):
    a = np.arange(n - 1)
    return a, a + 1


def cycle_edges(n):
    a = np.arange(n)
    return a, (a + 1) % n


def complete_edges(n):
    i, j = np.triu_indices(n, 1)
    return i.astype(np.int64), j.astype(np.int64)


def random_tree_edges(n, rng):
    """Random recursive tree: vertex v > 0 attaches to a uniform earlier one."""
    v = np.arange(1, n)
    parent = np.array([rng.integers(0, x) for x in v], np.int64)
    return parent, v


def connected_random_edges(n, extra, rng):
    """A random spanning tree plus ``extra`` random chords (simple graph)."""
    ti, tj = random_tree_edges(n, rng)
    ci = rng.integers(0, n, extra)
    cj = rng.integers(0, n, extra)
    return dedupe_edges(np.concatenate([ti, ci]), np.concatenate([tj, cj]))
