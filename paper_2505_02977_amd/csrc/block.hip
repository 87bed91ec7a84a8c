// block.hip -- the PCG kernels of several right-hand sides at once, on
// row-major blocks of nc <= 64 columns.  The preconditioner apply of a block
// runs in the dependency-driven sweeps (ready.hip), a slot per chunk of
// columns.
#include "device.hpp"
#include "internal.hpp"

namespace parac {

// ==========================================================================
// Block PCG.  One lane per column (G = 2^gshift >= nc lanes per row), rows
// in a grid-stride loop; per-column partial sums are reduced per block by a
// fixed LDS tree over the block's row groups and written as
// partial[block * nc + j], then summed in a fixed order by k_breduce.
//
// Per column j: bst[8j + ...] = ||b||^2, r.z, p.q, r.r, alpha, beta, rtol,
// true ||b - Ax||^2; bist[4j + ...] = iterations, done.  gfl[0] counts the
// columns still iterating, gfl[1] = 1 once none is (every kernel then
// returns at once).
// ==========================================================================
constexpr int kBRedT = 256;
constexpr int kBRedBlocks = 512;

// sum v over the row groups of the block; column j's total lands in sh[j]
__device__ __forceinline__ void colsum(double v, double *sh, int gshift) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = (kBRedT >> gshift) / 2; o > 0; o >>= 1) {
    if ((t >> gshift) < o) sh[t] = sh[t] + sh[t + (o << gshift)];
    __syncthreads();
  }
}

__device__ __forceinline__ void write_partials(double v, double *sh, int gshift, int nc,
                                               double *partial) {
  colsum(v, sh, gshift);
  if ((int)threadIdx.x < nc) partial[(int64_t)blockIdx.x * nc + threadIdx.x] = sh[threadIdx.x];
}

struct RowIter {
  int64_t row, stride;
  int j;
  __device__ RowIter(int gshift) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    row = t >> gshift;
    stride = ((int64_t)gridDim.x * blockDim.x) >> gshift;
    j = (int)(t & ((1 << gshift) - 1));
  }
};

// x = 0, r = b, partial b.b
__global__ __launch_bounds__(kBRedT) void k_binit(int64_t n, int nc, int gshift,
                                                  const double *__restrict__ b, int64_t ldb,
                                                  double *x, int64_t ldx, double *r, double *p,
                                                  double *partial) {
  __shared__ double sh[kBRedT];
  RowIter it(gshift);
  double acc = 0.0;
  if (it.j < nc)
    for (int64_t i = it.row; i < n; i += it.stride) {
      const double v = b[i * ldb + it.j];
      x[i * ldx + it.j] = 0.0;
      r[i * nc + it.j] = v;
      p[i * nc + it.j] = 0.0;
      acc = acc + v * v;
    }
  write_partials(acc, sh, gshift, nc, partial);
}

// q = A p, partial p.q.  The G lanes of a row load up to G of its entries
// (index and value) together, share them by shuffles, and issue the gathers
// of p for eight entries before adding any: the additions keep entry order
// (a left fold per column), and the gathers no longer wait one by one.
constexpr int kBSpmvBatch = 8;
__global__ __launch_bounds__(kBRedT) void k_bspmv_dot(int64_t n, int nc, int gshift,
                                                      const int64_t *__restrict__ rowptr,
                                                      const int32_t *__restrict__ col,
                                                      const double *__restrict__ val,
                                                      const double *__restrict__ p, double *q,
                                                      double *partial, const int *skip) {
  __shared__ double sh[kBRedT];
  if (*skip) return;
  RowIter it(gshift);
  const int G = 1 << gshift;
  const bool colv = it.j < nc;
  double acc = 0.0;
  for (int64_t i = it.row; i < n; i += it.stride) {
    double s = 0.0;
    const int64_t e0 = rowptr[i], e1 = rowptr[i + 1];
    for (int64_t b = e0; b < e1; b += G) {
      const int64_t kk = b + it.j;
      const int32_t cl = kk < e1 ? col[kk] : 0;
      const double vl = kk < e1 ? val[kk] : 0.0;
      const int m = e1 - b < G ? (int)(e1 - b) : G;
      for (int t0 = 0; t0 < m; t0 += kBSpmvBatch) {
        double vv[kBSpmvBatch], pv[kBSpmvBatch];
#pragma unroll
        for (int u = 0; u < kBSpmvBatch; ++u) {
          const int t = t0 + u < G ? t0 + u : G - 1;
          const int c = __shfl(cl, t, G);
          vv[u] = __shfl(vl, t, G);
          pv[u] = (t0 + u < m && colv) ? p[(int64_t)c * nc + it.j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kBSpmvBatch; ++u)
          if (t0 + u < m) s = s + vv[u] * pv[u];
      }
    }
    if (colv) {
      q[i * nc + it.j] = s;
      acc = acc + p[i * nc + it.j] * s;
    }
  }
  write_partials(acc, sh, gshift, nc, partial);
}

// y = b - A x, partial y.y
__global__ __launch_bounds__(kBRedT) void k_bresidual(int64_t n, int nc, int gshift,
                                                      const int64_t *__restrict__ rowptr,
                                                      const int32_t *__restrict__ col,
                                                      const double *__restrict__ val,
                                                      const double *__restrict__ x, int64_t ldx,
                                                      const double *__restrict__ b, int64_t ldb,
                                                      double *y, double *partial) {
  __shared__ double sh[kBRedT];
  RowIter it(gshift);
  double acc = 0.0;
  if (it.j < nc)
    for (int64_t i = it.row; i < n; i += it.stride) {
      double s = 0.0;
      const int64_t e1 = rowptr[i + 1];
      for (int64_t k = rowptr[i]; k < e1; ++k) s = s + val[k] * x[(int64_t)col[k] * ldx + it.j];
      const double t = b[i * ldb + it.j] - s;
      y[i * nc + it.j] = t;
      acc = acc + t * t;
    }
  write_partials(acc, sh, gshift, nc, partial);
}

// partial a.b
__global__ __launch_bounds__(kBRedT) void k_bdot(int64_t n, int nc, int gshift,
                                                 const double *__restrict__ a,
                                                 const double *__restrict__ b, double *partial,
                                                 const int *skip) {
  __shared__ double sh[kBRedT];
  if (*skip) return;
  RowIter it(gshift);
  double acc = 0.0;
  if (it.j < nc)
    for (int64_t i = it.row; i < n; i += it.stride) acc = acc + a[i * nc + it.j] * b[i * nc + it.j];
  write_partials(acc, sh, gshift, nc, partial);
}

// columns still iterating: x += alpha p, r -= alpha q; partial r.r
__global__ __launch_bounds__(kBRedT) void k_baxpy2(int64_t n, int nc, int gshift,
                                                   const double *__restrict__ p,
                                                   const double *__restrict__ q, double *x,
                                                   int64_t ldx, double *r, const double *bst,
                                                   const int *bist, double *partial,
                                                   const int *skip) {
  __shared__ double sh[kBRedT];
  if (*skip) return;
  RowIter it(gshift);
  double acc = 0.0;
  if (it.j < nc && !bist[4 * it.j + 1]) {
    const double alpha = bst[8 * it.j + 4];
    for (int64_t i = it.row; i < n; i += it.stride) {
      x[i * ldx + it.j] = x[i * ldx + it.j] + alpha * p[i * nc + it.j];
      const double ri = r[i * nc + it.j] - alpha * q[i * nc + it.j];
      r[i * nc + it.j] = ri;
      acc = acc + ri * ri;
    }
  }
  write_partials(acc, sh, gshift, nc, partial);
}

// columns still iterating: p = z + beta p
__global__ __launch_bounds__(kBRedT) void k_bxpby(int64_t n, int nc, int gshift,
                                                  const double *__restrict__ z, double *p,
                                                  const double *bst, const int *bist,
                                                  const int *skip) {
  if (*skip) return;
  RowIter it(gshift);
  if (it.j >= nc || bist[4 * it.j + 1]) return;
  const double beta = bst[8 * it.j + 5];
  for (int64_t i = it.row; i < n; i += it.stride)
    p[i * nc + it.j] = z[i * nc + it.j] + beta * p[i * nc + it.j];
}

__global__ void k_bsetup(int nc, double rtol, double *bst, int *bist, int *gfl) {
  const int j = threadIdx.x;
  if (j < nc) {
    for (int k = 0; k < 8; ++k) bst[8 * j + k] = 0.0;
    bst[8 * j + 6] = rtol;
    for (int k = 0; k < 4; ++k) bist[4 * j + k] = 0;
  }
  if (j == 0) {
    gfl[0] = nc;
    gfl[1] = 0;
  }
}

__device__ __forceinline__ void column_done(int *bist_j, int *gfl) {
  bist_j[1] = 1;
  if (atomicSub(&gfl[0], 1) == 1) gfl[1] = 1;
}

// block j reduces column j.  mode 0: ||b||^2 (a zero b is done at once);
// 1: r.z -> beta (first: 0); 2: p.q -> alpha; 3: r.r -> iteration count and
// stopping test; 4: true residual
__global__ __launch_bounds__(kBRedT) void k_breduce(const double *partial, int nb, int nc,
                                                    double *bst, int *bist, int *gfl, int mode,
                                                    int first) {
  __shared__ double sh[kBRedT];
  const int j = blockIdx.x;
  double *st = bst + 8 * j;
  int *ist = bist + 4 * j;
  if (mode != 0 && mode != 4 && (gfl[1] || ist[1])) return;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBRedT) acc = acc + partial[(int64_t)b * nc + j];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kBRedT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double s = sh[0];
  if (mode == 0) {
    st[0] = s;
    if (!(s > 0.0)) column_done(ist, gfl);
  } else if (mode == 1) {
    st[5] = first ? 0.0 : s / st[1];
    st[1] = s;
  } else if (mode == 2) {
    st[2] = s;
    st[4] = st[1] / s;
  } else if (mode == 3) {
    st[3] = s;
    ist[0] += 1;
    if (sqrt(s) <= st[6] * sqrt(st[0])) column_done(ist, gfl);
  } else {
    st[7] = s;
  }
}

static int gshift_for(int nc) {
  int g = 0;
  while ((1 << g) < nc) ++g;
  return g;
}

int bpcg_partials() { return kBRedBlocks; }

hipError_t bpcg_launch_init(int64_t n, int nc, double rtol, const double *b, int64_t ldb,
                            double *x, int64_t ldx, double *r, double *p, double *partial,
                            double *bst, int *bist, int *gfl, hipStream_t s) {
  const int g = gshift_for(nc);
  hipLaunchKernelGGL(k_bsetup, dim3(1), dim3(64), 0, s, nc, rtol, bst, bist, gfl);
  hipLaunchKernelGGL(k_binit, dim3(kBRedBlocks), dim3(kBRedT), 0, s, n, nc, g, b, ldb, x, ldx, r,
                     p, partial);
  hipLaunchKernelGGL(k_breduce, dim3(nc), dim3(kBRedT), 0, s, partial, kBRedBlocks, nc, bst, bist,
                     gfl, 0, 0);
  return hipGetLastError();
}

hipError_t bpcg_launch_rz(int64_t n, int nc, const double *r, const double *z, double *p,
                          double *partial, double *bst, int *bist, int *gfl, int first,
                          hipStream_t s) {
  const int g = gshift_for(nc);
  hipLaunchKernelGGL(k_bdot, dim3(kBRedBlocks), dim3(kBRedT), 0, s, n, nc, g, r, z, partial,
                     gfl + 1);
  hipLaunchKernelGGL(k_breduce, dim3(nc), dim3(kBRedT), 0, s, partial, kBRedBlocks, nc, bst, bist,
                     gfl, 1, first);
  hipLaunchKernelGGL(k_bxpby, dim3(kBRedBlocks), dim3(kBRedT), 0, s, n, nc, g, z, p, bst, bist,
                     gfl + 1);
  return hipGetLastError();
}

hipError_t bpcg_launch_step(int64_t n, int nc, const int64_t *rowptr, const int32_t *col,
                            const double *val, double *x, int64_t ldx, double *r, double *p,
                            double *q, double *partial, double *bst, int *bist, int *gfl,
                            hipStream_t s) {
  const int g = gshift_for(nc);
  hipLaunchKernelGGL(k_bspmv_dot, dim3(kBRedBlocks), dim3(kBRedT), 0, s, n, nc, g, rowptr, col,
                     val, p, q, partial, gfl + 1);
  hipLaunchKernelGGL(k_breduce, dim3(nc), dim3(kBRedT), 0, s, partial, kBRedBlocks, nc, bst, bist,
                     gfl, 2, 0);
  hipLaunchKernelGGL(k_baxpy2, dim3(kBRedBlocks), dim3(kBRedT), 0, s, n, nc, g, p, q, x, ldx, r,
                     bst, bist, partial, gfl + 1);
  hipLaunchKernelGGL(k_breduce, dim3(nc), dim3(kBRedT), 0, s, partial, kBRedBlocks, nc, bst, bist,
                     gfl, 3, 0);
  return hipGetLastError();
}

hipError_t bpcg_launch_true_res(int64_t n, int nc, const int64_t *rowptr, const int32_t *col,
                                const double *val, const double *x, int64_t ldx, const double *b,
                                int64_t ldb, double *tmp, double *partial, double *bst, int *bist,
                                int *gfl, hipStream_t s) {
  const int g = gshift_for(nc);
  hipLaunchKernelGGL(k_bresidual, dim3(kBRedBlocks), dim3(kBRedT), 0, s, n, nc, g, rowptr, col,
                     val, x, ldx, b, ldb, tmp, partial);
  hipLaunchKernelGGL(k_breduce, dim3(nc), dim3(kBRedT), 0, s, partial, kBRedBlocks, nc, bst, bist,
                     gfl, 4, 0);
  return hipGetLastError();
}

// consistency of every column of b per component (Laplacian mode): sums per
// (root, column); row groups whose root is the block's first root are
// reduced in LDS first, the rest add atomically
__global__ __launch_bounds__(kBRedT) void k_bcomp_sums(int64_t n, int nc, int gshift,
                                                       const int32_t *__restrict__ perm,
                                                       const int32_t *__restrict__ root,
                                                       const double *__restrict__ b, int64_t ldb,
                                                       double *sum, double *sabs) {
  __shared__ double sh[kBRedT];
  __shared__ int32_t r0;
  const int64_t rows = kBRedT >> gshift;
  const int64_t v = (int64_t)blockIdx.x * rows + (threadIdx.x >> gshift);
  const int j = threadIdx.x & ((1 << gshift) - 1);
  const bool valid = v < n && j < nc;
  const int32_t rt = v < n ? root[perm[v]] : -1;
  if (threadIdx.x == 0) r0 = rt;
  __syncthreads();
  const bool same = valid && rt == r0;
  const double bv = valid ? b[v * ldb + j] : 0.0;
  colsum(same ? bv : 0.0, sh, gshift);
  const double s1 = sh[threadIdx.x < (unsigned)(1 << gshift) ? threadIdx.x : 0];
  __syncthreads();
  colsum(same ? fabs(bv) : 0.0, sh, gshift);
  const double s2 = sh[threadIdx.x < (unsigned)(1 << gshift) ? threadIdx.x : 0];
  if ((int)threadIdx.x < nc && r0 >= 0) {
    atomicAdd(&sum[(int64_t)r0 * nc + threadIdx.x], s1);
    atomicAdd(&sabs[(int64_t)r0 * nc + threadIdx.x], s2);
  }
  if (valid && !same) {
    atomicAdd(&sum[(int64_t)rt * nc + j], bv);
    atomicAdd(&sabs[(int64_t)rt * nc + j], fabs(bv));
  }
}

__global__ void k_bcomp_check(int64_t n, int nc, int64_t ground, const int32_t *__restrict__ root,
                              const double *__restrict__ sum, const double *__restrict__ sabs,
                              int *bad) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n || root[k] != k) return;
  if (ground >= 0 && root[k] == ground) return;
  for (int j = 0; j < nc; ++j)
    if (fabs(sum[k * nc + j]) > 1e-8 * sabs[k * nc + j]) *bad = 1;
}

hipError_t launch_bcomp_check(int64_t n, int nc, int64_t ground, const int32_t *perm,
                              const int32_t *root, const double *b, int64_t ldb, double *sum,
                              double *sabs, int *bad, hipStream_t s) {
  const int g = gshift_for(nc);
  const int64_t rows = kBRedT >> g;
  hipLaunchKernelGGL(k_bcomp_sums, dim3((unsigned)((n + rows - 1) / rows)), dim3(kBRedT), 0, s, n,
                     nc, g, perm, root, b, ldb, sum, sabs);
  hipLaunchKernelGGL(k_bcomp_check, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, nc,
                     ground, root, sum, sabs, bad);
  return hipGetLastError();
}

}  // namespace parac
