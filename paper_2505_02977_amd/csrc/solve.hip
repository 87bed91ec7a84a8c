// solve.hip -- the preconditioner apply z = P^T F^-T D^+ F^-1 P r and the
// kernels of preconditioned conjugate gradients.
//
// Both triangular solves follow the elimination levels: the rows of one
// level depend only on rows of lower levels (forward) or higher levels
// (backward), so a level is solved in parallel once its predecessors are.
#include <float.h>

#include "device.hpp"
#include "internal.hpp"
#include "rows.hpp"

namespace parac {

// ---------------------------------------------------------------------------
// Preconditioner apply.  The factor is stored twice in level order: the rows
// of F for the forward solve and its columns (without the ground row) for
// the backward solve; position p of either copy is the row order[p].  Rows of
// one level are independent.
//
//  * wide levels (below L0): one launch per level, one thread per row;
//    the level's dependencies were written by earlier launches;
//  * the thin tail (L0 and above, at most kTailWidth rows per level): one
//    workgroup walks the levels; per level it gathers all products into LDS
//    with coalesced reads, then each row folds its own products.
//
// Every row is folded left in ascending column order, starting from the
// right-hand side (forward) or D^+ y (backward): the order of the CPU
// reference, so the result is the same bit for bit.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_level_fwd(SolveArgs a, int64_t p0, int64_t p1,
                                                   const double *__restrict__ r, T *y) {
  if (a.skip && *a.skip) return;
  const int64_t pos = p0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos < p1) fwd_row<T>(a, pos, r, y);
}

template <typename T>
__global__ __launch_bounds__(256) void k_level_bwd(SolveArgs a, int64_t p0, int64_t p1,
                                                   const T *__restrict__ y, T *x, double *z) {
  if (a.skip && *a.skip) return;
  const int64_t pos = p0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos < p1) bwd_row<T>(a, pos, y, x, z);
}

template <typename T>
__global__ __launch_bounds__(kTThreads) void k_tail_fwd(SolveArgs a, const double *__restrict__ r,
                                                        T *y) {
  __shared__ T stage[kTStage];
  if (a.skip && *a.skip) return;
  tail_fwd<T>(a, r, y, stage);
}

template <typename T>
__global__ __launch_bounds__(kTThreads) void k_tail_bwd(SolveArgs a, const T *__restrict__ y,
                                                        T *x, double *z) {
  __shared__ T stage[kTStage];
  if (a.skip && *a.skip) return;
  tail_bwd<T>(a, y, x, z, stage);
}

template <typename T>
static hipError_t apply_t(const SolveArgs &a, const int64_t *hlptr, const double *r, T *y, T *x,
                          double *z, hipStream_t s) {
  for (int64_t L = 0; L < a.L0; ++L) {
    const int64_t p0 = hlptr[L], p1 = hlptr[L + 1];
    if (p1 > p0)
      hipLaunchKernelGGL(k_level_fwd<T>, dim3((unsigned)((p1 - p0 + 255) / 256)), dim3(256), 0, s,
                         a, p0, p1, r, y);
  }
  if (a.L0 < a.depth) {
    hipLaunchKernelGGL(k_tail_fwd<T>, dim3(1), dim3(kTThreads), 0, s, a, r, y);
    hipLaunchKernelGGL(k_tail_bwd<T>, dim3(1), dim3(kTThreads), 0, s, a, (const T *)y, x, z);
  }
  for (int64_t L = a.L0 - 1; L >= 0; --L) {
    const int64_t p0 = hlptr[L], p1 = hlptr[L + 1];
    if (p1 > p0)
      hipLaunchKernelGGL(k_level_bwd<T>, dim3((unsigned)((p1 - p0 + 255) / 256)), dim3(256), 0, s,
                         a, p0, p1, (const T *)y, x, z);
  }
  return hipGetLastError();
}

hipError_t launch_apply(const SolveArgs &a, const int64_t *hlptr, const double *r, void *y, void *x,
                        double *z, int prec, hipStream_t s) {
  if (prec == PARAC_PREC_MIXED)
    return apply_t<float>(a, hlptr, r, (float *)y, (float *)x, z, s);
  return apply_t<double>(a, hlptr, r, (double *)y, (double *)x, z, s);
}

// level-ordered copies: position p holds row order[p]'s entries of F (rows
// for the forward solve; columns minus the ground row for the backward one)
__global__ void k_level_lengths(int64_t n, const int32_t *__restrict__ order,
                                const int64_t *__restrict__ rowptr_f,
                                const int64_t *__restrict__ colptr,
                                const int32_t *__restrict__ rowind, int32_t *flen, int32_t *blen) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t i = order[p];
  flen[p] = (int32_t)(rowptr_f[i + 1] - rowptr_f[i]);
  int64_t b = colptr[i], e = colptr[i + 1];
  if (e > b && rowind[e - 1] >= n) --e;  // the ground row is dropped
  blen[p] = (int32_t)(e - b);
}

// position maps: posof[label] = position, src[position] = original vertex,
// D^+ by position (zero pivots give zero: one per component)
__global__ void k_position_maps(int64_t n, const int32_t *__restrict__ order,
                                const int32_t *__restrict__ iperm, const double *__restrict__ D,
                                int32_t *posof, int32_t *src, double *pdinv, float *pdinv32) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t i = order[p];
  posof[i] = (int32_t)p;
  src[p] = iperm[i];
  const double d = D[i];
  const double v = d > 0.0 ? 1.0 / d : 0.0;
  pdinv[p] = v;
  if (pdinv32) pdinv32[p] = (float)v;
}

// position p holds row order[p]'s entries of F (rows for the forward solve;
// columns minus the ground row for the backward one), indices as positions
__global__ void k_level_copy(int64_t n, const int32_t *__restrict__ order,
                             const int32_t *__restrict__ posof,
                             const int64_t *__restrict__ rowptr_f,
                             const int32_t *__restrict__ colind_f, const double *__restrict__ val_f,
                             const int64_t *__restrict__ colptr, const int32_t *__restrict__ rowind,
                             const double *__restrict__ val, const int64_t *__restrict__ lf_ptr,
                             const int64_t *__restrict__ lb_ptr, int32_t *lf_idx, double *lf_val,
                             int32_t *lb_idx, double *lb_val) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t i = order[p];
  int64_t o = lf_ptr[p];
  for (int64_t e = rowptr_f[i]; e < rowptr_f[i + 1]; ++e, ++o) {
    lf_idx[o] = posof[colind_f[e]];
    lf_val[o] = val_f[e];
  }
  o = lb_ptr[p];
  const int64_t cnt = lb_ptr[p + 1] - lb_ptr[p];
  for (int64_t t = 0; t < cnt; ++t, ++o) {
    lb_idx[o] = posof[rowind[colptr[i] + t]];
    lb_val[o] = val[colptr[i] + t];
  }
}

hipError_t launch_level_layout(int64_t n, const int32_t *order, const int64_t *rowptr_f,
                               const int64_t *colptr, const int32_t *rowind, int32_t *flen,
                               int32_t *blen, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_level_lengths, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, order,
                     rowptr_f, colptr, rowind, flen, blen);
  return hipGetLastError();
}

__global__ void k_level_offsets(int64_t depth, const int64_t *__restrict__ lptr,
                                const int64_t *__restrict__ lf_ptr,
                                const int64_t *__restrict__ lb_ptr, int64_t *lqf, int64_t *lqb) {
  const int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (L > depth) return;
  lqf[L] = lf_ptr[lptr[L]];
  lqb[L] = lb_ptr[lptr[L]];
}

hipError_t launch_level_offsets(int64_t depth, const int64_t *lptr, const int64_t *lf_ptr,
                                const int64_t *lb_ptr, int64_t *lqf, int64_t *lqb, hipStream_t s) {
  hipLaunchKernelGGL(k_level_offsets, dim3((unsigned)((depth + 256) / 256)), dim3(256), 0, s,
                     depth, lptr, lf_ptr, lb_ptr, lqf, lqb);
  return hipGetLastError();
}

hipError_t launch_position_maps(int64_t n, const int32_t *order, const int32_t *iperm,
                                const double *D, int32_t *posof, int32_t *src, double *pdinv,
                                float *pdinv32, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_position_maps, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, order,
                     iperm, D, posof, src, pdinv, pdinv32);
  return hipGetLastError();
}

hipError_t launch_level_copy(int64_t n, const int32_t *order, const int32_t *posof,
                             const int64_t *rowptr_f, const int32_t *colind_f,
                             const double *val_f, const int64_t *colptr, const int32_t *rowind,
                             const double *val, const int64_t *lf_ptr, const int64_t *lb_ptr,
                             int32_t *lf_idx, double *lf_val, int32_t *lb_idx, double *lb_val,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_level_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, order,
                     posof, rowptr_f, colind_f, val_f, colptr, rowind, val, lf_ptr, lb_ptr, lf_idx,
                     lf_val, lb_idx, lb_val);
  return hipGetLastError();
}

// ==========================================================================
// Consistency of b with the null space: per connected component of the
// factor (labels joined by their first off-diagonal entry), the sum of b.
// ==========================================================================
constexpr int kRedT = 256;

__device__ __forceinline__ double block_sum(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = kRedT / 2; o > 0; o >>= 1) {
    if (t < o) sh[t] = sh[t] + sh[t + o];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// consistency of b per component: comp[label] = root label, sums per root
__global__ void k_comp_init(int64_t ntot, const int64_t *__restrict__ colptr,
                            const int32_t *__restrict__ rowind, int32_t *parent) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ntot) return;
  parent[k] = colptr[k + 1] > colptr[k] ? rowind[colptr[k]] : (int32_t)k;
}

__global__ void k_comp_jump(int64_t ntot, const int32_t *__restrict__ src, int32_t *dst,
                            int *changed) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ntot) return;
  int32_t p = src[k], pp = src[p];
  dst[k] = pp;
  if (pp != p) *changed = 1;
}

hipError_t launch_comp_init(int64_t ntot, const int64_t *colptr, const int32_t *rowind,
                            int32_t *parent, hipStream_t s) {
  hipLaunchKernelGGL(k_comp_init, dim3((unsigned)((ntot + 255) / 256)), dim3(256), 0, s, ntot,
                     colptr, rowind, parent);
  return hipGetLastError();
}

hipError_t launch_comp_jump(int64_t ntot, const int32_t *src, int32_t *dst, int *changed,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_comp_jump, dim3((unsigned)((ntot + 255) / 256)), dim3(256), 0, s, ntot, src,
                     dst, changed);
  return hipGetLastError();
}

// per-root sum and absolute sum of b (label space through perm); lanes of a
// block that share the block's first root are reduced in LDS first (the
// common single-component case), the rest add atomically
__global__ __launch_bounds__(kRedT) void k_comp_sums(int64_t n, const int32_t *__restrict__ perm,
                                                     const int32_t *__restrict__ root,
                                                     const double *__restrict__ b, double *sum,
                                                     double *sabs) {
  __shared__ double sh[kRedT];
  __shared__ int32_t r0;
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = v < n;
  const int32_t rt = valid ? root[perm[v]] : -1;
  if (threadIdx.x == 0) r0 = rt;
  __syncthreads();
  const bool same = valid && rt == r0;
  const double bv = valid ? b[v] : 0.0;
  double s1 = block_sum(same ? bv : 0.0, sh);
  double s2 = block_sum(same ? fabs(bv) : 0.0, sh);
  if (threadIdx.x == 0 && r0 >= 0) {
    atomicAdd(&sum[r0], s1);
    atomicAdd(&sabs[r0], s2);
  }
  if (valid && !same) {
    atomicAdd(&sum[rt], bv);
    atomicAdd(&sabs[rt], fabs(bv));
  }
}

// flag: a root (label < n, not joined to the ground) with |sum| > 1e-8 sum|b|
__global__ void k_comp_check(int64_t n, int64_t ground, const int32_t *__restrict__ root,
                             const double *__restrict__ sum, const double *__restrict__ sabs,
                             int *bad) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  if (root[k] != k) return;
  if (ground >= 0 && root[k] == ground) return;
  if (fabs(sum[k]) > 1e-8 * sabs[k]) *bad = 1;
}

hipError_t launch_comp_check(int64_t n, int64_t ground, const int32_t *perm, const int32_t *root,
                             const double *b, double *sum, double *sabs, int *bad, hipStream_t s) {
  hipLaunchKernelGGL(k_comp_sums, dim3((unsigned)((n + kRedT - 1) / kRedT)), dim3(kRedT), 0, s, n,
                     perm, root, b, sum, sabs);
  hipLaunchKernelGGL(k_comp_check, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, ground,
                     root, sum, sabs, bad);
  return hipGetLastError();
}

}  // namespace parac
