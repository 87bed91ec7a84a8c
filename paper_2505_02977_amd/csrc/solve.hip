// solve.hip -- the preconditioner apply z = P^T F^-T D^+ F^-1 P r and the
// kernels of preconditioned conjugate gradients.
//
// Both triangular solves follow the elimination levels: the rows of one
// level depend only on rows of lower levels (forward) or higher levels
// (backward), so a level is solved in parallel once its predecessors are.
#include <float.h>

#include "device.hpp"
#include "internal.hpp"

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
template <typename T> struct FactorVals;
template <> struct FactorVals<double> {
  static __device__ __forceinline__ const double *fwd(const SolveArgs &a) { return a.lf_val; }
  static __device__ __forceinline__ const double *bwd(const SolveArgs &a) { return a.lb_val; }
  static __device__ __forceinline__ const double *dinv(const SolveArgs &a) { return a.Dinv; }
};
template <> struct FactorVals<float> {
  static __device__ __forceinline__ const float *fwd(const SolveArgs &a) { return a.lf_val32; }
  static __device__ __forceinline__ const float *bwd(const SolveArgs &a) { return a.lb_val32; }
  static __device__ __forceinline__ const float *dinv(const SolveArgs &a) { return a.Dinv32; }
};

template <typename T>
__global__ __launch_bounds__(256) void k_level_fwd(SolveArgs a, int64_t p0, int64_t p1,
                                                   const double *__restrict__ r, T *y) {
  if (a.skip && *a.skip) return;
  const int64_t pos = p0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= p1) return;
  const int32_t i = a.order[pos];
  const T *fv = FactorVals<T>::fwd(a);
  T acc = (T)r[a.iperm[i]];
  for (int64_t e = a.lf_ptr[pos]; e < a.lf_ptr[pos + 1]; ++e) acc = acc - fv[e] * y[a.lf_idx[e]];
  y[i] = acc;
}

template <typename T>
__global__ __launch_bounds__(256) void k_level_bwd(SolveArgs a, int64_t p0, int64_t p1,
                                                   const T *__restrict__ y, T *x, double *z) {
  if (a.skip && *a.skip) return;
  const int64_t pos = p0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= p1) return;
  const int32_t i = a.order[pos];
  const T *fv = FactorVals<T>::bwd(a);
  T acc = FactorVals<T>::dinv(a)[i] * y[i];
  for (int64_t e = a.lb_ptr[pos]; e < a.lb_ptr[pos + 1]; ++e) acc = acc - fv[e] * x[a.lb_idx[e]];
  x[i] = acc;
  z[a.iperm[i]] = (double)acc;
}

constexpr int kTThreads = 1024;
constexpr int kTStage = 8192;  // products staged in LDS per pass

// one tail level: stage the products of the level's entries [q0, q1) in
// passes of kTStage, each row folding its own entries after every pass
template <typename T>
__device__ __forceinline__ T tail_level(T acc, int64_t e0, int64_t e1, int64_t q0, int64_t q1,
                                        const int32_t *__restrict__ idx,
                                        const T *__restrict__ fv, const T *vec, T *stage) {
  for (int64_t qc = q0; qc < q1; qc += kTStage) {
    const int64_t qe = qc + kTStage < q1 ? qc + kTStage : q1;
    for (int64_t q = qc + threadIdx.x; q < qe; q += kTThreads) stage[q - qc] = fv[q] * vec[idx[q]];
    __syncthreads();
    const int64_t lo = e0 > qc ? e0 : qc, hi = e1 < qe ? e1 : qe;
    for (int64_t e = lo; e < hi; ++e) acc = acc - stage[e - qc];
    __syncthreads();
  }
  return acc;
}

template <typename T>
__global__ __launch_bounds__(kTThreads) void k_tail_fwd(SolveArgs a, const double *__restrict__ r,
                                                        T *y) {
  __shared__ T stage[kTStage];
  if (a.skip && *a.skip) return;
  const T *fv = FactorVals<T>::fwd(a);
  for (int64_t L = a.L0; L < a.depth; ++L) {
    const int64_t p0 = a.lptr[L], p1 = a.lptr[L + 1];
    const int64_t pos = p0 + threadIdx.x;  // at most kTailWidth <= kTThreads rows
    const bool valid = pos < p1;
    const int32_t i = valid ? a.order[pos] : 0;
    T acc = valid ? (T)r[a.iperm[i]] : (T)0;
    const int64_t e0 = valid ? a.lf_ptr[pos] : 0, e1 = valid ? a.lf_ptr[pos + 1] : 0;
    acc = tail_level<T>(acc, e0, e1, a.lf_ptr[p0], a.lf_ptr[p1], a.lf_idx, fv, y, stage);
    if (valid) y[i] = acc;
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(kTThreads) void k_tail_bwd(SolveArgs a, const T *__restrict__ y,
                                                        T *x, double *z) {
  __shared__ T stage[kTStage];
  if (a.skip && *a.skip) return;
  const T *fv = FactorVals<T>::bwd(a);
  const T *dv = FactorVals<T>::dinv(a);
  for (int64_t L = a.depth - 1; L >= a.L0; --L) {
    const int64_t p0 = a.lptr[L], p1 = a.lptr[L + 1];
    const int64_t pos = p0 + threadIdx.x;
    const bool valid = pos < p1;
    const int32_t i = valid ? a.order[pos] : 0;
    T acc = valid ? dv[i] * y[i] : (T)0;
    const int64_t e0 = valid ? a.lb_ptr[pos] : 0, e1 = valid ? a.lb_ptr[pos + 1] : 0;
    acc = tail_level<T>(acc, e0, e1, a.lb_ptr[p0], a.lb_ptr[p1], a.lb_idx, fv, x, stage);
    if (valid) {
      x[i] = acc;
      z[a.iperm[i]] = (double)acc;
    }
    __syncthreads();
  }
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

__global__ void k_level_copy(int64_t n, const int32_t *__restrict__ order,
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
    lf_idx[o] = colind_f[e];
    lf_val[o] = val_f[e];
  }
  o = lb_ptr[p];
  const int64_t cnt = lb_ptr[p + 1] - lb_ptr[p];
  for (int64_t t = 0; t < cnt; ++t, ++o) {
    lb_idx[o] = rowind[colptr[i] + t];
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

hipError_t launch_level_copy(int64_t n, const int32_t *order, const int64_t *rowptr_f,
                             const int32_t *colind_f, const double *val_f, const int64_t *colptr,
                             const int32_t *rowind, const double *val, const int64_t *lf_ptr,
                             const int64_t *lb_ptr, int32_t *lf_idx, double *lf_val,
                             int32_t *lb_idx, double *lb_val, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_level_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, order,
                     rowptr_f, colind_f, val_f, colptr, rowind, val, lf_ptr, lb_ptr, lf_idx,
                     lf_val, lb_idx, lb_val);
  return hipGetLastError();
}

// ==========================================================================
// PCG building blocks (one right-hand side).  Reductions are deterministic:
// a fixed grid, a fixed LDS tree per block, then one block sums the partials
// in a fixed order.
// ==========================================================================
constexpr int kRedBlocks = 1024;
constexpr int kRedT = 256;
constexpr int kSG = 8;              // lanes per row (SpMV)
constexpr int kSRPW = kWave / kSG;  // SpMV rows per wave

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

// q = A p and partial sums of p.q ; kSG lanes per row
__global__ __launch_bounds__(kRedT) void k_spmv_dot(int64_t n, const int64_t *__restrict__ rowptr,
                                                    const int32_t *__restrict__ col,
                                                    const double *__restrict__ val,
                                                    const double *__restrict__ p, double *q,
                                                    double *partial, const int *skip) {
  __shared__ double sh[kRedT];
  if (skip && *skip) return;
  const int l = lane(), grp = l / kSG, sub = l % kSG;
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  double dot = 0.0;
  for (int64_t r0 = wid * kSRPW; r0 < n; r0 += nw * kSRPW) {
    const int64_t i = r0 + grp;
    double s = 0.0;
    if (i < n) {
      const int64_t b = rowptr[i], e = rowptr[i + 1];
      for (int64_t k = b + sub; k < e; k += kSG) s = s + val[k] * p[col[k]];
    }
#pragma unroll
    for (int o = kSG / 2; o >= 1; o >>= 1) s = s + __shfl_xor(s, o, kWave);
    if (i < n && sub == 0) {
      q[i] = s;
      dot = dot + p[i] * s;
    }
  }
  double bs = block_sum(dot, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = bs;
}

// y = b - A x and partial sums of y.y (true residual)
__global__ __launch_bounds__(kRedT) void k_residual(int64_t n, const int64_t *__restrict__ rowptr,
                                                    const int32_t *__restrict__ col,
                                                    const double *__restrict__ val,
                                                    const double *__restrict__ x,
                                                    const double *__restrict__ bvec, double *y,
                                                    double *partial) {
  __shared__ double sh[kRedT];
  const int l = lane(), grp = l / kSG, sub = l % kSG;
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  double acc = 0.0;
  for (int64_t r0 = wid * kSRPW; r0 < n; r0 += nw * kSRPW) {
    const int64_t i = r0 + grp;
    double s = 0.0;
    if (i < n) {
      const int64_t b = rowptr[i], e = rowptr[i + 1];
      for (int64_t k = b + sub; k < e; k += kSG) s = s + val[k] * x[col[k]];
    }
#pragma unroll
    for (int o = kSG / 2; o >= 1; o >>= 1) s = s + __shfl_xor(s, o, kWave);
    if (i < n && sub == 0) {
      double t = bvec[i] - s;
      y[i] = t;
      acc = acc + t * t;
    }
  }
  double bs = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = bs;
}

// partial sums of a.b over a grid-stride loop
__global__ __launch_bounds__(kRedT) void k_dot(int64_t n, const double *__restrict__ a,
                                               const double *__restrict__ b, double *partial,
                                               const int *skip) {
  __shared__ double sh[kRedT];
  if (skip && *skip) return;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc = acc + a[i] * b[i];
  double bs = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = bs;
}

// x = 0, r = b, partial sums of b.b
__global__ __launch_bounds__(kRedT) void k_pcg_init(int64_t n, const double *__restrict__ b,
                                                    double *x, double *r, double *partial) {
  __shared__ double sh[kRedT];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v = b[i];
    x[i] = 0.0;
    r[i] = v;
    acc = acc + v * v;
  }
  double bs = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = bs;
}

// x += alpha p ; r -= alpha q ; partial sums of r.r
__global__ __launch_bounds__(kRedT) void k_axpy2(int64_t n, const double *__restrict__ p,
                                                 const double *__restrict__ q, double *x, double *r,
                                                 const double *st, double *partial,
                                                 const int *skip) {
  __shared__ double sh[kRedT];
  if (skip && *skip) return;
  const double alpha = st[4];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    x[i] = x[i] + alpha * p[i];
    double ri = r[i] - alpha * q[i];
    r[i] = ri;
    acc = acc + ri * ri;
  }
  double bs = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = bs;
}

// p = z + beta p   (first iteration: beta = 0 via st[5])
__global__ void k_xpby(int64_t n, const double *__restrict__ z, double *p, const double *st,
                       const int *skip) {
  if (skip && *skip) return;
  const double beta = st[5];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = z[i] + beta * p[i];
}

// PCG scalars: st[0] ||b||^2, st[1] r.z, st[2] p.q, st[3] r.r, st[4] alpha,
// st[5] beta, st[6] rtol, st[7] true ||b-Ax||^2; ist[0] iterations,
// ist[1] done, ist[2] skip-apply (== done)
__device__ double sum_partials(const double *partial, int nb, double *sh) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += kRedT) acc = acc + partial[i];
  return block_sum(acc, sh);
}

// mode 0: ||b||^2 (done if zero); 1: r.z -> beta (first: beta = 0);
// 2: p.q -> alpha; 3: r.r -> iteration count and convergence; 4: true res
__global__ __launch_bounds__(kRedT) void k_reduce(const double *partial, int nb, double *st,
                                                  int *ist, int mode, int first) {
  __shared__ double sh[kRedT];
  if (mode != 0 && mode != 4 && ist[1]) return;
  double s = sum_partials(partial, nb, sh);
  if (threadIdx.x != 0) return;
  if (mode == 0) {
    st[0] = s;
    ist[0] = 0;
    ist[1] = s > 0.0 ? 0 : 1;
    ist[2] = ist[1];
  } else if (mode == 1) {
    st[5] = first ? 0.0 : s / st[1];
    st[1] = s;
  } else if (mode == 2) {
    st[2] = s;
    st[4] = st[1] / s;
  } else if (mode == 3) {
    st[3] = s;
    ist[0] += 1;
    if (sqrt(s) <= st[6] * sqrt(st[0])) {
      ist[1] = 1;
      ist[2] = 1;
    }
  } else {
    st[7] = s;
  }
}

hipError_t pcg_launch_init(int64_t n, const double *b, double *x, double *r, double *partial,
                           double *st, int *ist, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_init, dim3(kRedBlocks), dim3(kRedT), 0, s, n, b, x, r, partial);
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedT), 0, s, partial, kRedBlocks, st, ist, 0, 0);
  return hipGetLastError();
}

hipError_t pcg_launch_rz(int64_t n, const double *r, const double *z, double *p, double *partial,
                         double *st, int *ist, int first, hipStream_t s) {
  hipLaunchKernelGGL(k_dot, dim3(kRedBlocks), dim3(kRedT), 0, s, n, r, z, partial, ist + 1);
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedT), 0, s, partial, kRedBlocks, st, ist, 1, first);
  hipLaunchKernelGGL(k_xpby, dim3(kRedBlocks), dim3(kRedT), 0, s, n, z, p, st, ist + 1);
  return hipGetLastError();
}

hipError_t pcg_launch_step(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                           double *x, double *r, double *p, double *q, double *partial, double *st,
                           int *ist, hipStream_t s) {
  hipLaunchKernelGGL(k_spmv_dot, dim3(kRedBlocks), dim3(kRedT), 0, s, n, rowptr, col, val, p, q,
                     partial, ist + 1);
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedT), 0, s, partial, kRedBlocks, st, ist, 2, 0);
  hipLaunchKernelGGL(k_axpy2, dim3(kRedBlocks), dim3(kRedT), 0, s, n, p, q, x, r, st, partial,
                     ist + 1);
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedT), 0, s, partial, kRedBlocks, st, ist, 3, 0);
  return hipGetLastError();
}

hipError_t pcg_launch_true_res(int64_t n, const int64_t *rowptr, const int32_t *col,
                               const double *val, const double *x, const double *b, double *tmp,
                               double *partial, double *st, int *ist, hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3(kRedBlocks), dim3(kRedT), 0, s, n, rowptr, col, val, x, b,
                     tmp, partial);
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedT), 0, s, partial, kRedBlocks, st, ist, 4, 0);
  return hipGetLastError();
}

int pcg_partials() { return kRedBlocks; }

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
