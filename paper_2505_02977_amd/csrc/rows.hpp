// rows.hpp -- the row operations of the preconditioner apply, shared by the
// single-system, block and batched launches so that every launch shape
// computes each row with the same operations in the same order.
//
// Forward row i (level order position pos):  y_i = (P r)_i - sum_c F(i,c) y_c
// Backward row i:                            x_i = D^+_i y_i - sum_c F(c,i) x_c
// Both are left folds in ascending c, starting from the right-hand side
// (forward) or D^+ y (backward).
#pragma once

#include "device.hpp"
#include "internal.hpp"

namespace parac {

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
__device__ __forceinline__ void fwd_row(const SolveArgs &a, int64_t pos,
                                        const double *__restrict__ r, T *y) {
  const int32_t i = a.order[pos];
  const T *fv = FactorVals<T>::fwd(a);
  T acc = (T)r[a.iperm[i]];
  for (int64_t e = a.lf_ptr[pos]; e < a.lf_ptr[pos + 1]; ++e) acc = acc - fv[e] * y[a.lf_idx[e]];
  y[i] = acc;
}

template <typename T>
__device__ __forceinline__ void bwd_row(const SolveArgs &a, int64_t pos, const T *__restrict__ y,
                                        T *x, double *z) {
  const int32_t i = a.order[pos];
  const T *fv = FactorVals<T>::bwd(a);
  T acc = FactorVals<T>::dinv(a)[i] * y[i];
  for (int64_t e = a.lb_ptr[pos]; e < a.lb_ptr[pos + 1]; ++e) acc = acc - fv[e] * x[a.lb_idx[e]];
  x[i] = acc;
  z[a.iperm[i]] = (double)acc;
}

// the thin tail (levels L0 .. depth-1, at most kTThreads rows each) by one
// workgroup of kTThreads: per level the products of all its entries are
// staged in LDS with coalesced reads (passes of kTStage), then every row
// folds its own products in order
constexpr int kTThreads = 1024;
constexpr int kTStage = 8192;

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
__device__ __forceinline__ void tail_fwd(const SolveArgs &a, const double *__restrict__ r, T *y,
                                         T *stage) {
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
__device__ __forceinline__ void tail_bwd(const SolveArgs &a, const T *__restrict__ y, T *x,
                                         double *z, T *stage) {
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

}  // namespace parac
