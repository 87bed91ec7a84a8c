// rows.hpp -- the row operations of the preconditioner apply, shared by the
// single-system, block and batched launches so that every launch shape
// computes each row with the same operations in the same order.
//
// Forward row i (at level-order position p):  y_p = (P r)_i - sum_c F(i,c) y_c
// Backward row i:                              x_p = D^+_i y_p - sum_c F(c,i) x_c
// Both are left folds in ascending c, starting from the right-hand side
// (forward) or D^+ y (backward); vectors and indices are positions.
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

// acc - sum_e fv[e] vec[idx[e]] as a left fold in ascending e; the loads of
// eight entries are issued before their products are folded (same order,
// same roundings)
template <typename T>
__device__ __forceinline__ T fold_row(T acc, int64_t e, int64_t e1,
                                      const int32_t *__restrict__ idx,
                                      const T *__restrict__ fv, const T *vec) {
  for (; e + 8 <= e1; e += 8) {
    int32_t c[8];
    T f[8], v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      c[u] = idx[e + u];
      f[u] = fv[e + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = vec[c[u]];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = acc - f[u] * v[u];
  }
  for (; e < e1; ++e) acc = acc - fv[e] * vec[idx[e]];
  return acc;
}

template <typename T>
__device__ __forceinline__ void fwd_row(const SolveArgs &a, int64_t pos,
                                        const double *__restrict__ r, T *y) {
  const T acc = (T)r[a.src[pos]];
  y[pos] = fold_row<T>(acc, a.lf_ptr[pos], a.lf_ptr[pos + 1], a.lf_idx, FactorVals<T>::fwd(a), y);
}

template <typename T>
__device__ __forceinline__ void bwd_row(const SolveArgs &a, int64_t pos, const T *__restrict__ y,
                                        T *x, double *z) {
  const T acc = FactorVals<T>::dinv(a)[pos] * y[pos];
  const T v = fold_row<T>(acc, a.lb_ptr[pos], a.lb_ptr[pos + 1], a.lb_idx, FactorVals<T>::bwd(a), x);
  x[pos] = v;
  z[a.src[pos]] = (double)v;
}

// The thin tail (levels L0 .. depth-1, at most kTThreads rows each) by one
// workgroup of kTThreads.  Per level, the products of all its entries are
// staged in LDS (passes of kTStage), then every row folds its own products in
// order.  Level L+1's loads (row ranges, its first kTStage indices and
// values, its starting values) are issued while level L is folded, and level
// bounds are read two levels ahead, so each level waits on little more than
// the gather of earlier results.
constexpr int kTThreads = 1024;
constexpr int kTPer = 4;                      // staged entries per thread per pass
constexpr int kTStage = kTThreads * kTPer;   // 4096

struct TailBounds {
  int64_t p0, p1, q0, q1;  // positions and entries of one level
};

__device__ __forceinline__ TailBounds tail_bounds(const int64_t *lptr, const int64_t *lq,
                                                  int64_t L) {
  return TailBounds{lptr[L], lptr[L + 1], lq[L], lq[L + 1]};
}

template <typename T>
struct TailPre {
  T acc;           // starting value of this thread's row
  int64_t e0, e1;  // its entries
  int32_t c[kTPer];
  T f[kTPer];
};

// BWD: starting value D^+ y (else the pre-gathered right-hand side in y)
template <typename T, bool BWD>
__device__ __forceinline__ void tail_prefetch(const SolveArgs &a, const TailBounds &b,
                                              const int64_t *__restrict__ ptr,
                                              const int32_t *__restrict__ idx,
                                              const T *__restrict__ fv, const T *y,
                                              TailPre<T> &t) {
  const int64_t pos = b.p0 + threadIdx.x;
  const bool valid = pos < b.p1;
  t.e0 = valid ? ptr[pos] : 0;
  t.e1 = valid ? ptr[pos + 1] : 0;
  if (BWD) t.acc = valid ? FactorVals<T>::dinv(a)[pos] * y[pos] : (T)0;
  else t.acc = valid ? y[pos] : (T)0;
  const int64_t qe = b.q1 < b.q0 + kTStage ? b.q1 : b.q0 + kTStage;
#pragma unroll
  for (int u = 0; u < kTPer; ++u) {
    const int64_t q = b.q0 + threadIdx.x + (int64_t)u * kTThreads;
    t.c[u] = q < qe ? idx[q] : 0;
    t.f[u] = q < qe ? fv[q] : (T)0;
  }
}

// gather the vector values of a level's first pass (prefetched indices)
template <typename T>
__device__ __forceinline__ void tail_gather(const TailBounds &b, const TailPre<T> &cur,
                                            const T *vec, T (&v)[kTPer]) {
  const int64_t qe = b.q1 < b.q0 + kTStage ? b.q1 : b.q0 + kTStage;
#pragma unroll
  for (int u = 0; u < kTPer; ++u) {
    const int64_t q = b.q0 + threadIdx.x + (int64_t)u * kTThreads;
    v[u] = q < qe ? vec[cur.c[u]] : (T)0;
  }
}

// fold one level (first pass gathered in v); returns this thread's row value
template <typename T>
__device__ __forceinline__ T tail_fold(const TailBounds &b, const TailPre<T> &cur,
                                       const T (&v)[kTPer], const int32_t *__restrict__ idx,
                                       const T *__restrict__ fv, const T *vec, T *stage) {
  T acc = cur.acc;
  for (int64_t qc = b.q0; qc < b.q1; qc += kTStage) {
    const int64_t qe = qc + kTStage < b.q1 ? qc + kTStage : b.q1;
    if (qc == b.q0) {
#pragma unroll
      for (int u = 0; u < kTPer; ++u) {
        const int64_t q = qc + threadIdx.x + (int64_t)u * kTThreads;
        if (q < qe) stage[q - qc] = cur.f[u] * v[u];
      }
    } else {
#pragma unroll 4
      for (int64_t q = qc + threadIdx.x; q < qe; q += kTThreads) stage[q - qc] = fv[q] * vec[idx[q]];
    }
    __syncthreads();
    const int64_t lo = cur.e0 > qc ? cur.e0 : qc, hi = cur.e1 < qe ? cur.e1 : qe;
    int64_t e = lo;
    for (; e + 8 <= hi; e += 8) {  // eight LDS reads in flight, folded in order
      T w[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) w[u] = stage[e - qc + u];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = acc - w[u];
    }
    for (; e < hi; ++e) acc = acc - stage[e - qc];
    __syncthreads();
  }
  return acc;
}

// Per level: gather the current level's values first, then issue the next
// level's loads (vector loads complete in issue order, so waiting for the
// gather does not wait for the prefetch), then fold.
template <typename T>
__device__ __forceinline__ void tail_fwd(const SolveArgs &a, const double *__restrict__ r, T *y,
                                         T *stage) {
  if (a.L0 >= a.depth) return;
  const T *fv = FactorVals<T>::fwd(a);
  // the right-hand side of every tail row, gathered once into y
  for (int64_t pos = a.lptr[a.L0] + threadIdx.x; pos < a.n; pos += kTThreads)
    y[pos] = (T)r[a.src[pos]];
  __syncthreads();
  TailBounds b = tail_bounds(a.lptr, a.lqf, a.L0);
  TailBounds bn = a.L0 + 1 < a.depth ? tail_bounds(a.lptr, a.lqf, a.L0 + 1) : b;
  TailPre<T> cur;
  tail_prefetch<T, false>(a, b, a.lf_ptr, a.lf_idx, fv, y, cur);
  for (int64_t L = a.L0; L < a.depth; ++L) {
    T v[kTPer];
    tail_gather<T>(b, cur, y, v);
    TailPre<T> nxt;
    const bool more = L + 1 < a.depth;
    TailBounds bnn = bn;
    if (more) {
      tail_prefetch<T, false>(a, bn, a.lf_ptr, a.lf_idx, fv, y, nxt);
      if (L + 2 < a.depth) bnn = tail_bounds(a.lptr, a.lqf, L + 2);
    }
    const T val = tail_fold<T>(b, cur, v, a.lf_idx, fv, y, stage);
    const int64_t pos = b.p0 + threadIdx.x;
    if (pos < b.p1) y[pos] = val;
    __syncthreads();
    if (more) {
      cur = nxt;
      b = bn;
      bn = bnn;
    }
  }
}

template <typename T>
__device__ __forceinline__ void tail_bwd(const SolveArgs &a, const T *__restrict__ y, T *x,
                                         double *z, T *stage) {
  if (a.L0 >= a.depth) return;
  const T *fv = FactorVals<T>::bwd(a);
  const int64_t Lt = a.depth - 1;
  TailBounds b = tail_bounds(a.lptr, a.lqb, Lt);
  TailBounds bn = Lt - 1 >= a.L0 ? tail_bounds(a.lptr, a.lqb, Lt - 1) : b;
  TailPre<T> cur;
  tail_prefetch<T, true>(a, b, a.lb_ptr, a.lb_idx, fv, y, cur);
  for (int64_t L = Lt; L >= a.L0; --L) {
    T v[kTPer];
    tail_gather<T>(b, cur, x, v);
    TailPre<T> nxt;
    const bool more = L - 1 >= a.L0;
    TailBounds bnn = bn;
    if (more) {
      tail_prefetch<T, true>(a, bn, a.lb_ptr, a.lb_idx, fv, y, nxt);
      if (L - 2 >= a.L0) bnn = tail_bounds(a.lptr, a.lqb, L - 2);
    }
    const T val = tail_fold<T>(b, cur, v, a.lb_idx, fv, x, stage);
    const int64_t pos = b.p0 + threadIdx.x;
    if (pos < b.p1) {
      x[pos] = val;
      z[a.src[pos]] = (double)val;
    }
    __syncthreads();
    if (more) {
      cur = nxt;
      b = bn;
      bn = bnn;
    }
  }
}

}  // namespace parac
