// rows.hpp -- the row operations of the preconditioner apply, shared by the
// single-system, batched and block launches so that every launch shape
// computes each row with the same operations in the same order.
//
// Forward row i (at level-order position p):  y_p = (P r)_i - sum_c F(i,c) y_c
// Backward row i:                              x_p = D^+_i y_p - sum_c F(c,i) x_c
// Vectors and indices are positions.  The sum of a row is taken in chunks of
// kChunk consecutive products (ascending column): each chunk sum is a left
// fold from its first product, and the row value is the start value minus
// the chunk sums, folded left in chunk order.  Chunks are independent, so a
// long row is spread over a wave or a workgroup.
#pragma once

#include "device.hpp"
#include "internal.hpp"

namespace parac {

constexpr int kChunk = 64;

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

__device__ __forceinline__ double shfl_t(double v, int l) { return shfl_f64(v, l); }
__device__ __forceinline__ float shfl_t(float v, int l) { return __shfl(v, l, kWave); }

// sum of fv[e] vec[idx[e]] over e in [a, end) (end - a <= kChunk), a left
// fold from the first product; the loads of up to eight entries are issued
// together (the last batch predicated) before their products are added
template <typename T>
__device__ __forceinline__ T chunk_sum(int64_t a, int64_t end, const int32_t *__restrict__ idx,
                                       const T *__restrict__ fv, const T *vec) {
  T c = (T)0;
  for (int64_t e = a; e < end; e += 8) {
    int32_t ci[8];
    T f[8], v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const bool in = e + u < end;
      ci[u] = in ? idx[e + u] : 0;
      f[u] = in ? fv[e + u] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = e + u < end ? vec[ci[u]] : (T)0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (e + u < end) {
        const T p = f[u] * v[u];
        c = (e == a && u == 0) ? p : c + p;
      }
    }
  }
  return c;
}

// one thread: the whole row
template <typename T>
__device__ __forceinline__ T row_thread(T acc, int64_t e0, int64_t e1,
                                        const int32_t *__restrict__ idx,
                                        const T *__restrict__ fv, const T *vec) {
  for (int64_t a = e0; a < e1; a += kChunk) {
    const int64_t end = a + kChunk < e1 ? a + kChunk : e1;
    acc = acc - chunk_sum<T>(a, end, idx, fv, vec);
  }
  return acc;
}

// one wave: lane l sums chunk l of each round of 64 chunks; every lane folds
// the round's chunk sums in order (all lanes return the row value)
template <typename T>
__device__ __forceinline__ T row_wave(T acc, int64_t e0, int64_t e1,
                                      const int32_t *__restrict__ idx, const T *__restrict__ fv,
                                      const T *vec) {
  const int l = lane();
  for (int64_t base = e0; base < e1; base += (int64_t)kWave * kChunk) {
    const int64_t a = base + (int64_t)l * kChunk;
    T c = (T)0;
    if (a < e1) c = chunk_sum<T>(a, a + kChunk < e1 ? a + kChunk : e1, idx, fv, vec);
    const int64_t left = (e1 - base + kChunk - 1) / kChunk;
    const int nch = left < kWave ? (int)left : kWave;
    for (int k = 0; k < nch; ++k) acc = acc - shfl_t(c, k);
  }
  return acc;
}

// one workgroup of NT threads: thread t sums chunk t of each round, thread 0
// folds the round's chunk sums in order (the value is valid in thread 0)
constexpr int kGroupThreads = 1024;

template <typename T, int NT>
__device__ __forceinline__ T row_group(T acc, int64_t e0, int64_t e1,
                                       const int32_t *__restrict__ idx,
                                       const T *__restrict__ fv, const T *vec, T *cs) {
  const int t = threadIdx.x;
  for (int64_t base = e0; base < e1; base += (int64_t)NT * kChunk) {
    const int64_t a = base + (int64_t)t * kChunk;
    T c = (T)0;
    if (a < e1) c = chunk_sum<T>(a, a + kChunk < e1 ? a + kChunk : e1, idx, fv, vec);
    cs[t] = c;
    __syncthreads();
    if (t == 0) {
      const int64_t left = (e1 - base + kChunk - 1) / kChunk;
      const int nch = left < NT ? (int)left : NT;
      int k = 0;
      for (; k + 8 <= nch; k += 8) {
        T w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) w[u] = cs[k + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = acc - w[u];
      }
      for (; k < nch; ++k) acc = acc - cs[k];
    }
    __syncthreads();
  }
  return acc;
}

// row classes of a wide level: positions ordered [thread rows | wave rows |
// group rows] per direction, cnt[2L] thread rows and cnt[2L+1] wave rows.
// One launch per level, workgroups of kThrThreads: a level with thread rows
// only uses the lean kernel; otherwise the mixed one, whose workgroups take
// kThrThreads thread rows, kThrThreads / 64 wave rows, or one group row.
constexpr int kWaveRowMin = kChunk + 1;          // more entries: a wave
constexpr int kGroupRowMin = kWave * kChunk + 1;  // more entries: a workgroup
constexpr int kThrThreads = 256;
constexpr int kWavesPerGroup = kThrThreads / kWave;

struct LevelSplit {
  int64_t p0;
  int nthr, nwave, ngrp;
  int tb, wb;  // workgroups of thread rows, of wave rows
};

__device__ __forceinline__ LevelSplit level_split(const int64_t *lptr, const int32_t *cnt,
                                                  int64_t L) {
  LevelSplit s;
  s.p0 = lptr[L];
  const int nrows = (int)(lptr[L + 1] - s.p0);
  s.nthr = cnt[2 * L];
  s.nwave = cnt[2 * L + 1];
  s.ngrp = nrows - s.nthr - s.nwave;
  s.tb = (s.nthr + kThrThreads - 1) / kThrThreads;
  s.wb = (s.nwave + kWavesPerGroup - 1) / kWavesPerGroup;
  return s;
}

// workgroup lb of a level: row(pos, kind) for its rows, kind 0 thread,
// 1 wave, 2 group (uniform per thread, wave, workgroup respectively)
template <bool MIXED, typename RowFn>
__device__ __forceinline__ void level_rows(const int64_t *lptr, const int32_t *cnt,
                                           const int32_t *list, int64_t L, int lb, RowFn row) {
  if (!MIXED) {
    const int k = lb * kThrThreads + (int)threadIdx.x;
    if (k < cnt[2 * L]) row(list[lptr[L] + k], 0);
    return;
  }
  const LevelSplit s = level_split(lptr, cnt, L);
  if (lb < s.tb) {
    const int k = lb * kThrThreads + (int)threadIdx.x;
    if (k < s.nthr) row(list[s.p0 + k], 0);
  } else if (lb < s.tb + s.wb) {
    const int w = (lb - s.tb) * kWavesPerGroup + (int)(threadIdx.x >> 6);
    if (w < s.nwave) row(list[s.p0 + s.nthr + w], 1);
  } else {
    row(list[s.p0 + s.nthr + s.nwave + (lb - s.tb - s.wb)], 2);
  }
}

template <typename T>
__device__ __forceinline__ T row_kind(int kind, T start, int64_t e0, int64_t e1,
                                      const int32_t *__restrict__ idx, const T *__restrict__ fv,
                                      const T *vec, T *cs, bool &writer) {
  if (kind == 0) {
    writer = true;
    return row_thread<T>(start, e0, e1, idx, fv, vec);
  }
  if (kind == 1) {
    writer = lane() == 0;
    return row_wave<T>(start, e0, e1, idx, fv, vec);
  }
  writer = threadIdx.x == 0;
  return row_group<T, kThrThreads>(start, e0, e1, idx, fv, vec, cs);
}

template <typename T, bool MIXED>
__device__ __forceinline__ void fwd_level(const SolveArgs &a, int64_t L, int lb,
                                          const double *__restrict__ r, T *y, T *cs) {
  const T *fv = FactorVals<T>::fwd(a);
  level_rows<MIXED>(a.lptr, a.fcnt, a.flist, L, lb, [&](int64_t pos, int kind) {
    bool writer;
    const T v = row_kind<T>(kind, (T)r[a.src[pos]], a.lf_ptr[pos], a.lf_ptr[pos + 1], a.lf_idx,
                            fv, y, cs, writer);
    if (writer) y[pos] = v;
  });
}

template <typename T, bool MIXED>
__device__ __forceinline__ void bwd_level(const SolveArgs &a, int64_t L, int lb,
                                          const T *__restrict__ y, T *x, double *z, T *cs) {
  const T *fv = FactorVals<T>::bwd(a);
  level_rows<MIXED>(a.lptr, a.bcnt, a.blist, L, lb, [&](int64_t pos, int kind) {
    bool writer;
    const T v = row_kind<T>(kind, FactorVals<T>::dinv(a)[pos] * y[pos], a.lb_ptr[pos],
                            a.lb_ptr[pos + 1], a.lb_idx, fv, x, cs, writer);
    if (writer) {
      x[pos] = v;
      z[a.src[pos]] = (double)v;
    }
  });
}

// ---------------------------------------------------------------------------
// The thin tail (levels L0 .. depth-1, at most kTThreads rows and kTStage
// entries per level in each direction) by one workgroup of kTThreads.  Per
// level: the products of all entries are staged in LDS, every chunk of every
// row is summed by one thread, then every row folds its chunk sums.  Level
// L+1's loads (row ranges, indices, values, starting values) are issued
// while level L is folded, and level bounds are read two levels ahead.
// ---------------------------------------------------------------------------
constexpr int kTThreads = 1024;
constexpr int kTPer = 16;                     // staged entries per thread
constexpr int kTPre = 4;                      // of which prefetched a level ahead
constexpr int kTStage = kTThreads * kTPer;   // entries of one tail level at most
static_assert(kTStage == kTailEntries && kTThreads == kTailWidth, "tail limits");
static_assert(kWavesPerGroup == kWavesPerGroupHost && kThrThreads == kThrThreadsHost,
              "wide-level workgroups");
constexpr int kTChunks = kTStage / kChunk + kTThreads;  // chunks of one level at most

template <typename T>
struct TailShared {
  T stage[kTStage];
  T cs[kTChunks];
  int32_t choff[kTThreads + 1];  // first chunk of each row (exclusive scan)
  int32_t rs[kTThreads];         // first staged entry of each row
  int32_t re[kTThreads];         // end of each row's staged entries
  int32_t wsum[kTThreads / kWave];
};

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
  int32_t c[kTPre];
  T f[kTPre];
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
#pragma unroll
  for (int u = 0; u < kTPre; ++u) {
    const int64_t q = b.q0 + threadIdx.x + (int64_t)u * kTThreads;
    t.c[u] = q < b.q1 ? idx[q] : 0;
    t.f[u] = q < b.q1 ? fv[q] : (T)0;
  }
}

// gather the vector values of a level (prefetched indices)
template <typename T>
__device__ __forceinline__ void tail_gather(const TailBounds &b, const TailPre<T> &cur,
                                            const T *vec, T (&v)[kTPre]) {
#pragma unroll
  for (int u = 0; u < kTPre; ++u) {
    const int64_t q = b.q0 + threadIdx.x + (int64_t)u * kTThreads;
    v[u] = q < b.q1 ? vec[cur.c[u]] : (T)0;
  }
}

// one level: stage products, sum chunks, fold rows; returns this thread's
// row value
template <typename T>
__device__ __forceinline__ T tail_level(const TailBounds &b, const TailPre<T> &cur,
                                        const T (&v)[kTPre], const int32_t *__restrict__ idx,
                                        const T *__restrict__ fv, const T *vec,
                                        TailShared<T> &S) {
  const int t = threadIdx.x, l = lane(), w = t >> 6;
  const bool valid = b.p0 + t < b.p1;
#pragma unroll
  for (int u = 0; u < kTPre; ++u) {
    const int64_t q = b.q0 + t + (int64_t)u * kTThreads;
    if (q < b.q1) S.stage[q - b.q0] = cur.f[u] * v[u];
  }
  // the rest of a large level, four entries per thread at a time
  for (int ub = kTPre; ub < kTPer && b.q0 + (int64_t)ub * kTThreads < b.q1; ub += 4) {
    int32_t cc[4];
    T ff[4], vv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t q = b.q0 + t + (int64_t)(ub + u) * kTThreads;
      cc[u] = q < b.q1 ? idx[q] : 0;
      ff[u] = q < b.q1 ? fv[q] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t q = b.q0 + t + (int64_t)(ub + u) * kTThreads;
      vv[u] = q < b.q1 ? vec[cc[u]] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t q = b.q0 + t + (int64_t)(ub + u) * kTThreads;
      if (q < b.q1) S.stage[q - b.q0] = ff[u] * vv[u];
    }
  }
  // chunk offsets of the rows: exclusive scan of their chunk counts
  const int m = valid ? (int)(cur.e1 - cur.e0) : 0;
  const int nch = (m + kChunk - 1) / kChunk;
  int incl = nch;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(incl, o, kWave);
    if (l >= o) incl += y;
  }
  if (l == kWave - 1) S.wsum[w] = incl;
  __syncthreads();
  int wbase = 0;
  for (int k = 0; k < w; ++k) wbase += S.wsum[k];
  int total = 0;
  for (int k = 0; k < kTThreads / kWave; ++k) total += S.wsum[k];
  const int first = wbase + incl - nch;
  if (valid) {
    S.choff[t] = first;
    S.rs[t] = (int)(cur.e0 - b.q0);
    S.re[t] = (int)(cur.e1 - b.q0);
  }
  const int nr = (int)(b.p1 - b.p0);
  if (t == 0) S.choff[nr] = total;
  __syncthreads();
  // chunk sums: chunk j belongs to the row r with choff[r] <= j < choff[r+1]
  for (int j = t; j < total; j += kTThreads) {
    int lo = 0, hi = nr;  // choff[lo] <= j < choff[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (S.choff[mid] <= j) lo = mid;
      else hi = mid;
    }
    const int a = S.rs[lo] + (j - S.choff[lo]) * kChunk;
    const int end = a + kChunk < S.re[lo] ? a + kChunk : S.re[lo];
    T c = S.stage[a];
    int e = a + 1;
    for (; e + 8 <= end; e += 8) {
      T x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = S.stage[e + u];
#pragma unroll
      for (int u = 0; u < 8; ++u) c = c + x[u];
    }
    for (; e < end; ++e) c = c + S.stage[e];
    S.cs[j] = c;
  }
  __syncthreads();
  T acc = cur.acc;
  if (valid)
    for (int k = 0; k < nch; ++k) acc = acc - S.cs[first + k];
  return acc;
}

// Per level: gather the current level's values first, then issue the next
// level's loads (vector loads complete in issue order, so waiting for the
// gather does not wait for the prefetch), then stage and fold.
template <typename T>
__device__ __forceinline__ void tail_fwd(const SolveArgs &a, const double *__restrict__ r, T *y,
                                         TailShared<T> &S) {
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
    T v[kTPre];
    tail_gather<T>(b, cur, y, v);
    TailPre<T> nxt;
    const bool more = L + 1 < a.depth;
    TailBounds bnn = bn;
    if (more) {
      tail_prefetch<T, false>(a, bn, a.lf_ptr, a.lf_idx, fv, y, nxt);
      if (L + 2 < a.depth) bnn = tail_bounds(a.lptr, a.lqf, L + 2);
    }
    const T val = tail_level<T>(b, cur, v, a.lf_idx, fv, y, S);
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
                                         double *z, TailShared<T> &S) {
  if (a.L0 >= a.depth) return;
  const T *fv = FactorVals<T>::bwd(a);
  const int64_t Lt = a.depth - 1;
  TailBounds b = tail_bounds(a.lptr, a.lqb, Lt);
  TailBounds bn = Lt - 1 >= a.L0 ? tail_bounds(a.lptr, a.lqb, Lt - 1) : b;
  TailPre<T> cur;
  tail_prefetch<T, true>(a, b, a.lb_ptr, a.lb_idx, fv, y, cur);
  for (int64_t L = Lt; L >= a.L0; --L) {
    T v[kTPre];
    tail_gather<T>(b, cur, x, v);
    TailPre<T> nxt;
    const bool more = L - 1 >= a.L0;
    TailBounds bnn = bn;
    if (more) {
      tail_prefetch<T, true>(a, bn, a.lb_ptr, a.lb_idx, fv, y, nxt);
      if (L - 2 >= a.L0) bnn = tail_bounds(a.lptr, a.lqb, L - 2);
    }
    const T val = tail_level<T>(b, cur, v, a.lb_idx, fv, x, S);
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
