// solve.hip -- the preconditioner apply z = P^T F^-T D^+ F^-1 P r and the
// kernels of preconditioned conjugate gradients.
//
// Triangular solves are sync-free: every row waits for the rows it depends
// on by polling their values, which hold a sentinel bit pattern until they
// are computed (agent-scope loads and stores, so a value is its own ready
// flag).  Rows are processed in batches of one elimination level (rows of a
// level are independent); the forward solve walks the levels upwards, the
// backward solve downwards, so every dependency lies in an earlier batch and
// the lowest unfinished batch can always complete.  Each row is folded left
// in ascending column order, the order of the CPU reference.
#include <float.h>

#include "device.hpp"
#include "internal.hpp"

namespace parac {

template <typename T> struct Bits;
template <> struct Bits<double> {
  using U = unsigned long long;
  static __device__ __forceinline__ U sent() { return (U)kSent64; }
  static __device__ __forceinline__ U to(double v) {
    U b = (U)__double_as_longlong(v);
    return b == (U)kSent64 ? 0x7FF8000000000000ull : b;
  }
  static __device__ __forceinline__ double from(U b) { return __longlong_as_double((long long)b); }
};
template <> struct Bits<float> {
  using U = unsigned int;
  static __device__ __forceinline__ U sent() { return kSent32; }
  static __device__ __forceinline__ U to(float v) {
    U b = (U)__float_as_uint(v);
    return b == kSent32 ? 0x7FC00000u : b;
  }
  static __device__ __forceinline__ float from(U b) { return __uint_as_float(b); }
};

template <typename T> __device__ __forceinline__ const T *fvals_csr(const SolveArgs &a);
template <> __device__ __forceinline__ const double *fvals_csr<double>(const SolveArgs &a) { return a.val_f; }
template <> __device__ __forceinline__ const float *fvals_csr<float>(const SolveArgs &a) { return a.val_f32; }
template <typename T> __device__ __forceinline__ const T *fvals_csc(const SolveArgs &a);
template <> __device__ __forceinline__ const double *fvals_csc<double>(const SolveArgs &a) { return a.val; }
template <> __device__ __forceinline__ const float *fvals_csc<float>(const SolveArgs &a) { return a.val32; }
template <typename T> __device__ __forceinline__ const T *dinv_of(const SolveArgs &a);
template <> __device__ __forceinline__ const double *dinv_of<double>(const SolveArgs &a) { return a.Dinv; }
template <> __device__ __forceinline__ const float *dinv_of<float>(const SolveArgs &a) { return a.Dinv32; }

constexpr int kG = 4;                 // lanes per row (triangular solves)
constexpr int kU = 4;                 // entries per lane and round
constexpr int kRound = kG * kU;       // entries of a row per round
constexpr int kRPB = kWave / kG;      // rows per batch
constexpr int kSG = 8;                // lanes per row (SpMV)
constexpr int kSRPW = kWave / kSG;    // SpMV rows per wave

// level of batch b: the largest L with bptr[L] <= b
__device__ __forceinline__ int64_t batch_level(const SolveArgs &a, int64_t b) {
  int64_t lo = 0, hi = a.depth - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) >> 1;
    if (a.bptr[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Batches are claimed in increasing order from a counter, so the lowest
// unfinished batch is always held by a running wave: nothing assumes how many
// waves are resident.  The next claim is issued before the current batch is
// solved, hiding its latency.
__device__ __forceinline__ int64_t claim(int *ctr) {
  int v = 0;
  if (lane() == 0) v = atomicAdd(ctr, 1);
  return (int64_t)__shfl(v, 0, kWave);
}

// One row per kG lanes.  A row's entries are taken kRound at a time: all
// dependency values of a round are requested at once and polled until each
// is computed (it holds the sentinel until then); the products are folded
// left in entry order.
template <typename T>
__device__ __forceinline__ T row_fold(T acc, int64_t e0, int64_t e1,
                                      const int32_t *__restrict__ idx, const T *__restrict__ fv,
                                      const T *vec, int grp, int sub, uint64_t deadline,
                                      int *err) {
  using B = Bits<T>;
  using U = typename B::U;
  for (int64_t eb = e0; __any(eb < e1); eb += kRound) {
    U bits[kU];
    int32_t jj[kU];
    T f[kU];
    bool wait[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t e = eb + sub + (int64_t)u * kG;
      const bool has = e < e1;
      jj[u] = has ? idx[e] : 0;
      f[u] = has ? fv[e] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const bool has = eb + sub + (int64_t)u * kG < e1;
      bits[u] = has ? ld_acq_relaxed((const U *)(vec + jj[u])) : (U)0;
      wait[u] = has && bits[u] == B::sent();
    }
    bool any = false;
#pragma unroll
    for (int u = 0; u < kU; ++u) any |= wait[u];
    Backoff bo;
    while (__any(any)) {
      bo.pause();
      any = false;
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        if (wait[u]) {
          const U v = ld_acq_relaxed((const U *)(vec + jj[u]));
          if (v != B::sent()) {
            bits[u] = v;
            wait[u] = false;
          } else {
            any = true;
          }
        }
      }
      if (__any(any) && now_ticks() > deadline) {
        set_error(err, PARAC_ETIMEOUT);
        break;
      }
    }
    T prod[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) prod[u] = f[u] * B::from(bits[u]);
#pragma unroll
    for (int t = 0; t < kRound; ++t) {
      const T pt = shfl(prod[t / kG], grp * kG + (t % kG));
      if (eb + t < e1) acc = acc - pt;
    }
  }
  return acc;
}

template <typename T>
__device__ __forceinline__ void publish(T *p, T v) {
  using B = Bits<T>;
  st_relaxed((typename B::U *)p, B::to(v));
}

// forward: y_i = r_{perm^-1(i)} - sum_j F_ij y_j (left fold, j ascending);
// also re-arms x_i for the backward solve
template <typename T>
__global__ __launch_bounds__(256) void k_trsv_fwd(SolveArgs a, const double *__restrict__ r, T *y,
                                                  T *x) {
  if (a.skip && *a.skip) return;
  using B = Bits<T>;
  if (blockIdx.x == 0 && threadIdx.x == 0) st_relaxed(a.claim + kTailStride, 0);  // backward's
  const int l = lane(), grp = l / kG, sub = l % kG;
  const T *fv = fvals_csr<T>(a);
  const uint64_t deadline = now_ticks() + a.timeout_ticks;
  int64_t next = claim(a.claim);
  while (next < a.nbatch) {
    const int64_t b = next;
    next = claim(a.claim);
    const int64_t L = batch_level(a, b);
    const int64_t pos = a.lptr[L] + (b - a.bptr[L]) * kRPB + grp;
    const bool valid = pos < a.lptr[L + 1];
    const int32_t i = valid ? a.order[pos] : 0;
    const int64_t e0 = valid ? a.rowptr_f[i] : 0, e1 = valid ? a.rowptr_f[i + 1] : 0;
    T acc = valid ? (T)r[a.iperm[i]] : (T)0;
    acc = row_fold<T>(acc, e0, e1, a.colind_f, fv, y, grp, sub, deadline, a.err);
    if (valid && sub == 0) {
      publish<T>(y + i, acc);
      st_relaxed((typename B::U *)(x + i), B::sent());
    }
  }
}

// backward: x_i = Dinv_i y_i - sum_{u>i} F_ui x_u (left fold, u ascending;
// the ground row of an SDDM factor is dropped); z_{perm^-1(i)} = x_i; also
// re-arms y_i for the next forward solve
template <typename T>
__global__ __launch_bounds__(256) void k_trsv_bwd(SolveArgs a, T *y, T *x, double *z) {
  if (a.skip && *a.skip) return;
  using B = Bits<T>;
  int *ctr = a.claim + kTailStride;
  if (blockIdx.x == 0 && threadIdx.x == 0) st_relaxed(a.claim, 0);  // forward's
  const int l = lane(), grp = l / kG, sub = l % kG;
  const T *fv = fvals_csc<T>(a);
  const T *dv = dinv_of<T>(a);
  const uint64_t deadline = now_ticks() + a.timeout_ticks;
  int64_t next = claim(ctr);
  while (next < a.nbatch) {
    const int64_t b = a.nbatch - 1 - next;
    next = claim(ctr);
    const int64_t L = batch_level(a, b);
    const int64_t pos = a.lptr[L] + (b - a.bptr[L]) * kRPB + grp;
    const bool valid = pos < a.lptr[L + 1];
    const int32_t i = valid ? a.order[pos] : 0;
    int64_t e0 = valid ? a.colptr[i] : 0, e1 = valid ? a.colptr[i + 1] : 0;
    if (e1 > e0 && a.rowind[e1 - 1] >= a.n) --e1;  // ground is the last row
    const T yi = valid ? B::from(ld_acq_relaxed((const typename B::U *)(y + i))) : (T)0;
    T acc = valid ? dv[i] * yi : (T)0;
    acc = row_fold<T>(acc, e0, e1, a.rowind, fv, x, grp, sub, deadline, a.err);
    if (valid && sub == 0) {
      publish<T>(x + i, acc);
      z[a.iperm[i]] = (double)acc;
      st_relaxed((typename B::U *)(y + i), B::sent());
    }
  }
}

hipError_t launch_trsv_fwd(const SolveArgs &a, const double *r, void *y, void *x, int prec,
                           int waves, hipStream_t s) {
  const int wg = (waves + 3) / 4;
  if (prec == PARAC_PREC_MIXED)
    hipLaunchKernelGGL(k_trsv_fwd<float>, dim3(wg), dim3(256), 0, s, a, r, (float *)y, (float *)x);
  else
    hipLaunchKernelGGL(k_trsv_fwd<double>, dim3(wg), dim3(256), 0, s, a, r, (double *)y,
                       (double *)x);
  return hipGetLastError();
}

hipError_t launch_trsv_bwd(const SolveArgs &a, void *y, void *x, double *z, int prec, int waves,
                           hipStream_t s) {
  const int wg = (waves + 3) / 4;
  if (prec == PARAC_PREC_MIXED)
    hipLaunchKernelGGL(k_trsv_bwd<float>, dim3(wg), dim3(256), 0, s, a, (float *)y, (float *)x, z);
  else
    hipLaunchKernelGGL(k_trsv_bwd<double>, dim3(wg), dim3(256), 0, s, a, (double *)y, (double *)x,
                       z);
  return hipGetLastError();
}

int trsv_max_waves() {
  int dev = 0, a = 0, b = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_trsv_fwd<double>, 256, 0) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_trsv_bwd<double>, 256, 0) != hipSuccess)
    return 0;
  int m = a < b ? a : b;
  int c, d2;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&c, k_trsv_fwd<float>, 256, 0) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&d2, k_trsv_bwd<float>, 256, 0) != hipSuccess)
    return 0;
  m = m < c ? m : c;
  m = m < d2 ? m : d2;
  return m * prop.multiProcessorCount * 4;
}

// ==========================================================================
// PCG building blocks (one right-hand side).  Reductions are deterministic:
// a fixed grid, a fixed LDS tree per block, then one block sums the partials
// in a fixed order.
// ==========================================================================
constexpr int kRedBlocks = 1024;
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
