// setup.hip -- input classification, relabelling, label-space upper adjacency,
// initial dependency counters and ready queue; exclusive scans.
//
// The dependency counter of a label b starts at the number of its
// lower-labelled neighbours (the initialisation of §III); labels with no such
// neighbour form the initial ready queue.  Input classification follows the
// sign convention of §V: off-diagonals are -w_ij <= 0, and a positive row
// excess makes the matrix SDDM, factored through a ground vertex with the
// last label n.
#include <float.h>

#include "device.hpp"
#include "internal.hpp"

namespace parac {

// --------------------------------------------------------------------------
// CSR validation and excess s_i = a_ii - (left fold of w_ij, ascending j).
// Errors are reported deterministically: the key (phase, row, code) is
// min-reduced, so structural defects (phase 0) win over sign/symmetry/excess
// defects (phase 1), which win over permutation defects (phase 2), and within
// a phase the lowest row wins.
// --------------------------------------------------------------------------
__device__ __forceinline__ void report(unsigned long long *key, int phase, int64_t row, int code) {
  unsigned long long k = ((unsigned long long)phase << 60) | ((unsigned long long)row << 8) |
                         (unsigned long long)(-code);
  atomicMin(key, k);
}

__global__ void k_check_csr(int64_t n, int64_t nnz, const int64_t *__restrict__ rowptr,
                            const int32_t *__restrict__ col, const double *__restrict__ val,
                            double *__restrict__ excess, unsigned long long *errkey,
                            int *any_excess) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && (rowptr[0] != 0 || rowptr[n] != nnz)) report(errkey, 0, 0, PARAC_EINVAL);
  if (i >= n) return;
  int64_t b = rowptr[i], e = rowptr[i + 1];
  if (b < 0 || e < b || e > nnz) { report(errkey, 0, i, PARAC_EINVAL); return; }
  // structure: column range, strictly increasing, finite values
  int32_t prev = -1;
  for (int64_t p = b; p < e; ++p) {
    int32_t j = col[p];
    if (j < 0 || j >= n || j <= prev || !isfinite(val[p])) { report(errkey, 0, i, PARAC_EINVAL); return; }
    prev = j;
  }
  // sign convention, symmetry, excess
  double diag = 0.0, acc = 0.0;
  int64_t deg = 0;
  for (int64_t p = b; p < e; ++p) {
    int32_t j = col[p];
    double a = val[p];
    if (j == i) { diag = a; continue; }
    if (a == 0.0) continue;
    if (a > 0.0) { report(errkey, 1, i, PARAC_ENOTLAP); return; }
    // a_ji must be stored with the same value (row j is searched with its
    // bounds clamped, so a malformed row j cannot send the search astray)
    int64_t lo = rowptr[j], hi = rowptr[j + 1];
    lo = lo < 0 ? 0 : (lo > nnz ? nnz : lo);
    hi = hi < lo ? lo : (hi > nnz ? nnz : hi);
    const int64_t end_j = hi;
    while (lo < hi) {
      int64_t mid = lo + (hi - lo) / 2;
      if (col[mid] < (int32_t)i) lo = mid + 1; else hi = mid;
    }
    if (lo >= end_j || col[lo] != (int32_t)i || val[lo] != a) {
      report(errkey, 1, i, PARAC_EINVAL);
      return;
    }
    acc += -a;
    ++deg;
  }
  double s = diag - acc;
  double tol = 4.0 * (double)(deg + 1) * DBL_EPSILON * fabs(diag);
  if (s < -tol) { report(errkey, 1, i, PARAC_ENOTLAP); return; }
  if (s <= tol) s = 0.0;
  excess[i] = s;
  if (s > 0.0) __hip_atomic_store(any_excess, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

hipError_t launch_check_csr(int64_t n, int64_t nnz, const int64_t *rowptr, const int32_t *col,
                            const double *val, double *excess, unsigned long long *errkey,
                            int *any_excess, hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_check_csr, dim3((unsigned)blocks), dim3(256), 0, s, n, nnz, rowptr, col,
                     val, excess, errkey, any_excess);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// permutation check and inverse
// --------------------------------------------------------------------------
__global__ void k_check_perm(int64_t n, const int32_t *__restrict__ perm, int32_t *seen,
                             int32_t *iperm, unsigned long long *errkey) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int32_t l = perm ? perm[v] : (int32_t)v;
  if (l < 0 || l >= n) { report(errkey, 2, v, PARAC_EINVAL); return; }
  if (atomicExch(&seen[l], 1) != 0) { report(errkey, 2, v, PARAC_EINVAL); return; }
  iperm[l] = (int32_t)v;
}

hipError_t launch_check_perm(int64_t n, const int32_t *perm, int32_t *seen, int32_t *iperm,
                             unsigned long long *errkey, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_perm, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, perm,
                     seen, iperm, errkey);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// upper adjacency counts and initial dependency counters
// --------------------------------------------------------------------------
__global__ void k_upper_count(int64_t n, const int64_t *__restrict__ rowptr,
                              const int32_t *__restrict__ col, const double *__restrict__ val,
                              const int32_t *__restrict__ perm, const double *__restrict__ excess,
                              int sddm, int32_t *ucnt, int32_t *dp) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool ground_edge = false;
  if (i < n) {
    int32_t a = perm[i];
    int32_t up = 0, low = 0;
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
      int32_t j = col[p];
      if (j == i || val[p] == 0.0) continue;
      if (perm[j] > a) ++up; else ++low;
    }
    ground_edge = sddm && excess[i] > 0.0;
    if (ground_edge) ++up;
    ucnt[a] = up;
    dp[a] = low;
  }
  if (sddm) {
    // the ground vertex (label n) has every excess vertex below it
    uint64_t m = __ballot(ground_edge);
    if (lane() == 0 && m) atomicAdd(&dp[n], (int32_t)__popcll(m));
  }
}

hipError_t launch_upper_count(int64_t n, const int64_t *rowptr, const int32_t *col,
                              const double *val, const int32_t *perm, const double *excess,
                              int sddm, int32_t *ucnt, int32_t *dp, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_upper_count, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                     rowptr, col, val, perm, excess, sddm, ucnt, dp);
  return hipGetLastError();
}

__global__ void k_upper_fill(int64_t n, const int64_t *__restrict__ rowptr,
                             const int32_t *__restrict__ col, const double *__restrict__ val,
                             const int32_t *__restrict__ perm, const double *__restrict__ excess,
                             int sddm, const int64_t *__restrict__ uptr, int32_t *uidx,
                             double *uw) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t a = perm[i];
  int64_t o = uptr[a];
  for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
    int32_t j = col[p];
    if (j == i || val[p] == 0.0) continue;
    int32_t b = perm[j];
    if (b > a) {
      uidx[o] = b;
      uw[o] = -val[p];
      ++o;
    }
  }
  if (sddm && excess[i] > 0.0) {
    uidx[o] = (int32_t)n;
    uw[o] = excess[i];
  }
}

hipError_t launch_upper_fill(int64_t n, const int64_t *rowptr, const int32_t *col,
                             const double *val, const int32_t *perm, const double *excess,
                             int sddm, const int64_t *uptr, int32_t *uidx, double *uw,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_upper_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, rowptr,
                     col, val, perm, excess, sddm, uptr, uidx, uw);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// initial ready queue: labels with no lower neighbour, appended to the shard
// label & (kSubQueues - 1); one atomic per wave and shard
// --------------------------------------------------------------------------
__global__ void k_queue_init(int64_t ntot, const int32_t *__restrict__ dp, int32_t *q,
                             int32_t *qtail, int32_t cap_q) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool ready = v < ntot && dp[v] == 0;
  int x = (int)(v & (kSubQueues - 1));
  // lanes of one wave hold consecutive labels: shard = lane & 63 is distinct
  // per lane, so each ready lane appends on its own shard
  if (ready) {
    int pos = atomicAdd(&qtail[x * kTailStride], 1);
    q[(int64_t)x * cap_q + pos] = (int32_t)v;
  }
}

hipError_t launch_queue_init(int64_t ntot, const int32_t *dp, int32_t *q, int32_t *qtail,
                             int32_t cap_q, hipStream_t s) {
  if (ntot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_queue_init, dim3((unsigned)((ntot + 255) / 256)), dim3(256), 0, s, ntot,
                     dp, q, qtail, cap_q);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// exclusive scan of int32 counts into int64 offsets: tiles of 4096 elements
// scanned in LDS, tile totals scanned by one block, offsets added back
// --------------------------------------------------------------------------
constexpr int kScanT = 1024, kScanItems = 4, kScanTile = kScanT * kScanItems;

__device__ int64_t block_excl_scan(int64_t v, int64_t *sh, int64_t *total) {
  // Hillis-Steele over the block in LDS (integers: order irrelevant)
  int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanT; off <<= 1) {
    int64_t a = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  int64_t incl = sh[t];
  *total = sh[kScanT - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kScanT) void k_scan_tiles(const int32_t *__restrict__ cnt,
                                                       int64_t *out, int64_t n,
                                                       int64_t *tile_tot) {
  __shared__ int64_t sh[kScanT];
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t loc[kScanItems];
  int64_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    loc[k] = s;
    s += i < n ? cnt[i] : 0;
  }
  int64_t tot;
  int64_t pre = block_excl_scan(s, sh, &tot);
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    if (i < n) out[i] = pre + loc[k];
  }
  if (threadIdx.x == 0) tile_tot[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanT) void k_scan_totals(int64_t *tile_tot, int64_t ntiles,
                                                        int64_t *out_total) {
  __shared__ int64_t sh[kScanT];
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < ntiles; b0 += kScanT) {
    int64_t i = b0 + threadIdx.x;
    int64_t v = i < ntiles ? tile_tot[i] : 0;
    int64_t tot;
    int64_t pre = block_excl_scan(v, sh, &tot);
    if (i < ntiles) tile_tot[i] = carry + pre;
    carry += tot;
  }
  if (threadIdx.x == 0) *out_total = carry;
}

__global__ void k_scan_add(int64_t *out, int64_t n, const int64_t *__restrict__ tile_off) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += tile_off[i / kScanTile];
}

size_t scan_tmp_bytes(int64_t n) {
  int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  return (size_t)(ntiles + 1) * sizeof(int64_t);
}

hipError_t scan_counts(const int32_t *cnt, int64_t *out, int64_t n, void *tmp, size_t tmp_bytes,
                       hipStream_t s) {
  int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  if ((size_t)(ntiles + 1) * sizeof(int64_t) > tmp_bytes) return hipErrorInvalidValue;
  int64_t *tt = (int64_t *)tmp;
  if (n == 0) return hipMemsetAsync(out, 0, sizeof(int64_t), s);
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(kScanT), 0, s, cnt, out, n, tt);
  hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanT), 0, s, tt, ntiles, out + n);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n, tt);
  return hipGetLastError();
}

}  // namespace parac
