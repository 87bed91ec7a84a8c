// order.hip -- elimination orders computed on the device (the input of
// parac_factor's perm), for the ordering study of the paper's §V:
//   random  a uniformly random permutation: vertices sorted by a seeded hash;
//   NNZ     ascending stored entries per row (the order the paper recommends
//           for GPUs), ties broken by the hash;
//   MIS     local-minimum rounds (Jones-Plassmann): in round r every vertex
//           whose priority is below that of all its neighbours not yet placed
//           joins the round, so each round is an independent set of the
//           graph; priorities put low-degree vertices first.  Vertices are
//           labelled round by round.
// Every rule is integer arithmetic, so the permutation is the same bits for
// a given seed on any device.
//
// Definitions (deg = stored entries of the row, capped at 2^20 - 1;
// h(i) = SplitMix64 output for state seed + i):
//   pri(i)  = deg << 24 | h(i) >> 40               (44 bits)
//   random  : labels in ascending (h(i), i)
//   NNZ     : labels in ascending (pri(i), i)
//   MIS     : round(i) = the round in which (pri(i), i) is below (pri(u), u)
//             of every neighbour u not placed in an earlier round; labels in
//             ascending (round(i), pri(i), i)
#include "device.hpp"
#include "internal.hpp"

namespace parac {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortPer = 16;  // keys per thread of a sort tile
constexpr int kSortTile = kSortThreads * kSortPer;
constexpr int kRadixBits = 4;
constexpr int kRadix = 1 << kRadixBits;

__device__ __forceinline__ uint64_t splitmix_out(uint64_t state) {
  uint64_t z = state + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// per vertex: the sort key of the order kind (MIS: its priority, the round
// is added later), and the identity as the value
__global__ void k_order_keys(int64_t n, const int64_t *__restrict__ rowptr, uint64_t seed,
                             int kind, uint64_t *key, int32_t *val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t h = splitmix_out(seed + (uint64_t)i);
  int64_t deg = rowptr[i + 1] - rowptr[i];
  if (deg > (1 << 20) - 1) deg = (1 << 20) - 1;
  key[i] = kind == PARAC_ORDER_RANDOM ? h : ((uint64_t)deg << 24) | (h >> 40);
  val[i] = (int32_t)i;
}

// one local-minimum round: an unplaced vertex joins round r when its
// (priority, index) is below that of every neighbour not placed in an
// earlier round.  A neighbour read as placed in round r was unplaced when
// the round began, so it still counts.
__global__ void k_mis_round(int64_t n, const int64_t *__restrict__ rowptr,
                            const int32_t *__restrict__ col, const uint64_t *__restrict__ pri,
                            int32_t *round, int r, unsigned long long *placed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (__hip_atomic_load(round + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= 0) return;
  const uint64_t pv = pri[i];
  for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
    const int32_t u = col[e];
    if (u == i) continue;
    const int32_t ru = __hip_atomic_load(round + u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (ru >= 0 && ru != r) continue;
    const uint64_t pu = pri[u];
    if (pu < pv || (pu == pv && u < i)) return;
  }
  __hip_atomic_store(round + i, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  atomicAdd(placed, 1ull);
}

__global__ void k_mis_key(int64_t n, const int32_t *__restrict__ round, uint64_t *key) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  key[i] = ((uint64_t)round[i] << 44) | key[i];
}

// digit counts of one tile, bucket-major: hist[d * ntiles + tile]
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(int64_t n, const uint64_t *__restrict__ key,
                                                             int shift, int32_t *hist) {
  __shared__ int32_t cnt[kRadix];
  if (threadIdx.x < kRadix) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int k = 0; k < kSortPer; ++k) {
    const int64_t i = base + (int64_t)k * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(key[i] >> shift) & (kRadix - 1)], 1);
  }
  __syncthreads();
  if (threadIdx.x < kRadix) hist[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = cnt[threadIdx.x];
}

// stable scatter of one tile: thread t owns the tile's keys
// [t * kSortPer, (t + 1) * kSortPer); a key's place is its digit's global
// offset for this tile, plus the keys of that digit owned by lower threads,
// plus those before it in its own run
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    int64_t n, const uint64_t *__restrict__ key, const int32_t *__restrict__ val, int shift,
    const int64_t *__restrict__ off, uint64_t *key_out, int32_t *val_out) {
  __shared__ int32_t cnt[kRadix][kSortThreads];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)t * kSortPer;
  uint64_t k[kSortPer];
  int32_t v[kSortPer];
  int c[kRadix];
#pragma unroll
  for (int d = 0; d < kRadix; ++d) c[d] = 0;
#pragma unroll
  for (int j = 0; j < kSortPer; ++j) {
    const int64_t i = base + j;
    k[j] = i < n ? key[i] : 0;
    v[j] = i < n ? val[i] : 0;
    if (i < n) {
      const int d = (int)((k[j] >> shift) & (kRadix - 1));
#pragma unroll
      for (int dd = 0; dd < kRadix; ++dd) c[dd] += dd == d ? 1 : 0;
    }
  }
#pragma unroll
  for (int d = 0; d < kRadix; ++d) cnt[d][t] = c[d];
  __syncthreads();
  // exclusive scan of each digit's row over the threads: 16 threads per
  // digit, 16 entries each
  {
    const int d = t / (kSortThreads / kRadix), part = t % (kSortThreads / kRadix);
    constexpr int span = kSortThreads / (kSortThreads / kRadix);
    int32_t run = 0;
    for (int j = 0; j < span; ++j) run += cnt[d][part * span + j];
    // exclusive prefix of `run` over the 16 parts (lanes of one wave: 16
    // consecutive threads share a wave)
    int32_t pre = run;
    for (int o = 1; o < kSortThreads / kRadix; o <<= 1) {
      const int32_t y = __shfl_up(pre, o, kSortThreads / kRadix);
      if (part >= o) pre += y;
    }
    pre -= run;
    for (int j = 0; j < span; ++j) {
      const int32_t x = cnt[d][part * span + j];
      cnt[d][part * span + j] = pre;
      pre += x;
    }
  }
  __syncthreads();
#pragma unroll
  for (int d = 0; d < kRadix; ++d) c[d] = cnt[d][t] + (int32_t)0;
  int64_t dst[kRadix];
#pragma unroll
  for (int d = 0; d < kRadix; ++d) dst[d] = off[(int64_t)d * gridDim.x + blockIdx.x] + c[d];
#pragma unroll
  for (int j = 0; j < kSortPer; ++j) {
    if (base + j >= n) break;
    const int d = (int)((k[j] >> shift) & (kRadix - 1));
    int64_t p = 0;
#pragma unroll
    for (int dd = 0; dd < kRadix; ++dd)
      if (dd == d) p = dst[dd]++;
    key_out[p] = k[j];
    val_out[p] = v[j];
  }
}

// perm[val[p]] = p: the label of each vertex is its place in the sorted order
__global__ void k_rank_to_perm(int64_t n, const int32_t *__restrict__ val, int32_t *perm) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  perm[val[p]] = (int32_t)p;
}

unsigned grid_of(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

int64_t order_tiles(int64_t n) { return (n + kSortTile - 1) / kSortTile; }

hipError_t launch_order_keys(int64_t n, const int64_t *rowptr, uint64_t seed, int kind,
                             uint64_t *key, int32_t *val, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_order_keys, dim3(grid_of(n, 256)), dim3(256), 0, s, n, rowptr, seed, kind,
                     key, val);
  return hipGetLastError();
}

hipError_t launch_mis_round(int64_t n, const int64_t *rowptr, const int32_t *col,
                            const uint64_t *pri, int32_t *round, int r,
                            unsigned long long *placed, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mis_round, dim3(grid_of(n, 256)), dim3(256), 0, s, n, rowptr, col, pri,
                     round, r, placed);
  return hipGetLastError();
}

hipError_t launch_mis_key(int64_t n, const int32_t *round, uint64_t *key, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mis_key, dim3(grid_of(n, 256)), dim3(256), 0, s, n, round, key);
  return hipGetLastError();
}

// stable LSD radix sort of (key, val) pairs by the low `bits` bits of key;
// the result is in (key, val) (the second buffers are scratch)
hipError_t radix_sort_pairs(int64_t n, int bits, uint64_t *key, int32_t *val, uint64_t *key2,
                            int32_t *val2, int32_t *hist, int64_t *off, void *scan_tmp,
                            size_t scan_bytes, hipStream_t s) {
  if (n <= 1) return hipSuccess;
  const int64_t tiles = order_tiles(n);
  const int passes = (bits + kRadixBits - 1) / kRadixBits;
  uint64_t *ka = key, *kb = key2;
  int32_t *va = val, *vb = val2;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * kRadixBits;
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)tiles), dim3(kSortThreads), 0, s, n, ka, shift,
                       hist);
    hipError_t e = scan_counts(hist, off, tiles * kRadix, scan_tmp, scan_bytes, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)tiles), dim3(kSortThreads), 0, s, n, ka, va,
                       shift, off, kb, vb);
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (ka != key) {
    hipError_t e = hipMemcpyAsync(key, ka, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(val, va, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t launch_rank_to_perm(int64_t n, const int32_t *val, int32_t *perm, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rank_to_perm, dim3(grid_of(n, 256)), dim3(256), 0, s, n, val, perm);
  return hipGetLastError();
}

}  // namespace parac
