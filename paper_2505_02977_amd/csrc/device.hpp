// device.hpp -- wave64 building blocks for the gfx950 kernels: lane utilities,
// agent-scope atomics and fences, the counter-based sampler, bitonic networks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace parac {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// lanes
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  int l = lane();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// index of the j-th set bit of m (0-based); m must have more than j bits set
__device__ __forceinline__ int select_bit(uint64_t m, int j) {
  int base = 0;
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) {
    uint64_t low = m & ((w == 64) ? ~0ull : ((1ull << w) - 1));
    int c = __popcll(low);
    if (j >= c) {
      j -= c;
      m >>= w;
      base += w;
    } else {
      m = low;
    }
  }
  return base;
}

template <typename T>
__device__ __forceinline__ T shfl(T v, int src) { return __shfl(v, src, kWave); }

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
  return (uint64_t)__shfl((unsigned long long)v, src, kWave);
}

__device__ __forceinline__ double shfl_f64(double v, int src) {
  return __shfl(v, src, kWave);
}

__device__ __forceinline__ int first_lane_i32(int v) {
  return __builtin_amdgcn_readfirstlane(v);
}

// ---------------------------------------------------------------------------
// atomics and fences (agent scope: the whole device, across XCDs)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T ld_acq_relaxed(const T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_relaxed(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T fetch_add(T *p, T v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T fetch_max(T *p, T v) {
  return __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void fence_acquire() {
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}
__device__ __forceinline__ void fence_release() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
}
__device__ __forceinline__ void fence_acq_rel() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
}
// the compiler keeps memory accesses on their side of this point
__device__ __forceinline__ void compiler_fence() { __atomic_signal_fence(__ATOMIC_SEQ_CST); }
// wait until every earlier memory access of this wave has completed; with
// agent-scope (cache-coherent) stores this makes them visible to the agent
// before any later access is issued.  s_waitcnt vmcnt(0) expcnt(7)
// lgkmcnt(15) in the GFX9 encoding.
__device__ __forceinline__ void store_wait() {
  compiler_fence();
  __builtin_amdgcn_s_waitcnt(0x0F70);
  compiler_fence();
}
// orders this wave's own global/LDS accesses (same CU)
__device__ __forceinline__ void fence_wave_local() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// first error wins
__device__ __forceinline__ void set_error(int *err, int code) {
  int expected = 0;
  __hip_atomic_compare_exchange_strong(err, &expected, code, __ATOMIC_RELAXED,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t now_ticks() { return wall_clock64(); }

// exponential back-off for spin loops: 64 .. 512 cycles between polls.  A
// longer cap delays the pickup of a ready pivot on the critical path (a cap
// of 4096 cycles made the elimination 2% slower); callers whose wait is
// known to be long (a queue slot far behind its tail) sleep more on their own.
struct Backoff {
  int step = 0;
  __device__ __forceinline__ void pause() {
    switch (step) {
      case 0: __builtin_amdgcn_s_sleep(1); break;
      case 1: __builtin_amdgcn_s_sleep(2); break;
      case 2: __builtin_amdgcn_s_sleep(4); break;
      default: __builtin_amdgcn_s_sleep(8); break;
    }
    if (step < 3) ++step;
  }
};

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11): 2 x (64x64 -> 128) multiplies per
// round, Weyl key schedule.  Only the first output word is needed.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t philox_first_word(uint64_t c0, uint64_t c1, uint64_t c2,
                                                      uint64_t c3, uint64_t k0, uint64_t k1) {
  const uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
  const uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t h0 = __umul64hi(kM0, c0), l0 = kM0 * c0;
    uint64_t h1 = __umul64hi(kM1, c2), l1 = kM1 * c2;
    uint64_t n0 = h1 ^ c1 ^ k0, n2 = h0 ^ c3 ^ k1;
    c0 = n0;
    c1 = l1;
    c2 = n2;
    c3 = l0;
    k0 += kW0;
    k1 += kW1;
  }
  return c0;
}

// uniform double in [0,1) with 53 random bits: (x >> 11) * 2^-53 (exact)
__device__ __forceinline__ double draw_unit(uint64_t seed, uint32_t k, uint32_t s) {
  uint64_t x = philox_first_word((uint64_t)k, (uint64_t)s, 0, 0, seed, 0);
  return (double)(x >> 11) * 0x1.0p-53;
}

// ---------------------------------------------------------------------------
// Sort keys
// ---------------------------------------------------------------------------
// merge key: (u, src) with src = -1 for an input edge -> unique 64-bit key
__device__ __forceinline__ uint64_t merge_key(int32_t u, int32_t src) {
  return ((uint64_t)(uint32_t)u << 32) | (uint64_t)(uint32_t)(src + 1);
}

// positive doubles order like their bit patterns
__device__ __forceinline__ uint64_t dbits(double w) { return (uint64_t)__double_as_longlong(w); }
__device__ __forceinline__ double bitsd(uint64_t b) { return __longlong_as_double((long long)b); }

// (wbits, u) lexicographic
__device__ __forceinline__ bool less_wu(uint64_t wa, int32_t ua, uint64_t wb, int32_t ub) {
  return wa < wb || (wa == wb && ua < ub);
}

// One compare-exchange step of the bitonic network across lanes, in its
// direction-free form: stage `p` (block size), step `j`; the first step of
// each stage compares with the mirrored lane, later ones with lane ^ j.
// Lanes beyond the data hold +inf keys, so the network needs no padding.
__device__ __forceinline__ int bitonic_partner(int l, int p, int j, bool first) {
  return first ? (l ^ (p - 1)) : (l ^ j);
}


// ---------------------------------------------------------------------------
// Stable LSD radix sort of (key, payload) pairs, 8-bit digits at the given
// shifts, ping-ponging between two buffers.  A pass is a 256-bucket
// histogram in LDS, an exclusive scan of it, and a stable scatter in index
// order with in-wave ranks from ballots.  The histogram and the scatter work
// on an index range, so that several waves can share a pass (each takes a
// contiguous range, the scan orders the ranges).  Every lane issues the same
// global loads and stores in every chunk (lanes past the end read the last
// element of the range and store to a sink), so the wait for prefetched
// loads does not also wait for stores of the same group.
// ---------------------------------------------------------------------------
static __device__ uint64_t g_radix_sink[2];
constexpr int kRadixGroup = 8;  // chunks of 64 whose loads are issued together

// h[digit] += count of the keys in [lo, hi) (h in LDS, owned by this wave);
// a digit is the BITS bits of the key from bit sh on
template <typename K, int BITS = 8>
__device__ __forceinline__ void radix_count(const K *ks, int lo, int hi, int sh, int *h) {
  const int l = lane();
  for (int base = lo; base < hi; base += kRadixGroup * kWave) {
    K kk[kRadixGroup];
#pragma unroll
    for (int q = 0; q < kRadixGroup; ++q) {
      const int i = base + q * kWave + l;
      kk[q] = ks[i < hi ? i : hi - 1];
    }
#pragma unroll
    for (int q = 0; q < kRadixGroup; ++q)
      if (base + q * kWave + l < hi)
        atomicAdd(&h[(int)(((uint64_t)kk[q] >> sh) & ((1u << BITS) - 1))], 1);
  }
}

// stable scatter of [lo, hi) to the running bucket offsets h (LDS, owned by
// this wave), 64 elements at a time in index order; the loads of eight
// chunks are issued together, so waiting for them waits for the previous
// group's stores once per eight chunks (loads and stores share one counter)
template <typename K, typename V, int BITS = 8>
__device__ __forceinline__ void radix_scatter(const K *ks, const V *vs, K *kd, V *vd, int lo,
                                              int hi, int sh, int *h) {
  static_assert(sizeof(K) <= 8 && sizeof(V) <= 8, "sink holds 8-byte values");
  const int l = lane();
  K *const sink_k = (K *)&g_radix_sink[0];
  V *const sink_v = (V *)&g_radix_sink[1];
  for (int base = lo; base < hi; base += kRadixGroup * kWave) {
    K kk[kRadixGroup];
    V vv[kRadixGroup];
#pragma unroll
    for (int q = 0; q < kRadixGroup; ++q) {
      const int i = base + q * kWave + l;
      const int ic = i < hi ? i : hi - 1;
      kk[q] = ks[ic];
      vv[q] = vs[ic];
    }
#pragma unroll
    for (int q = 0; q < kRadixGroup; ++q) {
      if (base + q * kWave >= hi) break;  // uniform
      const int i = base + q * kWave + l;
      const bool valid = i < hi;
      const K k = kk[q];
      const V v = vv[q];
      const int d = (int)(((uint64_t)k >> sh) & ((1u << BITS) - 1));
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int b = 0; b < BITS; ++b) {
        const uint64_t bm = __ballot(valid && ((d >> b) & 1));
        peers &= ((d >> b) & 1) ? bm : ~bm;
      }
      const int off = valid ? h[d] : 0;
      fence_wave_local();
      const int rank = __popcll(peers & lanemask_lt());
      K *pk = valid ? kd + off + rank : sink_k;
      V *pv = valid ? vd + off + rank : sink_v;
      *pk = k;
      *pv = v;
      if (valid && rank == 0) h[d] = off + __popcll(peers);
      fence_wave_local();
    }
  }
}

// the whole sort by one wave; returns true when the sorted data ends in the
// first buffer
template <typename K, typename V>
__device__ bool wave_radix_sort(K *ka, V *va, K *kb, V *vb, int n, const int *shifts, int npass,
                                int *h) {
  if (n <= 0) return true;
  const int l = lane();
  bool in_a = true;
  for (int pass = 0; pass < npass; ++pass) {
    const int sh = shifts[pass];
    K *ks = in_a ? ka : kb;
    V *vs = in_a ? va : vb;
    for (int t = l; t < 256; t += kWave) h[t] = 0;
    fence_wave_local();
    radix_count(ks, 0, n, sh, h);
    fence_wave_local();
    // exclusive scan of the 256 buckets, four per lane
    const int c0 = h[4 * l], c1 = h[4 * l + 1], c2 = h[4 * l + 2], c3 = h[4 * l + 3];
    const int tot = c0 + c1 + c2 + c3;
    int incl = tot;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      int y = __shfl_up(incl, o, kWave);
      if (l >= o) incl += y;
    }
    const int ex = incl - tot;
    fence_wave_local();
    h[4 * l] = ex;
    h[4 * l + 1] = ex + c0;
    h[4 * l + 2] = ex + c0 + c1;
    h[4 * l + 3] = ex + c0 + c1 + c2;
    fence_wave_local();
    radix_scatter(ks, vs, in_a ? kb : ka, in_a ? vb : va, 0, n, sh, h);
    fence_wave_local();
    in_a = !in_a;
  }
  return in_a;
}

}  // namespace parac
