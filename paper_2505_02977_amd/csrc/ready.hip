// ready.hip -- the preconditioner apply z = P^T F^{-T} D^+ F^{-1} P r as two
// dependency-driven triangular sweeps (forward over the rows of F, backward
// over its columns).
//
// Level scheduling orders the rows: a row's inputs all lie in earlier
// levels, and the unit list of each direction is in level order.  Instead
// of a launch (or a barrier) per level, every wave of one persistent launch
// claims the next unit with a ticket counter and waits for exactly the
// inputs its rows read.  An entry of a work vector holds a sentinel (a
// signalling NaN that arithmetic never produces) until its row has been
// solved; a row is published by one agent-coherent store of its value, so a
// reader sees either the sentinel or the final value and needs no fence.
// A wave only waits on rows whose units hold smaller tickets, i.e. were
// claimed by waves that are already running, so the sweep always advances.
// Every wait is bounded by a wall-clock watchdog that records an error
// instead of hanging.
//
// The arithmetic of a row is that of the level-synchronous form: the sum is
// taken in chunks of 64 consecutive products (ascending column), each chunk
// a left fold from its first product, and the row value is the start value
// minus the chunk sums in chunk order.  Which wave computes which chunk
// changes nothing in the bits.
//
// Units (int4, kind in x).  A row of m entries is taken by a group of G
// lanes (G = 1 for m <= 16, 4 for m <= 64, 16 for m <= 256, 64 for
// m <= 1024); lane q of a group reads entries 16q .. 16q+15 of the row, so
// every lane issues all its loads at once and waits once.  A chunk of 64
// products spans four lanes and is folded along them through shuffles.
//   group G  : 64/G rows of one class of one level (y = first class-list
//              index, z = number of rows)
//   block    : chunks [z, z + 16) of a row of more than 1024 entries, by the
//              64 lanes as one group (y = position, w = offset of the row's
//              chunk sums in the chunk-sum buffer)
//   fold     : the chunk sums of such a row folded into its value
//              (y = position, z = number of chunks, w = offset)
// Work vectors y (forward) and x (backward) are indexed by position.  Each
// sweep leaves the other vector all-sentinel for the next apply: the forward
// sweep resets x, the backward sweep resets y once it has read it, and a
// fold resets the chunk sums it consumed.
#include "device.hpp"
#include "internal.hpp"

namespace parac {

namespace {

template <typename T> struct Bits;
template <> struct Bits<double> {
  using U = unsigned long long;
  static constexpr U kPending = kPending64;
  static constexpr U kQuietNaN = 0x7FF8000000000000ull;
  static __device__ __forceinline__ U of(double v) { return (U)__double_as_longlong(v); }
  static __device__ __forceinline__ double val(U u) { return __longlong_as_double((long long)u); }
};
template <> struct Bits<float> {
  using U = unsigned int;
  static constexpr U kPending = kPending32;
  static constexpr U kQuietNaN = 0x7FC00000u;
  static __device__ __forceinline__ U of(float v) { return (U)__float_as_uint(v); }
  static __device__ __forceinline__ float val(U u) { return __uint_as_float(u); }
};

template <typename T>
__device__ __forceinline__ typename Bits<T>::U load_bits(const T *p) {
  using U = typename Bits<T>::U;
  return __hip_atomic_load((const U *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// publish a value: one agent-coherent store; a computed NaN whose bits
// equal the sentinel is stored as the canonical quiet NaN
template <typename T>
__device__ __forceinline__ void publish(T *p, T v) {
  using B = Bits<T>;
  typename B::U u = B::of(v);
  if (u == B::kPending) u = B::kQuietNaN;
  __hip_atomic_store((typename B::U *)p, u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ void reset(T *p) {
  using B = Bits<T>;
  __hip_atomic_store((typename B::U *)p, B::kPending, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double shfl_t(double v, int l) { return shfl_f64(v, l); }
__device__ __forceinline__ float shfl_t(float v, int l) { return __shfl(v, l, kWave); }

__device__ __forceinline__ double readlane_t(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float readlane_t(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// DPP lane moves within rows of 16 lanes: row_shr:1 (lane l gets lane l-1;
// the first lane of a row keeps 0) and quad_perm [3,3,3,3] (every lane gets
// lane 3 of its group of four)
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_t(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_i32<CTRL>((int)(unsigned)(b & 0xffffffffll));
  const int hi = dpp_i32<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_t(float v) {
  return __int_as_float(dpp_i32<CTRL>(__float_as_int(v)));
}
constexpr int kDppRowShr1 = 0x111;
constexpr int kDppQuad3 = 0xFF;

// short back-off between polls of one address: 64, 128, 256 cycles
struct PollBackoff {
  int step = 0;
  __device__ __forceinline__ void pause() {
    if (step == 0) __builtin_amdgcn_s_sleep(1);
    else if (step == 1) __builtin_amdgcn_s_sleep(2);
    else __builtin_amdgcn_s_sleep(4);
    if (step < 2) ++step;
  }
};

// the watchdog of one wave: deadline, and the sweep's error word (another
// wave's timeout stops this one too)
struct Watch {
  uint64_t deadline;
  int *err;
  bool dead;
  int polls;
  __device__ __forceinline__ bool expired() {
    if (dead) return true;
    if ((++polls & 15) == 0) {
      if (now_ticks() > deadline) set_error(err, PARAC_ETIMEOUT);
      if (ld_acq_relaxed(err) != 0) dead = true;
    }
    return dead;
  }
};

// Wait until every lane's entries v[u], u < cnt, are solved.  The
// wave polls one address at a time: of its pending entries the one solved
// last in sweep order (positions follow the levels: the highest position
// forward, DESC: the lowest backward), then reloads the others, which are
// usually solved by then.  A single polled address per wave leaves the
// memory system to the loads and stores of the rows being solved.
template <typename T, int M, bool DESC>
__device__ __forceinline__ void wait_ready(const T *vec, const int32_t (&ci)[M],
                                           int cnt, typename Bits<T>::U (&v)[M],
                                           Watch &w) {
  using B = Bits<T>;
  auto reload = [&]() {
#pragma unroll
    for (int u = 0; u < M; ++u)
      if (u < cnt && v[u] == B::kPending) v[u] = load_bits(vec + ci[u]);
  };
  for (;;) {
    int key = INT32_MIN;
#pragma unroll
    for (int u = 0; u < M; ++u) {
      const int k = DESC ? -ci[u] : ci[u];
      if (u < cnt && v[u] == B::kPending && k > key) key = k;
    }
    if (!__ballot(key != INT32_MIN)) return;
#pragma unroll
    for (int o = kWave / 2; o >= 1; o >>= 1) {
      const int y = __shfl_xor(key, o, kWave);
      key = y > key ? y : key;
    }
    const int32_t at = __builtin_amdgcn_readfirstlane(DESC ? -key : key);
    PollBackoff bo;
    while (load_bits(vec + at) == B::kPending) {
      if (__ballot(w.expired())) {
#pragma unroll
        for (int u = 0; u < M; ++u)
          if (v[u] == B::kPending) v[u] = B::kQuietNaN;
        return;
      }
      bo.pause();
    }
    reload();
  }
}

// Lane q of a group reads the entries [b + 16q, b + 16q + 16) ∩ [b, e1)
// (b: the first entry of the group's share of the row); returns the sum of
// the chunk the lane belongs to (64 products, four lanes) in the chunk's
// fourth lane, and in every lane when G == 1 (one lane, at most 16
// products).  Chunks are left folds from their first product: the first
// lane of a chunk starts the fold, the next three continue it in turn.
template <typename T, int G, bool DESC>
__device__ __forceinline__ T group_chunks(int64_t b, int64_t e1, int q, bool valid,
                                          const int32_t *__restrict__ idx,
                                          const T *__restrict__ fv, const T *vec, Watch &w) {
  using B = Bits<T>;
  const int64_t a = b + 16 * (int64_t)q;
  int32_t ci[16];
  T f[16];
  // the lane's entries are a prefix of its 16 slots
  const int64_t left = valid ? e1 - a : 0;
  const int cnt = left <= 0 ? 0 : (left < 16 ? (int)left : 16);
  typename B::U v[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    ci[u] = u < cnt ? idx[a + u] : 0;
    f[u] = u < cnt ? fv[a + u] : (T)0;
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) v[u] = u < cnt ? load_bits(vec + ci[u]) : (typename B::U)0;
  wait_ready<T, 16, DESC>(vec, ci, cnt, v, w);
  // the lane's own products, folded from its first.  An absent entry
  // contributes -0.0, which leaves every sum unchanged (x + (-0.0) = x
  // exactly, for every x), so the fold is a plain chain of additions; a lane
  // without entries passes the running sum on.
  T p[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) p[u] = u < cnt ? f[u] * B::val(v[u]) : (T)-0.0;
  auto fold = [&](T t, bool first) {
    t = first ? p[0] : t + p[0];
#pragma unroll
    for (int u = 1; u < 16; ++u) t = t + p[u];
    return t;
  };
  if constexpr (G == 1) {
    return fold((T)0, true);
  } else {
    // the four lanes of a chunk lie in one DPP row: lane l takes the running
    // sum of lane l-1
    const int st = q & 3;
    T s = (T)0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const T prev = dpp_t<kDppRowShr1>(s);
      if (st == k) s = k == 0 ? fold((T)0, true) : fold(prev, false);
    }
    return s;
  }
}

template <typename T, bool BWD>
struct Sweep {
  const ApplySlot &q;  // the system's slot
  const int64_t *ptr;
  const int32_t *idx;
  const T *fv;
  T *in;   // vector read (y forward, x backward)
  T *out;  // vector written: the same vector
  __device__ __forceinline__ Sweep(const ApplySlot &q_) : q(q_) {
    ptr = BWD ? q.a.lb_ptr : q.a.lf_ptr;
    idx = BWD ? q.a.lb_idx : q.a.lf_idx;
    fv = BWD ? FactorVals<T>::bwd(q.a) : FactorVals<T>::fwd(q.a);
    in = (T *)(BWD ? q.x : q.y);
    out = in;
  }
  // start value of a row: (P r) forward, D^+ y backward
  __device__ __forceinline__ T start(int64_t pos) const {
    if constexpr (BWD) {
      return FactorVals<T>::dinv(q.a)[pos] * ((const T *)q.y)[pos];
    } else {
      return (T)q.r[(int64_t)q.a.src[pos] * q.ldr];
    }
  }
  // publish row pos; forward resets x[pos], backward resets y[pos] and
  // writes z in the original ordering
  __device__ __forceinline__ void finish(int64_t pos, T v) const {
    publish(out + pos, v);
    if constexpr (BWD) {
      reset((T *)q.y + pos);
      q.z[(int64_t)q.a.src[pos] * q.ldz] = (double)v;
    } else {
      reset((T *)q.x + pos);
    }
  }
};

// a group unit: 64/G rows, G lanes each
template <typename T, bool BWD, int G>
__device__ __forceinline__ void group_unit(const Sweep<T, BWD> &S, const int4 &u, Watch &w) {
  const int l = lane(), r = l / G, q = l % G;
  const bool valid = r < u.z;
  const int64_t pos = valid ? (BWD ? S.q.a.blist : S.q.a.flist)[u.y + r] : 0;
  const int64_t e0 = valid ? S.ptr[pos] : 0, e1 = valid ? S.ptr[pos + 1] : 0;
  T acc = valid && q == 0 ? S.start(pos) : (T)0;  // issued before the wait
  const T c = group_chunks<T, G, BWD>(e0, e1, q, valid, S.idx, S.fv, S.in, w);
  // the row value: start minus its chunk sums in chunk order (each in the
  // fourth lane of its chunk); the group's first lane publishes it
  if constexpr (G == 1) {
    if (e1 > e0) acc = acc - c;
  } else if constexpr (G == 4) {
    const T c0 = dpp_t<kDppQuad3>(c);
    if (e1 > e0) acc = acc - c0;
  } else if constexpr (G == 16) {
    const int base = r * G;
#pragma unroll
    for (int k = 0; k < G / 4; ++k) {
      const T ck = shfl_t(c, base + 4 * k + 3);
      if (e0 + kChunk * (int64_t)k < e1) acc = acc - ck;
    }
  } else {
#pragma unroll
    for (int k = 0; k < G / 4; ++k) {
      const T ck = readlane_t(c, 4 * k + 3);
      if (e0 + kChunk * (int64_t)k < e1) acc = acc - ck;
    }
  }
  if (valid && q == 0) S.finish(pos, acc);
}

template <typename T, bool BWD>
__global__ __launch_bounds__(kReadyThreads) void k_ready(const ApplySlot *AS,
                                                         const int32_t *wgmap) {
  const ApplySlot q = AS[wgmap[blockIdx.x]];
  if (*q.a.skip) return;
  const int l = lane();
  const Sweep<T, BWD> S(q);
  const int4 *units = BWD ? q.a.task_b : q.a.task_f;
  const int nt = BWD ? q.a.ntask_b : q.a.ntask_f;
  int32_t *ctr = q.ctr + (BWD ? 1 : 0);
  T *cs = (T *)q.cs;
  Watch w{now_ticks() + q.a.timeout_ticks, q.a.err, false, 0};
  for (;;) {
    int t = 0;
    if (l == 0) t = fetch_add(ctr, 1);
    t = first_lane_i32(__shfl(t, 0, kWave));
    if (t >= nt || __ballot(w.dead)) break;
    // the first unit of a sweep clears the other sweep's counter (that sweep
    // is finished, and the next one starts after this launch)
    if (t == 0 && l == 0) st_relaxed(q.ctr + (BWD ? 0 : 1), 0);
    const int4 u = units[t];
    const int kind = first_lane_i32(u.x);
    if (kind == kUnitGroup1) {
      group_unit<T, BWD, 1>(S, u, w);
    } else if (kind == kUnitGroup4) {
      group_unit<T, BWD, 4>(S, u, w);
    } else if (kind == kUnitGroup16) {
      group_unit<T, BWD, 16>(S, u, w);
    } else if (kind == kUnitGroup64) {
      group_unit<T, BWD, 64>(S, u, w);
    } else if (kind == kUnitBlock) {
      // chunks [c0, c0 + 16) of a long row: the 64 lanes as one group
      const int64_t pos = first_lane_i32(u.y);
      const int64_t e0 = S.ptr[pos], e1 = S.ptr[pos + 1];
      const int64_t c0 = u.z;
      const T c = group_chunks<T, 64, BWD>(e0 + kChunk * c0, e1, l, true, S.idx, S.fv, S.in, w);
      const int64_t ck = c0 + l / 4;
      if ((l & 3) == 3 && e0 + kChunk * ck < e1) publish(cs + u.w + ck, c);
    } else {  // fold
      const int64_t pos = first_lane_i32(u.y);
      const int nch = u.z;
      T acc = S.start(pos);
      for (int base = 0; base < nch; base += kWave) {
        const int m = nch - base < kWave ? nch - base : kWave;
        int32_t ci[1] = {u.w + base + l};
        const int cnt = l < m ? 1 : 0;
        typename Bits<T>::U v[1] = {cnt ? load_bits(cs + ci[0]) : (typename Bits<T>::U)0};
        wait_ready<T, 1, false>(cs, ci, cnt, v, w);
        if (cnt) reset(cs + ci[0]);
        const T c = Bits<T>::val(v[0]);
        for (int k = 0; k < m; ++k) acc = acc - readlane_t(c, k);
      }
      if (l == 0) S.finish(pos, acc);
    }
  }
}

template <typename T>
void ready_apply_t(const SlotBatch &B, hipStream_t s, hipEvent_t mid) {
  hipLaunchKernelGGL((k_ready<T, false>), dim3(B.nwg), dim3(kReadyThreads), 0, s, B.aslots,
                     B.wgmap);
  if (mid) (void)hipEventRecord(mid, s);
  hipLaunchKernelGGL((k_ready<T, true>), dim3(B.nwg), dim3(kReadyThreads), 0, s, B.aslots,
                     B.wgmap);
}

}  // namespace

hipError_t ready_apply(const SlotBatch &B, int prec, hipStream_t s, hipEvent_t mid) {
  if (B.nwg == 0) return mid ? hipEventRecord(mid, s) : hipSuccess;
  if (prec == PARAC_PREC_MIXED)
    ready_apply_t<float>(B, s, mid);
  else
    ready_apply_t<double>(B, s, mid);
  return hipGetLastError();
}

}  // namespace parac
