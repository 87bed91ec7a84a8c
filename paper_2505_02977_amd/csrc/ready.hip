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
// instead of hanging.  The final levels of few rows, when a factor has a
// long enough run of them, are not the sweeps' but k_narrow's: one workgroup
// per slot, launched between the two sweeps (see "Narrow levels" below).
//
// The arithmetic of a row: start value minus the sum of its products, the
// sum taken as a balanced binary tree whose shape depends only on the row's
// length.  Each lane adds its (up to) 16 products pairwise (4 levels, absent
// entries contributing -0.0, the exact identity of addition), the G lanes of
// a row combine their partial sums by a butterfly over lane-index bits
// (commutative pairs, so every lane ends with the same bits), and rows above
// 1024 entries add their block partials (1024 entries each) as a tree too.
// A row's dependent chain is about log2(entries) additions, where a left fold
// would take one per entry.  Which wave computes which part changes nothing
// in the bits.
//
// Units (int4, kind in x).  A row of m entries is taken by a group of G
// lanes (G = 1 for m <= 16, 4 for m <= 64, 16 for m <= 256, 64 for
// m <= 1024); lane q of a group reads entries 16q .. 16q+15 of the row, so
// every lane issues all its loads at once and waits once.  A chunk of 64
// products spans four lanes and is folded along them through shuffles.
//   group G  : 64/G rows of one class of one level (y = first class-list
//              index, z = number of rows)
//   block    : chunks [z, z + 16) of 64 entries of a row of more than 1024
//              entries, by the 64 lanes as one group: one block partial,
//              stored at w + z / 16 of the partial buffer (y = position,
//              w = offset of the row's partials)
//   fold     : the block partials of such a row added into its value
//              (y = position, z = number of 64-entry chunks, w = offset)
// Work vectors y (forward) and x (backward) are indexed by position.  Each
// sweep leaves the other vector all-sentinel for the next apply: the forward
// sweep resets x, the backward sweep resets y once it has read it, and a
// fold resets the chunk sums it consumed.
//
// Columns.  A slot solves CC right-hand sides at once (CC = 1, 2, 4 or 8,
// fixed per launch): entry (p, j) of its work vectors and chunk sums is at
// p * CC + j, so the CC values of one position share a line.  Every lane
// reads its entries' indices and factor values once and folds CC
// independent chains, one per column, each with exactly the association of
// the single-column sweep: a column's bits do not depend on CC.  Columns of
// a slot beyond its valid count carry zeros and are never written out.
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

// Pairs.  With the FP32 apply and an even number of columns per slot, the
// two columns 2i, 2i+1 of a position form one 8-byte-aligned pair, read and
// written by one 64-bit access: a gather moves one address per pair, and a
// row's two values become visible together.  Elements stay the unit of the
// pending test; a pair is reloaded when either element is pending (an
// element once solved keeps its bits for the rest of the sweep).
template <typename T, int CC>
__host__ __device__ constexpr int pack_width() {
  return (sizeof(T) == 4 && CC % 2 == 0) ? 2 : 1;
}

__device__ __forceinline__ unsigned long long load_pair(const float *p) {
  return __hip_atomic_load((const unsigned long long *)p, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// v[j], v[j+1] (PW = 2) or v[j] (PW = 1) from the element p
template <typename T, int PW, int CC>
__device__ __forceinline__ void load_elems(const T *p, typename Bits<T>::U (&v)[CC], int j) {
  if constexpr (PW == 2) {
    const unsigned long long w = load_pair((const float *)p);
    v[j] = (unsigned)(w & 0xffffffffull);
    v[j + 1] = (unsigned)(w >> 32);
  } else {
    v[j] = load_bits(p);
  }
}

template <typename T, int PW>
__device__ __forceinline__ void publish_elems(T *p, const T *v) {
  if constexpr (PW == 2) {
    using B = Bits<T>;
    typename B::U u0 = B::of(v[0]), u1 = B::of(v[1]);
    if (u0 == B::kPending) u0 = B::kQuietNaN;
    if (u1 == B::kPending) u1 = B::kQuietNaN;
    __hip_atomic_store((unsigned long long *)p,
                       (unsigned long long)u0 | ((unsigned long long)u1 << 32), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  } else {
    publish(p, v[0]);
  }
}

template <typename T, int PW>
__device__ __forceinline__ void reset_elems(T *p) {
  if constexpr (PW == 2) {
    using B = Bits<T>;
    __hip_atomic_store((unsigned long long *)p,
                       (unsigned long long)B::kPending | ((unsigned long long)B::kPending << 32),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    reset(p);
  }
}

__device__ __forceinline__ double shfl_xor_t(double v, int o) { return __shfl_xor(v, o, kWave); }
__device__ __forceinline__ float shfl_xor_t(float v, int o) { return __shfl_xor(v, o, kWave); }

__device__ __forceinline__ double readlane_t(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float readlane_t(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

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

// Wait until every lane's entries v[u][j], u < cnt, are solved.  The wave
// polls one address at a time: of its pending entries the one solved last
// in sweep order (positions follow the levels: the highest position
// forward, DESC: the lowest backward), then reloads the others, which are
// usually solved by then.  A single polled address per wave leaves the
// memory system to the loads and stores of the rows being solved.
// ci[u] must be a valid index for every u (callers pass one for u >= cnt).
//
// With one entry per lane (M = 1, the fold's partial sums) the reload is
// branch-free: every entry is loaded again and the new bits kept only where
// the old ones were pending.  The form with the load under a branch was
// compiled wrongly for the two-column FP32 sweep (hipcc of ROCm 7.2, -O3):
// the register holding an entry that was already solved was reused for the
// poll within the loop and not restored, so a column took another entry's
// value.  The 16-entry form (group units) is compiled correctly; the block
// apply tests compare every width bit for bit on graphs with long rows.
template <typename T, int M, int CC, bool DESC>
__device__ __forceinline__ void wait_ready(const T *vec, const int32_t (&ci)[M], int cnt,
                                           typename Bits<T>::U (&v)[M][CC], Watch &w) {
  using B = Bits<T>;
  constexpr int PW = pack_width<T, CC>();
  auto reload = [&]() {
#pragma unroll
    for (int u = 0; u < M; ++u)
#pragma unroll
      for (int j = 0; j < CC; j += PW) {
        bool pend = v[u][j] == B::kPending;
        if constexpr (PW == 2) pend = pend || v[u][j + 1] == B::kPending;
        if constexpr (M == 1) {
          typename B::U nv[CC];
          load_elems<T, PW, CC>(vec + ci[u] * CC + j, nv, j);
#pragma unroll
          for (int t = 0; t < PW; ++t) v[u][j + t] = (u < cnt && pend) ? nv[j + t] : v[u][j + t];
        } else if (u < cnt && pend) {
          load_elems<T, PW, CC>(vec + ci[u] * CC + j, v[u], j);
        }
      }
  };
  for (;;) {
    // key: the element index p * CC + j of a pending entry (negated: DESC)
    int key = INT32_MIN;
#pragma unroll
    for (int u = 0; u < M; ++u)
#pragma unroll
      for (int j = 0; j < CC; ++j) {
        const int e = ci[u] * CC + j;
        const int k = DESC ? -e : e;
        if (u < cnt && v[u][j] == B::kPending && k > key) key = k;
      }
    if (!__ballot(key != INT32_MIN)) return;
#pragma unroll
    for (int o = kWave / 2; o >= 1; o >>= 1) {
      const int y = __shfl_xor(key, o, kWave);
      key = y > key ? y : key;
    }
    const int32_t at = __builtin_amdgcn_readfirstlane(DESC ? -key : key);
    bool single = false;
    if constexpr (M == 1) {
      // a long row's partials: when the polled one is the only entry the
      // wave still waits for, its bits need no reload
      bool other = false;
#pragma unroll
      for (int j = 0; j < CC; ++j)
        other = other || (cnt > 0 && v[0][j] == B::kPending && ci[0] * CC + j != at);
      single = !__ballot(other);
    }
    PollBackoff bo;
    typename B::U pv;
    while ((pv = load_bits(vec + at)) == B::kPending) {
      if (__ballot(w.expired())) {
#pragma unroll
        for (int u = 0; u < M; ++u)
#pragma unroll
          for (int j = 0; j < CC; ++j)
            if (v[u][j] == B::kPending) v[u][j] = B::kQuietNaN;
        return;
      }
      bo.pause();
    }
    if constexpr (M == 1) {
      if (single) {
#pragma unroll
        for (int j = 0; j < CC; ++j)
          v[0][j] = (cnt > 0 && v[0][j] == B::kPending) ? pv : v[0][j];
        return;
      }
    }
    reload();
  }
}

// balanced sum of a lane's 16 products (pairs, then pairs of pairs, ...)
template <typename T>
__device__ __forceinline__ T tree16(const T (&p)[16]) {
  T a[8], c[4];
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = p[2 * i] + p[2 * i + 1];
#pragma unroll
  for (int i = 0; i < 4; ++i) c[i] = a[2 * i] + a[2 * i + 1];
  return (c[0] + c[1]) + (c[2] + c[3]);
}

// DPP lane moves inside rows of 16 lanes: quad_perm [1,0,3,2] (lane ^ 1),
// quad_perm [2,3,0,1] (lane ^ 2), row_half_mirror (lane i <-> 7 - i within
// 8) and row_mirror (i <-> 15 - i within 16)
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;
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

// sum over the G lanes of a row group (G a power of two, groups aligned to
// G lanes): a butterfly that pairs lanes 1, 2, 4, 8, 16, 32 apart (the
// partners at 4 and 8 by mirroring, which pairs the same two partial sums);
// the two lanes of a pair add the same two values, so every lane of the
// group ends with the same bits
template <typename T, int G>
__device__ __forceinline__ T group_reduce(T v) {
  if constexpr (G >= 2) v = v + dpp_t<kDppXor1>(v);
  if constexpr (G >= 4) v = v + dpp_t<kDppXor2>(v);
  if constexpr (G >= 8) v = v + dpp_t<kDppHalfMirror>(v);
  if constexpr (G >= 16) v = v + dpp_t<kDppMirror>(v);
  if constexpr (G >= 32) v = v + shfl_xor_t(v, 16);
  if constexpr (G >= 64) v = v + shfl_xor_t(v, 32);
  return v;
}

// Lane q of a group reads the entries [b + 16q, b + 16q + 16) ∩ [b, e1)
// (b: the first entry of the group's share of the row) and sets c[j] to the
// group's sum of column j over those entries, in every lane of the group.
template <typename T, int G, bool DESC, int CC>
__device__ __forceinline__ void group_sum(int64_t b, int64_t e1, int q, bool valid,
                                          const int32_t *__restrict__ idx,
                                          const T *__restrict__ fv, const T *vec, Watch &w,
                                          T (&c)[CC]) {
  using B = Bits<T>;
  const int64_t a = b + 16 * (int64_t)q;
  int32_t ci[16];
  T f[16];
  // the lane's entries are a prefix of its 16 slots
  const int64_t left = valid ? e1 - a : 0;
  const int cnt = left <= 0 ? 0 : (left < 16 ? (int)left : 16);
  typename B::U v[16][CC];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    ci[u] = u < cnt ? idx[a + u] : 0;
    f[u] = u < cnt ? fv[a + u] : (T)0;
  }
  constexpr int PW = pack_width<T, CC>();
#pragma unroll
  for (int u = 0; u < 16; ++u)
#pragma unroll
    for (int j = 0; j < CC; j += PW) {
      if (u < cnt) {
        load_elems<T, PW, CC>(vec + ci[u] * CC + j, v[u], j);
      } else {
#pragma unroll
        for (int t = 0; t < PW; ++t) v[u][j + t] = 0;
      }
    }
  wait_ready<T, 16, CC, DESC>(vec, ci, cnt, v, w);
#pragma unroll
  for (int j = 0; j < CC; ++j) {
    T p[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) p[u] = u < cnt ? f[u] * B::val(v[u][j]) : (T)-0.0;
    c[j] = group_reduce<T, G>(tree16(p));
  }
}

template <typename T, bool BWD, int CC>
struct Sweep {
  const ApplySlot &q;  // the slot
  const int64_t *ptr;
  const int32_t *idx;
  const T *fv;
  T *in;   // vector read (y forward, x backward)
  T *out;  // vector written: the same vector
  int nc;  // valid columns of the slot (the others carry zeros)
  __device__ __forceinline__ Sweep(const ApplySlot &q_) : q(q_) {
    ptr = BWD ? q.a.lb_ptr : q.a.lf_ptr;
    idx = BWD ? q.a.lb_idx : q.a.lf_idx;
    fv = BWD ? FactorVals<T>::bwd(q.a) : FactorVals<T>::fwd(q.a);
    in = (T *)(BWD ? q.x : q.y);
    out = in;
    nc = q.ncols;
  }
  // start values of a row: (P r) forward, D^+ y backward
  __device__ __forceinline__ void start(int64_t pos, T (&s)[CC]) const {
    if constexpr (BWD) {
      const T d = FactorVals<T>::dinv(q.a)[pos];
#pragma unroll
      for (int j = 0; j < CC; ++j) s[j] = d * ((const T *)q.y)[pos * CC + j];
    } else {
      const double *r = q.r + (int64_t)q.a.src[pos] * q.ldr;
#pragma unroll
      for (int j = 0; j < CC; ++j) s[j] = j < nc ? (T)r[j] : (T)0;
    }
  }
  // publish row pos; forward resets x[pos], backward resets y[pos] and
  // writes z in the original ordering
  __device__ __forceinline__ void finish(int64_t pos, const T (&v)[CC]) const {
    constexpr int PW = pack_width<T, CC>();
#pragma unroll
    for (int j = 0; j < CC; j += PW) publish_elems<T, PW>(out + pos * CC + j, v + j);
    if constexpr (BWD) {
      double *z = q.z + (int64_t)q.a.src[pos] * q.ldz;
#pragma unroll
      for (int j = 0; j < CC; j += PW) reset_elems<T, PW>((T *)q.y + pos * CC + j);
#pragma unroll
      for (int j = 0; j < CC; ++j)
        if (j < nc) z[j] = (double)v[j];
    } else {
#pragma unroll
      for (int j = 0; j < CC; j += PW) reset_elems<T, PW>((T *)q.x + pos * CC + j);
    }
  }
};

// a group unit: 64/G rows, G lanes each; the group's first lane publishes
// each row: start value minus the row's sum
template <typename T, bool BWD, int G, int CC>
__device__ __forceinline__ void group_unit(const Sweep<T, BWD, CC> &S, const int4 &u, Watch &w) {
  const int l = lane(), r = l / G, q = l % G;
  const bool valid = r < u.z;
  const int64_t pos = valid ? (BWD ? S.q.a.blist : S.q.a.flist)[u.y + r] : 0;
  const int64_t e0 = valid ? S.ptr[pos] : 0, e1 = valid ? S.ptr[pos + 1] : 0;
  T acc[CC];
  if (valid && q == 0) S.start(pos, acc);  // issued before the wait
  else
#pragma unroll
    for (int j = 0; j < CC; ++j) acc[j] = (T)0;
  T c[CC];
  group_sum<T, G, BWD, CC>(e0, e1, q, valid, S.idx, S.fv, S.in, w, c);
  if (valid && q == 0) {
    if (e1 > e0)
#pragma unroll
      for (int j = 0; j < CC; ++j) acc[j] = acc[j] - c[j];
    S.finish(pos, acc);
  }
}

template <typename T, bool BWD, int CC>
__global__ __launch_bounds__(kReadyThreads) void k_ready(const ApplySlot *AS,
                                                         const int32_t *wgmap) {
  const ApplySlot q = AS[wgmap[blockIdx.x]];
  // a slot whose columns are all done (block PCG) has nothing to solve
  bool skip = true;
  for (int j = 0; j < q.skip_n; ++j) skip = skip && q.a.skip[(int64_t)j * q.skip_stride] != 0;
  if (skip) return;
  const int l = lane();
  const Sweep<T, BWD, CC> S(q);
  // the narrow levels (the last forward, the first backward) are left to
  // k_narrow
  const int4 *units = BWD ? q.a.task_b + q.a.nskip_b : q.a.task_f;
  const int nt = BWD ? q.a.ntask_b - q.a.nskip_b : q.a.nwide_f;
  int32_t *ctr = q.ctr + (BWD ? 1 : 0);
  T *cs = (T *)q.cs;
  Watch w{now_ticks() + q.a.timeout_ticks, q.a.err, false, 0};
  for (;;) {
    int t = 0;
    if (l == 0) t = fetch_add(ctr, 1);
    t = first_lane_i32(__shfl(t, 0, kWave));
    // the first ticket of a sweep clears the other sweep's counter (that
    // sweep is finished, and the next one starts after this launch), also
    // when this sweep has no unit
    if (t == 0 && l == 0) st_relaxed(q.ctr + (BWD ? 0 : 1), 0);
    if (t >= nt || __ballot(w.dead)) break;
    const int4 u = units[t];
    const int kind = first_lane_i32(u.x);
    if (kind == kUnitGroup1) {
      group_unit<T, BWD, 1, CC>(S, u, w);
    } else if (kind == kUnitGroup4) {
      group_unit<T, BWD, 4, CC>(S, u, w);
    } else if (kind == kUnitGroup16) {
      group_unit<T, BWD, 16, CC>(S, u, w);
    } else if (kind == kUnitGroup64) {
      group_unit<T, BWD, 64, CC>(S, u, w);
    } else if (kind == kUnitBlock) {
      // entries [64 c0, 64 c0 + 1024) of a long row: the 64 lanes as one
      // group; the block's partial goes to slot w + c0 / 16
      const int64_t pos = first_lane_i32(u.y);
      const int64_t e0 = S.ptr[pos], e1 = S.ptr[pos + 1];
      const int64_t c0 = u.z;
      T c[CC];
      group_sum<T, 64, BWD, CC>(e0 + kChunk * c0, e1, l, true, S.idx, S.fv, S.in, w, c);
      if (l == 0)
#pragma unroll
        for (int j = 0; j < CC; j += pack_width<T, CC>())
          publish_elems<T, pack_width<T, CC>()>(cs + (u.w + c0 / kBlockChunks) * CC + j, c + j);
    } else {  // fold
      const int64_t pos = first_lane_i32(u.y);
      const int nb = (u.z + kBlockChunks - 1) / kBlockChunks;  // block partials
      T acc[CC], tot[CC];
      S.start(pos, acc);
#pragma unroll
      for (int j = 0; j < CC; ++j) tot[j] = (T)-0.0;  // -0.0 + s is s, bit for bit
      // partials 64 at a time, one per lane, each batch added as a tree
      // (butterfly over all 64 lanes), batches added in order
      for (int base = 0; base < nb; base += kWave) {
        const int m = nb - base < kWave ? nb - base : kWave;
        const int cnt = l < m ? 1 : 0;
        int32_t ci[1] = {cnt ? u.w + base + l : u.w};
        constexpr int PW = pack_width<T, CC>();
        typename Bits<T>::U v[1][CC];
#pragma unroll
        for (int j = 0; j < CC; j += PW) {
          load_elems<T, PW, CC>(cs + ci[0] * CC + j, v[0], j);
#pragma unroll
          for (int t = 0; t < PW; ++t) v[0][j + t] = cnt ? v[0][j + t] : 0;
        }
        wait_ready<T, 1, CC, false>(cs, ci, cnt, v, w);
        if (cnt)
#pragma unroll
          for (int j = 0; j < CC; j += PW) reset_elems<T, PW>(cs + ci[0] * CC + j);
#pragma unroll
        for (int j = 0; j < CC; ++j)
          tot[j] = tot[j] + group_reduce<T, kWave>(cnt ? Bits<T>::val(v[0][j]) : (T)-0.0);
      }
      if (l == 0) {
#pragma unroll
        for (int j = 0; j < CC; ++j) acc[j] = acc[j] - tot[j];
        S.finish(pos, acc);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Narrow levels: one workgroup per slot solves them level by level, with
// every narrow position's value in LDS and a barrier between levels, in
// place of a publish-to-detect hop through memory per level.  The forward
// narrow levels come after every other level, so they start once the
// forward sweep has ended; the backward ones come first, and the backward
// sweep starts once they are done.  Launch boundaries order all of it: no
// kernel here waits on another.
//
// The arithmetic is the sweeps' to the bit.  A row's sum is fixed by its
// entry order alone: products rounded once; per chunk of 16 entries a
// balanced tree; over the chunks of a row of at most 1,024 entries a
// balanced tree (padding with -0.0, the exact identity, to the 4, 16 or 64
// lanes of its group changes nothing); a longer row's blocks of 64 chunks as
// balanced trees, then added to -0.0 in batches of 64.  Here a thread takes
// half a chunk (a tree of 8), the two halves of a chunk are added by a lane
// move, and a wave adds the chunks of a row by the same butterfly.
// ---------------------------------------------------------------------------

// Products of the narrow entry slots, ahead of the narrow kernels: forward,
// an entry whose input lies before the narrow range (already solved) gets
// its product, an inside entry its factor value; backward (every input is
// inside) the factor value; padding -0.0.
template <typename T>
__global__ __launch_bounds__(256) void k_narrow_prep(const ApplySlot *AS) {
  const ApplySlot &q = AS[blockIdx.y];
  const NarrowDir &F = q.a.nf, &Bw = q.a.nb;
  if (F.nlev == 0) return;
  bool skip = true;
  for (int j = 0; j < q.skip_n; ++j) skip = skip && q.a.skip[(int64_t)j * q.skip_stride] != 0;
  if (skip) return;
  const int32_t *fidx = q.a.lf_idx;
  const T *ffv = FactorVals<T>::fwd(q.a), *bfv = FactorVals<T>::bwd(q.a);
  const T *y = (const T *)q.y;
  T *pv = (T *)q.pv;
  const int64_t total = F.nslots + Bw.nslots;
  for (int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; sl < total;
       sl += (int64_t)gridDim.x * blockDim.x) {
    T v = (T)-0.0;
    if (sl < F.nslots) {
      const int32_t e = F.smap[sl];
      if (e >= 0) {
        const int32_t c = fidx[e];
        v = c < q.a.np0 ? ffv[e] * y[c] : ffv[e];
      }
    } else {
      const int32_t e = Bw.smap[sl - F.nslots];
      if (e >= 0) v = bfv[e];
    }
    pv[sl] = v;
  }
}

// balanced sum of 8 products (the first or second half of tree16)
template <typename T>
__device__ __forceinline__ T tree8(const T (&p)[8]) {
  const T a0 = p[0] + p[1], a1 = p[2] + p[3], a2 = p[4] + p[5], a3 = p[6] + p[7];
  return (a0 + a1) + (a2 + a3);
}

// a global-memory view of a pointer: loads through it are global loads,
// counted by vmcnt alone (a flat load would also hold every LDS wait)
template <typename T>
using GlobalPtr = const __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ GlobalPtr<T> global_view(const T *p) {
  return (GlobalPtr<T>)p;
}

// a narrow row's value published as Sweep::finish does (single column),
// through global-memory stores: a flat store would also hold every LDS wait
template <typename T, bool BWD>
__device__ __forceinline__ void narrow_finish(const ApplySlot &q, int64_t pos, T v) {
  using B = Bits<T>;
  using U = typename B::U;
  using GU = __attribute__((address_space(1))) U *;
  U u = B::of(v);
  if (u == B::kPending) u = B::kQuietNaN;
  T *out = (T *)(BWD ? q.x : q.y), *other = (T *)(BWD ? q.y : q.x);
  __hip_atomic_store((GU)(out + pos), u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store((GU)(other + pos), B::kPending, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if constexpr (BWD) {
    using GD = __attribute__((address_space(1))) double *;
    *(GD)(q.z + (int64_t)q.a.src[pos] * q.ldz) = (double)v;
  }
}

// one half-chunk's slots of a level, loaded ahead of its level
// (the eight 16-bit inputs stay packed in four words until their level:
// split at the load, they would be waited for there)
template <typename T>
struct HalfChunk {
  int32_t lw;  // lane word (levels of one wave per row)
  uint32_t ni[4];
  T pv[8];
};

// the 64-lane butterfly's sum: rows of 16 lanes by lane moves, then the four
// row sums in the butterfly's pairs, read as uniform values
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  v = group_reduce<T, 16>(v);
  return (readlane_t(v, 0) + readlane_t(v, 16)) + (readlane_t(v, 32) + readlane_t(v, 48));
}

template <typename T, bool BWD, int D>
__global__ __launch_bounds__(kNarrowThreads) void k_narrow(const ApplySlot *AS) {
  const ApplySlot q = AS[blockIdx.x];
  const NarrowDir N = BWD ? q.a.nb : q.a.nf;
  if (N.nlev == 0) return;
  bool skip = true;
  for (int j = 0; j < q.skip_n; ++j) skip = skip && q.a.skip[(int64_t)j * q.skip_stride] != 0;
  if (skip) return;
  __shared__ T xs[kNarrowRows];          // values of the narrow positions
  __shared__ int32_t rows[kNarrowRows];  // (first chunk << 16) | chunks
  __shared__ int4 hdr[kNarrowLevels];
  __shared__ T cp[kNarrowChunks];        // chunk sums of the current level
  const Sweep<T, BWD, 1> S(q);
  const int tid = threadIdx.x, l = tid & (kWave - 1), wv = tid / kWave;
  const int np0 = q.a.np0, P = (int)(q.a.n - np0);
  // start values (P r forward, D^+ y backward), row and level tables
  for (int p = tid; p < P; p += kNarrowThreads) {
    T s0[1];
    S.start(np0 + p, s0);
    xs[p] = s0[0];
    rows[p] = N.rows[p];
  }
  for (int i = tid; i < N.nlev; i += kNarrowThreads) hdr[i] = N.hdr[i];
  __syncthreads();
  const GlobalPtr<T> pv = global_view((const T *)q.pv + (BWD ? q.a.nf.nslots : 0));
  const GlobalPtr<uint32_t> nidx = global_view((const uint32_t *)N.nidx);
  const GlobalPtr<int32_t> lwp = global_view(N.lw);
  // Every thread issues the same loads for every level (slot 0 where it has
  // no half-chunk or the level is past the last), so the number of loads
  // issued after a buffer's is known where the buffer is used, and a level
  // waits only for its own buffer.  Nothing in the level loop stores to
  // global memory: the rows are published after the last level.
  auto load = [&](int i, HalfChunk<T> &b) {
    int64_t s0 = 0;
    if (i < N.nlev) {
      const int4 h = hdr[i];
      if (tid < h.y) s0 = ((int64_t)h.x + tid) * 8;
    }
    b.lw = lwp[s0 / 8];
#pragma unroll
    for (int u = 0; u < 4; ++u) b.ni[u] = nidx[s0 / 2 + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) b.pv[u] = pv[s0 + u];
  };
  auto level = [&](int i, const HalfChunk<T> &b) {
    const int4 h = hdr[i];
    const bool one = (h.w & kNarrowOneWave) != 0;
    const int lw = tid < h.y ? b.lw : 0;
    const int pr1 = lw >> 8;
    const T x1 = (lw & 1) ? xs[pr1] : (T)0;  // a group's first lane: its row's start
    T hs = (T)-0.0;
    if (tid < h.y) {
      T p[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = (int16_t)(b.ni[u / 2] >> (16 * (u % 2)));
        const T x = xs[c >= 0 ? c : 0];
        p[u] = c >= 0 ? b.pv[u] * x : b.pv[u];
      }
      hs = tree8(p);
    }
    if (one) {
      // the row's group of 2^lg lanes: the butterfly's stages below lg
      const int lg = (lw >> 1) & 7;
      T v = hs, t;
      t = dpp_t<kDppXor1>(v);
      v = lg > 0 ? v + t : v;
      t = dpp_t<kDppXor2>(v);
      v = lg > 1 ? v + t : v;
      t = dpp_t<kDppHalfMirror>(v);
      v = lg > 2 ? v + t : v;
      t = dpp_t<kDppMirror>(v);
      v = lg > 3 ? v + t : v;
      // groups of 32 and 64 lanes: their rows of 16 lanes are uniform now;
      // the pairs of row sums read as uniform values (same sums as moves)
      const T ab = readlane_t(v, 0) + readlane_t(v, 16);
      const T cd = readlane_t(v, 32) + readlane_t(v, 48);
      v = lg > 4 ? (l < 32 ? ab : cd) : v;
      v = lg > 5 ? ab + cd : v;
      if (lw & 1) xs[pr1] = x1 - v;
      __syncthreads();
      return;
    }
    const T c = hs + dpp_t<kDppXor1>(hs);  // first half + second half
    if (tid < h.y && (tid & 1) == 0) cp[tid >> 1] = c;
    __syncthreads();
    for (int r = wv; r < (h.w & ~kNarrowOneWave); r += kNarrowThreads / kWave) {
      const int pr = h.z + r;
      const int32_t rd = rows[pr];
      const int c0 = rd >> 16, k = rd & 0xffff;
      T tot;
      if (k <= kWave) {
        tot = wave_sum<T>(l < k ? cp[c0 + l] : (T)-0.0);
      } else {
        // blocks of 64 chunks, then the fold of the block sums (one batch)
        T bl = (T)-0.0;
        for (int b2 = 0; b2 * kWave < k; ++b2) {
          const int m = k - b2 * kWave;
          const T sb = wave_sum<T>(l < m ? cp[c0 + b2 * kWave + l] : (T)-0.0);
          if (l == b2) bl = sb;
        }
        tot = (T)-0.0 + wave_sum<T>(bl);
      }
      if (l == 0 && k > 0) xs[pr] = xs[pr] - tot;
    }
    __syncthreads();
  };
  HalfChunk<T> buf[D];
#pragma unroll
  for (int d = 0; d < D; ++d) load(d, buf[d]);
  const int full = N.nlev / D * D;
  for (int i0 = 0; i0 < full; i0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      level(i0 + d, buf[d]);
      load(i0 + d + D, buf[d]);
    }
  }
#pragma unroll
  for (int d = 0; d < D - 1; ++d)
    if (full + d < N.nlev) level(full + d, buf[d]);
  // publish every narrow row (forward: y, and x reset; backward: x, y reset
  // and z)
  for (int p = tid; p < P; p += kNarrowThreads) narrow_finish<T, BWD>(q, np0 + p, xs[p]);
}

constexpr int kNarrowAhead = 3;  // levels whose slots are loaded ahead

template <typename T, int CC>
void ready_apply_t(const SlotBatch &B, hipStream_t s, hipEvent_t mid) {
  hipLaunchKernelGGL((k_ready<T, false, CC>), dim3(B.nwg), dim3(kReadyThreads), 0, s, B.aslots,
                     B.wgmap);
  const bool narrow = CC == 1 && B.nslots_max > 0;
  if constexpr (CC == 1) {
    if (narrow) {
      const int64_t g = std::min<int64_t>((B.nslots_max + 255) / 256, 1024);
      hipLaunchKernelGGL((k_narrow_prep<T>), dim3((unsigned)g, (unsigned)B.nslots), dim3(256), 0,
                         s, B.aslots);
      hipLaunchKernelGGL((k_narrow<T, false, kNarrowAhead>), dim3(B.nslots),
                         dim3(kNarrowThreads), 0, s, B.aslots);
    }
  }
  if (mid) (void)hipEventRecord(mid, s);
  if constexpr (CC == 1) {
    if (narrow)
      hipLaunchKernelGGL((k_narrow<T, true, kNarrowAhead>), dim3(B.nslots),
                         dim3(kNarrowThreads), 0, s, B.aslots);
  }
  hipLaunchKernelGGL((k_ready<T, true, CC>), dim3(B.nwg), dim3(kReadyThreads), 0, s, B.aslots,
                     B.wgmap);
}

}  // namespace

bool ready_cols_ok(int prec, int cc) {
  return cc == 1 || cc == 2 || cc == 4 || (prec == PARAC_PREC_MIXED && cc == 8);
}

hipError_t ready_apply(const SlotBatch &B, int prec, hipStream_t s, hipEvent_t mid) {
  if (B.nwg == 0) return mid ? hipEventRecord(mid, s) : hipSuccess;
  if (!ready_cols_ok(prec, B.cc)) return hipErrorInvalidValue;
  if (prec == PARAC_PREC_MIXED) {
    switch (B.cc) {
      case 1: ready_apply_t<float, 1>(B, s, mid); break;
      case 2: ready_apply_t<float, 2>(B, s, mid); break;
      case 4: ready_apply_t<float, 4>(B, s, mid); break;
      default: ready_apply_t<float, 8>(B, s, mid); break;
    }
  } else {
    switch (B.cc) {
      case 1: ready_apply_t<double, 1>(B, s, mid); break;
      case 2: ready_apply_t<double, 2>(B, s, mid); break;
      default: ready_apply_t<double, 4>(B, s, mid); break;
    }
  }
  return hipGetLastError();
}

}  // namespace parac
