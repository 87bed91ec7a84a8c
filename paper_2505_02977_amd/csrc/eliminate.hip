// eliminate.hip -- the persistent elimination kernel.
//
// Workers poll their slots of the ready queue round-robin (§IV-A, work
// scheduling), so the whole factorisation is one launch (§IV-C, persistent
// kernel).  A worker is one wave64 for a pivot of up to 128 gathered entries;
// a larger pivot is handed to a team, one of the workgroups reserved for them,
// whose eight waves share every step below.  For a pivot k the worker
//   1. gathers the input upper edges of k and every fill record addressed to k
//      (all present once k is ready: insertions precede deletions, §III);
//   2. merges parallel edges (sort by (u, src), left fold per run -- the
//      multiplicity is the run length);
//   3. sorts the merged neighbours by (w, u) ascending (Alg. 2) and forms the
//      suffix sums S with the 64-wide tiled association; D_k = S_1;
//   4. draws one partner per slot p = 1..d-1 with probability w_q / S_{p+1}
//      (Alg. 2) from a counter-based generator keyed by (k, slot) and appends
//      the sampled edge, of weight S_{p+1} w_p / D_k, to the inbox of its
//      smaller endpoint, incrementing the counter of the larger (§III);
//   5. writes column k of F, F(u,k) = -w_u / D_k, and D_k (§IV scaled form);
//   6. waits until its stores of steps 4-5 have completed (every datum another
//      pivot reads was written with agent-scope relaxed atomics, which bypass
//      the caches that are not coherent across XCDs), then decrements the
//      counters of its neighbours by their multiplicities and enqueues those
//      that reach zero (Alg. 3/4: insertions before deletions).
// The arithmetic follows fixed orders that do not depend on the schedule, so
// the factor is the same bit for bit for any grid size or timing.
#include "device.hpp"
#include "internal.hpp"

namespace parac {

struct Worker {
  int64_t f_base, f_left;    // reserved factor entries
  int64_t pg_base, pg_left;  // reserved fill-record pages
  int64_t sc_base, sc_size;  // scratch region of the large-neighbourhood path
};

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

// record r of an inbox: page j holds kInline << j records starting at
// record kInline (2^j - 1)
__device__ __forceinline__ void page_of(int r, int &j, int &off) {
  int q = r / kInline + 1;
  j = 31 - __clz(q);
  off = r - kInline * ((1 << j) - 1);
}

// Fill records and page-table entries cross waves (and XCDs).  They are
// written and read only by agent-scope relaxed accesses, which bypass the
// caches that are not coherent across XCDs; a producer waits for its stores
// to complete before it decrements any counter (store_wait), so a consumer
// that has seen its own counter at zero reads complete records without
// invalidating any cache.
__device__ __forceinline__ void store_rec(Rec *dst, int32_t other, int32_t src, double w) {
  uint64_t *d = (uint64_t *)dst;
  const uint64_t head = (uint64_t)(uint32_t)other | ((uint64_t)(uint32_t)src << 32);
  __hip_atomic_store(d, head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(d + 1, dbits(w), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ Rec load_rec(const ElimArgs &a, int32_t k, int r) {
  int j, off;
  page_of(r, j, off);
  const Rec *p;
  if (j == 0) {
    p = a.inl + (int64_t)k * kInline + off;
  } else {
    int32_t base = ld_acq_relaxed(&a.ptab[(int64_t)k * (kPages - 1) + j - 1]);
    if (base < 0) {  // never published: an invalid record (the caller's range check fails)
      Rec bad;
      bad.other = -1;
      bad.src = -1;
      bad.w = 0.0;
      return bad;
    }
    p = a.pool + (int64_t)base + off;
  }
  const uint64_t *q = (const uint64_t *)p;
  const uint64_t head = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint64_t wbits = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  Rec rc;
  rc.other = (int32_t)(uint32_t)head;
  rc.src = (int32_t)(uint32_t)(head >> 32);
  rc.w = bitsd(wbits);
  return rc;
}

__device__ __forceinline__ bool timed_out(const ElimArgs &a, uint64_t deadline) {
  if (now_ticks() > deadline) {
    set_error(a.err, PARAC_ETIMEOUT);
    return true;
  }
  return ld_acq_relaxed(a.err) != 0;
}

// Append one sampled edge per active lane and round to the inbox of
// tgt[q] and count it on oth[q] (insertion step of §III), for R rounds of
// lanes at once: the record indices of all rounds are reserved first (one
// round trip), then every page that one of them opens is allocated, and only
// then does a lane wait for a page opened by another lane or wave.  Returns
// false after setting an error.
template <int R>
__device__ bool insert_records(const ElimArgs &a, Worker &wk, const bool (&ins)[R],
                               const int32_t (&tgt)[R], const int32_t (&oth)[R], int32_t k,
                               const double (&c)[R], uint64_t deadline) {
  const int l = lane();
  int r[R], j[R], off[R];
#pragma unroll
  for (int q = 0; q < R; ++q) r[q] = ins[q] ? fetch_add(&a.fill_cnt[tgt[q]], 1) : 0;
  bool over = false;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    j[q] = 0;
    off[q] = 0;
    if (ins[q]) page_of(r[q], j[q], off[q]);
    over |= ins[q] && j[q] >= kPages;
  }
  if (__any(over)) {
    set_error(a.err, PARAC_EPOOL);
    return false;
  }
  // pages opened by this wave: reserve them together, publish their bases
  int64_t pbase[R];
  bool fail = false;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const bool alloc = ins[q] && j[q] > 0 && off[q] == 0;
    pbase[q] = -1;
    if (!__any(alloc)) continue;
    int32_t *pslot = alloc ? &a.ptab[(int64_t)tgt[q] * (kPages - 1) + j[q] - 1] : nullptr;
    const int need = alloc ? (kInline << j[q]) : 0;
    int incl = need;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      int y = __shfl_up(incl, o, kWave);
      if (l >= o) incl += y;
    }
    const int total = shfl(incl, kWave - 1);
    if ((int64_t)total > wk.pg_left) {
      int64_t grab = total > a.pg_chunk ? total : a.pg_chunk;
      long long b = 0;
      if (l == 0) b = (long long)atomicAdd(a.pool_top, (unsigned long long)grab);
      b = __shfl(b, 0, kWave);
      if (b + grab > a.pool_cap) {
        if (alloc) st_relaxed(pslot, (int32_t)-2);  // release waiters
        fail = true;
        continue;
      }
      wk.pg_base = b;
      wk.pg_left = grab;
    }
    const int64_t mybase = wk.pg_base + (incl - need);
    wk.pg_base += total;
    wk.pg_left -= total;
    if (alloc) {
      st_relaxed(pslot, (int32_t)mybase);
      pbase[q] = mybase;
    }
  }
  if (fail) {
    set_error(a.err, PARAC_EPOOL);
    return false;
  }
  // pages opened elsewhere: wait for their bases
#pragma unroll
  for (int q = 0; q < R; ++q) {
    bool wait = ins[q] && j[q] > 0 && pbase[q] < 0;
    if (!__any(wait)) continue;
    const int32_t *pslot = wait ? &a.ptab[(int64_t)tgt[q] * (kPages - 1) + j[q] - 1] : nullptr;
    Backoff bo;
    for (int it = 0; __any(wait); ++it) {
      if (wait) {
        int32_t v = ld_acq_relaxed(pslot);
        if (v != -1) {
          pbase[q] = v;
          wait = false;
        }
      }
      if (__any(wait)) {
        bo.pause();
        if ((it & 63) == 63 && timed_out(a, deadline)) return false;
      }
    }
    if (__any(ins[q] && j[q] > 0 && pbase[q] < 0)) {
      set_error(a.err, PARAC_EPOOL);
      return false;
    }
  }
  // the larger endpoint still counts k among its lower neighbours (k's own
  // edge to it is removed after the insertions), so its counter is >= 1
  bool bad = false;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    if (ins[q]) {
      Rec *dst = (j[q] == 0) ? a.inl + (int64_t)tgt[q] * kInline + off[q] : a.pool + pbase[q] + off[q];
      store_rec(dst, oth[q], k, c[q]);
      bad |= fetch_add(&a.dp[oth[q]], 1) < 1;
    }
  }
  if (__any(bad)) {
    set_error(a.err, PARAC_EINTERNAL);
    return false;
  }
  return true;
}

__device__ __forceinline__ bool alloc_column(const ElimArgs &a, Worker &wk, int d, int64_t &base) {
  if ((int64_t)d > wk.f_left) {
    int64_t grab = d > a.f_chunk ? d : a.f_chunk;
    long long b = 0;
    if (lane() == 0) b = (long long)atomicAdd(a.f_top, (unsigned long long)grab);
    b = __shfl(b, 0, kWave);
    if (b + grab > a.f_cap) {
      set_error(a.err, PARAC_EPOOL);
      return false;
    }
    wk.f_base = b;
    wk.f_left = grab;
  }
  base = wk.f_base;
  wk.f_base += d;
  wk.f_left -= d;
  return true;
}

// Synchronisation policies.  The wide kernel runs on every XCD: everything
// another pivot reads from this one (fill records, page-table entries,
// levels, counters, queue slots) goes through agent-scope atomics, so a pivot
// publishes by waiting for its stores to complete before its counter
// decrements (no cache write-back), and a consumer needs no cache
// invalidation after seeing its counter at zero.  The tail kernel is one
// workgroup on one CU: workgroup-scope fences suffice, and it has its own
// queue.
struct WideSync {
  static __device__ __forceinline__ void release() { store_wait(); }
  static __device__ __forceinline__ void acquire() { compiler_fence(); }
  static __device__ __forceinline__ bool enqueue(const ElimArgs &a, int32_t u) {
    const int x = u & (kSubQueues - 1);
    const int pos = fetch_add(&a.qtail[x * kTailStride], 1);
    if (pos >= a.cap_q) return false;
    __hip_atomic_exchange(&a.q[(int64_t)x * a.cap_q + pos], u, __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_AGENT);
    return true;
  }
};
struct TailSync {
  static __device__ __forceinline__ void release() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  }
  static __device__ __forceinline__ void acquire() {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
  static __device__ __forceinline__ bool enqueue(const ElimArgs &a, int32_t u) {
    const int pos = __hip_atomic_fetch_add(a.tq_tail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (pos >= a.ntot) return false;
    __hip_atomic_store(&a.tq[pos], u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    return true;
  }
};

// pivot-edge deletion of §III: d(u) -= m(u,k); enqueue on reaching zero
template <class Sync>
__device__ __forceinline__ bool decrement(const ElimArgs &a, bool valid, int32_t u, int m) {
  bool enq = false, bad = false;
  if (valid) {
    int prior = fetch_add(&a.dp[u], -m);
    enq = prior == m;
    bad = prior < m;
  }
  if (__any(bad)) {
    set_error(a.err, PARAC_EINTERNAL);
    return false;
  }
  if (__any(enq)) {
    // no fence here: the consumer synchronises with every producer of u
    // through u's counter (see claim_pivot); the slot only carries the label
    if (enq && !Sync::enqueue(a, u)) bad = true;
    if (__any(bad)) {
      set_error(a.err, PARAC_EINTERNAL);
      return false;
    }
  }
  return true;
}

// decrement() for Q rounds of lanes: the counter updates of all rounds go
// out together, then the labels that reached zero are enqueued
template <class Sync, int Q>
__device__ __forceinline__ bool decrement_batch(const ElimArgs &a, const bool (&valid)[Q],
                                                const int32_t (&u)[Q], const int (&m)[Q]) {
  int prior[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) prior[q] = valid[q] ? fetch_add(&a.dp[u[q]], -m[q]) : 0;
  bool bad = false;
#pragma unroll
  for (int q = 0; q < Q; ++q) bad |= valid[q] && prior[q] < m[q];
  if (__any(bad)) {
    set_error(a.err, PARAC_EINTERNAL);
    return false;
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const bool enq = valid[q] && prior[q] == m[q];
    if (__any(enq)) {
      if (enq && !Sync::enqueue(a, u[q])) bad = true;
      if (__any(bad)) {
        set_error(a.err, PARAC_EINTERNAL);
        return false;
      }
    }
  }
  return true;
}

// ---------------------------------------------------------------------------
// neighbourhoods of at most 64 gathered entries: one entry per lane
// ---------------------------------------------------------------------------
// the test hook's partner offset for slot s of pivot k (-1: draw)
__device__ __forceinline__ int forced_offset(const ElimArgs &a, int32_t k, int s) {
  if (s >= a.forced_stride) return -1;
  const int64_t i = (int64_t)k * a.forced_stride + s;
  return i < a.forced_count ? a.forced[i] : -1;
}

template <class Sync>
__device__ bool small_pivot(const ElimArgs &a, Worker &wk, int32_t k, int64_t u0, int nU, int g,
                            int levk, uint64_t deadline) {
  const int l = lane();
  // 1. gather
  uint64_t key = ~0ull;
  double w = 0.0;
  if (l < nU) {
    key = merge_key(a.uidx[u0 + l], -1);
    w = a.uw[u0 + l];
  } else if (l < g) {
    Rec rc = load_rec(a, k, l - nU);
    key = merge_key(rc.other, rc.src);
    w = rc.w;
  }
  // 2. sort by (u, src) (AC(k): by (u, src, w), keys may repeat; in the
  // plain method keys are distinct and w never decides): bitonic network
  // across the 64 lanes
  const bool tie = a.samples > 1;
#pragma unroll
  for (int p = 2; p <= kWave; p <<= 1) {
#pragma unroll
    for (int jj = p >> 1; jj >= 1; jj >>= 1) {
      int pl = (jj == (p >> 1)) ? (l ^ (p - 1)) : (l ^ jj);
      uint64_t ok = shfl_u64(key, pl);
      double ow = shfl_f64(w, pl);
      const uint64_t owb = dbits(ow), wbb = dbits(w);
      const bool lt = ok < key || (tie && ok == key && owb < wbb);
      const bool gt = ok > key || (tie && ok == key && owb > wbb);
      bool take = (pl > l) ? lt : gt;
      if (take) {
        key = ok;
        w = ow;
      }
    }
  }
  // merge runs of equal u: left fold in key order, multiplicity = run length
  const bool valid = l < g;
  const int32_t u = (int32_t)(key >> 32);
  const int32_t up = shfl(u, l > 0 ? l - 1 : 0);
  const bool head = valid && (l == 0 || up != u);
  double acc = w;
  int m = 1;
  bool active = head;
  for (int step = 1; step < kWave; ++step) {
    int sl = l + step < kWave ? l + step : kWave - 1;
    double ws = shfl_f64(w, sl);
    int32_t us = shfl(u, sl);
    bool cont = active && (l + step < g) && (us == u);
    if (cont) {
      acc = acc + ws;
      ++m;
    }
    active = cont;
    if (!__any(active)) break;
  }
  if (__any(valid && (u < 0 || u >= a.ntot || u <= k))) {  // labels above k only
    set_error(a.err, PARAC_EINTERNAL);
    return false;
  }
  const uint64_t hm = __ballot(head);
  const int d = __popcll(hm);
  const int src = l < d ? select_bit(hm, l) : 0;
  int32_t mu = shfl(u, src);
  double mw = shfl_f64(acc, src);
  int mm = shfl(m, src);
  if (l >= d) {
    mu = 0x7fffffff;
    mw = 0.0;
    mm = 0;
  }
  // 3. sampling order (w asc, u asc) and suffix sums
  uint64_t wb = l < d ? dbits(mw) : ~0ull;
  int32_t su = l < d ? mu : 0x7fffffff;
#pragma unroll
  for (int p = 2; p <= kWave; p <<= 1) {
#pragma unroll
    for (int jj = p >> 1; jj >= 1; jj >>= 1) {
      int pl = (jj == (p >> 1)) ? (l ^ (p - 1)) : (l ^ jj);
      uint64_t ow = shfl_u64(wb, pl);
      int32_t ou = shfl(su, pl);
      bool take = (pl > l) ? less_wu(ow, ou, wb, su) : less_wu(wb, su, ow, ou);
      if (take) {
        wb = ow;
        su = ou;
      }
    }
  }
  double sw = l < d ? bitsd(wb) : 0.0;
  // the sampling slots, one per lane: the merged neighbours, or (AC(k)) each
  // of them as ks consecutive slots of weight w / ks (ks d <= 64 here)
  const int ks = a.samples > 1 ? a.samples : 1;
  const int ds = d * ks;
  if (ks > 1) {
    const int src_i = l / ks < kWave ? l / ks : kWave - 1;
    const double wi = shfl_f64(sw, src_i);
    const int32_t ui = shfl(su, src_i);
    sw = l < ds ? wi / (double)ks : 0.0;
    su = l < ds ? ui : 0x7fffffff;
  }
  double S = sw;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    double y = shfl_f64(S, l + o < kWave ? l + o : kWave - 1);
    if (l + o < ds) S = S + y;
  }
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    double y = shfl_f64(S, l + o < kWave ? l + o : kWave - 1);
    if (l + o < ds && y > S) S = y;
  }
  const double Dk = shfl_f64(S, 0);
  // 4. one sampled edge per slot s = 0..ds-2 (position p = s+1)
  bool ins = l < ds - 1;
  const double Sp1 = shfl_f64(S, l + 1 < kWave ? l + 1 : kWave - 1);
  const double t = draw_unit(a.seed, (uint32_t)k, (uint32_t)l) * Sp1;
  int lo = l + 1, hi = ds - 1;
#pragma unroll
  for (int it = 0; it < 6; ++it) {
    int mid = (lo + hi) >> 1;
    int idx = mid + 1 < kWave ? mid + 1 : kWave - 1;
    double sn = shfl_f64(S, idx);
    if (mid + 1 >= ds) sn = 0.0;
    if (lo < hi) {
      if (sn <= t) hi = mid;
      else lo = mid + 1;
    }
  }
  if (a.forced && ins) {
    const int fo = forced_offset(a, k, l);
    if (fo >= 0 && fo >= ds - 1 - l) set_error(a.err, PARAC_EINVAL);
    else if (fo >= 0) lo = l + 1 + fo;
  }
  const int32_t ub = shfl(su, lo < kWave ? lo : kWave - 1);
  // AC(k): a partner on the same neighbour is a loop, dropped
  ins = ins && ub != su;
  const double c = (Sp1 * sw) / Dk;
  const int32_t tgt = su < ub ? su : ub, oth = su < ub ? ub : su;
  {
    const bool ins1[1] = {ins};
    const int32_t tgt1[1] = {tgt}, oth1[1] = {oth};
    const double c1[1] = {c};
    if (!insert_records<1>(a, wk, ins1, tgt1, oth1, k, c1, deadline)) return false;
  }
  // 5. column k of F (rows ascending) and D_k
  int64_t base;
  if (!alloc_column(a, wk, d, base)) return false;
  if (l < d) {
    a.frow[base + l] = mu;
    a.fval[base + l] = -(mw / Dk);
    fetch_max(&a.lev[mu], levk + 1);
  }
  if (l == 0) {
    a.D[k] = Dk;
    a.colstart[k] = base;
    a.colcnt[k] = d;
  }
  // 6. publish, then delete the pivot's edges
  Sync::release();
  return decrement<Sync>(a, l < d, mu, mm);
}

constexpr int kRankMax = 256;   // above this the radix sort replaces ranking
constexpr int kCoarse = 512;    // coarse suffix-sum points per wave (LDS)

// Rank sorts: an entry's rank is the number of entries before it in the
// order (keys are distinct), counted with readlanes over 64-key blocks; the
// blocks are loaded four at a time so that their latencies overlap.
// rank of each entry in (key, w) order; with TIE (AC(k): one pivot may draw
// the same pair twice, so keys repeat) equal keys are ordered by weight and
// entries equal in both by position (they are interchangeable); without it
// keys are unique
template <bool TIE>
__device__ __forceinline__ void rank_sort_key(const uint64_t *keyA, const double *wA,
                                              uint64_t *keyB, double *wB, int g) {
  const int l = lane();
  for (int ib = 0; ib < g; ib += kWave) {
    const int i = ib + l;
    const uint64_t ki = i < g ? keyA[i] : ~0ull;
    const double wi = i < g ? wA[i] : 0.0;
    const uint64_t wbi = dbits(wi);
    int rank = 0;
    for (int jb = 0; jb < g; jb += 4 * kWave) {
      uint64_t kj[4], wj[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = jb + r * kWave + l;
        kj[r] = j < g ? keyA[j] : ~0ull;
        wj[r] = TIE && j < g ? dbits(wA[j]) : 0ull;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int b0 = jb + r * kWave;
        const int lim = g - b0 < kWave ? g - b0 : kWave;
        for (int jj = 0; jj < lim; ++jj) {
          const uint64_t kk = readlane_u64(kj[r], jj);
          if (TIE) {
            const uint64_t ww = readlane_u64(wj[r], jj);
            rank += (kk < ki || (kk == ki && (ww < wbi || (ww == wbi && b0 + jj < i)))) ? 1 : 0;
          } else {
            rank += kk < ki ? 1 : 0;
          }
        }
      }
    }
    if (i < g) {
      keyB[rank] = ki;
      wB[rank] = wi;
    }
  }
}

__device__ __forceinline__ void rank_sort_wu(const double *mw, const int32_t *mu, double *sw,
                                             int32_t *su, int d) {
  const int l = lane();
  for (int ib = 0; ib < d; ib += kWave) {
    const int i = ib + l;
    const uint64_t wi = i < d ? dbits(mw[i]) : ~0ull;
    const int32_t ui = i < d ? mu[i] : 0x7fffffff;
    int rank = 0;
    for (int jb = 0; jb < d; jb += 4 * kWave) {
      uint64_t wj[4];
      int32_t uj[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = jb + r * kWave + l;
        wj[r] = j < d ? dbits(mw[j]) : ~0ull;
        uj[r] = j < d ? mu[j] : 0x7fffffff;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int b0 = jb + r * kWave;
        const int lim = d - b0 < kWave ? d - b0 : kWave;
        for (int jj = 0; jj < lim; ++jj) {
          const uint64_t ww = readlane_u64(wj[r], jj);
          const int32_t uu = __builtin_amdgcn_readlane(uj[r], jj);
          rank += less_wu(ww, uu, wi, ui) ? 1 : 0;
        }
      }
    }
    if (i < d) {
      su[rank] = ui;
      sw[rank] = bitsd(wi);
    }
  }
}

// Merge the runs of equal u whose first entry lies in [lo, hi) of the sorted
// list [0, g): each run's weights are summed left to right in key order, and
// the j-th run goes to position d0 + j.  Returns d0 + the number of runs.
// Chunks of 64 sorted entries are held one per lane: runs inside a chunk are
// folded in lockstep through shuffles, a run that reaches the end of a chunk
// is carried (label cu, partial sum cacc, length cm) into the next one.  A
// run that begins before lo belongs to the wave holding its beginning: it is
// carried as a phantom and dropped; the last run may run on past hi.
__device__ __forceinline__ int merge_runs(const uint64_t *keyS, const double *wS, int lo, int hi, int g, int d0,
                          int32_t *mu, double *mw, int32_t *mm) {
  const int l = lane();
  int d = d0;
  int32_t cu = -1;
  bool phantom = false;
  if (lo > 0 && lo < hi) {
    cu = (int32_t)(keyS[lo - 1] >> 32);
    phantom = true;
  }
  double cacc = 0.0;
  int cm = 0;
  auto emit_carry = [&]() {
    if (!phantom) {
      if (l == 0) {
        mu[d] = cu;
        mw[d] = cacc;
        mm[d] = cm;
      }
      ++d;
    }
    cu = -1;
    phantom = false;
  };
  uint64_t knext = lo + l < g ? keyS[lo + l] : ~0ull;
  double wnext = lo + l < g ? wS[lo + l] : 0.0;
  for (int ib = lo; ib < g; ib += kWave) {
    if (ib >= hi && cu < 0) break;
    const int i = ib + l;
    const int n = g - ib < kWave ? g - ib : kWave;
    const bool valid = i < g;
    const int32_t u = valid ? (int32_t)(knext >> 32) : -1;
    const double w = wnext;
    if (i + kWave < g) {
      knext = keyS[i + kWave];
      wnext = wS[i + kWave];
    }
    // lanes continuing the carried run form a prefix [0, c)
    int c = 0;
    if (cu >= 0) {
      const uint64_t cont = __ballot(valid && u == cu);
      c = ~cont == 0 ? kWave : __builtin_ctzll(~cont);
      if (!phantom)
        for (int j = 0; j < c; ++j) cacc = cacc + shfl_f64(w, j);
      cm += c;
      if (c < n) emit_carry();
      if (c == n) continue;  // the whole chunk continues the carried run
    }
    if (ib >= hi) break;  // runs that begin here belong to the next range
    const int32_t uprev = shfl(u, l > 0 ? l - 1 : 0);
    const bool head = valid && l >= c && (l == c || uprev != u);
    double acc = head ? w : 0.0;
    int m = head ? 1 : 0;
    bool active = head;
    for (int step = 1; step < kWave; ++step) {
      const int sl = l + step < kWave ? l + step : kWave - 1;
      const double ws = shfl_f64(w, sl);
      const int32_t us = shfl(u, sl);
      const bool cont2 = active && (l + step < n) && us == u;
      if (cont2) {
        acc = acc + ws;
        ++m;
      }
      active = cont2;
      if (!__any(active)) break;
    }
    const uint64_t hm = __ballot(head);
    uint64_t em = hm;
    if (hm && n == kWave && ib + kWave < g) {
      const int hl = 63 - __clzll(hm);  // the chunk's last run reaches lane 63?
      if (shfl(u, kWave - 1) == shfl(u, hl)) {
        em &= ~(1ull << hl);
        cu = shfl(u, hl);
        cacc = shfl_f64(acc, hl);
        cm = shfl(m, hl);
      }
    }
    if ((em >> l) & 1) {
      const int pos = d + __popcll(em & lanemask_lt());
      mu[pos] = u;
      mw[pos] = acc;
      mm[pos] = m;
    }
    d += __popcll(em);
  }
  if (cu >= 0) emit_carry();
  return d;
}

// Sampled edges of the slots ib + r*stride + [0, 64), r < 4, of a pivot with d merged
// neighbours in (w, u) order (weights sw, labels su, suffix sums S, D_k = S[0]).
// The partner of slot s is the first m > s with S[m+1] <= t (S
// non-increasing, S[d] = 0).  A coarse copy of S in LDS (coarse[j] =
// S[j st + 1], j < nco) narrows the search to st entries, and the searches
// of the four rounds of 64 slots run interleaved.
constexpr int kSampleRounds = 4;
__device__ __forceinline__ bool sample_rounds(const ElimArgs &a, Worker &wk, int32_t k, int d, int ib,
                              int stride, const double *S, const double *sw, const int32_t *su,
                              double Dk, const double *coarse, int st, int nco, uint64_t deadline) {
  constexpr int R = kSampleRounds;
  const int l = lane();
  int lo[R], hi[R];
  double t[R], Sp1[R];
  bool ins[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int sl = ib + r * stride + l;
    ins[r] = sl < d - 1;
    Sp1[r] = ins[r] ? S[sl + 1] : 0.0;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int sl = ib + r * stride + l;
    lo[r] = sl + 1;
    hi[r] = d - 1;
    if (!ins[r]) {
      lo[r] = hi[r] = 0;
      continue;
    }
    t[r] = draw_unit(a.seed, (uint32_t)k, (uint32_t)sl) * Sp1[r];
    // coarse: smallest j with m_j >= lo and coarse[j] <= t (exists unless
    // the answer lies beyond the last coarse point)
    int jl = (lo[r] + st - 1) / st, jh = nco;
    while (jl < jh) {
      const int mid = (jl + jh) >> 1;
      if (coarse[mid] <= t[r]) jh = mid;
      else jl = mid + 1;
    }
    if (jl < nco) hi[r] = jl * st;
    const int lo2 = (jl - 1) * st + 1;
    if (jl > 0 && lo2 > lo[r]) lo[r] = lo2;
  }
  // fine search in global memory, the four rounds' loads overlapping
  for (;;) {
    bool any = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (lo[r] < hi[r]) {
        const int mid = (lo[r] + hi[r]) >> 1;
        const double sn = mid + 1 < d ? S[mid + 1] : 0.0;
        if (sn <= t[r]) hi[r] = mid;
        else lo[r] = mid + 1;
        any = true;
      }
    }
    if (!__any(any)) break;
  }
  if (a.forced) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int sl = ib + r * stride + l;
      const int fo = ins[r] ? forced_offset(a, k, sl) : -1;
      if (fo >= 0 && fo >= d - 1 - sl) set_error(a.err, PARAC_EINVAL);
      else if (fo >= 0) lo[r] = sl + 1 + fo;
    }
  }
  int32_t tgt[R], oth[R];
  double c[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int sl = ib + r * stride + l;
    tgt[r] = oth[r] = 0;
    c[r] = 0.0;
    if (ins[r]) {
      const int32_t ua = su[sl], ub = su[lo[r]];
      // AC(k): a partner on the same neighbour is a loop, dropped (never
      // happens with one slot per neighbour: the labels are distinct)
      ins[r] = ua != ub;
      c[r] = (Sp1[r] * sw[sl]) / Dk;
      tgt[r] = ua < ub ? ua : ub;
      oth[r] = ua < ub ? ub : ua;
    }
  }
  return insert_records<R>(a, wk, ins, tgt, oth, k, c, deadline);
}

// ---------------------------------------------------------------------------
// larger neighbourhoods: the same steps over wave-private scratch in HBM;
// sorting by rank (keys are unique), suffix sums tile by tile
// ---------------------------------------------------------------------------
template <class Sync>
__device__ bool large_pivot(const ElimArgs &a, Worker &wk, int32_t k, int64_t u0, int nU, int g,
                            int levk, uint64_t deadline, int *h, double *coarse) {
  const int l = lane();
  // AC(k): k sampling slots per merged neighbour (at most g neighbours):
  // slot weights, labels and suffix sums after the per-pivot arrays
  const int ks = a.samples > 1 ? a.samples : 1;
  const int64_t slot_cap = ks > 1 ? (int64_t)g * ks : 0;
  const int64_t bytes = (((int64_t)g * 68 + slot_cap * 20 + 8) + 255) & ~(int64_t)255;
  if (bytes > wk.sc_size) {
    // the worker's region is reused across pivots; grow it geometrically
    int64_t want = bytes > 2 * wk.sc_size ? bytes : 2 * wk.sc_size;
    long long off = 0;
    if (l == 0) off = (long long)atomicAdd(a.arena_top, (unsigned long long)want);
    off = __shfl(off, 0, kWave);
    if (off + want > a.arena_cap) {
      set_error(a.err, PARAC_EPOOL);
      return false;
    }
    wk.sc_base = off;
    wk.sc_size = want;
  }
  char *base = a.arena + wk.sc_base;
  uint64_t *keyA = (uint64_t *)base;
  double *wA = (double *)(keyA + g);
  uint64_t *keyB = (uint64_t *)(wA + g);
  double *wB = (double *)(keyB + g);
  double *mw = wB + g;
  double *sw = mw + g;
  double *S = sw + g;
  int32_t *mu = (int32_t *)(S + g);
  int32_t *mm = mu + g;
  int32_t *su = mm + g;
  // slot weights [slot_cap] (AC(k)), 8-byte aligned
  double *xw2 = (double *)(((uintptr_t)(su + g) + 7) & ~(uintptr_t)7);
  double *S2 = xw2 + slot_cap;         // their suffix sums
  int32_t *xu2 = (int32_t *)(S2 + slot_cap);  // slot labels
  // 1. gather
#pragma unroll 4
  for (int i = l; i < g; i += kWave) {
    int32_t u, src;
    double w;
    if (i < nU) {
      u = a.uidx[u0 + i];
      src = -1;
      w = a.uw[u0 + i];
    } else {
      Rec rc = load_rec(a, k, i - nU);
      u = rc.other;
      src = rc.src;
      w = rc.w;
    }
    keyA[i] = merge_key(u, src);
    wA[i] = w;
  }
  fence_wave_local();
  // 2. sort by (u, src) (AC(k): by (u, src, w), keys may repeat)
  uint64_t *keyS = keyB;   // sorted keys and weights end up here
  double *wS = wB;
  if (g <= kRankMax) {
    if (ks > 1) rank_sort_key<true>(keyA, wA, keyB, wB, g);
    else rank_sort_key<false>(keyA, wA, keyB, wB, g);
  } else {
    if (ks > 1) {
      // least significant first: the weights (eight passes over the bits of
      // a positive double, whose order is that of its value), then the keys
      int wsh[8];
      for (int p2 = 0; p2 < 8; ++p2) wsh[p2] = 8 * p2;
      const bool w_in_a = wave_radix_sort<uint64_t, uint64_t>((uint64_t *)wA, keyA, (uint64_t *)wB,
                                                              keyB, g, wsh, 8, h);
      if (!w_in_a) {  // (an even pass count leaves them in place)
        set_error(a.err, PARAC_EINTERNAL);
        return false;
      }
      fence_wave_local();
    }
    // radix passes over the bits a key can use: src + 1 in the low word,
    // u in the high word, both below 2^bits(ntot + 1)
    const int nb = 32 - __clz(a.ntot + 1);
    int shifts[8], np = 0;
    for (int b = 0; b < nb; b += 8) shifts[np++] = b;
    for (int b = 0; b < nb; b += 8) shifts[np++] = 32 + b;
    const bool in_a = wave_radix_sort<uint64_t, uint64_t>(keyA, (uint64_t *)wA, keyB, (uint64_t *)wB, g, shifts, np, h);
    if (in_a) {
      keyS = keyA;
      wS = wA;
    }
  }
  fence_wave_local();
  // every gathered label must lie above k (and exist)
  {
    bool bad = false;
    for (int i = l; i < g; i += kWave) {
      int32_t u = (int32_t)(keyS[i] >> 32);
      bad |= u <= k || u >= a.ntot;
    }
    if (__any(bad)) {
      set_error(a.err, PARAC_EINTERNAL);
      return false;
    }
  }
  // merge runs of equal u
  const int d = merge_runs(keyS, wS, 0, g, g, 0, mu, mw, mm);
  fence_wave_local();
  // 3. sampling order (w asc, u asc)
  if (d <= kRankMax) {
    rank_sort_wu(mw, mu, sw, su, d);
  } else {
    // the merged list is in ascending u, so a stable sort on the bits of w
    // alone yields the (w, u) order
    uint64_t *kx = keyA, *vx = (uint64_t *)wA, *ky = keyB, *vy = (uint64_t *)wB;
    for (int i = l; i < d; i += kWave) {
      kx[i] = dbits(mw[i]);
      vx[i] = (uint64_t)(uint32_t)mu[i];
    }
    fence_wave_local();
    int shifts[8];
    for (int p2 = 0; p2 < 8; ++p2) shifts[p2] = 8 * p2;
    const bool in_x = wave_radix_sort<uint64_t, uint64_t>(kx, vx, ky, vy, d, shifts, 8, h);
    const uint64_t *kr = in_x ? kx : ky, *vr = in_x ? vx : vy;
    for (int i = l; i < d; i += kWave) {
      sw[i] = bitsd(kr[i]);
      su[i] = (int32_t)(uint32_t)vr[i];
    }
  }
  fence_wave_local();
  // the sampling slots: the merged neighbours in (w, u) order, or (AC(k))
  // each of them as ks consecutive slots of weight w / ks
  const double *xw = sw;
  const int32_t *xu = su;
  double *SS = S;
  int ds = d;
  if (ks > 1) {
    ds = d * ks;
    for (int i = l; i < ds; i += kWave) {
      xw2[i] = sw[i / ks] / (double)ks;
      xu2[i] = su[i / ks];
    }
    fence_wave_local();
    xw = xw2;
    xu = xu2;
    SS = S2;
  }
  // suffix sums: 64-wide tiles, Hillis-Steele inside, carries right to left
  // (the next tile's values are loaded while the current one is summed);
  // the exact suffix maximum that makes S non-increasing is taken in the
  // same right-to-left pass (a maximum does not depend on its order)
  const int ntile = (ds + kWave - 1) / kWave;
  double carry = 0.0, runmax = 0.0;
  double vnext = 0.0;
  {
    const int t0 = (ntile - 1) * kWave;
    vnext = t0 + l < ds ? xw[t0 + l] : 0.0;
  }
  for (int tt = ntile - 1; tt >= 0; --tt) {
    const int t0 = tt * kWave;
    const int len = ds - t0 < kWave ? ds - t0 : kWave;
    double v = vnext;
    if (tt > 0) vnext = xw[t0 - kWave + l];
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      double y = shfl_f64(v, l + o < kWave ? l + o : kWave - 1);
      if (l + o < len) v = v + y;
    }
    const double total = shfl_f64(v, 0);
    if (tt != ntile - 1) v = v + carry;
    carry = (tt == ntile - 1) ? total : total + carry;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      double y = shfl_f64(v, l + o < kWave ? l + o : kWave - 1);
      if (l + o < len && y > v) v = y;
    }
    if (runmax > v) v = runmax;
    runmax = shfl_f64(v, 0);
    if (l < len) SS[t0 + l] = v;
  }
  fence_wave_local();
  const double Dk = SS[0];
  // 4. sampled edges
  const int st = (ds + kCoarse - 1) / kCoarse;
  const int nco = (ds + st - 1) / st;  // coarse points m_j = j st, j < nco
  for (int j = l; j < nco; j += kWave) {
    const int m = j * st;
    coarse[j] = m + 1 < ds ? SS[m + 1] : 0.0;
  }
  fence_wave_local();
  for (int ib = 0; ib < ds - 1; ib += kSampleRounds * kWave)
    if (!sample_rounds(a, wk, k, ds, ib, kWave, SS, xw, xu, Dk, coarse, st, nco, deadline)) return false;
  // 5. column k of F
  int64_t fbase;
  if (!alloc_column(a, wk, d, fbase)) return false;
  for (int i = l; i < d; i += kWave) {
    const int32_t uu = mu[i];
    a.frow[fbase + i] = uu;
    a.fval[fbase + i] = -(mw[i] / Dk);
    fetch_max(&a.lev[uu], levk + 1);
  }
  if (l == 0) {
    a.D[k] = Dk;
    a.colstart[k] = fbase;
    a.colcnt[k] = d;
  }
  // 6. publish, then delete the pivot's edges (four chunks of the column
  // per round trip)
  Sync::release();
  for (int ib = 0; ib < d; ib += 4 * kWave) {
    bool valid[4];
    int32_t uu[4];
    int mmv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = ib + q * kWave + l;
      valid[q] = i < d;
      uu[q] = valid[q] ? mu[i] : 0;
      mmv[q] = valid[q] ? mm[i] : 0;
    }
    if (!decrement_batch<Sync, 4>(a, valid, uu, mmv)) return false;
  }
  return true;
}

// the gathered size of ready pivot k: nU input upper edges from u0, and its
// fill records
struct PivotSize {
  int64_t u0;
  int nU, g;
};
__device__ __forceinline__ PivotSize pivot_size(const ElimArgs &a, int32_t k) {
  PivotSize z;
  z.u0 = a.uptr[k];
  z.nU = (int)(a.uptr[k + 1] - z.u0);
  z.g = z.nU + ld_acq_relaxed(&a.fill_cnt[k]);
  return z;
}

template <class Sync>
__device__ __forceinline__ bool eliminate_pivot(const ElimArgs &a, Worker &wk, int32_t k,
                                                const PivotSize &z, uint64_t deadline, int *h,
                                                double *coarse) {
  if (z.g == 0) {  // empty neighbourhood: D_k = 0 (Alg. 3/4)
    if (lane() == 0) {
      a.D[k] = 0.0;
      a.colstart[k] = 0;
      a.colcnt[k] = 0;
    }
    return true;
  }
  const int levk = ld_acq_relaxed(&a.lev[k]);
  // AC(k) pivots sample over k slots per neighbour: in registers while
  // all slots fit one wave, else the scratch path
  if (z.g <= kWave && (a.samples <= 1 || (int64_t)z.g * a.samples <= kWave))
    return small_pivot<Sync>(a, wk, k, z.u0, z.nU, z.g, levk, deadline);
  return large_pivot<Sync>(a, wk, k, z.u0, z.nU, z.g, levk, deadline, h, coarse);
}

// After a slot has delivered label k: read k's counter (agent scope).  Zero
// means every pivot that could write to k's inbox has completed its stores
// and decremented the counter, so the records read afterwards are complete.
template <class Sync>
__device__ __forceinline__ bool sync_with_producers(const ElimArgs &a, int32_t k) {
  int v = 0;
  if (lane() == 0) v = fetch_add(&a.dp[k], 0);
  v = first_lane_i32(v);
  if (v != 0) {
    set_error(a.err, PARAC_EINTERNAL);
    return false;
  }
  Sync::acquire();
  return true;
}

// sum of the per-shard counts of eliminated pivots
__device__ __forceinline__ int64_t pivots_done(const ElimArgs &a) {
  int v = ld_acq_relaxed(&a.done[lane() * kTailStride]);
  int64_t t = v;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) t += __shfl_xor(t, o, kWave);
  return t;
}

// ---------------------------------------------------------------------------
// Larger neighbourhoods: the eight waves of a workgroup on one pivot.  The
// critical path of a factorisation is a chain of pivots, each depending on
// the one before, and the longest links are the pivots with many gathered
// entries (thousands on power-law graphs, a few hundred on 3D grids); a
// team shortens every such link.  Each step keeps the
// order of its arithmetic -- the same stable sorts, the same left folds of
// runs, the same 64-wide tiles and carries of the suffix sums, the same
// draws -- so the factor does not depend on which path eliminated a pivot.
// A wave that claims such a pivot hands it to the team queue; teams are
// workgroups of their own in the persistent grid.
// ---------------------------------------------------------------------------
constexpr int kTeamWaves = kElimWaves;
constexpr int kTeamThreads = kTeamWaves * kWave;
constexpr int kTeamCoarse = kTeamWaves * kCoarse;

struct TeamShared {
  int64_t sc_base;       // scratch of the pivot (in wave 0's region)
  int64_t fbase;         // column k of F
  int32_t k;             // the pivot; -1: leave
  int fail;              // a wave failed (the error word is set)
  int cnt[kTeamWaves];   // per-wave counts
};

__device__ __forceinline__ double readlane_f64(double v, int j) {
  return __longlong_as_double((long long)readlane_u64((uint64_t)__double_as_longlong(v), j));
}

// wave w's share of [0, n): an equal part of the chunks of 64, in order
__device__ __forceinline__ void team_range(int n, int w, int &lo, int &hi) {
  const int nch = (n + kWave - 1) / kWave;
  const int per = (nch + kTeamWaves - 1) / kTeamWaves;
  lo = w * per * kWave < n ? w * per * kWave : n;
  hi = (w + 1) * per * kWave < n ? (w + 1) * per * kWave : n;
}

// the stable LSD sort of wave_radix_sort by the team: wave w counts and
// scatters its share, and bucket b of share w starts after every smaller
// bucket and after bucket b of the shares before w.  The digits are the
// bytes 0 .. npass-1 of the key, or with half > 0 the bytes 0 .. half-1 of
// its low word and then of its high word.
template <typename K, typename V>
__device__ __forceinline__ bool team_radix_sort(K *ka, V *va, K *kb, V *vb, int n, int npass, int half,
                                int (*hist)[256], int *wtot) {
  const int t = threadIdx.x, l = lane(), w = t >> 6;
  int lo, hi;
  team_range(n, w, lo, hi);
  bool in_a = true;
  for (int pass = 0; pass < npass; ++pass) {
    const int sh = half > 0 && pass >= half ? 32 + 8 * (pass - half) : 8 * pass;
    K *ks = in_a ? ka : kb;
    V *vs = in_a ? va : vb;
    for (int b = l; b < 256; b += kWave) hist[w][b] = 0;
    fence_wave_local();
    if (lo < hi) radix_count(ks, lo, hi, sh, hist[w]);
    __syncthreads();
    // thread t < 256 owns bucket t (the first four waves)
    int c[kTeamWaves], tot = 0, incl = 0;
    if (t < 256) {
#pragma unroll
      for (int q = 0; q < kTeamWaves; ++q) {
        c[q] = hist[q][t];
        tot += c[q];
      }
      incl = tot;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        int y = __shfl_up(incl, o, kWave);
        if (l >= o) incl += y;
      }
      if (l == kWave - 1) wtot[w] = incl;
    }
    __syncthreads();
    if (t < 256) {
      int run = incl - tot;
      for (int q = 0; q < w; ++q) run += wtot[q];
#pragma unroll
      for (int q = 0; q < kTeamWaves; ++q) {
        hist[q][t] = run;
        run += c[q];
      }
    }
    __syncthreads();
    if (lo < hi) radix_scatter(ks, vs, in_a ? kb : ka, in_a ? vb : va, lo, hi, sh, hist[w]);
    __syncthreads();
    in_a = !in_a;
  }
  return in_a;
}

// The same stable LSD sort with 11-bit digits, for sorts above the LDS-sort
// size: fewer passes (a 22-bit label word in two instead of three, a 64-bit
// weight in six instead of eight), the 2,048-bucket histograms of the eight
// waves (64 KB) in the LDS of the in-LDS sort, idle at these sizes.  Bucket
// b of share w starts after every smaller bucket and after bucket b of the
// shares before w, as above.  shifts[] gives the low bit of each digit.
constexpr int kWideBits = 11;
constexpr int kWideBuckets = 1 << kWideBits;
template <typename K, typename V>
__device__ __forceinline__ bool team_radix_sort_wide(K *ka, V *va, K *kb, V *vb, int n,
                                                     const int *shifts, int npass, int *hl,
                                                     int *wtot) {
  constexpr int per = kWideBuckets / kTeamThreads;  // buckets a thread owns in the scan
  static_assert(per * kTeamThreads == kWideBuckets, "buckets split evenly over the team");
  const int t = threadIdx.x, l = lane(), w = t >> 6;
  int lo, hi;
  team_range(n, w, lo, hi);
  bool in_a = true;
  for (int pass = 0; pass < npass; ++pass) {
    const int sh = shifts[pass];
    K *ks = in_a ? ka : kb;
    V *vs = in_a ? va : vb;
    int *hw = hl + w * kWideBuckets;
    for (int b = l; b < kWideBuckets; b += kWave) hw[b] = 0;
    fence_wave_local();
    if (lo < hi) radix_count<K, kWideBits>(ks, lo, hi, sh, hw);
    __syncthreads();
    // thread t owns buckets [per t, per t + per): its totals over the shares,
    // then an exclusive scan of the per-thread totals over the team
    int c[per][kTeamWaves], tot = 0;
#pragma unroll
    for (int e = 0; e < per; ++e)
#pragma unroll
      for (int q = 0; q < kTeamWaves; ++q) {
        c[e][q] = hl[q * kWideBuckets + per * t + e];
        tot += c[e][q];
      }
    int incl = tot;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int y = __shfl_up(incl, o, kWave);
      if (l >= o) incl += y;
    }
    if (l == kWave - 1) wtot[w] = incl;
    __syncthreads();
    int run = incl - tot;
    for (int q = 0; q < w; ++q) run += wtot[q];
#pragma unroll
    for (int e = 0; e < per; ++e)
#pragma unroll
      for (int q = 0; q < kTeamWaves; ++q) {
        hl[q * kWideBuckets + per * t + e] = run;
        run += c[e][q];
      }
    __syncthreads();
    if (lo < hi)
      radix_scatter<K, V, kWideBits>(ks, vs, in_a ? kb : ka, in_a ? vb : va, lo, hi, sh, hw);
    __syncthreads();
    in_a = !in_a;
  }
  return in_a;
}

// Rank sort by the team for at most kTeamRankMax entries: the keys are staged
// in LDS (lk), and each thread counts, for each of its entries, the keys
// below it -- or equal to it at a smaller index, which makes the result the
// stable order, that of team_radix_sort -- and writes the entry to its rank.
constexpr int kTeamRankMax = 512;
static_assert(kTeamRankMax <= kTeamWaves * kCoarse, "rank-sort keys live in the coarse-table LDS");
__device__ __forceinline__ void team_rank_sort(const uint64_t *ks, const uint64_t *vs, uint64_t *kd,
                                               uint64_t *vd, int n, uint64_t *lk) {
  constexpr int E = (kTeamRankMax + kTeamThreads - 1) / kTeamThreads;
  const int t = threadIdx.x;
  for (int i = t; i < n; i += kTeamThreads) lk[i] = ks[i];
  __syncthreads();
  uint64_t mk[E];
  int r[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = t + e * kTeamThreads;
    mk[e] = i < n ? lk[i] : ~0ull;
    r[e] = 0;
  }
  for (int j = 0; j < n; ++j) {
    const uint64_t kj = lk[j];
#pragma unroll
    for (int e = 0; e < E; ++e) r[e] += (kj < mk[e] || (kj == mk[e] && j < t + e * kTeamThreads)) ? 1 : 0;
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = t + e * kTeamThreads;
    if (i < n) {
      kd[r[e]] = mk[e];
      vd[r[e]] = vs[i];
    }
  }
  __syncthreads();
}

// Radix sorts of at most kTeamLdsSort entries run in LDS: the pairs are
// copied in once, every pass reads and writes LDS (a workgroup has its CU to
// itself, so the LDS is otherwise idle), and the result is copied out once.
constexpr int kTeamLdsSort = 3072;
struct TeamSortLds {
  uint64_t k[2][kTeamLdsSort];
  uint64_t v[2][kTeamLdsSort];
};
static_assert(kTeamWaves * kWideBuckets * sizeof(int) <= sizeof(TeamSortLds),
              "the wide histograms live in the in-LDS sort's buffers");
// The team's stable sort of the pairs (ka, va) of n entries, with the
// buffers (kb, vb) beside them, all in global memory; the key bytes are given
// as for team_radix_sort, and `bits` is the number of bits the key uses (per
// word when half > 0).  Returns true when the result is in (ka, va), false
// when it is in (kb, vb).
__device__ __forceinline__ bool team_sort_pairs(uint64_t *ka, uint64_t *va, uint64_t *kb,
                                                uint64_t *vb, int n, int npass, int half, int bits,
                                                int (*hist)[256], int *wtot, uint64_t *lk,
                                                TeamSortLds &ls) {
  const int t = threadIdx.x;
  if (n <= kTeamRankMax) {
    team_rank_sort(ka, va, kb, vb, n, lk);
    return false;
  }
  if (n > kTeamLdsSort) {
    int shifts[12], np = 0;
    for (int b = 0; b < bits; b += kWideBits) shifts[np++] = b;
    if (half > 0)
      for (int b = 0; b < bits; b += kWideBits) shifts[np++] = 32 + b;
    return team_radix_sort_wide<uint64_t, uint64_t>(ka, va, kb, vb, n, shifts, np, (int *)&ls,
                                                    wtot);
  }
  for (int i = t; i < n; i += kTeamThreads) {
    ls.k[0][i] = ka[i];
    ls.v[0][i] = va[i];
  }
  __syncthreads();
  const bool in0 = team_radix_sort<uint64_t, uint64_t>(ls.k[0], ls.v[0], ls.k[1], ls.v[1], n, npass,
                                                       half, hist, wtot);
  const uint64_t *rk = ls.k[in0 ? 0 : 1], *rv = ls.v[in0 ? 0 : 1];
  for (int i = t; i < n; i += kTeamThreads) {
    kb[i] = rk[i];
    vb[i] = rv[i];
  }
  __syncthreads();
  return false;
}

// true when any wave of the team reported a failure (every wave must call it
// at the same point)
__device__ __forceinline__ bool team_failed(TeamShared &ts, bool mine) {
  if (mine && lane() == 0) ts.fail = 1;
  __syncthreads();
  return ts.fail != 0;
}

__device__ __forceinline__ bool team_pivot(const ElimArgs &a, Worker &wk, int32_t k, uint64_t deadline,
                           int (*hist)[256], double *coarse, TeamShared &ts, int *wtot,
                           TeamSortLds &ls) {
  const int t = threadIdx.x, l = lane(), w = t >> 6;
  const int64_t u0 = a.uptr[k];
  const int nU = (int)(a.uptr[k + 1] - u0);
  const int nF = ld_acq_relaxed(&a.fill_cnt[k]);
  const int g = nU + nF;
  const int levk = ld_acq_relaxed(&a.lev[k]);
  // scratch: wave 0's region, grown geometrically
  if (w == 0) {
    bool bad = false;
    const int64_t bytes = (((int64_t)g * 68) + 255) & ~(int64_t)255;
    if (bytes > wk.sc_size) {
      int64_t want = bytes > 2 * wk.sc_size ? bytes : 2 * wk.sc_size;
      long long off = 0;
      if (l == 0) off = (long long)atomicAdd(a.arena_top, (unsigned long long)want);
      off = __shfl(off, 0, kWave);
      if (off + want > a.arena_cap) {
        set_error(a.err, PARAC_EPOOL);
        bad = true;
      } else {
        wk.sc_base = off;
        wk.sc_size = want;
      }
    }
    if (l == 0) {
      ts.fail = bad ? 1 : 0;
      ts.sc_base = wk.sc_base;
    }
  }
  __syncthreads();
  if (ts.fail) return false;
  char *base = a.arena + ts.sc_base;
  uint64_t *keyA = (uint64_t *)base;
  double *wA = (double *)(keyA + g);
  uint64_t *keyB = (uint64_t *)(wA + g);
  double *wB = (double *)(keyB + g);
  double *mw = wB + g;
  double *sw = mw + g;
  double *S = sw + g;
  int32_t *mu = (int32_t *)(S + g);
  int32_t *mm = mu + g;
  int32_t *su = mm + g;
  // 1. gather
#pragma unroll 4
  for (int i = t; i < g; i += kTeamThreads) {
    int32_t u, src;
    double wt;
    if (i < nU) {
      u = a.uidx[u0 + i];
      src = -1;
      wt = a.uw[u0 + i];
    } else {
      Rec rc = load_rec(a, k, i - nU);
      u = rc.other;
      src = rc.src;
      wt = rc.w;
    }
    keyA[i] = merge_key(u, src);
    wA[i] = wt;
  }
  __syncthreads();
  // 2. sort by (u, src)
  {
    // the bytes a key can use: src + 1 in the low word, u in the high word,
    // both below 2^bits(ntot + 1)
    const int nb = 32 - __clz(a.ntot + 1);
    const int half = (nb + 7) / 8;
    const bool in_a = team_sort_pairs(keyA, (uint64_t *)wA, keyB, (uint64_t *)wB, g, 2 * half, half,
                                      nb, hist, wtot, (uint64_t *)coarse, ls);
    if (!in_a) {  // sorted data in the B buffers: swap names
      uint64_t *tk = keyA;
      keyA = keyB;
      keyB = tk;
      double *tw = wA;
      wA = wB;
      wB = tw;
    }
  }
  const uint64_t *keyS = keyA;
  const double *wS = wA;
  // labels above k, and the runs that begin in each wave's share
  int lo, hi;
  team_range(g, w, lo, hi);
  {
    bool bad = false;
    int cnt = 0;
    for (int ib = lo; ib < hi; ib += kWave) {
      const int i = ib + l;
      const bool valid = i < hi;
      const int32_t u = valid ? (int32_t)(keyS[i] >> 32) : 0;
      const int32_t up = valid && i > 0 ? (int32_t)(keyS[i - 1] >> 32) : -1;
      bad |= valid && (u <= k || u >= a.ntot);
      cnt += __popcll(__ballot(valid && (i == 0 || up != u)));
    }
    if (__any(bad)) set_error(a.err, PARAC_EINTERNAL);
    if (l == 0) ts.cnt[w] = cnt;
    if (team_failed(ts, __any(bad))) return false;
  }
  int d0 = 0, d = 0;
#pragma unroll
  for (int q = 0; q < kTeamWaves; ++q) {
    d0 += q < w ? ts.cnt[q] : 0;
    d += ts.cnt[q];
  }
  {
    const int d1 = merge_runs(keyS, wS, lo, hi, g, d0, mu, mw, mm);
    const bool bad = d1 != d0 + ts.cnt[w];
    if (bad) set_error(a.err, PARAC_EINTERNAL);
    if (team_failed(ts, bad)) return false;
  }
  // 3. sampling order (w asc, u asc): the merged list is in ascending u, so
  // a stable sort on the bits of w alone yields it
  {
    uint64_t *kx = keyB, *vx = (uint64_t *)wB, *ky = (uint64_t *)keyA, *vy = (uint64_t *)wA;
    for (int i = t; i < d; i += kTeamThreads) {
      kx[i] = dbits(mw[i]);
      vx[i] = (uint64_t)(uint32_t)mu[i];
    }
    __syncthreads();
    const bool in_x = team_sort_pairs(kx, vx, ky, vy, d, 8, 0, 64, hist, wtot, (uint64_t *)coarse,
                                      ls);
    const uint64_t *kr = in_x ? kx : ky, *vr = in_x ? vx : vy;
    for (int i = t; i < d; i += kTeamThreads) {
      sw[i] = bitsd(kr[i]);
      su[i] = (int32_t)(uint32_t)vr[i];
    }
    __syncthreads();
  }
  // suffix sums in the tiles and carries of the one-wave path: in-tile sums
  // by all waves, the carry chain (right to left) in wave 0, then in-tile
  // maxima, the maxima of the tiles to the right, and the final maximum
  const int ntile = (d + kWave - 1) / kWave;
  double *T = (double *)keyA;   // tile totals
  double *Cy = (double *)wA;    // carry each tile receives
  double *TM = (double *)keyB;  // tile maxima
  double *MX = (double *)wB;    // maximum of the tiles to the right
  for (int tt = w; tt < ntile; tt += kTeamWaves) {
    const int t0 = tt * kWave;
    const int len = d - t0 < kWave ? d - t0 : kWave;
    double v = l < len ? sw[t0 + l] : 0.0;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      double y = shfl_f64(v, l + o < kWave ? l + o : kWave - 1);
      if (l + o < len) v = v + y;
    }
    if (l < len) S[t0 + l] = v;
    if (l == 0) T[tt] = v;
  }
  __syncthreads();
  if (w == 0) {
    double carry = 0.0;
    for (int cb = ((ntile - 1) / kWave) * kWave; cb >= 0; cb -= kWave) {
      const double tv = cb + l < ntile ? T[cb + l] : 0.0;
      double cy = 0.0;
      const int jt = ntile - 1 - cb < kWave - 1 ? ntile - 1 - cb : kWave - 1;
      for (int j = jt; j >= 0; --j) {
        const double tj = readlane_f64(tv, j);
        if (l == j) cy = carry;
        carry = (cb + j == ntile - 1) ? tj : tj + carry;
      }
      if (cb + l < ntile) Cy[cb + l] = cy;
    }
  }
  __syncthreads();
  for (int tt = w; tt < ntile; tt += kTeamWaves) {
    const int t0 = tt * kWave;
    const int len = d - t0 < kWave ? d - t0 : kWave;
    double v = l < len ? S[t0 + l] : 0.0;
    if (tt != ntile - 1) v = v + Cy[tt];
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      double y = shfl_f64(v, l + o < kWave ? l + o : kWave - 1);
      if (l + o < len && y > v) v = y;
    }
    if (l < len) S[t0 + l] = v;
    if (l == 0) TM[tt] = v;
  }
  __syncthreads();
  if (w == 0) {
    double run = 0.0;
    for (int cb = ((ntile - 1) / kWave) * kWave; cb >= 0; cb -= kWave) {
      const double tv = cb + l < ntile ? TM[cb + l] : 0.0;
      double mx = 0.0;
      const int jt = ntile - 1 - cb < kWave - 1 ? ntile - 1 - cb : kWave - 1;
      for (int j = jt; j >= 0; --j) {
        const double tj = readlane_f64(tv, j);
        if (l == j) mx = run;
        if (tj > run) run = tj;
      }
      if (cb + l < ntile) MX[cb + l] = mx;
    }
  }
  __syncthreads();
  for (int tt = w; tt < ntile; tt += kTeamWaves) {
    const int t0 = tt * kWave;
    const int len = d - t0 < kWave ? d - t0 : kWave;
    const double mx = MX[tt];
    if (l < len) {
      const double v = S[t0 + l];
      if (mx > v) S[t0 + l] = mx;
    }
  }
  __syncthreads();
  const double Dk = S[0];
  // 4. sampled edges, the rounds of 64 slots dealt to the waves in turn
  {
    const int st = (d + kTeamCoarse - 1) / kTeamCoarse;
    const int nco = (d + st - 1) / st;
    for (int j = t; j < nco; j += kTeamThreads) {
      const int m = j * st;
      coarse[j] = m + 1 < d ? S[m + 1] : 0.0;
    }
    __syncthreads();
    bool bad = false;
    // wave w takes the 64-slot rounds w, w + 8, w + 16, ...: small pivots
    // spread over all waves
    for (int ib = w * kWave; ib < d - 1; ib += kTeamWaves * kSampleRounds * kWave)
      if (!sample_rounds(a, wk, k, d, ib, kTeamWaves * kWave, S, sw, su, Dk, coarse, st, nco,
                         deadline)) {
        bad = true;
        break;
      }
    if (team_failed(ts, bad)) return false;
  }
  // 5. column k of F
  {
    bool bad = false;
    if (w == 0) {
      int64_t fb = 0;
      bad = !alloc_column(a, wk, d, fb);
      if (l == 0) ts.fbase = fb;
    }
    if (team_failed(ts, bad)) return false;
  }
  const int64_t fbase = ts.fbase;
  for (int i = t; i < d; i += kTeamThreads) {
    const int32_t uu = mu[i];
    a.frow[fbase + i] = uu;
    a.fval[fbase + i] = -(mw[i] / Dk);
    fetch_max(&a.lev[uu], levk + 1);
  }
  if (t == 0) {
    a.D[k] = Dk;
    a.colstart[k] = fbase;
    a.colcnt[k] = d;
  }
  // 6. publish (every wave's stores complete before any counter drops),
  // then delete the pivot's edges
  WideSync::release();
  __syncthreads();
  bool bad = false;
  // wave w takes the 64-entry chunks w, w + 8, w + 16, ...
  for (int ib = w * kWave; ib < d; ib += kTeamWaves * 4 * kWave) {
    bool valid[4];
    int32_t uu[4];
    int mmv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = ib + q * kTeamWaves * kWave + l;
      valid[q] = i < d;
      uu[q] = valid[q] ? mu[i] : 0;
      mmv[q] = valid[q] ? mm[i] : 0;
    }
    if (!decrement_batch<WideSync, 4>(a, valid, uu, mmv)) {
      bad = true;
      break;
    }
  }
  return !team_failed(ts, bad);
}

// A team workgroup: claims slots of the team queue in increasing order, as
// the waves claim shard slots, and leaves once every pivot it could be
// waiting for is eliminated.
__device__ __forceinline__ void team_worker(const ElimArgs &a, int (*hist)[256], double *coarse, TeamShared &ts,
                            int *wtot, TeamSortLds &ls) {
  const int t = threadIdx.x, l = lane(), w = t >> 6;
  const uint64_t deadline = now_ticks() + a.timeout_ticks;
  const int64_t all = a.stop_at < (int64_t)a.ntot ? a.stop_at : (int64_t)a.ntot;
  Worker wk{0, 0, 0, 0, 0, 0};
  for (;;) {
    // a team claims a slot only when it is free, so that a handed-off pivot
    // never waits for a busy team while another one idles
    if (w == 0) {
      int slot = 0;
      if (l == 0) slot = atomicAdd(a.bq_head, 1);
      slot = first_lane_i32(slot);
      int32_t k = -1;
      Backoff bo;
      for (int it = 0;; ++it) {
        int32_t v = -1;
        if (l == 0 && slot < a.bq_cap) v = ld_acq_relaxed(&a.bq[slot]);
        k = first_lane_i32(v);
        if (k >= 0) break;
        if ((it & 15) == 15 && (timed_out(a, deadline) || pivots_done(a) >= all)) break;
        bo.pause();
      }
      // the wave that handed k over has seen its counter at zero
      if (l == 0) ts.k = k;
    }
    __syncthreads();
    const int32_t k = ts.k;
    if (k < 0) return;
    WideSync::acquire();
    if (!team_pivot(a, wk, k, deadline, hist, coarse, ts, wtot, ls)) return;
    if (t == 0) atomicAdd(&a.done[(k & (kSubQueues - 1)) * kTailStride], 1);
    __syncthreads();  // ts.k is rewritten for the next pivot
  }
}

static_assert(kElimWaves >= 4 && kElimWaves <= 8, "team sorts assume 4 to 8 waves");
__global__ __launch_bounds__(kElimWaves * kWave, 8 / kElimWaves) void k_eliminate(ElimArgs a) {
  __shared__ int hist[kElimWaves][256];          // radix-sort histogram of each wave
  __shared__ double coarse[kElimWaves][kCoarse];  // coarse suffix sums of each wave
  __shared__ TeamShared ts;
  __shared__ int wtot[kTeamWaves];
  __shared__ TeamSortLds tls;
  if (a.stop_at <= 0) return;
  if ((int)blockIdx.x >= a.team_wg0) {
    team_worker(a, hist, &coarse[0][0], ts, wtot, tls);
    return;
  }
  const int wid = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (wid >= a.nworkers) return;
  const uint64_t deadline = now_ticks() + a.timeout_ticks;
  // Shard x holds exactly the labels v = x (mod kSubQueues), so its slot
  // count is known.  Workers claim its slots in increasing order (the next
  // claim is taken before the current pivot is eliminated): the lowest ready
  // slot is always held by a running worker, whatever the residency.
  const int x = wid & (kSubQueues - 1);
  const int cnt = x < a.ntot ? (a.ntot - 1 - x) / kSubQueues + 1 : 0;
  const int32_t *qx = a.q + (int64_t)x * a.cap_q;
  int *head = a.qhead + x * kTailStride;
  const int *tailx = a.qtail + x * kTailStride;
  Worker wk{0, 0, 0, 0, 0, 0};
  int next = 0;
  if (lane() == 0) next = atomicAdd(head, 1);
  next = __shfl(next, 0, kWave);
  while (next < cnt) {
    const int slot = next;
    int32_t k;
    // Poll the slot.  A worker whose slot lies d places beyond the shard's
    // tail cannot be served before d more enqueues, so it waits ~d polls'
    // worth between reads: the front of each queue stays responsive while
    // the idle workers of a narrow phase stay quiet.  Once all but the thin
    // tail of the pivots are eliminated, idle workers leave: the tail kernel
    // finishes the factorisation.
    Backoff bo;
    for (int it = 0;; ++it) {
      int32_t v = 0;
      if (lane() == 0) v = ld_acq_relaxed(&qx[slot]);
      k = first_lane_i32(v);
      if (k >= 0) break;
      if ((it & 15) == 15) {
        if (timed_out(a, deadline)) return;
        if (pivots_done(a) >= a.stop_at) return;
        int t = 0;
        if (lane() == 0) t = ld_acq_relaxed(tailx);
        const int dist = first_lane_i32(slot - t);
        for (int w = 1; w < dist && w < 32; ++w) __builtin_amdgcn_s_sleep(64);
      }
      bo.pause();
    }
    if (!sync_with_producers<WideSync>(a, k)) return;
    // a pivot above team_min goes to the team queue (whose slots are never
    // reused) before the next claim
    const PivotSize z = pivot_size(a, k);
    const bool handed = a.team_min > 0 && z.g > a.team_min;
    if (handed && lane() == 0) {
      const int pos = fetch_add(a.bq_tail, 1);
      __hip_atomic_exchange(&a.bq[pos], k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane() == 0) next = atomicAdd(head, 1);
    next = __shfl(next, 0, kWave);
    if (handed) continue;
    if (!eliminate_pivot<WideSync>(a, wk, k, z, deadline, hist[threadIdx.x >> 6],
                                   coarse[threadIdx.x >> 6]))
      return;
    if (lane() == 0) atomicAdd(&a.done[x * kTailStride], 1);
  }
}

// The tail's starting point: labels not yet eliminated (colcnt < 0) are
// counted; those already ready (counter zero) seed the tail queue.
__global__ void k_tail_seed(ElimArgs a) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool left = v < a.ntot && a.colcnt[v] < 0;
  const bool ready = left && a.dp[v] == 0;
  const uint64_t ml = __ballot(left), mr = __ballot(ready);
  int base_r = 0;
  if (lane() == 0) {
    if (ml) atomicAdd(a.tq_count, (int)__popcll(ml));
    if (mr) base_r = atomicAdd(a.tq_tail, (int)__popcll(mr));
  }
  base_r = __shfl(base_r, 0, kWave);
  if (ready) a.tq[base_r + __popcll(mr & lanemask_lt())] = (int32_t)v;
}

// One workgroup (16 waves, one CU) eliminates the remaining pivots; the same
// pivot code with workgroup-scope fences and its own in-order queue.
__global__ __launch_bounds__(1024) void k_eliminate_tail(ElimArgs a) {
  __shared__ int hist[16][256];          // radix-sort histogram of each wave
  __shared__ double coarse[16][kCoarse];  // coarse suffix sums of each wave
  const int total = *a.tq_count;
  if (total == 0) return;
  const uint64_t deadline = now_ticks() + a.timeout_ticks;
  Worker wk{0, 0, 0, 0, 0, 0};
  int next = 0;
  if (lane() == 0) next = __hip_atomic_fetch_add(a.tq_head, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  next = __shfl(next, 0, kWave);
  while (next < total) {
    const int slot = next;
    int32_t k;
    Backoff bo;
    for (int it = 0;; ++it) {
      int32_t v = 0;
      if (lane() == 0) v = __hip_atomic_load(&a.tq[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      k = first_lane_i32(v);
      if (k >= 0) break;
      if ((it & 15) == 15 && timed_out(a, deadline)) return;
      bo.pause();
    }
    if (!sync_with_producers<TailSync>(a, k)) return;
    if (lane() == 0) next = __hip_atomic_fetch_add(a.tq_head, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    next = __shfl(next, 0, kWave);
    if (!eliminate_pivot<TailSync>(a, wk, k, pivot_size(a, k), deadline, hist[threadIdx.x >> 6],
                                   coarse[threadIdx.x >> 6]))
      return;
  }
}

hipError_t launch_eliminate(const ElimArgs &a, int wgs, hipStream_t s) {
  hipLaunchKernelGGL(k_eliminate, dim3((unsigned)wgs), dim3(kElimWaves * kWave), 0, s, a);
  hipLaunchKernelGGL(k_tail_seed, dim3((unsigned)((a.ntot + 255) / 256)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_eliminate_tail, dim3(1), dim3(1024), 0, s, a);
  return hipGetLastError();
}

int eliminate_max_workgroups() {
  int dev = 0, per_cu = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_eliminate, kElimWaves * kWave, 0) != hipSuccess)
    return 0;
  return per_cu * prop.multiProcessorCount;
}

}  // namespace parac
