// host_parac.cpp -- ParAC on the host's CPU cores: the paper's CPU design
// (§IV-B, Alg. 3).  Worker threads claim ready pivots from one shared queue
// and eliminate them concurrently; the dependency counters d(i) of §III
// decide when a vertex is ready (no lower-labelled neighbour left), and each
// pivot inserts its sampled fill before it removes its own edges, so a
// counter never reaches zero while fill for that vertex is still coming.
//
// The arithmetic follows the same canonical orders as the GPU elimination:
// gathered entries merged by the key (u, src) with a left fold per run,
// sampling order (w, u) ascending, suffix sums over 64-entry tiles with a
// fixed association, one Philox4x64-10 draw per (pivot label, slot), fill
// weight (S_{p+1} w_p) / D_k, factor entries -(w_u / D_k).  The factor is
// therefore the same bit for bit for any thread count and any timing, and
// equal to the GPU library's.
//
// Plain C++17 host code, built with -ffp-contract=off (no fused multiply-add)
// and no fast-math.  It runs only when called through parac_factor_host; no
// GPU entry point uses it.
#include <algorithm>
#include <atomic>
#include <cfloat>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "parac.h"

namespace {

thread_local std::string g_host_error;

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, two
// 64x64 -> 128-bit products per round, Weyl-sequence key schedule.  Only the
// first output word is used.
// ---------------------------------------------------------------------------
inline uint64_t philox_word0(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                             uint64_t k1) {
  const uint64_t m0 = 0xD2E7470EE14C6C93ull, m1 = 0xCA5A826395121157ull;
  const uint64_t w0 = 0x9E3779B97F4A7C15ull, w1 = 0xBB67AE8584CAA73Bull;
  for (int r = 0; r < 10; ++r) {
    const unsigned __int128 p0 = (unsigned __int128)m0 * c0;
    const unsigned __int128 p1 = (unsigned __int128)m1 * c2;
    const uint64_t h0 = (uint64_t)(p0 >> 64), l0 = (uint64_t)p0;
    const uint64_t h1 = (uint64_t)(p1 >> 64), l1 = (uint64_t)p1;
    const uint64_t n0 = h1 ^ c1 ^ k0, n2 = h0 ^ c3 ^ k1;
    c0 = n0;
    c1 = l1;
    c2 = n2;
    c3 = l0;
    k0 += w0;
    k1 += w1;
  }
  return c0;
}

// the draw of slot s of pivot k: 53 random bits as a double in [0, 1)
inline double unit_draw(uint64_t seed, int32_t k, int64_t s) {
  const uint64_t x = philox_word0((uint64_t)(uint32_t)k, (uint64_t)s, 0, 0, seed, 0);
  return (double)(x >> 11) * 0x1.0p-53;
}

struct FillRec {
  int32_t other, src;
  double w;
  int64_t next;  // next record of the same target, -1 at the end
};

struct Gathered {
  int32_t u, src;
  double w;
};

struct Merged {
  int32_t u, m;
  double w;
};

struct FailCode {
  int code;
  std::string msg;
};

// ---------------------------------------------------------------------------
// Suffix sums of x[0..d) into S[0..d): tiles of 64 positions from the first;
// inside a tile, log-steps with offsets 1, 2, ..., 32, each adding the value
// `off` places to the right (same tile) as it was before the step; tile
// totals carried from the last tile to the first by a running sum; then the
// exact suffix maximum, which makes S non-increasing.
// ---------------------------------------------------------------------------
void tiled_suffix_sums(const std::vector<double> &x, int64_t d, std::vector<double> &S,
                       std::vector<double> &prev) {
  for (int64_t i = 0; i < d; ++i) S[i] = x[i];
  for (int64_t base = 0; base < d; base += 64) {
    const int64_t len = std::min<int64_t>(64, d - base);
    for (int64_t off = 1; off < 64; off *= 2) {
      for (int64_t l = 0; l < len; ++l) prev[l] = S[base + l];
      for (int64_t l = 0; l + off < len; ++l) S[base + l] = prev[l] + prev[l + off];
    }
  }
  const int64_t ntiles = (d + 63) / 64;
  double carry = 0.0;
  for (int64_t t = ntiles - 1; t >= 0; --t) {
    const int64_t base = t * 64, len = std::min<int64_t>(64, d - base);
    const double total = S[base];
    const bool last = t == ntiles - 1;
    if (!last)
      for (int64_t l = 0; l < len; ++l) S[base + l] = S[base + l] + carry;
    carry = last ? total : total + carry;
  }
  for (int64_t i = d - 2; i >= 0; --i) S[i] = std::max(S[i], S[i + 1]);
}

// ---------------------------------------------------------------------------
// Input classification: w_ij = -a_ij, excess s_i = a_ii - (left fold of the
// w_ij over ascending j), |s_i| <= 4 (deg_i + 1) eps a_ii taken as zero.
// Errors by precedence: structure, then sign / symmetry / excess, then the
// permutation; the lowest row within a class.
// ---------------------------------------------------------------------------
struct RowCheck {
  int phase = 3;  // 3 = no error
  int64_t row = 0;
  int code = PARAC_OK;
  void note(int ph, int64_t r, int c) {
    if (ph < phase || (ph == phase && r < row)) {
      phase = ph;
      row = r;
      code = c;
    }
  }
};

template <class F>
void parallel_for(int64_t n, int threads, F fn) {
  if (threads <= 1 || n < 4096) {
    fn(0, (int64_t)0, n);
    return;
  }
  std::vector<std::thread> ts;
  const int64_t per = (n + threads - 1) / threads;
  for (int t = 0; t < threads; ++t) {
    const int64_t b = t * per, e = std::min(n, b + per);
    if (b >= e) break;
    ts.emplace_back([=, &fn] { fn(t, b, e); });
  }
  for (auto &th : ts) th.join();
}

int64_t find_col(const int64_t *rowptr, const int32_t *col, int64_t nnz, int64_t j, int32_t i) {
  int64_t lo = std::min(std::max<int64_t>(rowptr[j], 0), nnz);
  int64_t hi = std::min(std::max<int64_t>(rowptr[j + 1], lo), nnz);
  const int64_t end = hi;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (col[mid] < i)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < end && col[lo] == i) ? lo : -1;
}

struct Classified {
  int mode;
  std::vector<double> excess;
};

Classified classify(const parac_csr &A, int mode_req, const int32_t *perm, int threads) {
  const int64_t n = A.n, nnz = A.nnz;
  const int64_t *rowptr = A.rowptr;
  const int32_t *col = A.col;
  const double *val = A.val;
  if (n < 0 || n > (int64_t)INT32_MAX - 2 || nnz < 0)
    throw FailCode{PARAC_EINVAL, "bad matrix size"};
  if (mode_req < PARAC_MODE_AUTO || mode_req > PARAC_MODE_SDDM)
    throw FailCode{PARAC_EINVAL, "bad mode"};
  Classified out;
  out.excess.assign((size_t)n, 0.0);
  if (n == 0) {
    out.mode = mode_req == PARAC_MODE_SDDM ? PARAC_MODE_SDDM : PARAC_MODE_LAPLACIAN;
    return out;
  }
  if (!rowptr || !col || !val) throw FailCode{PARAC_EINVAL, "null matrix arrays"};
  std::vector<RowCheck> per(std::max(threads, 1));
  std::vector<char> any(std::max(threads, 1), 0);
  RowCheck head;
  if (rowptr[0] != 0 || rowptr[n] != nnz) head.note(0, 0, PARAC_EINVAL);
  parallel_for(n, threads, [&](int t, int64_t b0, int64_t e0) {
    RowCheck &rc = per[t];
    for (int64_t i = b0; i < e0; ++i) {
      const int64_t b = rowptr[i], e = rowptr[i + 1];
      if (b < 0 || e < b || e > nnz) {
        rc.note(0, i, PARAC_EINVAL);
        continue;
      }
      bool bad = false;
      int32_t prev = -1;
      for (int64_t p = b; p < e && !bad; ++p) {
        const int32_t j = col[p];
        if (j < 0 || j >= n || j <= prev || !std::isfinite(val[p])) bad = true;
        prev = j;
      }
      if (bad) {
        rc.note(0, i, PARAC_EINVAL);
        continue;
      }
      double diag = 0.0, acc = 0.0;
      int64_t deg = 0;
      for (int64_t p = b; p < e && !bad; ++p) {
        const int32_t j = col[p];
        const double a = val[p];
        if (j == i) {
          diag = a;
          continue;
        }
        if (a == 0.0) continue;
        if (a > 0.0) {
          rc.note(1, i, PARAC_ENOTLAP);
          bad = true;
          break;
        }
        const int64_t q = find_col(rowptr, col, nnz, j, (int32_t)i);
        if (q < 0 || val[q] != a) {
          rc.note(1, i, PARAC_EINVAL);
          bad = true;
          break;
        }
        acc += -a;
        ++deg;
      }
      if (bad) continue;
      double s = diag - acc;
      const double tol = 4.0 * (double)(deg + 1) * DBL_EPSILON * std::fabs(diag);
      if (s < -tol) {
        rc.note(1, i, PARAC_ENOTLAP);
        continue;
      }
      if (s <= tol) s = 0.0;
      out.excess[(size_t)i] = s;
      if (s > 0.0) any[t] = 1;
    }
  });
  for (auto &rc : per)
    if (rc.phase < 3) head.note(rc.phase, rc.row, rc.code);
  if (head.phase == 3 && perm) {
    std::vector<char> seen((size_t)n, 0);
    for (int64_t v = 0; v < n; ++v) {
      const int32_t l = perm[v];
      if (l < 0 || l >= n || seen[(size_t)l]) {
        head.note(2, v, PARAC_EINVAL);
        break;
      }
      seen[(size_t)l] = 1;
    }
  }
  if (head.phase < 3)
    throw FailCode{head.code, "input rejected at row " + std::to_string(head.row)};
  const bool has_excess = std::find(any.begin(), any.end(), 1) != any.end();
  int mode = mode_req;
  if (mode == PARAC_MODE_AUTO) mode = has_excess ? PARAC_MODE_SDDM : PARAC_MODE_LAPLACIAN;
  if (mode == PARAC_MODE_LAPLACIAN && has_excess)
    throw FailCode{PARAC_ENOTLAP, "positive excess in Laplacian mode"};
  out.mode = mode;
  return out;
}

// ---------------------------------------------------------------------------
// The concurrent elimination
// ---------------------------------------------------------------------------
struct Shared {
  int64_t ntot = 0;
  uint64_t seed = 0;
  // label-space upper adjacency (input edges, with the ground edges)
  std::vector<int64_t> uptr;
  std::vector<int32_t> uidx;
  std::vector<double> uw;
  // dependency counters, ready queue, levels
  std::unique_ptr<std::atomic<int32_t>[]> dp;
  std::unique_ptr<std::atomic<int32_t>[]> q;
  std::atomic<int64_t> q_tail{0}, q_next{0};
  std::unique_ptr<std::atomic<int32_t>[]> level;
  // fill records: a lock-free stack per target label, records from one pool
  std::unique_ptr<std::atomic<int64_t>[]> inbox;
  FillRec *pool = nullptr;
  int64_t pool_cap = 0;
  std::atomic<int64_t> pool_top{0};
  std::atomic<int> error{0};
  // factor columns: per-thread buffers
  std::vector<int32_t> col_thread;
  std::vector<int64_t> col_off;
  std::vector<int32_t> col_cnt;
  std::vector<double> D;
  std::atomic<int64_t> n_fill{0};
};

struct ThreadCols {
  std::vector<int32_t> row;
  std::vector<double> val;
};

// a vertex is enqueued once, when its counter reaches zero; more than ntot
// enqueues means some vertex came twice
void enqueue(Shared &S, int32_t u) {
  const int64_t at = S.q_tail.fetch_add(1, std::memory_order_relaxed);
  if (at >= S.ntot) {
    S.error.store(PARAC_EINTERNAL, std::memory_order_relaxed);
    return;
  }
  S.q[at].store(u, std::memory_order_release);
}

void atomic_max(std::atomic<int32_t> &a, int32_t v) {
  int32_t cur = a.load(std::memory_order_relaxed);
  while (cur < v && !a.compare_exchange_weak(cur, v, std::memory_order_relaxed)) {
  }
}

void worker(Shared &S, int tid, ThreadCols &cols) {
  std::vector<Gathered> g;
  std::vector<Merged> byu, order;
  std::vector<double> x, Sx, tmp;
  for (;;) {
    if (S.error.load(std::memory_order_relaxed)) return;
    const int64_t slot = S.q_next.fetch_add(1, std::memory_order_relaxed);
    if (slot >= S.ntot) return;
    int32_t k;
    // the slot is written once the vertex it will hold becomes ready; the
    // lowest unfinished label is always ready, so this wait ends
    while ((k = S.q[slot].load(std::memory_order_acquire)) < 0) {
      if (S.error.load(std::memory_order_relaxed)) return;
      std::this_thread::yield();
    }
    // gather: input upper edges and the fill addressed to k
    g.clear();
    for (int64_t e = S.uptr[k]; e < S.uptr[k + 1]; ++e) g.push_back({S.uidx[e], -1, S.uw[e]});
    for (int64_t r = S.inbox[k].load(std::memory_order_acquire); r >= 0; r = S.pool[r].next)
      g.push_back({S.pool[r].other, S.pool[r].src, S.pool[r].w});
    S.col_thread[k] = tid;
    S.col_off[k] = (int64_t)cols.row.size();
    if (g.empty()) {  // isolated: D_k = 0, empty column
      S.col_cnt[k] = 0;
      S.D[k] = 0.0;
      continue;
    }
    // merge parallel edges: key (u, src) is unique; left fold per run of u
    std::sort(g.begin(), g.end(), [](const Gathered &a, const Gathered &b) {
      return a.u != b.u ? a.u < b.u : a.src < b.src;
    });
    byu.clear();
    for (size_t i = 0; i < g.size();) {
      size_t j = i;
      double w = g[i].w;
      while (j + 1 < g.size() && g[j + 1].u == g[i].u) w = w + g[++j].w;
      byu.push_back({g[i].u, (int32_t)(j - i + 1), w});
      i = j + 1;
    }
    const int64_t d = (int64_t)byu.size();
    // sampling order (w, u) ascending, suffix sums, D_k = S_1
    order = byu;
    std::sort(order.begin(), order.end(), [](const Merged &a, const Merged &b) {
      return a.w != b.w ? a.w < b.w : a.u < b.u;
    });
    x.resize((size_t)d);
    Sx.resize((size_t)d);
    tmp.resize(64);
    for (int64_t i = 0; i < d; ++i) x[(size_t)i] = order[(size_t)i].w;
    tiled_suffix_sums(x, d, Sx, tmp);
    const double Dk = Sx[0];
    S.D[k] = Dk;
    const int32_t lk = S.level[k].load(std::memory_order_relaxed);
    // one sampled edge per slot: partner q > s drawn with probability
    // w_q / S_{s+1}, i.e. the first q whose remaining suffix S_{q+1} <= t
    if (d > 1) {
      const int64_t base = S.pool_top.fetch_add(d - 1, std::memory_order_relaxed);
      if (base + d - 1 > S.pool_cap) {
        S.error.store(PARAC_EPOOL, std::memory_order_relaxed);
        return;
      }
      for (int64_t s = 0; s + 1 < d; ++s) {
        const double t = unit_draw(S.seed, k, s) * Sx[(size_t)s + 1];
        int64_t lo = s + 1, hi = d - 1;  // S_{hi+1} = 0 <= t always
        while (lo < hi) {
          const int64_t mid = lo + (hi - lo) / 2;
          const double next = Sx[(size_t)mid + 1];
          if (next <= t)
            hi = mid;
          else
            lo = mid + 1;
        }
        const int32_t a = order[(size_t)s].u, b = order[(size_t)lo].u;
        const double c = (Sx[(size_t)s + 1] * order[(size_t)s].w) / Dk;
        const int32_t tgt = std::min(a, b), oth = std::max(a, b);
        FillRec &rec = S.pool[base + s];
        rec.other = oth;
        rec.src = k;
        rec.w = c;
        // the larger endpoint gains a lower neighbour before k's own edge to
        // it is removed below (insert before delete)
        if (S.dp[oth].fetch_add(1, std::memory_order_relaxed) < 1)
          S.error.store(PARAC_EINTERNAL, std::memory_order_relaxed);
        int64_t head = S.inbox[tgt].load(std::memory_order_relaxed);
        do {
          rec.next = head;
        } while (!S.inbox[tgt].compare_exchange_weak(head, base + s, std::memory_order_release,
                                                     std::memory_order_relaxed));
      }
      S.n_fill.fetch_add(d - 1, std::memory_order_relaxed);
    }
    // column k of F, rows ascending
    for (const Merged &m : byu) {
      cols.row.push_back(m.u);
      cols.val.push_back(-(m.w / Dk));
    }
    S.col_cnt[k] = (int32_t)d;
    // remove k's edges: counters drop by the multiplicities; a counter
    // reaching zero makes its vertex ready
    for (const Merged &m : byu) {
      atomic_max(S.level[m.u], lk + 1);
      const int32_t prior = S.dp[m.u].fetch_sub(m.m, std::memory_order_acq_rel);
      if (prior < m.m) S.error.store(PARAC_EINTERNAL, std::memory_order_relaxed);
      if (prior == m.m) enqueue(S, m.u);
    }
  }
}

void run_elimination(const parac_csr &A, const parac_factor_opts &o, int threads,
                     parac_host_factor *out) {
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t n = A.n;
  Classified cl = classify(A, o.mode, o.perm, threads);
  const bool sddm = cl.mode == PARAC_MODE_SDDM;
  const int64_t ntot = n + (sddm ? 1 : 0);
  std::vector<int32_t> label((size_t)n);
  for (int64_t v = 0; v < n; ++v) label[(size_t)v] = o.perm ? o.perm[v] : (int32_t)v;
  Shared S;
  S.ntot = ntot;
  S.seed = o.seed;
  S.uptr.assign((size_t)ntot + 1, 0);
  S.dp.reset(new std::atomic<int32_t>[(size_t)std::max<int64_t>(ntot, 1)]);
  S.q.reset(new std::atomic<int32_t>[(size_t)std::max<int64_t>(ntot, 1)]);
  S.level.reset(new std::atomic<int32_t>[(size_t)std::max<int64_t>(ntot, 1)]);
  S.inbox.reset(new std::atomic<int64_t>[(size_t)std::max<int64_t>(ntot, 1)]);
  for (int64_t v = 0; v < ntot; ++v) {
    S.dp[v].store(0, std::memory_order_relaxed);
    S.q[v].store(-1, std::memory_order_relaxed);
    S.level[v].store(0, std::memory_order_relaxed);
    S.inbox[v].store(-1, std::memory_order_relaxed);
  }
  // upper adjacency in label space and the initial counters d_0(b) = number
  // of lower-labelled neighbours (§III initialisation)
  auto edge_ok = [&](int64_t i, int64_t p) { return A.col[p] != i && A.val[p] != 0.0; };
  for (int64_t i = 0; i < n; ++i) {
    const int32_t a = label[(size_t)i];
    for (int64_t p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p)
      if (edge_ok(i, p) && label[(size_t)A.col[p]] > a) S.uptr[(size_t)a + 1]++;
    if (sddm && cl.excess[(size_t)i] > 0.0) S.uptr[(size_t)a + 1]++;
  }
  for (int64_t v = 0; v < ntot; ++v) S.uptr[(size_t)v + 1] += S.uptr[(size_t)v];
  const int64_t ne = S.uptr[(size_t)ntot];
  S.uidx.resize((size_t)ne);
  S.uw.resize((size_t)ne);
  {
    std::vector<int64_t> cur(S.uptr.begin(), S.uptr.end() - 1);
    for (int64_t i = 0; i < n; ++i) {
      const int32_t a = label[(size_t)i];
      for (int64_t p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) {
        if (!edge_ok(i, p)) continue;
        const int32_t b = label[(size_t)A.col[p]];
        if (b <= a) continue;
        S.uidx[(size_t)cur[(size_t)a]] = b;
        S.uw[(size_t)cur[(size_t)a]++] = -A.val[p];
        S.dp[b].fetch_add(1, std::memory_order_relaxed);
      }
      if (sddm && cl.excess[(size_t)i] > 0.0) {
        S.uidx[(size_t)cur[(size_t)a]] = (int32_t)n;
        S.uw[(size_t)cur[(size_t)a]++] = cl.excess[(size_t)i];
        S.dp[n].fetch_add(1, std::memory_order_relaxed);
      }
    }
  }
  S.col_thread.assign((size_t)ntot, 0);
  S.col_off.assign((size_t)ntot, 0);
  S.col_cnt.assign((size_t)ntot, 0);
  S.D.assign((size_t)ntot, 0.0);
  double pf = o.pool_factor > 0 ? o.pool_factor : 4.0;
  std::vector<ThreadCols> cols((size_t)threads);
  for (int attempt = 0;; ++attempt) {
    // fill pool: pool_factor records per stored entry of L
    S.pool_cap = std::max<int64_t>((int64_t)(pf * (double)std::max<int64_t>(A.nnz, 64)), 64);
    std::unique_ptr<FillRec[]> pool(new (std::nothrow) FillRec[(size_t)S.pool_cap]);
    if (!pool) throw FailCode{PARAC_ENOMEM, "host fill pool allocation failed"};
    S.pool = pool.get();
    S.pool_top.store(0);
    S.error.store(0);
    S.n_fill.store(0);
    S.q_tail.store(0);
    S.q_next.store(0);
    std::vector<int32_t> dp0((size_t)ntot);
    for (int64_t v = 0; v < ntot; ++v) dp0[(size_t)v] = S.dp[v].load(std::memory_order_relaxed);
    for (int64_t v = 0; v < ntot; ++v)
      if (dp0[(size_t)v] == 0) enqueue(S, (int32_t)v);
    std::vector<std::thread> ts;
    for (int t = 0; t < threads; ++t)
      ts.emplace_back([&S, &cols, t] { worker(S, t, cols[(size_t)t]); });
    for (auto &th : ts) th.join();
    const int err = S.error.load();
    if (err == PARAC_EPOOL && attempt < 12) {
      // the factor does not depend on storage: a larger pool reproduces it
      pf *= 2.5;
      for (int64_t v = 0; v < ntot; ++v) {
        S.dp[v].store(dp0[(size_t)v], std::memory_order_relaxed);
        S.q[v].store(-1, std::memory_order_relaxed);
        S.level[v].store(0, std::memory_order_relaxed);
        S.inbox[v].store(-1, std::memory_order_relaxed);
      }
      for (auto &c : cols) {
        c.row.clear();
        c.val.clear();
      }
      continue;
    }
    if (err)
      throw FailCode{err, err == PARAC_EINTERNAL ? "a dependency counter invariant failed"
                                                 : "host elimination failed"};
    if (S.q_tail.load() != ntot) throw FailCode{PARAC_EINTERNAL, "not every vertex was eliminated"};
    break;
  }
  // canonical CSC of F in label space
  std::vector<int64_t> colptr((size_t)ntot + 1, 0);
  for (int64_t k = 0; k < ntot; ++k) colptr[(size_t)k + 1] = colptr[(size_t)k] + S.col_cnt[(size_t)k];
  const int64_t nnz_off = colptr[(size_t)ntot];
  out->colptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ntot + 1));
  out->rowind = (int32_t *)malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz_off, 1));
  out->val = (double *)malloc(sizeof(double) * (size_t)std::max<int64_t>(nnz_off, 1));
  out->D = (double *)malloc(sizeof(double) * (size_t)std::max<int64_t>(ntot, 1));
  out->level = (int32_t *)malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(ntot, 1));
  if (!out->colptr || !out->rowind || !out->val || !out->D || !out->level)
    throw FailCode{PARAC_ENOMEM, "host factor allocation failed"};
  memcpy(out->colptr, colptr.data(), sizeof(int64_t) * (size_t)(ntot + 1));
  int64_t depth = 0;
  parallel_for(ntot, threads, [&](int, int64_t b, int64_t e) {
    for (int64_t k = b; k < e; ++k) {
      const ThreadCols &c = cols[(size_t)S.col_thread[(size_t)k]];
      const int64_t off = S.col_off[(size_t)k], cnt = S.col_cnt[(size_t)k];
      memcpy(out->rowind + colptr[(size_t)k], c.row.data() + off, sizeof(int32_t) * (size_t)cnt);
      memcpy(out->val + colptr[(size_t)k], c.val.data() + off, sizeof(double) * (size_t)cnt);
      out->D[k] = S.D[(size_t)k];
      out->level[k] = S.level[k].load(std::memory_order_relaxed);
    }
  });
  for (int64_t k = 0; k < ntot; ++k) depth = std::max<int64_t>(depth, out->level[k] + 1);
  out->n = n;
  out->ntot = ntot;
  out->mode = cl.mode;
  out->nnz_off = nnz_off;
  out->n_fill = S.n_fill.load();
  out->depth = depth;
  out->threads = threads;
  out->ms_total =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

extern "C" {

parac_status parac_factor_host(const parac_csr *A, const parac_factor_opts *o, int32_t threads,
                               parac_host_factor *out) {
  if (!A || !out || A->on_device) {
    g_host_error = "parac_factor_host needs a host matrix and an output struct";
    return PARAC_EINVAL;
  }
  memset(out, 0, sizeof(*out));
  parac_factor_opts opt{};
  opt.pool_factor = 4.0;
  if (o) opt = *o;
  if (opt.samples > 1) {
    g_host_error = "parac_factor_host builds the plain factor only (samples must be 0 or 1)";
    return PARAC_EINVAL;
  }
  if (threads <= 0) threads = (int32_t)std::max(1u, std::thread::hardware_concurrency());
  try {
    run_elimination(*A, opt, threads, out);
    return PARAC_OK;
  } catch (FailCode &e) {
    parac_host_factor_free(out);
    g_host_error = e.msg;
    return e.code;
  } catch (std::bad_alloc &) {
    parac_host_factor_free(out);
    g_host_error = "host allocation failed";
    return PARAC_ENOMEM;
  }
}

void parac_host_factor_free(parac_host_factor *f) {
  if (!f) return;
  free(f->colptr);
  free(f->rowind);
  free(f->val);
  free(f->D);
  free(f->level);
  f->colptr = nullptr;
  f->rowind = nullptr;
  f->val = nullptr;
  f->D = nullptr;
  f->level = nullptr;
}

const char *parac_host_last_error(void) { return g_host_error.c_str(); }

}  // extern "C"
