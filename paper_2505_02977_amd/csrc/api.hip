// api.hip -- the C ABI: parac_factor, parac_apply, parac_pcg and the factor
// handle's accessors.  Host code only orchestrates: every step of the path
// runs in the library's own kernels.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace parac;

namespace {

thread_local std::string g_last_error;

struct Err {
  int code;
  std::string msg;
};

void chk(hipError_t e, const char *what) {
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Err{e == hipErrorOutOfMemory ? PARAC_ENOMEM : PARAC_EDEVICE,
              std::string(what) + ": " + hipGetErrorString(e)};
  }
}

// device allocations freed at scope exit unless kept
struct Scratch {
  std::vector<void *> ptrs;
  std::vector<size_t> sizes;
  int64_t total = 0;  // bytes currently held
  template <class T>
  T *alloc(int64_t n, const char *what) {
    void *p = nullptr;
    size_t bytes = (size_t)std::max<int64_t>(n, 1) * sizeof(T);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Err{PARAC_ENOMEM, std::string("device allocation of ") + std::to_string(bytes) +
                                  " bytes for " + what + " failed"};
    }
    ptrs.push_back(p);
    sizes.push_back(bytes);
    total += (int64_t)bytes;
    return (T *)p;
  }
  // hand p over to dst (not freed here any more); returns its size
  int64_t keep(void *p, std::vector<void *> &dst) {
    auto it = std::find(ptrs.begin(), ptrs.end(), p);
    if (it == ptrs.end()) return 0;
    const size_t k = (size_t)(it - ptrs.begin());
    const int64_t b = (int64_t)sizes[k];
    ptrs.erase(it);
    sizes.erase(sizes.begin() + (std::ptrdiff_t)k);
    total -= b;
    dst.push_back(p);
    return b;
  }
  void release_all() {
    for (void *p : ptrs) (void)hipFree(p);
    ptrs.clear();
    sizes.clear();
    total = 0;
  }
  ~Scratch() { release_all(); }
};

template <class T>
T read1(const T *dev, hipStream_t s) {
  T v;
  chk(hipMemcpyAsync(&v, dev, sizeof(T), hipMemcpyDeviceToHost, s), "read back");
  chk(hipStreamSynchronize(s), "stream sync");
  return v;
}

struct Events {
  hipEvent_t e[6];
  int n = 0;
  Events() {
    for (auto &x : e) x = nullptr;
  }
  void create() {
    for (auto &x : e) chk(hipEventCreate(&x), "hipEventCreate");
    n = 6;
  }
  ~Events() {
    for (int i = 0; i < n; ++i) (void)hipEventDestroy(e[i]);
  }
  double ms(int a, int b) {
    float v = 0.f;
    chk(hipEventElapsedTime(&v, e[a], e[b]), "hipEventElapsedTime");
    return (double)v;
  }
};

int g_wall_khz = 0;
int wall_khz() {
  if (!g_wall_khz) {
    int dev = 0, v = 0;
    chk(hipGetDevice(&dev), "hipGetDevice");
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, dev) != hipSuccess || v <= 0)
      v = 100000;  // 100 MHz
    g_wall_khz = v;
  }
  return g_wall_khz;
}

int status_from(Err &e) {
  g_last_error = e.msg;
  return e.code;
}

}  // namespace

// first level of the single-workgroup tail for a width threshold: every
// level from it on has at most `rows` rows and at most kTailEntries entries
// in each direction
constexpr double kSweepTimeoutS = 20.0;  // watchdog of one triangular sweep

static int64_t tail_start(parac_factor_t f, int64_t rows) {
  int64_t L0 = f->depth;
  while (L0 > 0) {
    const int64_t L = L0 - 1;
    if (f->hlptr[L + 1] - f->hlptr[L] > rows) break;
    if (f->hlqf[L + 1] - f->hlqf[L] > kTailEntries) break;
    if (f->hlqb[L + 1] - f->hlqb[L] > kTailEntries) break;
    --L0;
  }
  return L0;
}

// ---------------------------------------------------------------------------
// factor
// ---------------------------------------------------------------------------
static void ensure_work(parac_factor_t f, int prec, hipStream_t s);

static parac_factor_t factor_impl(const parac_csr *A, const parac_factor_opts *o, hipStream_t s) {
  if (!A) throw Err{PARAC_EINVAL, "null matrix"};
  const int64_t n = A->n, nnz = A->nnz;
  if (n < 0 || nnz < 0 || n > (int64_t)INT32_MAX - 2 || nnz > (int64_t)INT32_MAX * 4)
    throw Err{PARAC_EINVAL, "matrix sizes out of range"};
  if (n > 0 && (!A->rowptr || !A->col || !A->val)) throw Err{PARAC_EINVAL, "null CSR array"};
  parac_factor_opts opt{};
  opt.pool_factor = 4.0;
  opt.timeout_s = 30.0;
  if (o) {
    opt = *o;
    if (!(opt.pool_factor > 0)) opt.pool_factor = 4.0;
    if (!(opt.timeout_s > 0)) opt.timeout_s = 30.0;
  }
  if (opt.mode < 0 || opt.mode > 2) throw Err{PARAC_EINVAL, "bad mode"};

  Events ev;
  ev.create();
  chk(hipEventRecord(ev.e[0], s), "event");
  Scratch tmp;
  auto *F = new parac_factor_s();
  struct Guard {
    parac_factor_s *f;
    bool ok = false;
    ~Guard() {
      if (!ok && f) {
        for (void *p : f->owned) (void)hipFree(p);
        delete f;
      }
    }
  } guard{F};

  // inputs on the device
  const int64_t *rowptr = A->rowptr;
  const int32_t *col = A->col;
  const double *val = A->val;
  const int32_t *perm_in = opt.perm;
  if (!A->on_device && n > 0) {
    int64_t *r = tmp.alloc<int64_t>(n + 1, "rowptr");
    int32_t *c = tmp.alloc<int32_t>(nnz, "col");
    double *v = tmp.alloc<double>(nnz, "val");
    chk(hipMemcpyAsync(r, A->rowptr, (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s), "copy");
    chk(hipMemcpyAsync(c, A->col, nnz * sizeof(int32_t), hipMemcpyHostToDevice, s), "copy");
    chk(hipMemcpyAsync(v, A->val, nnz * sizeof(double), hipMemcpyHostToDevice, s), "copy");
    rowptr = r;
    col = c;
    val = v;
    if (opt.perm) {
      int32_t *pp = tmp.alloc<int32_t>(n, "perm");
      chk(hipMemcpyAsync(pp, opt.perm, n * sizeof(int32_t), hipMemcpyHostToDevice, s), "copy");
      perm_in = pp;
    }
  }

  // A1: classification; permutation check
  int *flags = tmp.alloc<int>(8, "flags");  // 0 err, 1 any_excess, 2 n_long, 3 changed
  chk(hipMemsetAsync(flags, 0, 8 * sizeof(int), s), "memset");
  unsigned long long *errkey = tmp.alloc<unsigned long long>(1, "error key");
  chk(hipMemsetAsync(errkey, 0xff, sizeof(unsigned long long), s), "memset");
  double *excess = tmp.alloc<double>(n, "excess");
  int32_t *seen = tmp.alloc<int32_t>(n, "seen");
  F->perm = tmp.alloc<int32_t>(n, "perm");
  int32_t *iperm = tmp.alloc<int32_t>(n + 1, "iperm");
  chk(hipMemsetAsync(seen, 0, std::max<int64_t>(n, 1) * sizeof(int32_t), s), "memset");
  if (n > 0) {
    chk(launch_check_csr(n, nnz, rowptr, col, val, excess, errkey, flags + 1, s), "check_csr");
    chk(launch_check_perm(n, perm_in, seen, iperm, errkey, s), "check_perm");
    if (perm_in)
      chk(hipMemcpyAsync(F->perm, perm_in, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s), "copy");
  }
  int hflags[2];
  unsigned long long hkey = ~0ull;
  chk(hipMemcpyAsync(hflags, flags, 2 * sizeof(int), hipMemcpyDeviceToHost, s), "read");
  chk(hipMemcpyAsync(&hkey, errkey, sizeof(hkey), hipMemcpyDeviceToHost, s), "read");
  chk(hipStreamSynchronize(s), "sync");
  hflags[0] = hkey == ~0ull ? 0 : -(int)(hkey & 0xff);
  if (hflags[0]) throw Err{hflags[0], hflags[0] == PARAC_ENOTLAP
                                          ? "matrix is not a Laplacian/SDDM matrix"
                                          : "malformed CSR, asymmetric matrix or bad permutation"};
  int mode = opt.mode;
  if (mode == PARAC_MODE_AUTO) mode = hflags[1] ? PARAC_MODE_SDDM : PARAC_MODE_LAPLACIAN;
  if (mode == PARAC_MODE_LAPLACIAN && hflags[1])
    throw Err{PARAC_ENOTLAP, "row excess present but Laplacian mode requested"};
  const int sddm = mode == PARAC_MODE_SDDM;
  if (!perm_in && n > 0) {
    // identity permutation: iperm holds it already
    chk(hipMemcpyAsync(F->perm, iperm, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s), "copy");
  }
  const int64_t ntot = n + sddm;
  F->n = n;
  F->ntot = ntot;
  F->mode = mode;
  if (sddm) chk(hipMemsetAsync(iperm + n, 0xff, sizeof(int32_t), s), "memset");
  F->iperm = iperm;

  // A2: label-space upper adjacency and counters
  int32_t *ucnt = tmp.alloc<int32_t>(ntot, "ucnt");
  int32_t *dp = tmp.alloc<int32_t>(ntot, "dp");
  int64_t *uptr = tmp.alloc<int64_t>(ntot + 1, "uptr");
  const size_t scan_bytes = scan_tmp_bytes(ntot + 2);
  void *scan_tmp = tmp.alloc<char>((int64_t)scan_bytes, "scan");
  const int64_t emax = nnz + n + 1;
  int32_t *uidx = tmp.alloc<int32_t>(emax, "uidx");
  double *uw = tmp.alloc<double>(emax, "uw");
  chk(hipMemsetAsync(ucnt, 0, std::max<int64_t>(ntot, 1) * sizeof(int32_t), s), "memset");
  chk(launch_upper_count(n, rowptr, col, val, F->perm, excess, sddm, ucnt, dp, s), "upper_count");
  chk(scan_counts(ucnt, uptr, ntot, scan_tmp, scan_bytes, s), "scan");
  chk(launch_upper_fill(n, rowptr, col, val, F->perm, excess, sddm, uptr, uidx, uw, s),
      "upper_fill");
  const int64_t n_edges = read1(uptr + ntot, s);

  // persistent grid
  int maxwg = eliminate_max_workgroups();
  if (maxwg <= 0) throw Err{PARAC_EDEVICE, "occupancy query failed"};
  // one workgroup in kTeamShare is a team for the largest pivots (none when
  // the graph is too small to have any)
  const int nteam = ntot > 4 * kTeamMin ? maxwg / kTeamShare : 0;
  int workers = ((maxwg - nteam) * kElimWaves) / kSubQueues * kSubQueues;
  // no more workers than a quarter of the pivots could keep busy
  workers = std::min<int64_t>(workers, std::max<int64_t>(kSubQueues, (ntot / 4) / kSubQueues * kSubQueues));
  if (opt.workers > 0) workers = std::min(workers, std::max(kSubQueues, opt.workers / kSubQueues * kSubQueues));
  if (workers < kSubQueues) throw Err{PARAC_EDEVICE, "device too small for the persistent grid"};
  const int wgs = workers / kElimWaves;

  // per-attempt state
  const int32_t cap_q = (int32_t)((ntot + kSubQueues - 1) / kSubQueues);
  int32_t *q = tmp.alloc<int32_t>((int64_t)cap_q * kSubQueues, "queue");
  int32_t *qtail = tmp.alloc<int32_t>(3 * kSubQueues * kTailStride + 3 * kTailStride, "qtail");
  int32_t *qhead = qtail + kSubQueues * kTailStride;
  int32_t *qdone = qhead + kSubQueues * kTailStride;
  int32_t *tqc = qdone + kSubQueues * kTailStride;  // tail head, tail, count
  int32_t *tq = tmp.alloc<int32_t>(ntot, "tail queue");
  // team queue: every handed-off pivot takes a fresh slot, and each team
  // holds at most one claimed slot beyond them
  const int32_t bq_cap = (int32_t)(ntot + nteam + 1);
  int32_t *bq = tmp.alloc<int32_t>(bq_cap, "team queue");
  int32_t *bqc = tmp.alloc<int32_t>(2 * kTailStride, "team queue counters");
  int32_t *fill_cnt = tmp.alloc<int32_t>(ntot, "fill_cnt");
  Rec *inl = tmp.alloc<Rec>(ntot * kInline, "inline inbox");
  int32_t *ptab = tmp.alloc<int32_t>(ntot * (kPages - 1), "page table");
  int64_t *colstart = tmp.alloc<int64_t>(ntot, "colstart");
  int32_t *colcnt = tmp.alloc<int32_t>(ntot, "colcnt");
  F->D = tmp.alloc<double>(ntot, "D");
  F->lev = tmp.alloc<int32_t>(ntot, "level");
  unsigned long long *tops = tmp.alloc<unsigned long long>(8, "tops");
  int *err = flags;

  double pf = opt.pool_factor;
  int retries = 0;
  Rec *pool = nullptr;
  int32_t *frow = nullptr;
  double *fval = nullptr;
  char *arena = nullptr;
  int64_t pool_cap = 0, f_cap = 0, arena_cap = 0;
  unsigned long long htops[3] = {0, 0, 0};
  double ms_elim = 0.0;
  for (;;) {
    const int64_t base_entries = std::max<int64_t>(nnz, 64);
    // pages double in size, so up to half of a target's page chain can be
    // unused: twice the expected record count
    const int64_t pool_base = (int64_t)(2.0 * pf * (double)base_entries);
    // factor entries: about 1.6 nnz on grids, about 3 nnz on power-law graphs
    const int64_t f_base = (int64_t)(pf * (double)base_entries) + ntot;
    // per-worker reservations: small enough that their slack stays a fraction
    // of the pools
    const int pg_chunk = (int)std::min<int64_t>(kPageChunk, std::max<int64_t>(64, pool_base / (8 * workers)));
    const int f_chunk = (int)std::min<int64_t>(kFChunk, std::max<int64_t>(64, f_base / (8 * workers)));
    pool_cap = std::min<int64_t>(pool_base + (int64_t)workers * pg_chunk, (int64_t)INT32_MAX - 1);
    f_cap = f_base + (int64_t)workers * f_chunk;
    // scratch of the large-neighbourhood path: every worker keeps its own
    // region (grown geometrically), so besides a share of the fill volume
    // each worker gets room for a few thousand entries (68 bytes each)
    arena_cap = (int64_t)(pf * (double)base_entries) * 16 + (int64_t)workers * 68 * 4096;
    pool = tmp.alloc<Rec>(pool_cap, "fill pool");
    frow = tmp.alloc<int32_t>(f_cap, "factor rows");
    fval = tmp.alloc<double>(f_cap, "factor values");
    arena = tmp.alloc<char>(arena_cap, "scratch arena");
    // reset
    chk(hipMemsetAsync(ucnt, 0, std::max<int64_t>(ntot, 1) * sizeof(int32_t), s), "memset");
    chk(hipMemsetAsync(dp, 0, std::max<int64_t>(ntot, 1) * sizeof(int32_t), s), "memset");
    chk(launch_upper_count(n, rowptr, col, val, F->perm, excess, sddm, ucnt, dp, s), "upper_count");
    chk(hipMemsetAsync(q, 0xff, (size_t)cap_q * kSubQueues * sizeof(int32_t), s), "memset");
    chk(hipMemsetAsync(qtail, 0, (3 * kSubQueues * kTailStride + 3 * kTailStride) * sizeof(int32_t), s),
        "memset");
    chk(hipMemsetAsync(tq, 0xff, std::max<int64_t>(ntot, 1) * sizeof(int32_t), s), "memset");
    chk(hipMemsetAsync(bq, 0xff, (size_t)bq_cap * sizeof(int32_t), s), "memset");
    chk(hipMemsetAsync(bqc, 0, 2 * kTailStride * sizeof(int32_t), s), "memset");
    chk(hipMemsetAsync(fill_cnt, 0, std::max<int64_t>(ntot, 1) * sizeof(int32_t), s), "memset");
    chk(hipMemsetAsync(ptab, 0xff, std::max<int64_t>(ntot * (kPages - 1), 1) * sizeof(int32_t), s),
        "memset");
    chk(hipMemsetAsync(F->lev, 0, std::max<int64_t>(ntot, 1) * sizeof(int32_t), s), "memset");
    chk(hipMemsetAsync(colcnt, 0xff, std::max<int64_t>(ntot, 1) * sizeof(int32_t), s), "memset");
    chk(hipMemsetAsync(tops, 0, 8 * sizeof(unsigned long long), s), "memset");
    chk(hipMemsetAsync(err, 0, sizeof(int), s), "memset");
    chk(launch_queue_init(ntot, dp, q, qtail, cap_q, s), "queue_init");
    chk(hipEventRecord(ev.e[1], s), "event");

    // A4: the persistent elimination
    ElimArgs ea{};
    ea.ntot = (int32_t)ntot;
    ea.uptr = uptr;
    ea.uidx = uidx;
    ea.uw = uw;
    ea.dp = dp;
    ea.q = q;
    ea.qtail = qtail;
    ea.qhead = qhead;
    ea.cap_q = cap_q;
    ea.fill_cnt = fill_cnt;
    ea.inl = inl;
    ea.ptab = ptab;
    ea.pool = pool;
    ea.pool_cap = pool_cap;
    ea.pool_top = tops + 0;
    ea.frow = frow;
    ea.fval = fval;
    ea.f_cap = f_cap;
    ea.f_top = tops + 1;
    ea.colstart = colstart;
    ea.colcnt = colcnt;
    ea.D = F->D;
    ea.lev = F->lev;
    ea.arena = arena;
    ea.arena_cap = arena_cap;
    ea.arena_top = tops + 2;
    ea.seed = opt.seed;
    ea.err = err;
    ea.timeout_ticks = (uint64_t)(opt.timeout_s * 1000.0 * (double)wall_khz());
    ea.nworkers = workers;
    ea.pg_chunk = pg_chunk;
    ea.f_chunk = f_chunk;
    ea.done = qdone;
    {
      // the wide kernel leaves the last `tail_fraction` of the pivots (the
      // thin end of the dependency DAG) to the single-workgroup kernel
      const double tf = opt.tail_fraction == 0.0 ? -1.0 : opt.tail_fraction;
      if (tf >= 1.0) {
        ea.stop_at = 0;
      } else if (tf < 0.0) {
        ea.stop_at = ntot + 1;
      } else {
        const int64_t left = (int64_t)(tf * (double)ntot);
        ea.stop_at = left < 256 ? ntot + 1 : ntot - left;
      }
    }
    ea.tq = tq;
    ea.tq_head = tqc;
    ea.tq_tail = tqc + kTailStride;
    ea.tq_count = tqc + 2 * kTailStride;
    ea.bq = bq;
    ea.bq_head = bqc;
    ea.bq_tail = bqc + kTailStride;
    ea.bq_cap = bq_cap;
    ea.team_min = nteam > 0 ? kTeamMin : 0;
    ea.team_wg0 = wgs;
    if (ntot > 0) chk(launch_eliminate(ea, wgs + nteam, s), "eliminate");
    chk(hipEventRecord(ev.e[2], s), "event");
    int herr = 0;
    chk(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s), "read");
    chk(hipMemcpyAsync(htops, tops, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s),
        "read");
    chk(hipStreamSynchronize(s), "sync");
    ms_elim += ev.ms(1, 2);
    if (herr == PARAC_EPOOL && retries < 12) {
      // fill capacity exhausted: the factor does not depend on storage, so a
      // larger pool reproduces it exactly
      ++retries;
      pf *= 2.5;
      for (void *p : {(void *)pool, (void *)frow, (void *)fval, (void *)arena}) {
        auto it = std::find(tmp.ptrs.begin(), tmp.ptrs.end(), p);
        if (it != tmp.ptrs.end()) {
          (void)hipFree(p);
          tmp.ptrs.erase(it);
        }
      }
      continue;
    }
    if (herr) {
      throw Err{herr, herr == PARAC_ETIMEOUT ? "elimination watchdog expired"
                      : herr == PARAC_EPOOL  ? "fill pool exhausted after retries"
                                             : "elimination invariant failed"};
    }
    break;
  }

  // A5: finalize
  chk(hipEventRecord(ev.e[3], s), "event");
  F->colptr = tmp.alloc<int64_t>(ntot + 1, "colptr");
  chk(scan_counts(colcnt, F->colptr, ntot, scan_tmp, scan_bytes, s), "scan");
  const int64_t nnz_off = read1(F->colptr + ntot, s);
  F->nnz_off = nnz_off;
  F->rowind = tmp.alloc<int32_t>(nnz_off, "rowind");
  F->val = tmp.alloc<double>(nnz_off, "val");
  if (ntot > 0)
    chk(launch_compact_csc(ntot, colstart, colcnt, frow, fval, F->colptr, F->rowind, F->val, s),
        "compact");
  int32_t *rowcnt = tmp.alloc<int32_t>(ntot, "rowcnt");
  chk(hipMemsetAsync(rowcnt, 0, std::max<int64_t>(ntot, 1) * sizeof(int32_t), s), "memset");
  chk(launch_row_count(nnz_off, F->rowind, rowcnt, s), "row_count");
  int64_t *rowptr_f = tmp.alloc<int64_t>(ntot + 1, "rowptr_f");
  chk(scan_counts(rowcnt, rowptr_f, ntot, scan_tmp, scan_bytes, s), "scan");
  chk(hipMemsetAsync(rowcnt, 0, std::max<int64_t>(ntot, 1) * sizeof(int32_t), s), "memset");
  int32_t *colind_f = tmp.alloc<int32_t>(nnz_off, "colind_f");
  double *val_f = tmp.alloc<double>(nnz_off, "val_f");
  int32_t *long_rows = tmp.alloc<int32_t>(ntot, "long rows");
  if (ntot > 0) {
    chk(launch_transpose(ntot, F->colptr, F->rowind, F->val, rowptr_f, rowcnt, colind_f,
                         val_f, s),
        "transpose");
    chk(launch_sort_rows(ntot, rowptr_f, colind_f, val_f, long_rows, flags + 2, s),
        "sort_rows");
    chk(launch_sort_long_rows(rowptr_f, colind_f, val_f, long_rows, flags + 2, frow, fval, ntot,
                              s),
        "sort_long_rows");
  }
  // statistics (and the depth needed for the level grouping)
  unsigned long long *st = tops + 3;
  chk(hipMemsetAsync(st, 0, 5 * sizeof(unsigned long long), s), "memset");
  if (ntot > 0) chk(launch_max_stats(ntot, uptr, fill_cnt, colcnt, F->lev, st, s), "stats");
  unsigned long long hst[5];
  chk(hipMemcpyAsync(hst, st, sizeof(hst), hipMemcpyDeviceToHost, s), "read");
  chk(hipStreamSynchronize(s), "sync");
  const int64_t depth = ntot > 0 ? (int64_t)hst[3] + 1 : 0;
  F->depth = depth;
  // rows (labels < n) grouped by level
  int32_t *lcount = tmp.alloc<int32_t>(depth + 1, "lcount");
  F->lptr = tmp.alloc<int64_t>(depth + 2, "lptr");
  F->order = tmp.alloc<int32_t>(n, "order");
  chk(hipMemsetAsync(lcount, 0, (depth + 1) * sizeof(int32_t), s), "memset");
  if (n > 0) {
    chk(launch_level_count(n, F->lev, lcount, s), "level_count");
    chk(scan_counts(lcount, F->lptr, depth, scan_tmp, scan_bytes, s), "scan");
    chk(hipMemsetAsync(lcount, 0, (depth + 1) * sizeof(int32_t), s), "memset");
    chk(launch_level_place(n, F->lev, F->lptr, lcount, F->order, s), "level_place");
    F->hlptr.resize(depth + 1);
    chk(hipMemcpyAsync(F->hlptr.data(), F->lptr, (depth + 1) * sizeof(int64_t),
                       hipMemcpyDeviceToHost, s),
        "read");
    chk(hipStreamSynchronize(s), "sync");
    // level-ordered copies of the rows (forward) and columns (backward) of F
    int32_t *flen = tmp.alloc<int32_t>(n, "flen");
    int32_t *blen = tmp.alloc<int32_t>(n, "blen");
    chk(launch_level_layout(n, F->order, rowptr_f, F->colptr, F->rowind, flen, blen, s),
        "level_layout");
    F->lf_ptr = tmp.alloc<int64_t>(n + 1, "lf_ptr");
    F->lb_ptr = tmp.alloc<int64_t>(n + 1, "lb_ptr");
    chk(scan_counts(flen, F->lf_ptr, n, scan_tmp, scan_bytes, s), "scan");
    chk(scan_counts(blen, F->lb_ptr, n, scan_tmp, scan_bytes, s), "scan");
    const int64_t nf = read1(F->lf_ptr + n, s), nbk = read1(F->lb_ptr + n, s);
    F->lf_idx = tmp.alloc<int32_t>(nf, "lf_idx");
    F->lf_val = tmp.alloc<double>(nf, "lf_val");
    F->lb_idx = tmp.alloc<int32_t>(nbk, "lb_idx");
    F->lb_val = tmp.alloc<double>(nbk, "lb_val");
    // position space of the solves: posof / src maps and D^+ by position
    int32_t *posof = tmp.alloc<int32_t>(n, "posof");
    F->src = tmp.alloc<int32_t>(n, "src");
    F->Dinv = tmp.alloc<double>(n, "Dinv");
    if (opt.keep_fp32) F->Dinv32 = tmp.alloc<float>(n, "Dinv32");
    chk(launch_position_maps(n, F->order, F->iperm, F->D, posof, F->src, F->Dinv, F->Dinv32, s),
        "position maps");
    chk(launch_level_copy(n, F->order, posof, rowptr_f, colind_f, val_f, F->colptr, F->rowind,
                          F->val, F->lf_ptr, F->lb_ptr, F->lf_idx, F->lf_val, F->lb_idx,
                          F->lb_val, s),
        "level_copy");
    int64_t *lqf = tmp.alloc<int64_t>(depth + 1, "lqf");
    int64_t *lqb = tmp.alloc<int64_t>(depth + 1, "lqb");
    chk(launch_level_offsets(depth, F->lptr, F->lf_ptr, F->lb_ptr, lqf, lqb, s),
        "level offsets");
    F->hlqf.resize(depth + 1);
    F->hlqb.resize(depth + 1);
    chk(hipMemcpyAsync(F->hlqf.data(), lqf, (depth + 1) * sizeof(int64_t),
                       hipMemcpyDeviceToHost, s),
        "read");
    chk(hipMemcpyAsync(F->hlqb.data(), lqb, (depth + 1) * sizeof(int64_t),
                       hipMemcpyDeviceToHost, s),
        "read");
    // per direction: the positions of each level listed by row class, then
    // the units of the dependency-driven sweep cut from these lists
    const int64_t ncl = (int64_t)kRowClasses * depth;
    int32_t *ccount = tmp.alloc<int32_t>(ncl, "class counts");
    int64_t *cbase = tmp.alloc<int64_t>(ncl, "class bases");
    int32_t *ucount = tmp.alloc<int32_t>(n, "unit counts");
    int32_t *ccnt = tmp.alloc<int32_t>(n, "chunk counts");
    int64_t *uoff = tmp.alloc<int64_t>(n + 1, "unit offsets");
    int64_t *coff = tmp.alloc<int64_t>(n + 1, "chunk offsets");
    std::vector<int32_t> hcc(ncl);
    std::vector<int64_t> hcb(ncl);
    for (int dir = 0; dir < 2; ++dir) {
      const int64_t *ptr = dir == 0 ? F->lf_ptr : F->lb_ptr;
      int32_t *&list = dir == 0 ? F->flist : F->blist;
      chk(hipMemsetAsync(ccount, 0, ncl * sizeof(int32_t), s), "memset");
      chk(launch_class_count(n, F->order, F->lev, ptr, ccount, s), "class count");
      chk(hipMemcpyAsync(hcc.data(), ccount, ncl * sizeof(int32_t), hipMemcpyDeviceToHost, s),
          "read");
      chk(hipStreamSynchronize(s), "sync");
      for (int64_t L = 0; L < depth; ++L) {
        int64_t b = F->hlptr[L];
        for (int c = 0; c < kRowClasses; ++c) {
          hcb[kRowClasses * L + c] = b;
          b += hcc[kRowClasses * L + c];
        }
      }
      list = tmp.alloc<int32_t>(n, "class list");
      chk(hipMemcpyAsync(cbase, hcb.data(), ncl * sizeof(int64_t), hipMemcpyHostToDevice, s),
          "upload");
      chk(hipMemsetAsync(ccount, 0, ncl * sizeof(int32_t), s), "memset");
      chk(launch_class_place(n, F->order, F->lev, ptr, cbase, ccount, list, s), "class place");
      // units of the dependency-driven sweep of this direction
      chk(launch_unit_count(n, depth, F->lptr, cbase, list, ptr, ucount, ccnt, dir == 1, s),
          "unit count");
      chk(scan_counts(ucount, uoff, n, scan_tmp, scan_bytes, s), "scan");
      chk(scan_counts(ccnt, coff, n, scan_tmp, scan_bytes, s), "scan");
      const int64_t nu = read1(uoff + n, s), nch = read1(coff + n, s);
      if (nu > INT32_MAX || nch > INT32_MAX)
        throw Err{PARAC_EINVAL, "factor too large for the sweep's 32-bit unit tables"};
      int4 *units = tmp.alloc<int4>(nu, "sweep units");
      chk(launch_unit_write(n, depth, F->lptr, cbase, list, ptr, uoff, coff, units, dir == 1,
                            s),
          "unit write");
      (dir == 0 ? F->task_f : F->task_b) = units;
      (dir == 0 ? F->ntask_f : F->ntask_b) = (int32_t)nu;
      F->ncs = std::max(F->ncs, nch);
      chk(hipStreamSynchronize(s), "sync");  // host tables reused by the next direction
    }
    if (opt.keep_fp32) {
      F->lf_val32 = tmp.alloc<float>(nf, "lf_val32");
      F->lb_val32 = tmp.alloc<float>(nbk, "lb_val32");
      chk(launch_cast32(nf, F->lf_val, F->lf_val32, s), "cast");
      chk(launch_cast32(nbk, F->lb_val, F->lb_val32, s), "cast");
    }
  }
  if (!F->Dinv) F->Dinv = tmp.alloc<double>(1, "Dinv");  // n = 0
  F->zero = tmp.alloc<int>(1, "zero flag");
  chk(hipMemsetAsync(F->zero, 0, sizeof(int), s), "memset");
  F->ctr = tmp.alloc<int32_t>(2, "sweep counters");
  F->serr = tmp.alloc<int>(1, "sweep error");
  chk(hipMemsetAsync(F->ctr, 0, 2 * sizeof(int32_t), s), "memset");
  chk(hipMemsetAsync(F->serr, 0, sizeof(int), s), "memset");
  if (opt.keep_fp32 && !F->Dinv32) F->Dinv32 = tmp.alloc<float>(1, "Dinv32");
  // component roots (last label of each component) by pointer jumping
  F->root = tmp.alloc<int32_t>(ntot, "root");
  if (ntot > 0) {
    int32_t *alt = tmp.alloc<int32_t>(ntot, "root tmp");
    chk(launch_comp_init(ntot, F->colptr, F->rowind, F->root, s), "comp_init");
    int32_t *src = F->root, *dst = alt;
    for (int it = 0; it < 64; ++it) {
      chk(hipMemsetAsync(flags + 3, 0, sizeof(int), s), "memset");
      for (int k2 = 0; k2 < 4; ++k2) {
        chk(launch_comp_jump(ntot, src, dst, flags + 3, s), "comp_jump");
        std::swap(src, dst);
      }
      if (!read1(flags + 3, s)) break;
    }
    if (src != F->root)
      chk(hipMemcpyAsync(F->root, src, ntot * sizeof(int32_t), hipMemcpyDeviceToDevice, s), "copy");
  }
  chk(hipEventRecord(ev.e[4], s), "event");
  chk(hipStreamSynchronize(s), "sync");

  parac_factor_stats &S = F->stats;
  S.n = n;
  S.ntot = ntot;
  S.mode = mode;
  S.nnz_off = nnz_off;
  S.n_input_edges = n_edges;
  S.max_gather = (int64_t)hst[0];
  S.max_deg = (int64_t)hst[1];
  S.n_fill = (int64_t)hst[2];
  S.depth = depth;
  S.n_zero_pivots = (int64_t)hst[4];
  S.workers = workers;
  S.retries = retries;
  S.pool_factor = pf;
  S.ms_setup = ev.ms(0, 1);
  S.ms_eliminate = ms_elim;
  S.ms_finalize = ev.ms(3, 4);
  S.ms_total = ev.ms(0, 4);

  // keep the handle's arrays; everything else is freed with `tmp`
  for (void *p : {(void *)F->perm, (void *)F->iperm, (void *)F->colptr, (void *)F->rowind,
                  (void *)F->val, (void *)F->D, (void *)F->Dinv, (void *)F->Dinv32,
                  (void *)F->lev, (void *)F->order, (void *)F->root, (void *)F->lptr,
                  (void *)F->src, (void *)F->flist, (void *)F->blist, (void *)F->zero,
                  (void *)F->task_f, (void *)F->task_b, (void *)F->ctr, (void *)F->serr,
                  (void *)F->lf_ptr, (void *)F->lf_idx, (void *)F->lf_val, (void *)F->lf_val32,
                  (void *)F->lb_ptr, (void *)F->lb_idx, (void *)F->lb_val, (void *)F->lb_val32})
    if (p) F->bytes += tmp.keep(p, F->owned);
  // the sweeps' work vectors, so that solving with the factor needs no
  // further device allocation
  ensure_work(F, PARAC_PREC_FP64, s);
  if (opt.keep_fp32) ensure_work(F, PARAC_PREC_MIXED, s);
  chk(hipStreamSynchronize(s), "sync");
  guard.ok = true;
  return F;
}

// ---------------------------------------------------------------------------
// apply
// ---------------------------------------------------------------------------
static int prec_slot(int prec) { return prec == PARAC_PREC_MIXED ? 1 : 0; }


static SolveArgs solve_args(parac_factor_t f, const int *skip) {
  SolveArgs a{};
  a.n = f->n;
  a.lptr = f->lptr;
  a.depth = f->depth;
  a.lf_ptr = f->lf_ptr;
  a.lf_idx = f->lf_idx;
  a.lf_val = f->lf_val;
  a.lf_val32 = f->lf_val32;
  a.lb_ptr = f->lb_ptr;
  a.lb_idx = f->lb_idx;
  a.lb_val = f->lb_val;
  a.lb_val32 = f->lb_val32;
  a.Dinv = f->Dinv;
  a.Dinv32 = f->Dinv32;
  a.src = f->src;
  a.flist = f->flist;
  a.blist = f->blist;
  a.skip = skip;
  a.task_f = f->task_f;
  a.task_b = f->task_b;
  a.ntask_f = f->ntask_f;
  a.ntask_b = f->ntask_b;
  a.err = f->serr;
  a.timeout_ticks = (uint64_t)(kSweepTimeoutS * 1000.0 * (double)wall_khz());
  return a;
}

// label-space work vectors of the two triangular solves
// every entry of the sweep vectors and chunk sums pending, counters and
// error word cleared: the state each sweep pair starts from and leaves
static void reset_work(parac_factor_t f, int prec, hipStream_t s) {
  const int64_t m = std::max<int64_t>(f->ntot, 1), c = std::max<int64_t>(f->ncs, 1);
  if (prec == PARAC_PREC_MIXED) {
    for (void *p : {f->wy32, f->wx32})
      chk(launch_fill_u32((uint32_t *)p, kPending32, m, s), "fill");
    chk(launch_fill_u32((uint32_t *)f->cs32, kPending32, c, s), "fill");
  } else {
    for (void *p : {f->wy64, f->wx64})
      chk(launch_fill_u64((uint64_t *)p, kPending64, m, s), "fill");
    chk(launch_fill_u64((uint64_t *)f->cs64, kPending64, c, s), "fill");
  }
  chk(hipMemsetAsync(f->ctr, 0, 2 * sizeof(int32_t), s), "memset");
  chk(hipMemsetAsync(f->serr, 0, sizeof(int), s), "memset");
}

static void ensure_work(parac_factor_t f, int prec, hipStream_t s) {
  const bool mixed = prec == PARAC_PREC_MIXED;
  void **py = mixed ? &f->wy32 : &f->wy64;
  void **px = mixed ? &f->wx32 : &f->wx64;
  void **pc = mixed ? &f->cs32 : &f->cs64;
  if (*py) return;
  const size_t el = mixed ? 4 : 8;
  const int64_t m = std::max<int64_t>(f->ntot, 1), c = std::max<int64_t>(f->ncs, 1);
  chk(hipMalloc(py, m * el), "work vector");
  f->owned.push_back(*py);
  chk(hipMalloc(px, m * el), "work vector");
  f->owned.push_back(*px);
  chk(hipMalloc(pc, c * el), "chunk sums");
  f->owned.push_back(*pc);
  f->bytes += (int64_t)((2 * m + c) * el);
  reset_work(f, prec, s);
}

// after sweeps have run: a watchdog error leaves the sweep state
// inconsistent, so it is reset before the error is reported
static void check_sweeps(parac_factor_t f, int prec, hipStream_t s) {
  if (read1(f->serr, s) == 0) return;
  reset_work(f, prec, s);
  chk(hipStreamSynchronize(s), "sync");
  throw Err{PARAC_ETIMEOUT, "triangular sweep watchdog expired"};
}

// ---------------------------------------------------------------------------
// block apply (several right-hand sides, chunks of at most kBlockCols)
// ---------------------------------------------------------------------------
static void ensure_bwork(parac_factor_t f, int prec, int nc) {
  const int k = prec_slot(prec);
  if (f->bcols[k] >= nc) return;
  const size_t el = k ? 4 : 8;
  for (void **pp : {&f->bwy[k], &f->bwx[k]}) {
    if (!*pp) continue;
    f->owned.erase(std::remove(f->owned.begin(), f->owned.end(), *pp), f->owned.end());
    (void)hipFree(*pp);
    *pp = nullptr;
    f->bytes -= (int64_t)((size_t)std::max<int64_t>(f->ntot, 1) * (size_t)f->bcols[k] * el);
  }
  f->bcols[k] = 0;
  const size_t m = (size_t)std::max<int64_t>(f->ntot, 1) * (size_t)nc;
  chk(hipMalloc(&f->bwy[k], m * el), "block work vector");
  f->owned.push_back(f->bwy[k]);
  chk(hipMalloc(&f->bwx[k], m * el), "block work vector");
  f->owned.push_back(f->bwx[k]);
  f->bcols[k] = nc;
  f->bytes += 2 * (int64_t)(m * el);
}

// column sweeps: every column's work vectors and chunk sums pending, its
// counters clear (the state each sweep pair starts from and leaves)
static void reset_cwork(parac_factor_t f, int prec, hipStream_t s) {
  const int k = prec_slot(prec);
  const int64_t nc = f->ccols[k];
  if (nc == 0) return;
  const int64_t m = std::max<int64_t>(f->ntot, 1) * nc, c = std::max<int64_t>(f->ncs, 1) * nc;
  if (k) {
    for (void *p : {f->cy[k], f->cx[k]}) chk(launch_fill_u32((uint32_t *)p, kPending32, m, s), "fill");
    chk(launch_fill_u32((uint32_t *)f->ccs[k], kPending32, c, s), "fill");
  } else {
    for (void *p : {f->cy[k], f->cx[k]}) chk(launch_fill_u64((uint64_t *)p, kPending64, m, s), "fill");
    chk(launch_fill_u64((uint64_t *)f->ccs[k], kPending64, c, s), "fill");
  }
  chk(hipMemsetAsync(f->cctr[k], 0, 2 * nc * sizeof(int32_t), s), "memset");
}

static void ensure_cwork(parac_factor_t f, int prec, int nc, hipStream_t s) {
  const int k = prec_slot(prec);
  if (f->ccols[k] >= nc) return;
  const size_t el = k ? 4 : 8;
  const int64_t m0 = std::max<int64_t>(f->ntot, 1), c0 = std::max<int64_t>(f->ncs, 1);
  for (void **pp : {&f->cy[k], &f->cx[k], &f->ccs[k], (void **)&f->cctr[k]}) {
    if (!*pp) continue;
    f->owned.erase(std::remove(f->owned.begin(), f->owned.end(), *pp), f->owned.end());
    (void)hipFree(*pp);
    *pp = nullptr;
  }
  f->bytes -= f->ccols[k] * (int64_t)((2 * m0 + c0) * el + 2 * sizeof(int32_t));
  f->ccols[k] = 0;
  chk(hipMalloc(&f->cy[k], (size_t)(m0 * nc) * el), "column work vector");
  f->owned.push_back(f->cy[k]);
  chk(hipMalloc(&f->cx[k], (size_t)(m0 * nc) * el), "column work vector");
  f->owned.push_back(f->cx[k]);
  chk(hipMalloc(&f->ccs[k], (size_t)(c0 * nc) * el), "column chunk sums");
  f->owned.push_back(f->ccs[k]);
  chk(hipMalloc((void **)&f->cctr[k], (size_t)(2 * nc) * sizeof(int32_t)), "column counters");
  f->owned.push_back(f->cctr[k]);
  f->ccols[k] = nc;
  f->bytes += nc * (int64_t)((2 * m0 + c0) * el + 2 * sizeof(int32_t));
  reset_cwork(f, prec, s);
}

struct Batch;
static void build_cols(Batch &bt, parac_factor_t f, int nc, const double *r, int64_t ldr,
                       double *z, int64_t ldz, int prec, const int *skip, int skip_stride,
                       hipStream_t s);
static void apply_cols(parac_factor_t f, int nc, const double *r, int64_t ldr, double *z,
                       int64_t ldz, int prec, hipStream_t s);

// a block of nc columns: with cpl = 0 one dependency-driven sweep pair per
// column, all columns in the same two launches; else level-synchronous block
// launches of that shape (the factor read once for all columns)
static void apply_block(parac_factor_t f, const parac_block_shape &shp, int nc, const double *r,
                        int64_t ldr, double *z, int64_t ldz, int prec, const int *skip,
                        hipStream_t s) {
  if (f->n == 0) return;
  if (shp.cpl == 0) {
    apply_cols(f, nc, r, ldr, z, ldz, prec, s);
    return;
  }
  ensure_bwork(f, prec, nc);
  SolveArgs a = solve_args(f, skip);
  BlockShape sh{shp.cpl, tail_start(f, shp.tail_rows)};
  const int k = prec_slot(prec);
  chk(launch_block_apply(a, f->hlptr.data(), sh, nc, r, ldr, f->bwy[k], f->bwx[k], z, ldz, prec,
                         s),
      "block apply");
}

// the shape for (nc, prec): fixed by the caller, else column sweeps
static parac_block_shape block_shape(parac_factor_t f, int nc, int prec) {
  const auto key = std::make_pair(nc, prec_slot(prec));
  auto it = f->shapes.find(key);
  if (it != f->shapes.end()) return it->second;
  // column sweeps unless the caller fixed a level-synchronous shape
  const parac_block_shape sweeps{0, kTailDefault};
  f->shapes[key] = sweeps;
  return sweeps;
}

static bool shape_ok(const parac_block_shape &c) {
  return (c.cpl == 0 || c.cpl == 1 || c.cpl == 2 || c.cpl == 4) && c.tail_rows >= 0;
}

// ---------------------------------------------------------------------------
// PCG (one right-hand side; several columns run as independent recurrences)
// ---------------------------------------------------------------------------
// sum, sabs (ntot entries each) and bad may come from the caller; else they
// are allocated here
static void check_consistent(parac_factor_t f, const double *b, hipStream_t s,
                             double *sum = nullptr, double *sabs = nullptr, int *bad = nullptr) {
  const int64_t n = f->n;
  if (n == 0) return;
  Scratch tmp;
  if (!sum) sum = tmp.alloc<double>(f->ntot, "sums");
  if (!sabs) sabs = tmp.alloc<double>(f->ntot, "sums");
  if (!bad) bad = tmp.alloc<int>(1, "flag");
  chk(launch_fill_u64((uint64_t *)sum, 0, f->ntot, s), "fill");
  chk(launch_fill_u64((uint64_t *)sabs, 0, f->ntot, s), "fill");
  chk(launch_fill_u32((uint32_t *)bad, 0, 1, s), "fill");
  chk(launch_comp_check(n, f->ntot > n ? n : -1, f->perm, f->root, b, sum, sabs, bad, s),
      "comp_check");
  if (read1(bad, s))
    throw Err{PARAC_EINCONSISTENT, "b has a nonzero sum on a component without excess"};
}

// device memory for the tables of a batch of one system, when the caller
// provides it (else the tables are allocated in Batch::mem)
struct TableMem {
  PcgSlot *slots = nullptr;
  int32_t *bslot = nullptr;
  int64_t bslot_cap = 0;
  ApplySlot *aslots = nullptr;
  int32_t *wgmap = nullptr;
  int64_t wgmap_cap = 0;
};

// device tables of one batch of systems (see serve.hip)
struct Batch {
  Scratch mem;
  SlotBatch B;
  const TableMem *pre = nullptr;
};

struct SlotView {
  PcgSlot ps;  // blk0 / nblk are filled in by build_batch
  parac_factor_t f;
};

// the apply tables of a batch: its apply slots and the workgroups of the
// sweeps, each system's dealt out round-robin so that every system starts
// at once.  Uploads into bt.mem.
static void build_apply_tables(Batch &bt, const std::vector<ApplySlot> &as,
                               const std::vector<parac_factor_t> &fs, hipStream_t s) {
  const int ns = (int)as.size();
  std::vector<int32_t> g(ns);
  int32_t gmax = 0;
  for (int k = 0; k < ns; ++k) {
    const int64_t nt = std::max(fs[k]->ntask_f, fs[k]->ntask_b);
    const int64_t waves = kReadyThreads / 64;
    g[k] = (int32_t)std::min<int64_t>((nt + waves - 1) / waves, kReadyGroupsMax);
    gmax = std::max(gmax, g[k]);
  }
  std::vector<int32_t> map;
  for (int32_t r = 0; r < gmax; ++r)
    for (int k = 0; k < ns; ++k)
      if (r < g[k]) map.push_back(k);
  ApplySlot *das;
  int32_t *dmap;
  if (bt.pre) {
    if (ns != 1 || (int64_t)map.size() > bt.pre->wgmap_cap)
      throw Err{PARAC_EINTERNAL, "caller-provided batch tables too small"};
    das = bt.pre->aslots;
    dmap = bt.pre->wgmap;
  } else {
    das = bt.mem.alloc<ApplySlot>(ns, "batch apply slots");
    dmap = bt.mem.alloc<int32_t>(std::max<int64_t>((int64_t)map.size(), 1), "sweep map");
  }
  chk(hipMemcpyAsync(das, as.data(), ns * sizeof(ApplySlot), hipMemcpyHostToDevice, s), "upload");
  if (!map.empty())
    chk(hipMemcpyAsync(dmap, map.data(), map.size() * sizeof(int32_t), hipMemcpyHostToDevice, s),
        "upload");
  chk(hipStreamSynchronize(s), "sync");  // the host tables above go out of scope
  SlotBatch &B = bt.B;
  B.aslots = das;
  B.wgmap = dmap;
  B.nwg = (int)map.size();
}

// lay out the workgroups of a batch and upload its tables; partial must
// hold the sum of slot_blocks(n) over the batch
static void build_batch(Batch &bt, const std::vector<SlotView> &v, int prec, double *partial,
                        hipStream_t s) {
  bt.mem.release_all();
  const int ns = (int)v.size();
  std::vector<PcgSlot> ps(ns);
  std::vector<ApplySlot> as(ns);
  std::vector<parac_factor_t> fs(ns);
  std::vector<int32_t> bslot;
  int blk = 0;
  for (int k = 0; k < ns; ++k) {
    ps[k] = v[k].ps;
    ps[k].nblk = slot_blocks(ps[k].n);
    ps[k].blk0 = blk;
    bslot.insert(bslot.end(), (size_t)ps[k].nblk, k);
    blk += ps[k].nblk;
    parac_factor_t f = v[k].f;
    fs[k] = f;
    ensure_work(f, prec, s);
    as[k].a = solve_args(f, ps[k].ist + 1);
    as[k].ldr = as[k].ldz = 1;
    as[k].r = ps[k].r;
    as[k].y = prec == PARAC_PREC_MIXED ? f->wy32 : f->wy64;
    as[k].x = prec == PARAC_PREC_MIXED ? f->wx32 : f->wx64;
    as[k].cs = prec == PARAC_PREC_MIXED ? f->cs32 : f->cs64;
    as[k].ctr = f->ctr;
    as[k].z = ps[k].z;
  }
  PcgSlot *dps;
  int32_t *dbs;
  if (bt.pre) {
    if (ns != 1 || blk > bt.pre->bslot_cap)
      throw Err{PARAC_EINTERNAL, "caller-provided batch tables too small"};
    dps = bt.pre->slots;
    dbs = bt.pre->bslot;
  } else {
    dps = bt.mem.alloc<PcgSlot>(ns, "batch slots");
    dbs = bt.mem.alloc<int32_t>(blk, "batch block map");
  }
  chk(hipMemcpyAsync(dps, ps.data(), ns * sizeof(PcgSlot), hipMemcpyHostToDevice, s), "upload");
  chk(hipMemcpyAsync(dbs, bslot.data(), bslot.size() * sizeof(int32_t), hipMemcpyHostToDevice, s),
      "upload");
  build_apply_tables(bt, as, fs, s);  // synchronises the stream
  SlotBatch &B = bt.B;
  B.nslots = ns;
  B.nblocks = blk;
  B.slots = dps;
  B.bslot = dbs;
  B.partial = partial;
}

// z = M^+ r for one vector: the batched apply with a batch of one
static void apply_one(parac_factor_t f, const double *r, double *z, int prec, hipStream_t s) {
  if (f->n == 0) return;
  ensure_work(f, prec, s);
  std::vector<ApplySlot> as(1);
  as[0].a = solve_args(f, f->zero);
  as[0].ldr = as[0].ldz = 1;
  as[0].r = r;
  as[0].y = prec == PARAC_PREC_MIXED ? f->wy32 : f->wy64;
  as[0].x = prec == PARAC_PREC_MIXED ? f->wx32 : f->wx64;
  as[0].cs = prec == PARAC_PREC_MIXED ? f->cs32 : f->cs64;
  as[0].ctr = f->ctr;
  as[0].z = z;
  Batch bt;
  build_apply_tables(bt, as, {f}, s);
  bt.B.nslots = 1;
  chk(slots_apply(bt.B, prec, s), "apply");
  chk(hipStreamSynchronize(s), "sync");
  check_sweeps(f, prec, s);
}

// the column sweeps of a block: column j of r (stride ldr) into column j of
// z, each a slot of its own over the same factor; skip (optional) gives
// column j's done flag at skip + j * skip_stride
static void build_cols(Batch &bt, parac_factor_t f, int nc, const double *r, int64_t ldr,
                       double *z, int64_t ldz, int prec, const int *skip, int skip_stride,
                       hipStream_t s) {
  ensure_cwork(f, prec, nc, s);
  const int k = prec_slot(prec);
  const size_t el = k ? 4 : 8;
  const int64_t m = std::max<int64_t>(f->ntot, 1), c = std::max<int64_t>(f->ncs, 1);
  std::vector<ApplySlot> as(nc);
  for (int j = 0; j < nc; ++j) {
    as[j].a = solve_args(f, skip ? skip + (int64_t)j * skip_stride : f->zero);
    as[j].ldr = ldr;
    as[j].ldz = ldz;
    as[j].r = r + j;
    as[j].y = (char *)f->cy[k] + (size_t)(j * m) * el;
    as[j].x = (char *)f->cx[k] + (size_t)(j * m) * el;
    as[j].cs = (char *)f->ccs[k] + (size_t)(j * c) * el;
    as[j].ctr = f->cctr[k] + 2 * j;
    as[j].z = z + j;
  }
  build_apply_tables(bt, as, std::vector<parac_factor_t>(nc, f), s);
  bt.B.nslots = nc;
}

static void check_col_sweeps(parac_factor_t f, int prec, hipStream_t s) {
  if (read1(f->serr, s) == 0) return;
  reset_cwork(f, prec, s);
  chk(hipMemsetAsync(f->serr, 0, sizeof(int), s), "memset");
  chk(hipStreamSynchronize(s), "sync");
  throw Err{PARAC_ETIMEOUT, "triangular sweep watchdog expired"};
}

static void apply_cols(parac_factor_t f, int nc, const double *r, int64_t ldr, double *z,
                       int64_t ldz, int prec, hipStream_t s) {
  Batch bt;
  build_cols(bt, f, nc, r, ldr, z, ldz, prec, nullptr, 0, s);
  chk(slots_apply(bt.B, prec, s), "column sweeps");
  chk(hipStreamSynchronize(s), "sync");
  check_col_sweeps(f, prec, s);
}

// device memory of one single-vector PCG: vectors r, z, p, q (n each),
// block partial sums (slot_blocks(n)), 8 scalars, 4 flags, and optionally
// the batch tables
struct PcgWork {
  double *r, *z, *p, *q, *partial, *dst;
  int *ist;
  const TableMem *tables;
  bool events;  // time the call with HIP events (false: no event is created)
};

// one system as a batch of one: the same launches, hence the same bits, as
// when the system is served together with others
static int pcg_run(const parac_csr *A, parac_factor_t f, const double *b, double *x,
                   const parac_pcg_opts &o, parac_pcg_stats *st, hipStream_t s, const PcgWork &w) {
  const int64_t n = f->n;
  double *r = w.r, *z = w.z, *p = w.p, *q = w.q, *partial = w.partial, *dst = w.dst;
  int *ist = w.ist;
  const double hst0[8] = {0, 0, 0, 0, 0, 0, o.rtol, 0};
  const int hist0[4] = {0, 0, o.maxit, 0};
  chk(hipMemcpyAsync(dst, hst0, sizeof(hst0), hipMemcpyHostToDevice, s), "upload");
  chk(hipMemcpyAsync(ist, hist0, sizeof(hist0), hipMemcpyHostToDevice, s), "upload");
  Batch bt;
  bt.pre = w.tables;
  build_batch(bt, {SlotView{PcgSlot{n, A->rowptr, A->col, A->val, b, x, r, z, p, q, dst, ist, 0, 0},
                            f}},
              o.precision, partial, s);
  const SlotBatch &B = bt.B;
  // optional phase timing: events bracket every apply
  std::vector<hipEvent_t> evs;
  struct EvFree {
    std::vector<hipEvent_t> &v;
    ~EvFree() {
      for (auto e : v) (void)hipEventDestroy(e);
    }
  } evfree{evs};
  auto mark = [&](bool always) {
    if (!w.events || (!o.timing && !always)) return;
    hipEvent_t e;
    chk(hipEventCreate(&e), "hipEventCreate");
    chk(hipEventRecord(e, s), "hipEventRecord");
    evs.push_back(e);
  };
  // events between the two sweeps of every timed apply
  std::vector<hipEvent_t> mids;
  struct MidFree {
    std::vector<hipEvent_t> &v;
    ~MidFree() {
      for (auto e : v) (void)hipEventDestroy(e);
    }
  } midfree{mids};
  auto mid = [&]() -> hipEvent_t {
    if (!w.events || !o.timing) return nullptr;
    hipEvent_t e;
    chk(hipEventCreate(&e), "hipEventCreate");
    mids.push_back(e);
    return e;
  };
  mark(true);  // evs[0]: start
  chk(slots_init(B, s), "pcg init");
  int applies = 0;
  mark(false);
  chk(slots_apply(B, o.precision, s, mid()), "apply");
  mark(false);
  ++applies;
  chk(slots_rz(B, 1, s), "pcg rz");
  const int K = o.check_every > 0 ? o.check_every : 8;
  int launched = 0;
  int hist[2] = {0, 0};
  for (;;) {
    const int chunk = std::min(K, o.maxit - launched);
    if (chunk <= 0) break;
    for (int it = 0; it < chunk; ++it) {
      chk(slots_step(B, s), "pcg step");
      mark(false);
      chk(slots_apply(B, o.precision, s, mid()), "apply");
      mark(false);
      ++applies;
      chk(slots_rz(B, 0, s), "pcg rz");
    }
    launched += chunk;
    chk(hipMemcpyAsync(hist, ist, 2 * sizeof(int), hipMemcpyDeviceToHost, s), "read");
    chk(hipStreamSynchronize(s), "sync");
    if (hist[1]) break;
  }
  chk(slots_true_res(B, s), "true residual");
  mark(true);  // last: end
  check_sweeps(f, o.precision, s);
  double hst[8];
  chk(hipMemcpyAsync(hst, dst, sizeof(hst), hipMemcpyDeviceToHost, s), "read");
  chk(hipMemcpyAsync(hist, ist, 2 * sizeof(int), hipMemcpyDeviceToHost, s), "read");
  chk(hipStreamSynchronize(s), "sync");
  const bool ok = hist[1] == 1;
  const double bn = sqrt(hst[0]);
  if (st) {
    // applies that ran (those after convergence return at once)
    const int ran = std::min(applies, hist[0] + 1);
    st->iterations = hist[0];
    st->relres = (bn > 0 && hist[0] > 0) ? sqrt(hst[3]) / bn : 0.0;
    st->true_relres = bn > 0 ? sqrt(hst[7]) / bn : 0.0;
    st->status = ok ? PARAC_OK : PARAC_ENOCONV;
    float ms = 0.f;
    if (evs.size() >= 2) chk(hipEventElapsedTime(&ms, evs.front(), evs.back()), "elapsed");
    st->ms_total = ms;
    st->ms_apply = 0.0;
    st->ms_fwd = 0.0;
    st->applies = ran;
    for (size_t i = 1; i + 2 < evs.size() && (int)((i - 1) / 2) < ran; i += 2) {
      chk(hipEventElapsedTime(&ms, evs[i], evs[i + 1]), "elapsed");
      st->ms_apply += ms;
      const size_t k = (i - 1) / 2;
      if (k < mids.size()) {
        chk(hipEventElapsedTime(&ms, evs[i], mids[k]), "elapsed");
        st->ms_fwd += ms;
      }
    }
  }
  return ok ? PARAC_OK : PARAC_ENOCONV;
}

static int pcg_one(const parac_csr *A, parac_factor_t f, const double *b, double *x,
                   const parac_pcg_opts &o, parac_pcg_stats *st, hipStream_t s) {
  const int64_t n = f->n;
  Scratch tmp;
  PcgWork w{};
  w.r = tmp.alloc<double>(n, "r");
  w.z = tmp.alloc<double>(n, "z");
  w.p = tmp.alloc<double>(n, "p");
  w.q = tmp.alloc<double>(n, "q");
  w.partial = tmp.alloc<double>(slot_blocks(n), "partials");
  w.dst = tmp.alloc<double>(8, "pcg scalars");
  w.ist = tmp.alloc<int>(4, "pcg flags");
  w.tables = nullptr;
  w.events = true;
  return pcg_run(A, f, b, x, o, st, s, w);
}

// ---------------------------------------------------------------------------
// PCG without device allocation (parac_pcg_static)
// ---------------------------------------------------------------------------
// Every per-call buffer of a single-vector PCG (r, z, p, q, partial sums,
// scalars, flags, the batch tables, and the consistency check's sums, which
// share r and z before the iteration starts) lives in this fixed array, one
// copy per GPU for the life of the process.  In host code its name is a
// host-side stand-in, never a device address: each device's address comes
// from hipGetSymbolAddress, once per device with that device current, and
// only that address is handed to kernels and copies.
static __device__ __align__(256) unsigned char scratch[PARAC_STATIC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::vector<void *> g_scratch_dev;  // device address of scratch, by device

static char *static_scratch() {
  int dev = 0;
  chk(hipGetDevice(&dev), "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_dev.size() <= dev) g_scratch_dev.resize((size_t)dev + 1, nullptr);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      throw Err{PARAC_EDEVICE,
                std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
    }
    g_scratch_dev[dev] = p;
  }
  return (char *)g_scratch_dev[dev];
}

// byte offsets of the buffers in the array for a system of ntot rows
struct StaticLayout {
  size_t r, z, p, q, partial, dst, ist, bad, slots, bslot, aslots, wgmap, end;
};
static StaticLayout static_layout(int64_t ntot) {
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t vb = up((size_t)std::max<int64_t>(ntot, 1) * sizeof(double));
  StaticLayout L{};
  size_t o = 0;
  L.r = o, o += vb;
  L.z = o, o += vb;
  L.p = o, o += vb;
  L.q = o, o += vb;
  L.partial = o, o += up(kSlotMaxBlocks * sizeof(double));
  L.dst = o, o += up(8 * sizeof(double));
  L.ist = o, o += up(4 * sizeof(int));
  L.bad = o, o += up(sizeof(int));
  L.slots = o, o += up(sizeof(PcgSlot));
  L.bslot = o, o += up(kSlotMaxBlocks * sizeof(int32_t));
  L.aslots = o, o += up(sizeof(ApplySlot));
  L.wgmap = o, o += up(kReadyGroupsMax * sizeof(int32_t));
  L.end = o;
  return L;
}

static void check_consistent_block(parac_factor_t f, const double *b, int64_t nrhs,
                                   hipStream_t s) {
  const int64_t n = f->n;
  if (n == 0) return;
  for (int64_t c0 = 0; c0 < nrhs; c0 += kBlockCols) {
    const int nc = (int)std::min<int64_t>(kBlockCols, nrhs - c0);
    Scratch tmp;
    const int64_t m = f->ntot * nc;
    double *sum = tmp.alloc<double>(m, "sums");
    double *sabs = tmp.alloc<double>(m, "sums");
    int *bad = tmp.alloc<int>(1, "flag");
    chk(hipMemsetAsync(sum, 0, m * sizeof(double), s), "memset");
    chk(hipMemsetAsync(sabs, 0, m * sizeof(double), s), "memset");
    chk(hipMemsetAsync(bad, 0, sizeof(int), s), "memset");
    chk(launch_bcomp_check(n, nc, f->ntot > n ? n : -1, f->perm, f->root, b + c0, nrhs, sum,
                           sabs, bad, s),
        "comp_check");
    if (read1(bad, s))
      throw Err{PARAC_EINCONSISTENT,
                "a column of b has a nonzero sum on a component without excess"};
  }
}

// block PCG: chunks of at most kBlockCols columns, each chunk one sequence
// of block launches with per-column scalars
static int pcg_block(const parac_csr *A, parac_factor_t f, const double *b, double *x,
                     int64_t nrhs, const parac_pcg_opts &o, parac_pcg_stats *st, hipStream_t s) {
  const int64_t n = f->n;
  int rc = PARAC_OK;
  for (int64_t c0 = 0; c0 < nrhs; c0 += kBlockCols) {
    const int nc = (int)std::min<int64_t>(kBlockCols, nrhs - c0);
    Scratch tmp;
    const int64_t m = std::max<int64_t>(n, 1) * nc;
    double *r = tmp.alloc<double>(m, "r");
    double *z = tmp.alloc<double>(m, "z");
    double *p = tmp.alloc<double>(m, "p");
    double *q = tmp.alloc<double>(m, "q");
    const int nb = bpcg_partials();
    double *partial = tmp.alloc<double>((int64_t)nb * nc, "partials");
    double *bst = tmp.alloc<double>(8 * nc, "pcg scalars");
    int *bist = tmp.alloc<int>(4 * nc, "pcg flags");
    int *gfl = tmp.alloc<int>(2, "pcg flags");
    std::vector<hipEvent_t> evs;
    struct EvFree {
      std::vector<hipEvent_t> &v;
      ~EvFree() {
        for (auto e : v) (void)hipEventDestroy(e);
      }
    } evfree{evs};
    auto mark = [&](bool always) {
      if (!o.timing && !always) return;
      hipEvent_t e;
      chk(hipEventCreate(&e), "hipEventCreate");
      chk(hipEventRecord(e, s), "hipEventRecord");
      evs.push_back(e);
    };
    mark(true);  // evs[0]: start
    chk(bpcg_launch_init(n, nc, o.rtol, b + c0, nrhs, x + c0, nrhs, r, p, partial, bst, bist, gfl,
                         s),
        "bpcg_init");
    const parac_block_shape shp = block_shape(f, nc, o.precision);
    // column sweeps: one batch for the whole solve, a converged column's
    // sweeps skipped through its done flag
    Batch cols;
    if (shp.cpl == 0 && n > 0) build_cols(cols, f, nc, r, nc, z, nc, o.precision, bist + 1, 4, s);
    auto apply = [&]() {
      if (shp.cpl == 0) {
        if (n > 0) chk(slots_apply(cols.B, o.precision, s), "column sweeps");
      } else {
        apply_block(f, shp, nc, r, nc, z, nc, o.precision, gfl + 1, s);
      }
    };
    int applies = 0;
    mark(false);
    apply();
    mark(false);
    ++applies;
    chk(bpcg_launch_rz(n, nc, r, z, p, partial, bst, bist, gfl, 1, s), "bpcg_rz");
    const int K = o.check_every > 0 ? o.check_every : 8;
    int launched = 0;
    int g[2] = {0, 0};
    for (;;) {
      const int chunk = std::min(K, o.maxit - launched);
      if (chunk <= 0) break;
      for (int it = 0; it < chunk; ++it) {
        chk(bpcg_launch_step(n, nc, A->rowptr, A->col, A->val, x + c0, nrhs, r, p, q, partial, bst,
                             bist, gfl, s),
            "bpcg_step");
        mark(false);
        apply();
        mark(false);
        ++applies;
        chk(bpcg_launch_rz(n, nc, r, z, p, partial, bst, bist, gfl, 0, s), "bpcg_rz");
      }
      launched += chunk;
      chk(hipMemcpyAsync(g, gfl, sizeof(g), hipMemcpyDeviceToHost, s), "read");
      chk(hipStreamSynchronize(s), "sync");
      if (g[1]) break;
    }
    chk(bpcg_launch_true_res(n, nc, A->rowptr, A->col, A->val, x + c0, nrhs, b + c0, nrhs, q,
                             partial, bst, bist, gfl, s),
        "bpcg_true_res");
    mark(true);  // last: end
    if (shp.cpl == 0 && n > 0) check_col_sweeps(f, o.precision, s);
    std::vector<double> hst(8 * nc);
    std::vector<int> hist(4 * nc);
    chk(hipMemcpyAsync(hst.data(), bst, hst.size() * sizeof(double), hipMemcpyDeviceToHost, s),
        "read");
    chk(hipMemcpyAsync(hist.data(), bist, hist.size() * sizeof(int), hipMemcpyDeviceToHost, s),
        "read");
    chk(hipStreamSynchronize(s), "sync");
    int maxit_seen = 0;
    for (int j = 0; j < nc; ++j) maxit_seen = std::max(maxit_seen, hist[4 * j]);
    const int ran = std::min(applies, maxit_seen + 1);
    float ms = 0.f;
    chk(hipEventElapsedTime(&ms, evs.front(), evs.back()), "elapsed");
    const double ms_total = ms;
    double ms_apply = 0.0;
    for (size_t i = 1; i + 2 < evs.size() && (int)((i - 1) / 2) < ran; i += 2) {
      chk(hipEventElapsedTime(&ms, evs[i], evs[i + 1]), "elapsed");
      ms_apply += ms;
    }
    for (int j = 0; j < nc; ++j) {
      const double bn = sqrt(hst[8 * j]);
      const bool done = hist[4 * j + 1] != 0;
      if (!done) rc = PARAC_ENOCONV;
      if (!st) continue;
      parac_pcg_stats &o1 = st[c0 + j];
      o1.iterations = hist[4 * j];
      o1.relres = (bn > 0 && hist[4 * j] > 0) ? sqrt(hst[8 * j + 3]) / bn : 0.0;
      o1.true_relres = bn > 0 ? sqrt(hst[8 * j + 7]) / bn : 0.0;
      o1.status = done ? PARAC_OK : PARAC_ENOCONV;
      o1.ms_total = ms_total;
      o1.ms_apply = ms_apply;
      o1.ms_fwd = 0.0;
      o1.applies = ran;
    }
  }
  return rc;
}

// ---------------------------------------------------------------------------
// serving loop
// ---------------------------------------------------------------------------
namespace {

// one admitted system: its device copy of the request, factor and PCG state
struct ServeSlot {
  int64_t req = -1;
  int id = -1;  // row of the per-call scalar pools
  parac_factor_t f = nullptr;
  Scratch mem;
  int64_t n = 0;
  const int64_t *rowptr = nullptr;
  const int32_t *col = nullptr;
  const double *val = nullptr;
  double *b = nullptr, *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  int64_t est = 0, bytes = 0;
  int status = PARAC_OK;
  std::string err;
  ~ServeSlot() {
    if (f) {
      for (void *ptr : f->owned) (void)hipFree(ptr);
      delete f;
    }
  }
};

// estimated peak device bytes of one request: input, PCG vectors, and the
// elimination's pools and factor arrays at their largest (pool_factor 4)
int64_t serve_estimate(int64_t n, int64_t nnz) {
  const int64_t ntot = n + 1;
  return 12 * nnz + 8 * (n + 1) + 6 * 8 * n + 170 * nnz + 340 * ntot + (1 << 20);
}

struct SetupQueue {
  std::mutex m;
  std::condition_variable cv_work, cv_done;
  std::deque<std::unique_ptr<ServeSlot>> todo, done;
  bool stop = false;
};

// upload and factor one admitted request (worker thread, its own stream)
void serve_setup(ServeSlot &sl, const parac_request &rq, int prec, int maxit, double *st_pool,
                 int *ist_pool, hipStream_t s) {
  const int64_t n = rq.A.n, nnz = rq.A.nnz;
  if (n < 0 || nnz < 0 || rq.A.on_device ||
      (n > 0 && (!rq.A.rowptr || !rq.A.col || !rq.A.val || !rq.b || !rq.x)))
    throw Err{PARAC_EINVAL, "a request needs host CSR arrays, b and x"};
  Scratch &M = sl.mem;
  int64_t *rp = M.alloc<int64_t>(n + 1, "request rowptr");
  int32_t *c = M.alloc<int32_t>(nnz, "request col");
  double *v = M.alloc<double>(nnz, "request val");
  double *b = M.alloc<double>(n, "request b");
  int32_t *pm = rq.perm ? M.alloc<int32_t>(n, "request perm") : nullptr;
  if (n > 0) {
    chk(hipMemcpyAsync(rp, rq.A.rowptr, (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s),
        "upload");
    chk(hipMemcpyAsync(c, rq.A.col, nnz * sizeof(int32_t), hipMemcpyHostToDevice, s), "upload");
    chk(hipMemcpyAsync(v, rq.A.val, nnz * sizeof(double), hipMemcpyHostToDevice, s), "upload");
    chk(hipMemcpyAsync(b, rq.b, n * sizeof(double), hipMemcpyHostToDevice, s), "upload");
    if (pm) chk(hipMemcpyAsync(pm, rq.perm, n * sizeof(int32_t), hipMemcpyHostToDevice, s), "upload");
  }
  parac_csr dA{n, nnz, rp, c, v, 1};
  parac_factor_opts fo{};
  fo.seed = rq.seed;
  fo.perm = pm;
  fo.mode = PARAC_MODE_AUTO;
  fo.pool_factor = 4.0;
  fo.keep_fp32 = prec == PARAC_PREC_MIXED;
  fo.timeout_s = 30.0;
  sl.f = factor_impl(&dA, &fo, s);
  if (sl.f->mode == PARAC_MODE_LAPLACIAN) check_consistent(sl.f, b, s);
  sl.n = n;
  sl.rowptr = rp;
  sl.col = c;
  sl.val = v;
  sl.b = b;
  sl.x = M.alloc<double>(n, "x");
  sl.r = M.alloc<double>(n, "r");
  sl.z = M.alloc<double>(n, "z");
  sl.p = M.alloc<double>(n, "p");
  sl.q = M.alloc<double>(n, "q");
  ensure_work(sl.f, prec, s);
  const double rtol = rq.rtol >= 0 ? rq.rtol : 1e-6;
  const double hst0[8] = {0, 0, 0, 0, 0, 0, rtol, 0};
  const int hist0[4] = {0, 0, maxit, 0};
  chk(hipMemcpyAsync(st_pool + 8 * sl.id, hst0, sizeof(hst0), hipMemcpyHostToDevice, s), "upload");
  chk(hipMemcpyAsync(ist_pool + 4 * sl.id, hist0, sizeof(hist0), hipMemcpyHostToDevice, s),
      "upload");
  chk(hipStreamSynchronize(s), "sync");
  sl.bytes = M.total + sl.f->bytes;
}

SlotView slot_view(ServeSlot &sl, double *st_pool, int *ist_pool) {
  return SlotView{PcgSlot{sl.n, sl.rowptr, sl.col, sl.val, sl.b, sl.x, sl.r, sl.z, sl.p, sl.q,
                          st_pool + 8 * sl.id, ist_pool + 4 * sl.id, 0, 0},
                  sl.f};
}

}  // namespace

static int serve_impl(const parac_request *reqs, int64_t nreq, const parac_serve_opts &o,
                      parac_result *out) {
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  auto now = [&]() { return std::chrono::duration<double>(clk::now() - t0).count(); };
  const int prec = o.precision;
  const int max_slots = o.max_slots;
  const int K = o.check_every;
  int dev = 0;
  chk(hipGetDevice(&dev), "hipGetDevice");
  size_t budget = o.hbm_budget;
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    chk(hipMemGetInfo(&fr, &tot), "hipMemGetInfo");
    budget = (size_t)(0.8 * (double)fr);
  }
  for (int64_t i = 0; i < nreq; ++i) {
    out[i] = parac_result{};
    out[i].status = PARAC_OK;
    out[i].t_arrive = reqs[i].arrival_s;
  }
  std::vector<int64_t> order(nreq);
  for (int64_t i = 0; i < nreq; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    return reqs[a].arrival_s < reqs[b].arrival_s;
  });

  Scratch pools;
  double *st_pool = pools.alloc<double>(8 * (int64_t)max_slots, "serve scalars");
  int *ist_pool = pools.alloc<int>(4 * (int64_t)max_slots, "serve flags");
  double *partial = pools.alloc<double>((int64_t)max_slots * kSlotMaxBlocks, "serve partials");
  hipStream_t cs = nullptr;
  chk(hipStreamCreate(&cs), "hipStreamCreate");
  struct StreamFree {
    hipStream_t &s;
    ~StreamFree() {
      if (s) (void)hipStreamDestroy(s);
    }
  } csfree{cs};

  // the setup worker
  SetupQueue Q;
  std::thread worker([&]() {
    (void)hipSetDevice(dev);
    hipStream_t ss = nullptr;
    const bool have_stream = hipStreamCreate(&ss) == hipSuccess;
    for (;;) {
      std::unique_ptr<ServeSlot> sl;
      {
        std::unique_lock<std::mutex> lk(Q.m);
        Q.cv_work.wait(lk, [&] { return Q.stop || !Q.todo.empty(); });
        if (Q.todo.empty()) break;
        sl = std::move(Q.todo.front());
        Q.todo.pop_front();
      }
      try {
        if (!have_stream) throw Err{PARAC_EDEVICE, "setup stream"};
        serve_setup(*sl, reqs[sl->req], prec, o.maxit, st_pool, ist_pool, ss);
      } catch (Err &e) {
        sl->status = e.code;
        sl->err = e.msg;
      } catch (std::exception &e) {
        sl->status = PARAC_EINTERNAL;
        sl->err = e.what();
      }
      {
        std::lock_guard<std::mutex> lk(Q.m);
        Q.done.push_back(std::move(sl));
      }
      Q.cv_done.notify_one();
    }
    if (ss) (void)hipStreamDestroy(ss);
  });
  struct Joiner {
    SetupQueue &Q;
    std::thread &t;
    ~Joiner() {
      {
        std::lock_guard<std::mutex> lk(Q.m);
        Q.stop = true;
      }
      Q.cv_work.notify_all();
      if (t.joinable()) t.join();
    }
  } joiner{Q, worker};

  std::vector<int> free_ids;
  for (int k = max_slots - 1; k >= 0; --k) free_ids.push_back(k);
  std::vector<std::unique_ptr<ServeSlot>> active;
  int64_t next = 0, finished = 0, inflight = 0;
  size_t reserved = 0;
  Batch bt;
  bool dirty = true;
  std::vector<int> hflags(4 * (size_t)max_slots);

  auto retire = [&](ServeSlot &sl, int status) {
    parac_result &r = out[sl.req];
    r.status = status;
    r.t_done = now();
    r.bytes_resident = sl.bytes;
    reserved -= (size_t)(sl.bytes ? sl.bytes : sl.est);
    free_ids.push_back(sl.id);
    --inflight;
    ++finished;
  };

  while (finished < nreq) {
    // 1. admission in arrival order
    const double t = now();
    while (next < nreq && reqs[order[next]].arrival_s <= t) {
      const int64_t i = order[next];
      const int64_t est = serve_estimate(std::max<int64_t>(reqs[i].A.n, 0),
                                         std::max<int64_t>(reqs[i].A.nnz, 0));
      if ((size_t)est > budget) {
        out[i].status = PARAC_ENOMEM;
        out[i].t_admit = out[i].t_done = t;
        ++next;
        ++finished;
        continue;
      }
      if (free_ids.empty() || reserved + (size_t)est > budget) break;
      auto sl = std::make_unique<ServeSlot>();
      sl->req = i;
      sl->id = free_ids.back();
      free_ids.pop_back();
      sl->est = est;
      reserved += (size_t)est;
      ++inflight;
      out[i].t_admit = t;
      {
        std::lock_guard<std::mutex> lk(Q.m);
        Q.todo.push_back(std::move(sl));
      }
      Q.cv_work.notify_one();
      ++next;
    }
    // 2. systems the worker has set up: start their PCG, then join the batch
    std::vector<std::unique_ptr<ServeSlot>> fresh;
    {
      std::lock_guard<std::mutex> lk(Q.m);
      while (!Q.done.empty()) {
        fresh.push_back(std::move(Q.done.front()));
        Q.done.pop_front();
      }
    }
    std::vector<std::unique_ptr<ServeSlot>> started;
    for (auto &sl : fresh) {
      if (sl->status != PARAC_OK) {
        retire(*sl, sl->status);
        continue;
      }
      reserved = reserved - (size_t)sl->est + (size_t)sl->bytes;
      started.push_back(std::move(sl));
    }
    if (!started.empty()) {
      std::vector<SlotView> v;
      for (auto &sl : started) v.push_back(slot_view(*sl, st_pool, ist_pool));
      Batch nb;
      build_batch(nb, v, prec, partial, cs);
      chk(slots_init(nb.B, cs), "serve init");
      chk(slots_apply(nb.B, prec, cs), "serve apply");
      chk(slots_rz(nb.B, 1, cs), "serve rz");
      chk(hipStreamSynchronize(cs), "sync");
      for (auto &sl : started) active.push_back(std::move(sl));
      dirty = true;
    }
    if (active.empty()) {
      // nothing to iterate: wait for the worker or the next arrival
      std::unique_lock<std::mutex> lk(Q.m);
      double wait = 1e-3;
      if (inflight == 0 && next < nreq)
        wait = std::max(0.0, reqs[order[next]].arrival_s - now());
      if (Q.done.empty())
        Q.cv_done.wait_for(lk, std::chrono::duration<double>(std::min(wait, 0.05)));
      continue;
    }
    // 3. K batched iterations over every system in flight
    if (dirty) {
      std::vector<SlotView> v;
      for (auto &sl : active) v.push_back(slot_view(*sl, st_pool, ist_pool));
      build_batch(bt, v, prec, partial, cs);
      dirty = false;
    }
    for (int it = 0; it < K; ++it) {
      chk(slots_step(bt.B, cs), "serve step");
      chk(slots_apply(bt.B, prec, cs), "serve apply");
      chk(slots_rz(bt.B, 0, cs), "serve rz");
    }
    chk(hipMemcpyAsync(hflags.data(), ist_pool, hflags.size() * sizeof(int),
                       hipMemcpyDeviceToHost, cs),
        "read");
    chk(hipStreamSynchronize(cs), "sync");
    // 4. finished systems: true residual, x back to the caller, release
    // (the batch tables point into every active slot: slots leave `active`
    // only together with a rebuild of the batch)
    bool any_done = false;
    for (auto &sl : active) any_done |= hflags[4 * sl->id + 1] != 0;
    if (!any_done) continue;
    std::vector<std::unique_ptr<ServeSlot>> fin, keep;
    for (auto &sl : active) {
      if (hflags[4 * sl->id + 1]) fin.push_back(std::move(sl));
      else keep.push_back(std::move(sl));
    }
    active = std::move(keep);
    dirty = true;
    {
      std::vector<SlotView> v;
      for (auto &sl : fin) v.push_back(slot_view(*sl, st_pool, ist_pool));
      Batch fb;
      build_batch(fb, v, prec, partial, cs);
      chk(slots_true_res(fb.B, cs), "serve residual");
    }
    std::vector<double> hst(8 * (size_t)max_slots);
    chk(hipMemcpyAsync(hst.data(), st_pool, hst.size() * sizeof(double), hipMemcpyDeviceToHost,
                       cs),
        "read");
    chk(hipMemcpyAsync(hflags.data(), ist_pool, hflags.size() * sizeof(int),
                       hipMemcpyDeviceToHost, cs),
        "read");
    for (auto &sl : fin)
      if (sl->n > 0)
        chk(hipMemcpyAsync(reqs[sl->req].x, sl->x, sl->n * sizeof(double), hipMemcpyDeviceToHost,
                           cs),
            "result copy");
    chk(hipStreamSynchronize(cs), "sync");
    for (auto &sl : fin) {
      const int id = sl->id;
      const double bn = sqrt(hst[8 * id]);
      parac_result &r = out[sl->req];
      r.iterations = hflags[4 * id];
      r.true_relres = bn > 0 ? sqrt(hst[8 * id + 7]) / bn : 0.0;
      int stat = hflags[4 * id + 1] == 1 ? PARAC_OK : PARAC_ENOCONV;
      if (sl->f && read1(sl->f->serr, cs) != 0) stat = PARAC_ETIMEOUT;
      retire(*sl, stat);
    }
  }
  return PARAC_OK;
}

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------
extern "C" {

parac_status parac_factor(const parac_csr *A, const parac_factor_opts *o, void *stream,
                          parac_factor_t *out) {
  if (!out) {
    g_last_error = "null output handle";
    return PARAC_EINVAL;
  }
  *out = nullptr;
  try {
    *out = factor_impl(A, o, (hipStream_t)stream);
    return PARAC_OK;
  } catch (Err &e) {
    return status_from(e);
  } catch (std::exception &e) {
    g_last_error = e.what();
    return PARAC_EINTERNAL;
  }
}

parac_status parac_factor_info(parac_factor_t f, parac_factor_stats *s) {
  if (!f || !s) {
    g_last_error = "null argument";
    return PARAC_EINVAL;
  }
  *s = f->stats;
  return PARAC_OK;
}

parac_status parac_factor_export(parac_factor_t f, int64_t *colptr, int32_t *rowind, double *val,
                                 double *D, int32_t *level) {
  if (!f) {
    g_last_error = "null handle";
    return PARAC_EINVAL;
  }
  try {
    auto cp = [](void *dst, const void *src, size_t bytes) {
      if (dst && src && bytes) chk(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost), "export");
    };
    cp(colptr, f->colptr, (f->ntot + 1) * sizeof(int64_t));
    cp(rowind, f->rowind, f->nnz_off * sizeof(int32_t));
    cp(val, f->val, f->nnz_off * sizeof(double));
    cp(D, f->D, f->ntot * sizeof(double));
    cp(level, f->lev, f->ntot * sizeof(int32_t));
    return PARAC_OK;
  } catch (Err &e) {
    return status_from(e);
  }
}

parac_status parac_apply(parac_factor_t f, const double *r, double *z, int64_t nrhs,
                         int32_t precision, void *stream) {
  if (!f || (!r && f->n) || (!z && f->n) || nrhs < 1) {
    g_last_error = "bad apply arguments";
    return PARAC_EINVAL;
  }
  if (precision == PARAC_PREC_MIXED && !f->Dinv32) {
    g_last_error = "mixed precision needs a factor built with keep_fp32";
    return PARAC_EINVAL;
  }
  if (precision != PARAC_PREC_FP64 && precision != PARAC_PREC_MIXED) {
    g_last_error = "bad precision";
    return PARAC_EINVAL;
  }
  try {
    hipStream_t s = (hipStream_t)stream;
    if (nrhs == 1) {
      apply_one(f, r, z, precision, s);
    } else {
      for (int64_t c0 = 0; c0 < nrhs; c0 += kBlockCols) {
        const int nc = (int)std::min<int64_t>(kBlockCols, nrhs - c0);
        const parac_block_shape shp = block_shape(f, nc, precision);
        apply_block(f, shp, nc, r + c0, nrhs, z + c0, nrhs, precision, nullptr, s);
      }
    }
    chk(hipStreamSynchronize(s), "sync");
    return PARAC_OK;
  } catch (Err &e) {
    return status_from(e);
  }
}

parac_status parac_pcg(const parac_csr *A, parac_factor_t f, const double *b, double *x,
                       int64_t nrhs, const parac_pcg_opts *o, parac_pcg_stats *st, void *stream) {
  if (!A || !f || nrhs < 1 || A->n != f->n || !A->on_device || (f->n && (!b || !x))) {
    g_last_error = "bad pcg arguments (matrix must be on the device and match the factor)";
    return PARAC_EINVAL;
  }
  parac_pcg_opts opt{};
  opt.rtol = 1e-6;
  opt.maxit = 10000;
  if (o) {
    opt = *o;
    if (!(opt.rtol >= 0)) opt.rtol = 1e-6;
    if (opt.maxit <= 0) opt.maxit = 10000;
  }
  if (opt.precision == PARAC_PREC_MIXED && !f->Dinv32) {
    g_last_error = "mixed precision needs a factor built with keep_fp32";
    return PARAC_EINVAL;
  }
  try {
    hipStream_t s = (hipStream_t)stream;
    if (nrhs == 1) {
      check_consistent(f, b, s);
      return pcg_one(A, f, b, x, opt, st, s);
    }
    check_consistent_block(f, b, nrhs, s);
    return pcg_block(A, f, b, x, nrhs, opt, st, s);
  } catch (Err &e) {
    if (st)
      for (int64_t j = 0; j < nrhs; ++j) st[j].status = e.code;
    return status_from(e);
  }
}

parac_status parac_pcg_static(const parac_csr *A, parac_factor_t f, const double *b, double *x,
                              const parac_pcg_opts *o, parac_pcg_stats *st, void *stream) {
  if (!A || !f || A->n != f->n || !A->on_device || (f->n && (!b || !x))) {
    g_last_error = "bad pcg arguments (matrix must be on the device and match the factor)";
    return PARAC_EINVAL;
  }
  const StaticLayout L = static_layout(f->ntot);
  if (L.end > (size_t)PARAC_STATIC_SCRATCH_BYTES) {
    g_last_error = "system too large for parac_pcg_static: " + std::to_string(f->ntot) +
                   " rows need " + std::to_string(L.end) + " bytes of the " +
                   std::to_string((size_t)PARAC_STATIC_SCRATCH_BYTES) +
                   "-byte static scratch (at most " +
                   std::to_string(parac_pcg_static_max_rows()) + " rows)";
    return PARAC_EINVAL;
  }
  parac_pcg_opts opt{};
  opt.rtol = 1e-6;
  opt.maxit = 10000;
  if (o) {
    opt = *o;
    if (!(opt.rtol >= 0)) opt.rtol = 1e-6;
    if (opt.maxit <= 0) opt.maxit = 10000;
  }
  opt.timing = 0;
  if (opt.precision != PARAC_PREC_FP64 && opt.precision != PARAC_PREC_MIXED) {
    g_last_error = "bad precision";
    return PARAC_EINVAL;
  }
  if (opt.precision == PARAC_PREC_MIXED && !f->Dinv32) {
    g_last_error = "mixed precision needs a factor built with keep_fp32";
    return PARAC_EINVAL;
  }
  // the factor's sweep work vectors come with it; nothing is allocated here
  if (f->n && !(opt.precision == PARAC_PREC_MIXED ? f->wy32 : f->wy64)) {
    g_last_error = "factor has no sweep work vectors for this precision";
    return PARAC_EINVAL;
  }
  try {
    hipStream_t s = (hipStream_t)stream;
    char *base = static_scratch();
    check_consistent(f, b, s, (double *)(base + L.r), (double *)(base + L.z),
                     (int *)(base + L.bad));
    TableMem tm;
    tm.slots = (PcgSlot *)(base + L.slots);
    tm.bslot = (int32_t *)(base + L.bslot);
    tm.bslot_cap = kSlotMaxBlocks;
    tm.aslots = (ApplySlot *)(base + L.aslots);
    tm.wgmap = (int32_t *)(base + L.wgmap);
    tm.wgmap_cap = kReadyGroupsMax;
    PcgWork w{};
    w.r = (double *)(base + L.r);
    w.z = (double *)(base + L.z);
    w.p = (double *)(base + L.p);
    w.q = (double *)(base + L.q);
    w.partial = (double *)(base + L.partial);
    w.dst = (double *)(base + L.dst);
    w.ist = (int *)(base + L.ist);
    w.tables = &tm;
    w.events = false;
    return pcg_run(A, f, b, x, opt, st, s, w);
  } catch (Err &e) {
    if (st) st->status = e.code;
    return status_from(e);
  }
}

int64_t parac_pcg_static_max_rows(void) {
  // the largest ntot whose layout fits: the fixed part, then 4 vectors
  const StaticLayout L0 = static_layout(1);
  const size_t fixed = L0.end - 4 * 256;
  const size_t avail = (size_t)PARAC_STATIC_SCRATCH_BYTES - fixed;
  return (int64_t)((avail / 4) & ~(size_t)255) / (int64_t)sizeof(double);
}

parac_status parac_block_shape_set(parac_factor_t f, int32_t cols, int32_t precision,
                                   const parac_block_shape *shape) {
  if (!f || cols < 2 || cols > kBlockCols ||
      (precision != PARAC_PREC_FP64 && precision != PARAC_PREC_MIXED) ||
      (shape && !shape_ok(*shape))) {
    g_last_error = "bad block shape arguments";
    return PARAC_EINVAL;
  }
  const auto key = std::make_pair((int)cols, prec_slot(precision));
  if (shape)
    f->shapes[key] = *shape;
  else
    f->shapes.erase(key);
  return PARAC_OK;
}

parac_status parac_block_shape_get(parac_factor_t f, int32_t cols, int32_t precision,
                                   parac_block_shape *shape) {
  if (!f || !shape) {
    g_last_error = "null argument";
    return PARAC_EINVAL;
  }
  auto it = f->shapes.find(std::make_pair((int)cols, prec_slot(precision)));
  if (it == f->shapes.end()) {
    g_last_error = "no block shape fixed for these columns and precision";
    return PARAC_EINVAL;
  }
  *shape = it->second;
  return PARAC_OK;
}

parac_status parac_serve(const parac_request *reqs, int64_t n, const parac_serve_opts *o,
                         parac_result *out) {
  if (n < 0 || (n > 0 && (!reqs || !out))) {
    g_last_error = "bad serve arguments";
    return PARAC_EINVAL;
  }
  parac_serve_opts opt{};
  if (o) opt = *o;
  if (opt.max_slots == 0) opt.max_slots = 32;
  if (opt.maxit <= 0) opt.maxit = 10000;
  if (opt.check_every <= 0) opt.check_every = 4;
  if (opt.max_slots < 1 || opt.max_slots > 256 ||
      (opt.precision != PARAC_PREC_FP64 && opt.precision != PARAC_PREC_MIXED)) {
    g_last_error = "bad serve options";
    return PARAC_EINVAL;
  }
  try {
    return serve_impl(reqs, n, opt, out);
  } catch (Err &e) {
    return status_from(e);
  } catch (std::exception &e) {
    g_last_error = e.what();
    return PARAC_EINTERNAL;
  }
}

void parac_factor_free(parac_factor_t f) {
  if (!f) return;
  for (void *p : f->owned) (void)hipFree(p);
  delete f;
}

const char *parac_status_str(parac_status s) {
  switch (s) {
    case PARAC_OK: return "ok";
    case PARAC_EINVAL: return "invalid argument";
    case PARAC_ENOTLAP: return "not a Laplacian/SDDM matrix";
    case PARAC_EPOOL: return "fill pool exhausted";
    case PARAC_ENOMEM: return "out of device memory";
    case PARAC_ETIMEOUT: return "elimination watchdog expired";
    case PARAC_EDEVICE: return "HIP runtime error";
    case PARAC_EINCONSISTENT: return "inconsistent right-hand side";
    case PARAC_ENOCONV: return "PCG did not converge";
    case PARAC_EINTERNAL: return "internal invariant failed";
    default: return "unknown status";
  }
}

const char *parac_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
