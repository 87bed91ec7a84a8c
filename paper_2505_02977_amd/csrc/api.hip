// api.hip -- the C ABI: parac_factor, parac_apply, parac_pcg and the factor
// handle's accessors.  Host code only orchestrates: every step of the path
// runs in the library's own kernels.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
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
    return (T *)p;
  }
  void keep(void *p, std::vector<void *> &dst) {
    auto it = std::find(ptrs.begin(), ptrs.end(), p);
    if (it != ptrs.end()) {
      ptrs.erase(it);
      dst.push_back(p);
    }
  }
  void release_all() {
    for (void *p : ptrs) (void)hipFree(p);
    ptrs.clear();
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

// ---------------------------------------------------------------------------
// factor
// ---------------------------------------------------------------------------
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
  int workers = (maxwg * 4) / kSubQueues * kSubQueues;
  // no more workers than a quarter of the pivots could keep busy
  workers = std::min<int64_t>(workers, std::max<int64_t>(kSubQueues, (ntot / 4) / kSubQueues * kSubQueues));
  if (opt.workers > 0) workers = std::min(workers, std::max(kSubQueues, opt.workers / kSubQueues * kSubQueues));
  if (workers < kSubQueues) throw Err{PARAC_EDEVICE, "device too small for the persistent grid"};
  const int wgs = workers / 4;

  // per-attempt state
  const int32_t cap_q = (int32_t)((ntot + kSubQueues - 1) / kSubQueues);
  int32_t *q = tmp.alloc<int32_t>((int64_t)cap_q * kSubQueues, "queue");
  int32_t *qtail = tmp.alloc<int32_t>(3 * kSubQueues * kTailStride + 3 * kTailStride, "qtail");
  int32_t *qhead = qtail + kSubQueues * kTailStride;
  int32_t *qdone = qhead + kSubQueues * kTailStride;
  int32_t *tqc = qdone + kSubQueues * kTailStride;  // tail head, tail, count
  int32_t *tq = tmp.alloc<int32_t>(ntot, "tail queue");
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
    const int64_t pool_base = (int64_t)(pf * (double)base_entries);
    const int64_t f_base = (int64_t)(0.5 * pf * (double)base_entries) + ntot;
    // per-worker reservations: small enough that their slack stays a fraction
    // of the pools
    const int pg_chunk = (int)std::min<int64_t>(kPageChunk, std::max<int64_t>(64, pool_base / (8 * workers)));
    const int f_chunk = (int)std::min<int64_t>(kFChunk, std::max<int64_t>(64, f_base / (8 * workers)));
    pool_cap = std::min<int64_t>(pool_base + (int64_t)workers * pg_chunk, (int64_t)INT32_MAX - 1);
    f_cap = f_base + (int64_t)workers * f_chunk;
    arena_cap = (int64_t)(pf * (double)base_entries) * 16 + (int64_t)workers * 8192;
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
      const double tf = opt.tail_fraction == 0.0 ? 0.04 : opt.tail_fraction;
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
    if (ntot > 0) chk(launch_eliminate(ea, wgs, s), "eliminate");
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
    chk(launch_sort_long_rows(rowptr_f, colind_f, val_f, long_rows, flags + 2, frow, fval,
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
    // the thin tail: the smallest level from which every level has at most
    // kTailWidth rows
    int64_t L0 = depth;
    while (L0 > 0 && F->hlptr[L0] - F->hlptr[L0 - 1] <= kTailWidth) --L0;
    F->L0 = L0;
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
    chk(launch_level_copy(n, F->order, rowptr_f, colind_f, val_f, F->colptr, F->rowind,
                          F->val, F->lf_ptr, F->lb_ptr, F->lf_idx, F->lf_val, F->lb_idx,
                          F->lb_val, s),
        "level_copy");
    if (opt.keep_fp32) {
      F->lf_val32 = tmp.alloc<float>(nf, "lf_val32");
      F->lb_val32 = tmp.alloc<float>(nbk, "lb_val32");
      chk(launch_cast32(nf, F->lf_val, F->lf_val32, s), "cast");
      chk(launch_cast32(nbk, F->lb_val, F->lb_val32, s), "cast");
    }
  }
  F->Dinv = tmp.alloc<double>(ntot, "Dinv");
  float *Dinv32 = nullptr;
  if (opt.keep_fp32) Dinv32 = tmp.alloc<float>(ntot, "Dinv32");
  F->Dinv32 = Dinv32;
  if (ntot > 0) chk(launch_dinv(ntot, F->D, F->Dinv, Dinv32, s), "dinv");
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
                  (void *)F->lf_ptr, (void *)F->lf_idx, (void *)F->lf_val, (void *)F->lf_val32,
                  (void *)F->lb_ptr, (void *)F->lb_idx, (void *)F->lb_val, (void *)F->lb_val32})
    if (p) tmp.keep(p, F->owned);
  guard.ok = true;
  return F;
}

// ---------------------------------------------------------------------------
// apply
// ---------------------------------------------------------------------------
static SolveArgs solve_args(parac_factor_t f, const int *skip) {
  SolveArgs a{};
  a.n = f->n;
  a.order = f->order;
  a.lptr = f->lptr;
  a.depth = f->depth;
  a.L0 = f->L0;
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
  a.iperm = f->iperm;
  a.skip = skip;
  return a;
}

// label-space work vectors of the two triangular solves
static void ensure_work(parac_factor_t f, int prec) {
  void **py = prec == PARAC_PREC_MIXED ? &f->wy32 : &f->wy64;
  void **px = prec == PARAC_PREC_MIXED ? &f->wx32 : &f->wx64;
  if (*py) return;
  const size_t el = prec == PARAC_PREC_MIXED ? 4 : 8;
  const int64_t m = std::max<int64_t>(f->ntot, 1);
  chk(hipMalloc(py, m * el), "work vector");
  f->owned.push_back(*py);
  chk(hipMalloc(px, m * el), "work vector");
  f->owned.push_back(*px);
}

static void apply_one(parac_factor_t f, const double *r, double *z, int prec, const int *skip,
                      hipStream_t s) {
  if (f->n == 0) return;
  ensure_work(f, prec);
  SolveArgs a = solve_args(f, skip);
  void *y = prec == PARAC_PREC_MIXED ? f->wy32 : f->wy64;
  void *x = prec == PARAC_PREC_MIXED ? f->wx32 : f->wx64;
  chk(launch_apply(a, f->hlptr.data(), r, y, x, z, prec, s), "apply");
}

// ---------------------------------------------------------------------------
// PCG (one right-hand side; several columns run as independent recurrences)
// ---------------------------------------------------------------------------
static void check_consistent(parac_factor_t f, const double *b, hipStream_t s) {
  const int64_t n = f->n;
  if (n == 0) return;
  Scratch tmp;
  double *sum = tmp.alloc<double>(f->ntot, "sums");
  double *sabs = tmp.alloc<double>(f->ntot, "sums");
  int *bad = tmp.alloc<int>(1, "flag");
  chk(hipMemsetAsync(sum, 0, f->ntot * sizeof(double), s), "memset");
  chk(hipMemsetAsync(sabs, 0, f->ntot * sizeof(double), s), "memset");
  chk(hipMemsetAsync(bad, 0, sizeof(int), s), "memset");
  chk(launch_comp_check(n, f->ntot > n ? n : -1, f->perm, f->root, b, sum, sabs, bad, s),
      "comp_check");
  if (read1(bad, s))
    throw Err{PARAC_EINCONSISTENT, "b has a nonzero sum on a component without excess"};
}

static int pcg_one(const parac_csr *A, parac_factor_t f, const double *b, double *x,
                   const parac_pcg_opts &o, parac_pcg_stats *st, hipStream_t s) {
  const int64_t n = f->n;
  Scratch tmp;
  double *r = tmp.alloc<double>(n, "r");
  double *z = tmp.alloc<double>(n, "z");
  double *p = tmp.alloc<double>(n, "p");
  double *q = tmp.alloc<double>(n, "q");
  const int nb = pcg_partials();
  double *partial = tmp.alloc<double>(nb, "partials");
  double *dst = tmp.alloc<double>(8, "pcg scalars");
  int *ist = tmp.alloc<int>(4, "pcg flags");
  // optional phase timing: events bracket every apply
  std::vector<hipEvent_t> evs;
  auto mark = [&]() {
    if (!o.timing) return;
    hipEvent_t e;
    chk(hipEventCreate(&e), "hipEventCreate");
    chk(hipEventRecord(e, s), "hipEventRecord");
    evs.push_back(e);
  };
  struct EvFree {
    std::vector<hipEvent_t> &v;
    ~EvFree() {
      for (auto e : v) (void)hipEventDestroy(e);
    }
  } evfree{evs};
  hipEvent_t t0, t1;
  chk(hipEventCreate(&t0), "hipEventCreate");
  chk(hipEventCreate(&t1), "hipEventCreate");
  evs.push_back(t0);
  evs.push_back(t1);
  const size_t napply_marks = 2;  // evs[0..1] are t0/t1
  chk(hipEventRecord(t0, s), "hipEventRecord");
  chk(hipMemsetAsync(dst, 0, 8 * sizeof(double), s), "memset");
  chk(hipMemsetAsync(ist, 0, 4 * sizeof(int), s), "memset");
  chk(hipMemsetAsync(p, 0, std::max<int64_t>(n, 1) * sizeof(double), s), "memset");
  chk(hipMemcpyAsync(dst + 6, &o.rtol, sizeof(double), hipMemcpyHostToDevice, s), "copy");
  chk(pcg_launch_init(n, b, x, r, partial, dst, ist, s), "pcg_init");
  int applies = 0;
  mark();
  apply_one(f, r, z, o.precision, ist + 2, s);
  mark();
  ++applies;
  chk(pcg_launch_rz(n, r, z, p, partial, dst, ist, 1, s), "pcg_rz");
  const int K = o.check_every > 0 ? o.check_every : 8;
  int launched = 0;
  int hist[2] = {0, 0};
  for (;;) {
    int chunk = std::min(K, o.maxit - launched);
    if (chunk <= 0) break;
    for (int it = 0; it < chunk; ++it) {
      chk(pcg_launch_step(n, A->rowptr, A->col, A->val, x, r, p, q, partial, dst, ist, s), "step");
      mark();
      apply_one(f, r, z, o.precision, ist + 2, s);
      mark();
      ++applies;
      chk(pcg_launch_rz(n, r, z, p, partial, dst, ist, 0, s), "pcg_rz");
    }
    launched += chunk;
    chk(hipMemcpyAsync(hist, ist, 2 * sizeof(int), hipMemcpyDeviceToHost, s), "read");
    chk(hipStreamSynchronize(s), "sync");
    if (hist[1]) break;
  }
  chk(pcg_launch_true_res(n, A->rowptr, A->col, A->val, x, b, q, partial, dst, ist, s), "true_res");
  chk(hipEventRecord(t1, s), "hipEventRecord");
  double hst[8];
  chk(hipMemcpyAsync(hst, dst, sizeof(hst), hipMemcpyDeviceToHost, s), "read");
  chk(hipMemcpyAsync(hist, ist, 2 * sizeof(int), hipMemcpyDeviceToHost, s), "read");
  chk(hipStreamSynchronize(s), "sync");
  const int done = hist[1];
  const double bn = sqrt(hst[0]);
  if (st) {
    // applies that ran (skipped ones after convergence return at once)
    const int ran = std::min(applies, hist[0] + 1);
    st->iterations = hist[0];
    st->relres = bn > 0 ? sqrt(hst[3]) / bn : 0.0;
    st->true_relres = bn > 0 ? sqrt(hst[7]) / bn : 0.0;
    if (hist[0] == 0) st->relres = 0.0;
    st->status = done ? PARAC_OK : PARAC_ENOCONV;
    float ms = 0.f;
    chk(hipEventElapsedTime(&ms, t0, t1), "elapsed");
    st->ms_total = ms;
    st->ms_apply = 0.0;
    st->applies = ran;
    for (size_t i = napply_marks; i + 1 < evs.size() && (int)((i - napply_marks) / 2) < ran;
         i += 2) {
      chk(hipEventElapsedTime(&ms, evs[i], evs[i + 1]), "elapsed");
      st->ms_apply += ms;
    }
  }
  return done ? PARAC_OK : PARAC_ENOCONV;
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
  if (nrhs != 1) {
    g_last_error = "apply: use parac_pcg for several right-hand sides";
    return PARAC_EINVAL;
  }
  try {
    hipStream_t s = (hipStream_t)stream;
    apply_one(f, r, z, precision, nullptr, s);
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
    if (nrhs != 1) throw Err{PARAC_EINVAL, "block PCG not available in this build"};
    check_consistent(f, b, s);
    return pcg_one(A, f, b, x, opt, st, s);
  } catch (Err &e) {
    if (st) st->status = e.code;
    return status_from(e);
  }
}

parac_status parac_serve(const parac_request *reqs, int64_t n, const parac_serve_opts *o,
                         parac_result *out) {
  (void)reqs;
  (void)n;
  (void)o;
  (void)out;
  g_last_error = "serving loop not available in this build";
  return PARAC_EINVAL;
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
