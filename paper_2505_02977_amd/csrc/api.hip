// api.hip -- the C ABI: parac_factor, parac_apply, parac_pcg and the factor
// handle's accessors.  Host code only orchestrates: every step of the path
// runs in the library's own kernels.
#include <math.h>
#include <stdio.h>
#include <unistd.h>
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

// device bytes the library holds (every allocation goes through dev_alloc /
// dev_free), and the peak since the last reset
std::mutex g_mem_mu;
std::map<void *, size_t> g_mem_size;
int64_t g_mem_live = 0, g_mem_peak = 0;

// A serving worker allocates and frees in its own stream's order: hipMalloc
// and hipFree wait for the whole device, so a small system being set up
// would wait for a large one's solve to finish.
thread_local hipStream_t g_alloc_stream = nullptr;

hipError_t dev_alloc(void **p, size_t bytes) {
  const hipError_t e = g_alloc_stream ? hipMallocAsync(p, bytes, g_alloc_stream)
                                      : hipMalloc(p, bytes);
  if (e == hipSuccess) {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    g_mem_size[*p] = bytes;
    g_mem_live += (int64_t)bytes;
    g_mem_peak = std::max(g_mem_peak, g_mem_live);
  }
  return e;
}

void dev_free(void *p) {
  if (!p) return;
  {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    auto it = g_mem_size.find(p);
    if (it != g_mem_size.end()) {
      g_mem_live -= (int64_t)it->second;
      g_mem_size.erase(it);
    }
  }
  if (g_alloc_stream)
    (void)hipFreeAsync(p, g_alloc_stream);
  else
    (void)hipFree(p);
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
    hipError_t e = dev_alloc(&p, bytes);
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
    for (void *p : ptrs) dev_free(p);
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

// PARAC_VERBOSE=1: long solves report their progress on stderr at every
// host convergence check, and the block-shape tuner its candidates
bool verbose() {
  static const bool v = [] {
    const char *e = getenv("PARAC_VERBOSE");
    return e && *e && *e != '0';
  }();
  return v;
}

}  // namespace

constexpr double kSweepTimeoutS = 20.0;  // watchdog of one triangular sweep

// ---------------------------------------------------------------------------
// factor
// ---------------------------------------------------------------------------
// the persistent elimination grid of a system of ntot vertices
struct ElimSizing {
  int nteam = 0, workers = 0, wgs = 0;
};
static ElimSizing elim_sizing(int64_t ntot, int opt_workers) {
  const int maxwg = eliminate_max_workgroups();
  if (maxwg <= 0) throw Err{PARAC_EDEVICE, "occupancy query failed"};
  ElimSizing z;
  // one workgroup in kTeamShare is a team for the largest pivots (none when
  // the graph is too small to have any)
  z.nteam = ntot > 4 * kTeamMin ? maxwg / kTeamShare : 0;
  int64_t workers = ((maxwg - z.nteam) * kElimWaves) / kSubQueues * kSubQueues;
  // no more workers than a sixteenth of the pivots could keep busy
  workers = std::min<int64_t>(workers,
                              std::max<int64_t>(kSubQueues, (ntot / 16) / kSubQueues * kSubQueues));
  if (opt_workers > 0)
    workers = std::min<int64_t>(workers, std::max(kSubQueues, opt_workers / kSubQueues * kSubQueues));
  if (workers < kSubQueues) throw Err{PARAC_EDEVICE, "device too small for the persistent grid"};
  z.workers = (int)workers;
  z.wgs = z.workers / kElimWaves;
  return z;
}

// capacities of the elimination's pools for pool factor pf
struct PoolSizing {
  int64_t pool_cap = 0, f_cap = 0, arena_cap = 0;
  int pg_chunk = 0, f_chunk = 0;
};
static PoolSizing pool_sizing(int64_t ntot, int64_t nnz, double pf, int workers) {
  PoolSizing p;
  const int64_t base_entries = std::max<int64_t>(nnz, 64);
  // pages double in size, so up to half of a target's page chain can be
  // unused: twice the expected record count
  const int64_t pool_base = (int64_t)(2.0 * pf * (double)base_entries);
  // factor entries: about 1.6 nnz on grids, about 3 nnz on power-law graphs
  const int64_t f_base = (int64_t)(pf * (double)base_entries) + ntot;
  // per-worker reservations: small enough that their slack stays a fraction
  // of the pools
  p.pg_chunk = (int)std::min<int64_t>(kPageChunk, std::max<int64_t>(64, pool_base / (8 * workers)));
  p.f_chunk = (int)std::min<int64_t>(kFChunk, std::max<int64_t>(64, f_base / (8 * workers)));
  p.pool_cap = std::min<int64_t>(pool_base + (int64_t)workers * p.pg_chunk, (int64_t)INT32_MAX - 1);
  p.f_cap = f_base + (int64_t)workers * p.f_chunk;
  // scratch of the large-neighbourhood path: every worker keeps its own
  // region (grown geometrically), so besides a share of the fill volume
  // each worker gets room for up to 4096 entries (68 bytes each), fewer on
  // small graphs (an overflow is retried with a larger pool factor)
  const int64_t per_worker = std::min<int64_t>(4096, std::max<int64_t>(64, ntot / 4));
  p.arena_cap = (int64_t)(pf * (double)base_entries) * 16 + (int64_t)workers * 68 * per_worker;
  return p;
}

// an upper bound of the device bytes parac_factor holds at its peak for a
// system of n vertices and nnz stored entries (ntot = n + sddm), at the
// default pool factor: inputs (when copied from the host), checks, upper
// adjacency, queues and inboxes, pools, and the finalised factor with its
// solve layout and work vectors, factor entries bounded by the pool's f_cap
static int64_t factor_peak_bytes(int64_t n, int64_t nnz, int sddm, bool host_input, bool keep32,
                                 int opt_workers) {
  const int64_t ntot = n + sddm;
  const ElimSizing z = elim_sizing(ntot, opt_workers);
  const PoolSizing ps = pool_sizing(ntot, nnz, 4.0, z.workers);
  const int64_t nf = ps.f_cap, nch = nf / 64 + 1;
  int64_t b = 0;
  if (host_input) b += 8 * (n + 1) + 12 * nnz + 4 * n;
  b += 64 + 8 * n + 4 * n + 4 * n + 4 * (n + 1);                                   // A1
  b += 8 * ntot + 8 * (ntot + 1) + (int64_t)scan_tmp_bytes(ntot + 2) + 12 * (nnz + n + 1);  // A2
  b += 4 * (ntot + kSubQueues) + 4 * (3 * kSubQueues * kTailStride + 3 * kTailStride) +
       4 * ntot + 4 * (ntot + z.nteam + 1) + 8 * kTailStride + 4 * ntot + 16 * kInline * ntot +
       4 * (kPages - 1) * ntot + 28 * ntot + 64;                                   // queues, inboxes
  b += 16 * ps.pool_cap + 12 * ps.f_cap + ps.arena_cap;                             // pools
  b += 2 * (8 * (ntot + 1) + 12 * nf + 4 * ntot);                                   // CSC, CSR
  b += 4 * (ntot + 1) + 8 * (ntot + 2) + 4 * n + 8 * n + 16 * (n + 1) + 24 * nf;    // level copies
  b += 16 * n + 16 * (ntot + 1) + 60 * ntot + 8 * n + 16 * (n + 1) + 8 * n;        // maps, lists
  b += 2 * 16 * (n + nch) + 8 * ntot + 16 * ntot + 8 * nch;                         // units, roots, work
  if (keep32) b += 4 * n + 8 * nf + 8 * ntot + 4 * nch;
  return b + (1 << 20);
}

static void ensure_work(parac_factor_t f, int prec, hipStream_t s);

// forced (host, optional): the test hook's partner offsets, forced_count
// entries of forced_stride per pivot label

// Narrow levels of a factor (NarrowDir): the longest run of final levels in
// which every level has at most kNarrowChunks chunks of 16 entries in either
// direction, with at most kNarrowRows positions and kNarrowLevels levels in
// all, and at least kNarrowMinLevels levels.  Builds both directions' tables.
static void narrow_plan(parac_factor_t F, int64_t n, int64_t depth, Scratch &tmp, hipStream_t s) {
  F->nlev0 = depth;
  F->np0 = (int32_t)n;
  F->nf = NarrowDir{};
  F->nb = NarrowDir{};
  if (depth == 0 || n == 0) return;
  const std::vector<int64_t> &lp = F->hlptr;
  int64_t lc = depth;  // lowest candidate level
  while (lc > 0 && n - lp[lc - 1] <= kNarrowRows && depth - (lc - 1) <= kNarrowLevels) --lc;
  if (depth - lc < kNarrowMinLevels) return;
  const int64_t pc = lp[lc], m = n - pc;
  std::vector<int64_t> fp(m + 1), bp(m + 1);
  chk(hipMemcpyAsync(fp.data(), F->lf_ptr + pc, (m + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s),
      "read");
  chk(hipMemcpyAsync(bp.data(), F->lb_ptr + pc, (m + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s),
      "read");
  chk(hipStreamSynchronize(s), "sync");
  if (fp[m] > INT32_MAX || bp[m] > INT32_MAX) return;  // entry indices are 32-bit in the tables
  auto chunks = [](int64_t len) { return (len + 15) / 16; };
  int64_t lo = depth;
  for (int64_t L = depth - 1; L >= lc; --L) {
    int64_t cf = 0, cb = 0;
    for (int64_t p = lp[L]; p < lp[L + 1]; ++p) {
      cf += chunks(fp[p - pc + 1] - fp[p - pc]);
      cb += chunks(bp[p - pc + 1] - bp[p - pc]);
    }
    if (cf > kNarrowChunks || cb > kNarrowChunks) break;
    lo = L;
  }
  const int64_t nlev = depth - lo;
  if (nlev < kNarrowMinLevels) return;
  const int64_t p0 = lp[lo];
  const int32_t P = (int32_t)(n - p0);
  for (int dir = 0; dir < 2; ++dir) {
    const std::vector<int64_t> &pp = dir == 0 ? fp : bp;
    std::vector<int4> hdr;
    std::vector<int32_t> rows(P, 0), smap, lw;
    for (int64_t i = 0; i < nlev; ++i) {
      const int64_t L = dir == 0 ? lo + i : depth - 1 - i;  // the direction's order
      const int64_t a = lp[L], b = lp[L + 1];
      const int64_t hc0 = (int64_t)smap.size() / 8;
      // one wave per row: every row within 32 chunks, groups of 2^lg lanes
      // (lg >= 1) that fit the workgroup
      bool one = true;
      int64_t lanes = 0;
      std::vector<std::pair<int, int64_t>> grp;  // (lg, position) of rows with entries
      for (int64_t p = a; p < b && one; ++p) {
        const int64_t k = chunks(pp[p - pc + 1] - pp[p - pc]);
        if (k > 32) one = false;
        if (k == 0) continue;
        int lg = 1;
        while ((1 << lg) < 2 * k) ++lg;
        lanes += 1 << lg;
        grp.push_back({lg, p});
      }
      if (one && lanes > kNarrowThreads) one = false;
      if (one) {
        // largest groups first: each lands aligned to its size, inside a wave
        std::stable_sort(grp.begin(), grp.end(),
                         [](const std::pair<int, int64_t> &x, const std::pair<int, int64_t> &y) {
                           return x.first > y.first;
                         });
        for (const auto &g : grp) {
          const int64_t p = g.second, e0 = pp[p - pc], e1 = pp[p - pc + 1];
          const int G = 1 << g.first;
          for (int t = 0; t < G; ++t) {
            lw.push_back(t == 0 ? (int32_t)(((p - p0) << 8) | (g.first << 1) | 1) : g.first << 1);
            for (int u = 0; u < 8; ++u) {
              const int64_t e = e0 + 8 * t + u;
              smap.push_back(e < e1 ? (int32_t)e : -1);
            }
          }
        }
        hdr.push_back(make_int4((int)hc0, (int)lanes, (int)(a - p0), (int)(b - a) | kNarrowOneWave));
        continue;
      }
      int32_t c = 0;
      for (int64_t p = a; p < b; ++p) {
        const int64_t e0 = pp[p - pc], e1 = pp[p - pc + 1];
        const int32_t k = (int32_t)chunks(e1 - e0);
        rows[p - p0] = (c << 16) | k;
        for (int64_t e = e0; e < e0 + 16 * (int64_t)k; ++e) smap.push_back(e < e1 ? (int32_t)e : -1);
        c += k;
      }
      lw.resize(smap.size() / 8, 0);
      hdr.push_back(make_int4((int)hc0, 2 * c, (int)(a - p0), (int)(b - a)));
    }
    // at least one half-chunk of slots: threads without one load slot 0
    if (smap.empty()) smap.assign(8, -1);
    lw.resize(smap.size() / 8, 0);
    NarrowDir &N = dir == 0 ? F->nf : F->nb;
    int4 *dh = tmp.alloc<int4>(nlev, "narrow levels");
    int32_t *dr = tmp.alloc<int32_t>(P, "narrow rows");
    const int64_t ns = (int64_t)smap.size();
    int32_t *dm = tmp.alloc<int32_t>(ns, "narrow slots");
    int32_t *dw = tmp.alloc<int32_t>(ns / 8, "narrow lane words");
    chk(hipMemcpyAsync(dw, lw.data(), (ns / 8) * sizeof(int32_t), hipMemcpyHostToDevice, s),
        "upload");
    int16_t *dn = tmp.alloc<int16_t>(ns, "narrow inputs");
    chk(hipMemcpyAsync(dh, hdr.data(), nlev * sizeof(int4), hipMemcpyHostToDevice, s), "upload");
    chk(hipMemcpyAsync(dr, rows.data(), P * sizeof(int32_t), hipMemcpyHostToDevice, s), "upload");
    chk(hipMemcpyAsync(dm, smap.data(), ns * sizeof(int32_t), hipMemcpyHostToDevice, s), "upload");
    chk(launch_narrow_index(ns, dm, dir == 0 ? F->lf_idx : F->lb_idx, (int32_t)p0, dn, s),
        "narrow index");
    chk(hipStreamSynchronize(s), "sync");  // the host tables go out of scope
    N.hdr = dh;
    N.rows = dr;
    N.lw = dw;
    N.smap = dm;
    N.nidx = dn;
    N.nslots = ns;
    N.nlev = (int32_t)nlev;
  }
  F->nlev0 = lo;
  F->np0 = (int32_t)p0;
}

static parac_factor_t factor_impl(const parac_csr *A, const parac_factor_opts *o, hipStream_t s,
                                  const int32_t *forced = nullptr, int32_t forced_stride = 0,
                                  int64_t forced_count = 0) {
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
  if (opt.samples < 0 || opt.samples > 16) throw Err{PARAC_EINVAL, "bad samples per entry"};
  const int samples = opt.samples > 1 ? opt.samples : 1;

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
        for (void *p : f->owned) dev_free(p);
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
  const ElimSizing ez = elim_sizing(ntot, opt.workers);
  const int nteam = ez.nteam, workers = ez.workers, wgs = ez.wgs;

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

  // AC(k) draws about k times the fill: pools scale with it
  double pf = opt.pool_factor * samples;
  int retries = 0;
  Rec *pool = nullptr;
  int32_t *frow = nullptr;
  double *fval = nullptr;
  char *arena = nullptr;
  int64_t pool_cap = 0, f_cap = 0, arena_cap = 0;
  unsigned long long htops[3] = {0, 0, 0};
  double ms_elim = 0.0;
  for (;;) {
    const PoolSizing ps = pool_sizing(ntot, nnz, pf, workers);
    const int pg_chunk = ps.pg_chunk, f_chunk = ps.f_chunk;
    pool_cap = ps.pool_cap;
    f_cap = ps.f_cap;
    arena_cap = ps.arena_cap;
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
    ea.team_min = nteam > 0 && samples == 1 ? kTeamMin : 0;
    ea.samples = samples;
    ea.team_wg0 = wgs;
    if (forced && forced_count > 0) {
      int32_t *df = tmp.alloc<int32_t>(forced_count, "forced choices");
      chk(hipMemcpyAsync(df, forced, forced_count * sizeof(int32_t), hipMemcpyHostToDevice, s),
          "upload");
      ea.forced = df;
      ea.forced_stride = forced_stride;
      ea.forced_count = forced_count;
    }
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
          const size_t k = (size_t)(it - tmp.ptrs.begin());
          tmp.total -= (int64_t)tmp.sizes[k];
          tmp.sizes.erase(tmp.sizes.begin() + (std::ptrdiff_t)k);
          tmp.ptrs.erase(it);
          dev_free(p);
        }
      }
      continue;
    }
    if (herr) {
      throw Err{herr, herr == PARAC_ETIMEOUT ? "elimination watchdog expired"
                      : herr == PARAC_EPOOL  ? "fill pool exhausted after retries"
                      : herr == PARAC_EINVAL ? "a forced partner offset is out of range"
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
  // scheduler invariants (besides the kernel's own: a counter never goes
  // below zero, a queue shard never takes more labels than it holds, so no
  // vertex is enqueued twice): every vertex was eliminated, i.e. wrote its
  // column count (-1 until then, read here as the largest unsigned value)
  if (ntot > 0 && hst[1] > (unsigned long long)ntot)
    throw Err{PARAC_EINTERNAL, "a vertex was not eliminated"};
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
    narrow_plan(F, n, depth, tmp, s);
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
      // the sweeps leave the narrow levels to k_narrow: forward the units of
      // the levels below, backward those after the narrow levels' units
      if (dir == 0)
        F->nwide_f = F->nf.nlev ? (int32_t)read1(uoff + F->hlptr[F->nlev0], s) : (int32_t)nu;
      else
        F->nskip_b = F->nb.nlev ? (int32_t)read1(uoff + (n - F->hlptr[F->nlev0]), s) : 0;
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
  S.narrow_levels = F->nf.nlev;

  // keep the handle's arrays; everything else is freed with `tmp`
  for (void *p : {(void *)F->perm, (void *)F->iperm, (void *)F->colptr, (void *)F->rowind,
                  (void *)F->val, (void *)F->D, (void *)F->Dinv, (void *)F->Dinv32,
                  (void *)F->lev, (void *)F->order, (void *)F->root, (void *)F->lptr,
                  (void *)F->src, (void *)F->flist, (void *)F->blist, (void *)F->zero,
                  (void *)F->task_f, (void *)F->task_b, (void *)F->ctr, (void *)F->serr,
                  (void *)F->lf_ptr, (void *)F->lf_idx, (void *)F->lf_val, (void *)F->lf_val32,
                  (void *)F->lb_ptr, (void *)F->lb_idx, (void *)F->lb_val, (void *)F->lb_val32,
                  (void *)F->nf.hdr, (void *)F->nf.rows, (void *)F->nf.lw, (void *)F->nf.smap,
                  (void *)F->nf.nidx, (void *)F->nb.hdr, (void *)F->nb.rows, (void *)F->nb.lw,
                  (void *)F->nb.smap, (void *)F->nb.nidx})
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
  a.nf = f->nf;
  a.nb = f->nb;
  const bool narrow = f->nf.nlev > 0;
  a.np0 = narrow ? f->np0 : (int32_t)f->n;
  a.nwide_f = narrow ? f->nwide_f : f->ntask_f;
  a.nskip_b = narrow ? f->nskip_b : 0;
  return a;
}

// the sweeps take every level (slots of several columns, or work vectors
// other than the factor's own: no narrow-level kernel for them)
static void wide_only(SolveArgs &a) {
  a.nf = NarrowDir{};
  a.nb = NarrowDir{};
  a.np0 = (int32_t)a.n;
  a.nwide_f = a.ntask_f;
  a.nskip_b = 0;
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
  void **pv = mixed ? &f->npv32 : &f->npv64;
  if (*py) return;
  const size_t el = mixed ? 4 : 8;
  const int64_t m = std::max<int64_t>(f->ntot, 1), c = std::max<int64_t>(f->ncs, 1);
  const int64_t nv = std::max<int64_t>(f->nf.nslots + f->nb.nslots, 1);
  chk(dev_alloc(py, m * el), "work vector");
  f->owned.push_back(*py);
  chk(dev_alloc(px, m * el), "work vector");
  f->owned.push_back(*px);
  chk(dev_alloc(pc, c * el), "chunk sums");
  f->owned.push_back(*pc);
  chk(dev_alloc(pv, nv * el), "narrow products");
  f->owned.push_back(*pv);
  f->bytes += (int64_t)((2 * m + c + nv) * el);
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

// columns of the sweep state for nc columns in slots of up to kMaxSweepCols
// (the last slot of a block may be partly filled)
constexpr int kMaxSweepCols = 8;
static int padded_cols(int nc) { return (nc + kMaxSweepCols - 1) / kMaxSweepCols * kMaxSweepCols; }

static void ensure_cwork(parac_factor_t f, int prec, int nc_, hipStream_t s) {
  const int k = prec_slot(prec);
  const int nc = padded_cols(nc_);
  if (f->ccols[k] >= nc) return;
  const size_t el = k ? 4 : 8;
  const int64_t m0 = std::max<int64_t>(f->ntot, 1), c0 = std::max<int64_t>(f->ncs, 1);
  for (void **pp : {&f->cy[k], &f->cx[k], &f->ccs[k], (void **)&f->cctr[k]}) {
    if (!*pp) continue;
    f->owned.erase(std::remove(f->owned.begin(), f->owned.end(), *pp), f->owned.end());
    dev_free(*pp);
    *pp = nullptr;
  }
  f->bytes -= f->ccols[k] * (int64_t)((2 * m0 + c0) * el + 2 * sizeof(int32_t));
  f->ccols[k] = 0;
  chk(dev_alloc(&f->cy[k], (size_t)(m0 * nc) * el), "column work vector");
  f->owned.push_back(f->cy[k]);
  chk(dev_alloc(&f->cx[k], (size_t)(m0 * nc) * el), "column work vector");
  f->owned.push_back(f->cx[k]);
  chk(dev_alloc(&f->ccs[k], (size_t)(c0 * nc) * el), "column chunk sums");
  f->owned.push_back(f->ccs[k]);
  chk(dev_alloc((void **)&f->cctr[k], (size_t)(2 * nc) * sizeof(int32_t)), "column counters");
  f->owned.push_back(f->cctr[k]);
  f->ccols[k] = nc;
  f->bytes += nc * (int64_t)((2 * m0 + c0) * el + 2 * sizeof(int32_t));
  reset_cwork(f, prec, s);
}

struct Batch;
static void build_cols(Batch &bt, parac_factor_t f, int nc, const parac_block_shape &shp,
                       const double *r, int64_t ldr, double *z, int64_t ldz, int prec,
                       const int *skip, int skip_stride, hipStream_t s);
static void apply_cols(parac_factor_t f, int nc, const parac_block_shape &shp, const double *r,
                       int64_t ldr, double *z, int64_t ldz, int prec, hipStream_t s,
                       float *ms = nullptr);

static bool shape_ok(const parac_block_shape &c, int prec) {
  return ready_cols_ok(prec, c.cols_per_sweep) && c.workgroups >= 0 &&
         c.workgroups <= kReadyGroupsMax;
}

// ---------------------------------------------------------------------------
// block-shape autotuner: the block apply of nc columns runs one sweep slot per
// chunk of cols_per_sweep columns (the factor is read once per chunk); which
// chunk width is fastest depends on the factor and the precision.  On first
// use for (columns, precision) the candidates are timed on the caller's
// vectors (every shape gives the same bits, so the timing runs are ordinary
// applies) within a bounded budget, and the choice is kept in the handle and
// in a JSON cache file keyed by device architecture, precision, columns and
// the factor's shape class, so that later processes skip the timing.
// ---------------------------------------------------------------------------
constexpr double kTuneBudgetMs = 4000.0;  // stop timing further candidates past this

static std::mutex g_shape_mu;
static bool g_shape_loaded = false;
static std::map<std::string, parac_block_shape> g_shape_cache;

static std::string shape_cache_path() {
  const char *e = getenv("PARAC_SHAPE_CACHE");
  if (e) return std::string(e);  // empty: no cache file
  const char *h = getenv("HOME");
  if (!h || !*h) return std::string();
  return std::string(h) + "/.cache/parac_block_shapes.json";
}

// the cache file: one object, "key": [cols_per_sweep, workgroups, ms]
static void shape_cache_load() {
  if (g_shape_loaded) return;
  g_shape_loaded = true;
  const std::string path = shape_cache_path();
  if (path.empty()) return;
  FILE *fp = fopen(path.c_str(), "r");
  if (!fp) return;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof(buf), fp)) > 0) text.append(buf, got);
  fclose(fp);
  size_t i = 0;
  for (;;) {
    const size_t k0 = text.find('"', i);
    if (k0 == std::string::npos) break;
    const size_t k1 = text.find('"', k0 + 1);
    const size_t b0 = text.find('[', k1);
    const size_t b1 = text.find(']', b0);
    if (k1 == std::string::npos || b0 == std::string::npos || b1 == std::string::npos) break;
    int cps = 0, wg = 0;
    double ms = 0.0;
    if (sscanf(text.c_str() + b0, "[%d , %d , %lf]", &cps, &wg, &ms) == 3) {
      parac_block_shape sh{};
      sh.cols_per_sweep = cps;
      sh.workgroups = wg;
      sh.source = 2;
      sh.ms = (float)ms;
      g_shape_cache[text.substr(k0 + 1, k1 - k0 - 1)] = sh;
    }
    i = b1 + 1;
  }
}

static void shape_cache_store() {
  const std::string path = shape_cache_path();
  if (path.empty()) return;
  const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
  FILE *fp = fopen(tmp.c_str(), "w");
  if (!fp) return;
  fprintf(fp, "{\n");
  size_t k = 0;
  for (const auto &kv : g_shape_cache)
    fprintf(fp, "  \"%s\": [%d, %d, %.4f]%s\n", kv.first.c_str(), kv.second.cols_per_sweep,
            kv.second.workgroups, (double)kv.second.ms,
            ++k < g_shape_cache.size() ? "," : "");
  fprintf(fp, "}\n");
  const bool ok = fclose(fp) == 0;
  if (!ok || rename(tmp.c_str(), path.c_str()) != 0) remove(tmp.c_str());
}

static int log2_bucket(double v) { return v < 1.0 ? 0 : (int)floor(log2(v)); }

// architecture, precision, columns and the factor's shape class: size,
// depth and entries per row, each to the nearest power of two below
static std::string shape_key(parac_factor_t f, int nc, int prec) {
  int dev = 0;
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t c = arch.find(':');
    if (c != std::string::npos) arch = arch.substr(0, c);
  }
  char key[256];
  snprintf(key, sizeof(key), "%s|%s|cols%d|n2^%d|depth2^%d|epr2^%d", arch.c_str(),
           prec == PARAC_PREC_MIXED ? "fp32" : "fp64", nc, log2_bucket((double)f->ntot),
           log2_bucket((double)f->depth),
           log2_bucket((double)f->nnz_off / (double)std::max<int64_t>(f->ntot, 1)));
  return key;
}

// candidates in the order they are timed: the widest chunks first (the
// likeliest winners when the factor dominates the traffic)
static std::vector<int> tune_candidates(int nc, int prec) {
  std::vector<int> c;
  for (int cps : {8, 4, 2, 1})
    if (ready_cols_ok(prec, cps) && (cps == 1 || cps <= nc)) c.push_back(cps);
  return c;
}

// the shape for (nc, prec): fixed by the caller, tuned earlier, cached, or
// timed now on r -> z, which then holds the apply's result (*applied set)
static parac_block_shape block_shape(parac_factor_t f, int nc, int prec, const double *r,
                                     int64_t ldr, double *z, int64_t ldz, hipStream_t s,
                                     bool *applied = nullptr) {
  if (applied) *applied = false;
  const auto key = std::make_pair(nc, prec_slot(prec));
  auto it = f->shapes.find(key);
  if (it != f->shapes.end()) return it->second;
  const std::string ck = shape_key(f, nc, prec);
  {
    std::lock_guard<std::mutex> lk(g_shape_mu);
    shape_cache_load();
    auto c = g_shape_cache.find(ck);
    if (c != g_shape_cache.end() && shape_ok(c->second, prec)) {
      parac_block_shape sh = c->second;
      sh.source = 2;
      f->shapes[key] = sh;
      return sh;
    }
  }
  parac_block_shape best{};
  best.cols_per_sweep = 1;
  best.source = 1;
  best.ms = 0.f;
  if (f->n == 0) {
    f->shapes[key] = best;
    return best;
  }
  double spent = 0.0;
  bool have = false;
  for (int cps : tune_candidates(nc, prec)) {
    parac_block_shape cand{};
    cand.cols_per_sweep = cps;
    cand.workgroups = 0;
    float ms = 0.f;
    apply_cols(f, nc, cand, r, ldr, z, ldz, prec, s, &ms);
    spent += ms;
    if (verbose()) {
      fprintf(stderr, "parac block shape: %d columns, %d per sweep slot: %.3f ms\n", nc, cps,
              (double)ms);
      fflush(stderr);
    }
    if (!have || ms < best.ms) {
      best = cand;
      best.ms = ms;
      have = true;
    }
    if (applied) *applied = true;
    if (spent > kTuneBudgetMs) break;
  }
  best.source = 1;
  f->shapes[key] = best;
  {
    std::lock_guard<std::mutex> lk(g_shape_mu);
    g_shape_cache[ck] = best;
    shape_cache_store();
  }
  return best;
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
                               const std::vector<parac_factor_t> &fs, hipStream_t s,
                               int wgcap = 0) {
  const int64_t cap = wgcap > 0 ? wgcap : kReadyGroupsDefault;
  const int ns = (int)as.size();
  std::vector<int32_t> g(ns);
  int32_t gmax = 0;
  for (int k = 0; k < ns; ++k) {
    const int64_t nt = std::max(fs[k]->ntask_f, fs[k]->ntask_b);
    const int64_t waves = kReadyThreads / 64;
    g[k] = (int32_t)std::min<int64_t>((nt + waves - 1) / waves, cap);
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
  B.nslots_max = 0;
  for (const ApplySlot &a : as)
    if (a.a.nf.nlev > 0) B.nslots_max = std::max(B.nslots_max, a.a.nf.nslots + a.a.nb.nslots);
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
    as[k].pv = prec == PARAC_PREC_MIXED ? f->npv32 : f->npv64;
    as[k].ctr = f->ctr;
    as[k].z = ps[k].z;
    as[k].ncols = 1;
    as[k].skip_n = 1;
    as[k].skip_stride = 0;
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
  as[0].pv = prec == PARAC_PREC_MIXED ? f->npv32 : f->npv64;
  as[0].ctr = f->ctr;
  as[0].z = z;
  as[0].ncols = 1;
  as[0].skip_n = 1;
  as[0].skip_stride = 0;
  Batch bt;
  build_apply_tables(bt, as, {f}, s);
  bt.B.nslots = 1;
  chk(slots_apply(bt.B, prec, s), "apply");
  chk(hipStreamSynchronize(s), "sync");
  check_sweeps(f, prec, s);
}

// the column sweeps of a block: columns [j c, (j + 1) c) of r (row stride
// ldr) into the same columns of z, c = shp.cols_per_sweep columns per sweep
// slot over the same factor; skip (optional) gives column i's done flag at
// skip + i * skip_stride (a slot is skipped once all of its columns are done)
static void build_cols(Batch &bt, parac_factor_t f, int nc, const parac_block_shape &shp,
                       const double *r, int64_t ldr, double *z, int64_t ldz, int prec,
                       const int *skip, int skip_stride, hipStream_t s) {
  ensure_cwork(f, prec, nc, s);
  const int k = prec_slot(prec);
  const size_t el = k ? 4 : 8;
  const int cc = shp.cols_per_sweep;
  const int64_t m = std::max<int64_t>(f->ntot, 1), c = std::max<int64_t>(f->ncs, 1);
  const int ns = (nc + cc - 1) / cc;
  std::vector<ApplySlot> as(ns);
  for (int j = 0; j < ns; ++j) {
    const int c0 = j * cc;
    as[j].a = solve_args(f, skip ? skip + (int64_t)c0 * skip_stride : f->zero);
    wide_only(as[j].a);
    as[j].pv = nullptr;
    as[j].ldr = ldr;
    as[j].ldz = ldz;
    as[j].r = r + c0;
    as[j].y = (char *)f->cy[k] + (size_t)(c0 * m) * el;
    as[j].x = (char *)f->cx[k] + (size_t)(c0 * m) * el;
    as[j].cs = (char *)f->ccs[k] + (size_t)(c0 * c) * el;
    as[j].ctr = f->cctr[k] + 2 * j;
    as[j].z = z + c0;
    as[j].ncols = std::min(cc, nc - c0);
    as[j].skip_n = skip ? as[j].ncols : 1;
    as[j].skip_stride = skip ? skip_stride : 0;
  }
  build_apply_tables(bt, as, std::vector<parac_factor_t>(ns, f), s, shp.workgroups);
  bt.B.nslots = ns;
  bt.B.cc = cc;
}

static void check_col_sweeps(parac_factor_t f, int prec, hipStream_t s) {
  if (read1(f->serr, s) == 0) return;
  reset_cwork(f, prec, s);
  chk(hipMemsetAsync(f->serr, 0, sizeof(int), s), "memset");
  chk(hipStreamSynchronize(s), "sync");
  throw Err{PARAC_ETIMEOUT, "triangular sweep watchdog expired"};
}

// one block apply; ms (optional) receives its time on the stream
static void apply_cols(parac_factor_t f, int nc, const parac_block_shape &shp, const double *r,
                       int64_t ldr, double *z, int64_t ldz, int prec, hipStream_t s, float *ms) {
  Batch bt;
  build_cols(bt, f, nc, shp, r, ldr, z, ldz, prec, nullptr, 0, s);
  Events ev;
  if (ms) {
    ev.create();
    chk(hipEventRecord(ev.e[0], s), "event");
  }
  chk(slots_apply(bt.B, prec, s), "column sweeps");
  if (ms) chk(hipEventRecord(ev.e[1], s), "event");
  chk(hipStreamSynchronize(s), "sync");
  check_col_sweeps(f, prec, s);
  if (ms) *ms = (float)ev.ms(0, 1);
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
    if (verbose() && launched % 64 == 0) {
      fprintf(stderr, "parac pcg: %d iterations\n", hist[0]);
      fflush(stderr);
    }
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
    // the block apply's shape (timed on r -> z on first use: part of this
    // call's time), then one batch of sweep slots for the whole solve, a
    // slot skipped once all of its columns have converged
    const parac_block_shape shp = block_shape(f, nc, o.precision, r, nc, z, nc, s);
    Batch cols;
    if (n > 0) build_cols(cols, f, nc, shp, r, nc, z, nc, o.precision, bist + 1, 4, s);
    auto apply = [&]() {
      if (n > 0) chk(slots_apply(cols.B, o.precision, s), "column sweeps");
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
      if (verbose()) {
        fprintf(stderr, "parac pcg: %d columns, %d iterations, %d columns iterating\n", nc,
                launched, g[0]);
        fflush(stderr);
      }
      if (g[1]) break;
    }
    chk(bpcg_launch_true_res(n, nc, A->rowptr, A->col, A->val, x + c0, nrhs, b + c0, nrhs, q,
                             partial, bst, bist, gfl, s),
        "bpcg_true_res");
    mark(true);  // last: end
    if (n > 0) check_col_sweeps(f, o.precision, s);
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
      for (void *ptr : f->owned) dev_free(ptr);
      delete f;
    }
  }
};

// peak device bytes of one request: its device copy (CSR, b, perm), the
// factorisation at its peak (the sizing parac_factor uses, pool factor 4; an
// SDDM request has a ground vertex), and the PCG vectors and tables
int64_t serve_estimate(int64_t n, int64_t nnz, int prec) {
  const int64_t request = 8 * (n + 1) + 12 * nnz + 8 * n + 4 * n;
  const int64_t pcg = 5 * 8 * n + 8 * kSlotMaxBlocks + 4096;
  return request + factor_peak_bytes(n, nnz, 1, false, prec == PARAC_PREC_MIXED, 0) + pcg;
}

// one request from upload to result, on the calling worker's stream: the
// device copy of the request, parac_factor's factorisation, and parac_pcg's
// single-system PCG (the same code, so the result is the same bits as those
// two calls give for the request alone).  `bytes` is called with the bytes
// the system holds once it is set up.
template <class OnBytes>
void serve_one(const parac_request &rq, const parac_serve_opts &o, parac_result &res,
               hipStream_t s, OnBytes on_bytes) {
  const int64_t n = rq.A.n, nnz = rq.A.nnz;
  if (n < 0 || nnz < 0 || rq.A.on_device ||
      (n > 0 && (!rq.A.rowptr || !rq.A.col || !rq.A.val || !rq.b || !rq.x)))
    throw Err{PARAC_EINVAL, "a request needs host CSR arrays, b and x"};
  ServeSlot sl;
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
  fo.keep_fp32 = o.precision == PARAC_PREC_MIXED;
  fo.timeout_s = 30.0;
  sl.f = factor_impl(&dA, &fo, s);
  if (sl.f->mode == PARAC_MODE_LAPLACIAN) check_consistent(sl.f, b, s);
  double *x = M.alloc<double>(n, "x");
  PcgWork w{};
  w.r = M.alloc<double>(n, "r");
  w.z = M.alloc<double>(n, "z");
  w.p = M.alloc<double>(n, "p");
  w.q = M.alloc<double>(n, "q");
  w.partial = M.alloc<double>(slot_blocks(n), "partials");
  w.dst = M.alloc<double>(8, "pcg scalars");
  w.ist = M.alloc<int>(4, "pcg flags");
  w.tables = nullptr;
  w.events = false;
  res.bytes_resident = M.total + sl.f->bytes;
  on_bytes(res.bytes_resident);
  parac_pcg_opts po{};
  po.rtol = rq.rtol >= 0 ? rq.rtol : 1e-6;
  po.maxit = o.maxit;
  po.precision = o.precision;
  po.check_every = o.check_every;
  parac_pcg_stats st{};
  const int rc = pcg_run(&dA, sl.f, b, x, po, &st, s, w);
  if (n > 0) chk(hipMemcpyAsync(rq.x, x, n * sizeof(double), hipMemcpyDeviceToHost, s), "result");
  chk(hipStreamSynchronize(s), "sync");
  res.status = rc;
  res.iterations = st.iterations;
  res.true_relres = st.true_relres;
}

}  // namespace

// Continuous serving: requests are admitted in arrival order while fewer than
// `streams` systems are in flight and the memory budget holds the request's
// peak footprint; each admitted system runs from upload to result on a
// worker thread with its own stream, so systems overlap on the device and a
// small system never waits for a large one's launches.
static int serve_impl(const parac_request *reqs, int64_t nreq, const parac_serve_opts &o,
                      parac_result *out) {
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  auto now = [&]() { return std::chrono::duration<double>(clk::now() - t0).count(); };
  const int nstreams = std::max(1, o.max_slots);
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

  struct Job {
    int64_t req;
    int64_t est;
  };
  std::mutex m;
  std::condition_variable cv_work, cv_done;
  std::deque<Job> todo;
  bool stop = false;
  size_t reserved = 0;
  int inflight = 0;
  int64_t finished = 0;

  auto worker = [&]() {
    (void)hipSetDevice(dev);
    hipStream_t ws = nullptr;
    const bool have_stream = hipStreamCreate(&ws) == hipSuccess;
    // this thread's device memory comes and goes in its stream's order
    if (have_stream) g_alloc_stream = ws;
    for (;;) {
      Job job;
      {
        std::unique_lock<std::mutex> lk(m);
        cv_work.wait(lk, [&] { return stop || !todo.empty(); });
        if (todo.empty()) break;
        job = todo.front();
        todo.pop_front();
      }
      parac_result &res = out[job.req];
      int64_t held = job.est;
      try {
        if (!have_stream) throw Err{PARAC_EDEVICE, "serving stream"};
        serve_one(reqs[job.req], o, res, ws, [&](int64_t bytes) {
          // once set up, the reservation shrinks to the bytes actually held
          std::lock_guard<std::mutex> lk(m);
          reserved = reserved - (size_t)held + (size_t)bytes;
          held = bytes;
        });
      } catch (Err &e) {
        res.status = e.code;
      } catch (std::exception &) {
        res.status = PARAC_EINTERNAL;
      }
      if (ws) (void)hipStreamSynchronize(ws);
      {
        std::lock_guard<std::mutex> lk(m);
        res.t_done = now();
        reserved -= (size_t)held;
        --inflight;
        ++finished;
      }
      cv_done.notify_one();
    }
    g_alloc_stream = nullptr;
    if (ws) {
      (void)hipStreamSynchronize(ws);
      (void)hipStreamDestroy(ws);
    }
  };
  std::vector<std::thread> pool;
  struct Joiner {
    std::mutex &m;
    std::condition_variable &cv;
    bool &stop;
    std::vector<std::thread> &t;
    ~Joiner() {
      {
        std::lock_guard<std::mutex> lk(m);
        stop = true;
      }
      cv.notify_all();
      for (auto &th : t)
        if (th.joinable()) th.join();
    }
  } joiner{m, cv_work, stop, pool};
  for (int k = 0; k < nstreams; ++k) pool.emplace_back(worker);

  int64_t next = 0;
  std::unique_lock<std::mutex> lk(m);
  while (finished < nreq) {
    // admission in arrival order
    const double t = now();
    while (next < nreq && reqs[order[next]].arrival_s <= t) {
      const int64_t i = order[next];
      const int64_t est = serve_estimate(std::max<int64_t>(reqs[i].A.n, 0),
                                         std::max<int64_t>(reqs[i].A.nnz, 0), o.precision);
      if ((size_t)est > budget) {
        out[i].status = PARAC_ENOMEM;
        out[i].t_admit = out[i].t_done = t;
        ++next;
        ++finished;
        continue;
      }
      if (inflight >= nstreams || reserved + (size_t)est > budget) break;
      reserved += (size_t)est;
      ++inflight;
      out[i].t_admit = t;
      todo.push_back(Job{i, est});
      cv_work.notify_one();
      ++next;
    }
    if (finished >= nreq) break;
    // wait for a completion or the next arrival
    double wait = 0.05;
    if (next < nreq && inflight < nstreams)
      wait = std::min(wait, std::max(0.0, reqs[order[next]].arrival_s - now()));
    cv_done.wait_for(lk, std::chrono::duration<double>(wait));
  }
  lk.unlock();
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

parac_status parac_debug_factor_forced(const parac_csr *A, const parac_factor_opts *o,
                                       const int32_t *forced, int32_t stride, int64_t count,
                                       void *stream, parac_factor_t *out) {
  if (!out) {
    g_last_error = "null output handle";
    return PARAC_EINVAL;
  }
  *out = nullptr;
  if (stride <= 0 || count < 0 || (count > 0 && !forced)) {
    g_last_error = "bad forced-choice table";
    return PARAC_EINVAL;
  }
  try {
    *out = factor_impl(A, o, (hipStream_t)stream, forced, stride, count);
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
        bool applied = false;
        const parac_block_shape shp =
            block_shape(f, nc, precision, r + c0, nrhs, z + c0, nrhs, s, &applied);
        if (!applied) apply_cols(f, nc, shp, r + c0, nrhs, z + c0, nrhs, precision, s);
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
      (shape && !shape_ok(*shape, precision))) {
    g_last_error = "bad block shape arguments";
    return PARAC_EINVAL;
  }
  const auto key = std::make_pair((int)cols, prec_slot(precision));
  if (shape) {
    parac_block_shape sh = *shape;
    sh.source = 0;
    sh.ms = 0.f;
    f->shapes[key] = sh;
  } else {
    f->shapes.erase(key);
  }
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
    g_last_error = "no block shape fixed, timed or cached yet for these columns and precision";
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
  if (opt.max_slots == 0) opt.max_slots = 4;
  if (opt.maxit <= 0) opt.maxit = 10000;
  if (opt.check_every <= 0) opt.check_every = 4;
  if (opt.max_slots < 1 || opt.max_slots > 64 ||
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

parac_status parac_order(const parac_csr *A, int32_t kind, uint64_t seed, int32_t *perm,
                         int32_t *rounds, void *stream) {
  if (!A || A->n < 0 || A->nnz < 0 || (A->n > 0 && (!A->rowptr || !A->col || !perm)) ||
      (kind != PARAC_ORDER_RANDOM && kind != PARAC_ORDER_NNZ && kind != PARAC_ORDER_MIS)) {
    g_last_error = "bad order arguments";
    return PARAC_EINVAL;
  }
  if (A->n > INT32_MAX) {
    g_last_error = "too many vertices for 32-bit labels";
    return PARAC_EINVAL;
  }
  try {
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = A->n, nnz = A->nnz;
    if (rounds) *rounds = 0;
    if (n == 0) return PARAC_OK;
    Scratch tmp;
    const int64_t *rowptr = A->rowptr;
    const int32_t *col = A->col;
    int32_t *dperm = perm;
    if (!A->on_device) {
      int64_t *r = tmp.alloc<int64_t>(n + 1, "rowptr");
      chk(hipMemcpyAsync(r, A->rowptr, (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s), "copy");
      rowptr = r;
      if (kind == PARAC_ORDER_MIS) {
        int32_t *c = tmp.alloc<int32_t>(nnz, "col");
        chk(hipMemcpyAsync(c, A->col, nnz * sizeof(int32_t), hipMemcpyHostToDevice, s), "copy");
        col = c;
      }
      dperm = tmp.alloc<int32_t>(n, "perm");
    }
    uint64_t *key = tmp.alloc<uint64_t>(n, "keys");
    uint64_t *key2 = tmp.alloc<uint64_t>(n, "keys");
    int32_t *val = tmp.alloc<int32_t>(n, "values");
    int32_t *val2 = tmp.alloc<int32_t>(n, "values");
    const int64_t nh = 16 * order_tiles(n);
    int32_t *hist = tmp.alloc<int32_t>(nh, "histograms");
    int64_t *off = tmp.alloc<int64_t>(nh + 1, "offsets");
    const size_t scan_bytes = scan_tmp_bytes(nh + 1);
    void *scan_tmp = tmp.alloc<char>((int64_t)scan_bytes, "scan");
    chk(launch_order_keys(n, rowptr, seed, kind, key, val, s), "order keys");
    int bits = kind == PARAC_ORDER_RANDOM ? 64 : 44;
    if (kind == PARAC_ORDER_MIS) {
      int32_t *round = tmp.alloc<int32_t>(n, "rounds");
      unsigned long long *placed = tmp.alloc<unsigned long long>(1, "placed");
      chk(launch_fill_u32((uint32_t *)round, 0xffffffffu, n, s), "fill");
      chk(launch_fill_u64((uint64_t *)placed, 0, 1, s), "fill");
      unsigned long long done = 0;
      int r = 0;
      // at least the unplaced vertex of least (priority, index) joins each
      // round, so the loop ends
      while ((int64_t)done < n) {
        if (r >= (1 << 20)) throw Err{PARAC_EINTERNAL, "too many rounds"};
        chk(launch_mis_round(n, rowptr, col, key, round, r, placed, s), "mis round");
        done = read1(placed, s);
        ++r;
      }
      chk(launch_mis_key(n, round, key, s), "mis key");
      bits = 64;
      if (rounds) *rounds = r;
    }
    chk(radix_sort_pairs(n, bits, key, val, key2, val2, hist, off, scan_tmp, scan_bytes, s), "sort");
    chk(launch_rank_to_perm(n, val, dperm, s), "perm");
    if (!A->on_device)
      chk(hipMemcpyAsync(perm, dperm, n * sizeof(int32_t), hipMemcpyDeviceToHost, s), "copy");
    chk(hipStreamSynchronize(s), "sync");
    return PARAC_OK;
  } catch (Err &e) {
    return status_from(e);
  }
}

int64_t parac_device_bytes(int32_t what) {
  std::lock_guard<std::mutex> lk(g_mem_mu);
  if (what == 0) return g_mem_live;
  if (what == 1) return g_mem_peak;
  if (what == 2) {
    g_mem_peak = g_mem_live;
    return g_mem_peak;
  }
  return -1;
}

void parac_factor_free(parac_factor_t f) {
  if (!f) return;
  for (void *p : f->owned) dev_free(p);
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
