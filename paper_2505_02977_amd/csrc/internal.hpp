// internal.hpp -- host-side types shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <map>
#include <utility>
#include <vector>

#include "parac.h"

namespace parac {

// fill record: an edge (target = the smaller label, other) of weight w,
// produced by pivot src.  Stored at its target's inbox.
struct __attribute__((aligned(16))) Rec {
  int32_t other;
  int32_t src;
  double w;
};

// inbox geometry: page 0 (kInline records) is preallocated per vertex; page
// j >= 1 holds kInline << j records and is allocated on first use, its base
// published in the vertex's page table (kPages - 1 entries).
constexpr int kInline = 8;
constexpr int kPages = 17;             // capacity 8 (2^17 - 1) ~ 1M records
constexpr int kSubQueues = 64;         // ready-queue shards (power of two)
constexpr int kTailStride = 32;        // ints between shard tails (128 B)
constexpr int kElimWaves = 8;          // waves per workgroup of the persistent elimination
constexpr int kTeamMin = 128;          // gathered entries above which a team eliminates
constexpr int kTeamShare = 16;         // one workgroup in this many is a team
constexpr int kFChunk = 2048;          // largest factor-entry reservation
constexpr int kPageChunk = 4096;       // largest fill-record reservation

struct ElimArgs {
  int32_t ntot;
  const int64_t *uptr;
  const int32_t *uidx;
  const double *uw;
  int32_t *dp;
  int32_t *q;          // kSubQueues shards of cap_q slots
  int32_t *qtail;      // shard tails, kTailStride apart
  int32_t *qhead;      // shard claim counters, kTailStride apart
  int32_t cap_q;
  int32_t *fill_cnt;
  Rec *inl;            // ntot * kInline
  int32_t *ptab;       // ntot * (kPages - 1)
  Rec *pool;
  int64_t pool_cap;
  unsigned long long *pool_top;
  int32_t *frow;
  double *fval;
  int64_t f_cap;
  unsigned long long *f_top;
  int64_t *colstart;
  int32_t *colcnt;
  double *D;
  int32_t *lev;
  char *arena;         // scratch of the large-neighbourhood path
  int64_t arena_cap;
  unsigned long long *arena_top;
  uint64_t seed;
  int *err;
  uint64_t timeout_ticks;
  int32_t nworkers;
  int32_t pg_chunk;    // fill records a worker reserves at a time
  int32_t f_chunk;     // factor entries a worker reserves at a time
  int32_t *done;       // per-shard eliminated-pivot counts, kTailStride apart
  int64_t stop_at;     // the wide kernel leaves once this many are eliminated
  int32_t *tq;         // tail queue [ntot] (-1 = empty slot)
  int32_t *tq_head, *tq_tail, *tq_count;  // tail claim, append, pivots left
  int32_t *bq;         // team queue [bq_cap] (-1 = empty slot)
  int32_t *bq_head, *bq_tail;  // team claim, append
  int32_t bq_cap;
  int32_t team_min;    // pivots with more gathered entries go to teams (0: none)
  int32_t samples;     // AC(k): sampling slots per merged neighbour (1: plain)
  int32_t team_wg0;    // workgroups from this index on are teams
  // test hook (worked examples): forced[k * forced_stride + s], when present
  // and >= 0, is the partner offset of slot s of pivot k in place of a draw
  const int32_t *forced;
  int32_t forced_stride;
  int64_t forced_count;
};

// --- launchers (setup.hip) ---
// input errors are min-reduced into *errkey (all ones = no error); the low
// byte holds -status
hipError_t launch_check_csr(int64_t n, int64_t nnz, const int64_t *rowptr, const int32_t *col,
                            const double *val, double *excess, unsigned long long *errkey,
                            int *any_excess, hipStream_t s);
hipError_t launch_check_perm(int64_t n, const int32_t *perm, int32_t *seen, int32_t *iperm,
                             unsigned long long *errkey, hipStream_t s);
hipError_t launch_upper_count(int64_t n, const int64_t *rowptr, const int32_t *col,
                              const double *val, const int32_t *perm, const double *excess,
                              int sddm, int32_t *ucnt, int32_t *dp, hipStream_t s);
hipError_t launch_upper_fill(int64_t n, const int64_t *rowptr, const int32_t *col,
                             const double *val, const int32_t *perm, const double *excess,
                             int sddm, const int64_t *uptr, int32_t *uidx, double *uw,
                             hipStream_t s);
hipError_t launch_queue_init(int64_t ntot, const int32_t *dp, int32_t *q, int32_t *qtail,
                             int32_t cap_q, hipStream_t s);
// exclusive scan of int32 counts into int64 offsets (out[n] = total)
hipError_t scan_counts(const int32_t *cnt, int64_t *out, int64_t n, void *tmp, size_t tmp_bytes,
                       hipStream_t s);
size_t scan_tmp_bytes(int64_t n);

// --- order.hip (elimination orders on the device) ---
int64_t order_tiles(int64_t n);
hipError_t launch_order_keys(int64_t n, const int64_t *rowptr, uint64_t seed, int kind,
                             uint64_t *key, int32_t *val, hipStream_t s);
hipError_t launch_mis_round(int64_t n, const int64_t *rowptr, const int32_t *col,
                            const uint64_t *pri, int32_t *round, int r,
                            unsigned long long *placed, hipStream_t s);
hipError_t launch_mis_key(int64_t n, const int32_t *round, uint64_t *key, hipStream_t s);
// stable LSD radix sort of (key, val) by the low `bits` bits of key; hist
// holds 16 * order_tiles(n) counts, off one more offset
hipError_t radix_sort_pairs(int64_t n, int bits, uint64_t *key, int32_t *val, uint64_t *key2,
                            int32_t *val2, int32_t *hist, int64_t *off, void *scan_tmp,
                            size_t scan_bytes, hipStream_t s);
hipError_t launch_rank_to_perm(int64_t n, const int32_t *val, int32_t *perm, hipStream_t s);

// --- eliminate.hip ---
hipError_t launch_eliminate(const ElimArgs &a, int wgs, hipStream_t s);
int eliminate_max_workgroups();

// --- finalize.hip ---
hipError_t launch_compact_csc(int64_t ntot, const int64_t *colstart, const int32_t *colcnt,
                              const int32_t *frow, const double *fval, const int64_t *colptr,
                              int32_t *rowind, double *val, hipStream_t s);
hipError_t launch_row_count(int64_t nnz, const int32_t *rowind, int32_t *rowcnt, hipStream_t s);
hipError_t launch_transpose(int64_t ntot, const int64_t *colptr, const int32_t *rowind,
                            const double *val, const int64_t *rowptr_f, int32_t *cursor,
                            int32_t *colind_f, double *val_f, hipStream_t s);
hipError_t launch_sort_rows(int64_t ntot, const int64_t *rowptr_f, int32_t *colind_f,
                            double *val_f, int32_t *long_rows, int32_t *n_long, hipStream_t s);
hipError_t launch_level_count(int64_t nrows, const int32_t *lev, int32_t *lcount, hipStream_t s);
hipError_t launch_level_place(int64_t nrows, const int32_t *lev, const int64_t *lptr,
                              int32_t *lcursor, int32_t *order, hipStream_t s);
hipError_t launch_sort_long_rows(const int64_t *rowptr_f, int32_t *colind_f, double *val_f,
                                 const int32_t *long_rows, const int32_t *n_long, int32_t *tmp_c,
                                 double *tmp_v, int64_t ntot, hipStream_t s);
hipError_t launch_cast32(int64_t n, const double *a, float *b, hipStream_t s);
hipError_t launch_max_stats(int64_t ntot, const int64_t *uptr, const int32_t *fill_cnt,
                            const int32_t *colcnt, const int32_t *lev, unsigned long long *out,
                            hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);

// --- solve.hip ---
// The solves work in position space: position p is the p-th row in level
// order (rows of one level are contiguous), the work vectors are indexed by
// position, and the level-ordered copies of F store positions as indices.
// Narrow levels.  The last levels of a factor often hold few rows each; a
// sweep spends a publish-to-detect hop per level there.  One workgroup per
// slot solves them instead, with the level's values in LDS and a barrier per
// level.  Per direction, in the order the direction solves the levels:
//   hdr[i]  = (first half-chunk, half-chunks, first row - np0, rows)
//   rows[p] = (first chunk of the level << 16) | chunks, p = position - np0
// A row of m entries has ceil(m / 16) chunks of 16 entries, each cut in two
// half-chunks of 8 entry slots (slots past the row's end are padding).
//   smap[s] = the slot's entry in the level-ordered copy, -1 for padding
//   nidx[s] = position - np0 of an entry inside the narrow range, else -1
// A level whose rows all have at most 32 chunks and fit the workgroup's
// lanes in groups of a power of two (two lanes per chunk, rounded up) is a
// one-wave-per-row level (bit 30 of hdr.w): each row's half-chunks lie in one
// aligned lane group, lane word
//   lw[h] = (row position - np0) << 8 | log2(group lanes) << 1 | first lane
// and the row is summed inside its wave.  Other levels list each row's
// half-chunks in position order, and rows[] gives their chunk ranges.
constexpr int kNarrowOneWave = 1 << 30;
struct NarrowDir {
  const int4 *hdr;
  const int32_t *rows;
  const int32_t *lw;
  const int32_t *smap;
  const int16_t *nidx;
  int64_t nslots;  // entry slots (8 per half-chunk)
  int32_t nlev;
};
constexpr int kNarrowThreads = 1024;     // one workgroup of 16 waves
constexpr int kNarrowChunks = 512;       // chunks of one narrow level, at most
constexpr int kNarrowRows = 8192;        // narrow positions, at most
constexpr int kNarrowLevels = 2048;      // narrow levels, at most
constexpr int kNarrowMinLevels = 16;     // fewer: not worth the extra launches
struct SolveArgs {
  int64_t n;             // solved rows (labels 0..n-1)
  const int64_t *lptr;   // position prefix over levels [depth+1]
  int64_t depth;
  // level-ordered copies of F: forward rows, backward columns (no ground)
  const int64_t *lf_ptr; const int32_t *lf_idx; const double *lf_val; const float *lf_val32;
  const int64_t *lb_ptr; const int32_t *lb_idx; const double *lb_val; const float *lb_val32;
  const double *Dinv; const float *Dinv32;  // D^+ by position
  const int32_t *src;    // position -> vertex of the original ordering
  // positions of each level ordered by row class, per direction
  const int32_t *flist, *blist;
  const int *skip;       // device flag: nonzero => return immediately
  // dependency-driven sweeps: units of work per direction in level order
  const int4 *task_f, *task_b;
  int32_t ntask_f, ntask_b;
  int *err;                // error word of the sweeps (watchdog)
  uint64_t timeout_ticks;  // watchdog of one sweep, wall-clock ticks
  // narrow levels (positions >= np0, solved by one workgroup per slot, see
  // NarrowDir); the sweeps then take forward units [0, nwide_f) and backward
  // units [nskip_b, ntask_b).  No narrow levels: np0 = n, nwide_f = ntask_f,
  // nskip_b = 0, nf.nlev = nb.nlev = 0.
  int32_t np0, nwide_f, nskip_b;
  NarrowDir nf, nb;
};
// the factor values of an apply precision
template <typename T> struct FactorVals;
template <> struct FactorVals<double> {
  static __device__ __forceinline__ const double *fwd(const SolveArgs &a) { return a.lf_val; }
  static __device__ __forceinline__ const double *bwd(const SolveArgs &a) { return a.lb_val; }
  static __device__ __forceinline__ const double *dinv(const SolveArgs &a) { return a.Dinv; }
};
template <> struct FactorVals<float> {
  static __device__ __forceinline__ const float *fwd(const SolveArgs &a) { return a.lf_val32; }
  static __device__ __forceinline__ const float *bwd(const SolveArgs &a) { return a.lb_val32; }
  static __device__ __forceinline__ const float *dinv(const SolveArgs &a) { return a.Dinv32; }
};
// Rows are cut in chunks of kChunk entries.  Row classes by entries (per
// direction): at most 16, 64, 256, 1024, more; a row of class c < 4 is
// solved by a group of 4^c lanes (16 entries per lane), 64 / 4^c rows to a
// wave; a longer row in blocks of kBlockChunks chunks (one partial sum per
// block) and a fold that adds the partials.
constexpr int kChunk = 64;
constexpr int kRowClasses = 5;
__host__ __device__ __forceinline__ int row_class(int64_t m) {
  return m <= 16 ? 0 : m <= 64 ? 1 : m <= 256 ? 2 : m <= 1024 ? 3 : 4;
}
// units of a sweep (x = kind): group of 4^kind lanes per row (y = first
// class-list index, z = rows), block (y = position, z = first chunk,
// w = partial-sum offset), fold (y = position, z = chunks, w = partial-sum
// offset)
constexpr int kUnitGroup1 = 0, kUnitGroup4 = 1, kUnitGroup16 = 2, kUnitGroup64 = 3;
constexpr int kUnitBlock = 4, kUnitFold = 5;
constexpr int kBlockChunks = 16;                // chunks of one block unit
constexpr int kReadyThreads = 256;              // four independent waves
constexpr int kReadyGroupsMax = 1024;           // workgroups of one system's sweep, at most
// by default: as fast as more on the 3D grid and Chung-Lu benchmarks, and a
// quarter of the waves the device holds, so other systems' kernels still fit
constexpr int kReadyGroupsDefault = 256;
// a work-vector entry whose row is not solved yet (signalling NaNs)
constexpr unsigned long long kPending64 = 0x7FF4DEADBEEF0001ull;
constexpr unsigned int kPending32 = 0x7FA0BEEFu;
// units of each direction (rev: levels in descending order, the backward
// sweep) from the class lists and the class bases cls[kRowClasses L + c]:
// counts per class-list entry in sweep order, then the units
hipError_t launch_unit_count(int64_t n, int64_t depth, const int64_t *lptr, const int64_t *cls,
                             const int32_t *list, const int64_t *ptr, int32_t *ucnt,
                             int32_t *ccnt, bool rev, hipStream_t s);
hipError_t launch_unit_write(int64_t n, int64_t depth, const int64_t *lptr, const int64_t *cls,
                             const int32_t *list, const int64_t *ptr, const int64_t *uoff,
                             const int64_t *coff, int4 *units, bool rev, hipStream_t s);
hipError_t launch_level_layout(int64_t n, const int32_t *order, const int64_t *rowptr_f,
                               const int64_t *colptr, const int32_t *rowind, int32_t *flen,
                               int32_t *blen, hipStream_t s);
// row classes (row_class); counts per (level, class), then placement into
// per-level lists
hipError_t launch_class_count(int64_t n, const int32_t *order, const int32_t *lev,
                              const int64_t *ptr, int32_t *ccount, hipStream_t s);
hipError_t launch_class_place(int64_t n, const int32_t *order, const int32_t *lev,
                              const int64_t *ptr, const int64_t *cbase, int32_t *ccursor,
                              int32_t *list, hipStream_t s);
hipError_t launch_narrow_index(int64_t ns, const int32_t *smap, const int32_t *idx, int32_t np0,
                               int16_t *nidx, hipStream_t s);
hipError_t launch_level_offsets(int64_t depth, const int64_t *lptr, const int64_t *lf_ptr,
                                const int64_t *lb_ptr, int64_t *lqf, int64_t *lqb, hipStream_t s);
hipError_t launch_position_maps(int64_t n, const int32_t *order, const int32_t *iperm,
                                const double *D, int32_t *posof, int32_t *src, double *pdinv,
                                float *pdinv32, hipStream_t s);
hipError_t launch_level_copy(int64_t n, const int32_t *order, const int32_t *posof,
                             const int64_t *rowptr_f, const int32_t *colind_f,
                             const double *val_f, const int64_t *colptr, const int32_t *rowind,
                             const double *val, const int64_t *lf_ptr, const int64_t *lb_ptr,
                             int32_t *lf_idx, double *lf_val, int32_t *lb_idx, double *lb_val,
                             hipStream_t s);
hipError_t launch_comp_init(int64_t ntot, const int64_t *colptr, const int32_t *rowind,
                            int32_t *parent, hipStream_t s);
hipError_t launch_comp_jump(int64_t ntot, const int32_t *src, int32_t *dst, int *changed,
                            hipStream_t s);
hipError_t launch_comp_check(int64_t n, int64_t ground, const int32_t *perm, const int32_t *root,
                             const double *b, double *sum, double *sabs, int *bad, hipStream_t s);

// --- block.hip (several right-hand sides, row-major blocks of nc columns) ---
constexpr int kBlockCols = 64;  // columns per block PCG launch sequence
int bpcg_partials();
hipError_t bpcg_launch_init(int64_t n, int nc, double rtol, const double *b, int64_t ldb,
                            double *x, int64_t ldx, double *r, double *p, double *partial,
                            double *bst, int *bist, int *gfl, hipStream_t s);
hipError_t bpcg_launch_rz(int64_t n, int nc, const double *r, const double *z, double *p,
                          double *partial, double *bst, int *bist, int *gfl, int first,
                          hipStream_t s);
hipError_t bpcg_launch_step(int64_t n, int nc, const int64_t *rowptr, const int32_t *col,
                            const double *val, double *x, int64_t ldx, double *r, double *p,
                            double *q, double *partial, double *bst, int *bist, int *gfl,
                            hipStream_t s);
hipError_t bpcg_launch_true_res(int64_t n, int nc, const int64_t *rowptr, const int32_t *col,
                                const double *val, const double *x, int64_t ldx, const double *b,
                                int64_t ldb, double *tmp, double *partial, double *bst, int *bist,
                                int *gfl, hipStream_t s);
hipError_t launch_bcomp_check(int64_t n, int nc, int64_t ground, const int32_t *perm,
                              const int32_t *root, const double *b, int64_t ldb, double *sum,
                              double *sabs, int *bad, hipStream_t s);

// --- serve.hip (PCG over a batch of independent systems) ---
constexpr int kSlotMaxBlocks = 1024;  // reduction workgroups of one system
struct PcgSlot {
  int64_t n;
  const int64_t *rowptr; const int32_t *col; const double *val;  // A (device)
  const double *b;
  double *x, *r, *z, *p, *q;
  double *st;  // 8 scalars: ||b||^2, r.z, p.q, r.r, alpha, beta, rtol, true res^2
  int *ist;    // iterations, done (1 converged, 2 iteration cap), cap, unused
  int32_t blk0, nblk;  // the system's workgroups in a batched launch
};
struct ApplySlot {
  SolveArgs a;  // a.skip points at the system's done flag
  int64_t ldr, ldz;  // element strides of r and z (1, or the columns of a block)
  const double *r;
  void *y, *x;  // position-space work vectors (precision of the apply), all pending
  void *cs;     // block partial sums of long rows (precision of the apply), all pending
  int32_t *ctr;  // ticket counters of the forward and backward sweeps
  double *z;
  void *pv;        // narrow entry slots' products (precision of the apply)
  int32_t ncols;  // valid columns of the slot (at most the launch's columns per slot)
  // the slot is skipped when all of a.skip[j * skip_stride], j < skip_n, are set
  int32_t skip_n, skip_stride;
};
struct SlotBatch {
  int nslots = 0, nblocks = 0;
  const PcgSlot *slots = nullptr;   // device [nslots]
  const int32_t *bslot = nullptr;   // device [nblocks]: slot of each workgroup
  double *partial = nullptr;        // device [nblocks]
  const ApplySlot *aslots = nullptr;  // device [nslots]
  // sweeps: one launch per direction; workgroup b serves slot wgmap[b]
  const int32_t *wgmap = nullptr;  // device [nwg]
  int nwg = 0;
  int cc = 1;  // columns per sweep slot (1, 2, 4; 8 with the FP32 apply)
  int64_t nslots_max = 0;  // narrow entry slots of the batch's largest system (0: none)
};
int slot_blocks(int64_t n);
hipError_t slots_init(const SlotBatch &B, hipStream_t s);
hipError_t slots_rz(const SlotBatch &B, int first, hipStream_t s);
hipError_t slots_step(const SlotBatch &B, hipStream_t s);
hipError_t slots_true_res(const SlotBatch &B, hipStream_t s);
// mid: optional event recorded between the forward and the backward sweep
hipError_t slots_apply(const SlotBatch &B, int prec, hipStream_t s, hipEvent_t mid = nullptr);
// --- ready.hip ---
hipError_t ready_apply(const SlotBatch &B, int prec, hipStream_t s, hipEvent_t mid = nullptr);
// columns per sweep slot the apply supports in a precision
bool ready_cols_ok(int prec, int cc);

}  // namespace parac

// the opaque handle
struct parac_factor_s {
  int64_t n = 0, ntot = 0;
  int32_t mode = 0;
  int64_t nnz_off = 0, depth = 0;
  parac_factor_stats stats{};
  // device arrays
  int32_t *perm = nullptr, *iperm = nullptr;
  int64_t *colptr = nullptr;   // canonical CSC of F (label space)
  int32_t *rowind = nullptr;
  double *val = nullptr;
  double *D = nullptr, *Dinv = nullptr;
  float *Dinv32 = nullptr;
  int32_t *lev = nullptr, *order = nullptr, *root = nullptr, *src = nullptr;
  int32_t *flist = nullptr, *blist = nullptr;
  int *zero = nullptr;  // device flag that stays 0 (apply without a skip flag)
  int64_t *lptr = nullptr;
  int64_t *lf_ptr = nullptr, *lb_ptr = nullptr;
  int32_t *lf_idx = nullptr, *lb_idx = nullptr;
  double *lf_val = nullptr, *lb_val = nullptr;
  float *lf_val32 = nullptr, *lb_val32 = nullptr;
  std::vector<int64_t> hlptr;  // host copy of lptr
  std::vector<int64_t> hlqf, hlqb;  // host copies of the level entry offsets
  // sweep units per direction, chunk-sum entries they need (the larger)
  int4 *task_f = nullptr, *task_b = nullptr;
  int32_t ntask_f = 0, ntask_b = 0;
  int64_t ncs = 0;
  // narrow levels (levels >= nlev0 when nf.nlev > 0) and the sweeps' cut
  int64_t nlev0 = 0;
  int32_t np0 = 0, nwide_f = 0, nskip_b = 0;
  parac::NarrowDir nf{}, nb{};
  void *npv64 = nullptr, *npv32 = nullptr;  // products of the narrow slots, per precision
  int32_t *ctr = nullptr;  // sweep ticket counters [2]
  int *serr = nullptr;     // sweep error word
  // solve work vectors (position space) and chunk sums per precision
  void *wy64 = nullptr, *wx64 = nullptr, *wy32 = nullptr, *wx32 = nullptr;
  void *cs64 = nullptr, *cs32 = nullptr;
  // column sweeps of a block apply, per precision: work vectors and chunk
  // sums of ccols columns (column-major), ticket counters (2 per column)
  void *cy[2] = {nullptr, nullptr}, *cx[2] = {nullptr, nullptr}, *ccs[2] = {nullptr, nullptr};
  int32_t *cctr[2] = {nullptr, nullptr};
  int64_t ccols[2] = {0, 0};
  // launch shape of the block apply per (columns, precision): fixed by the
  // caller, or timed on first use (else taken from the shape cache)
  std::map<std::pair<int, int>, parac_block_shape> shapes;
  std::vector<void *> owned;
  int64_t bytes = 0;  // device bytes held by the factor's own arrays
};
