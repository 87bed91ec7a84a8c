/*
 * parac_oracle.c -- sequential CPU oracle for ParAC: the randomized
 * approximate-Cholesky elimination of rchol (Alg. 1 with the SampleClique
 * rule of Alg. 2), scheduled by the dependency counters of §III, producing
 * L ~= F D F^T (§IV), and the PCG solve that applies it (§V methodology).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the GPU library is
 * checked against.  Only the tests, the smoke check and the benchmark's CPU
 * baseline may load it; no product path may call it.  It shares no source
 * with the GPU library.
 *
 * Plain C11, FP64, single thread, -O2 -ffp-contract=off, no fast-math.
 *
 * Readings of points the paper leaves open (each is also listed in the design
 * notes of the repository):
 *  R1  input: w_ij = -a_ij for stored a_ij < 0 (i != j); excess
 *      s_i = a_ii - (left fold of w_ij over ascending j); |s_i| within
 *      4 (deg_i+1) eps a_ii counts as zero; a negative excess beyond it is
 *      "not a Laplacian".  SDDM inputs get a ground vertex with the last
 *      label n, joined to every i with s_i > 0 by an edge of weight s_i
 *      (§V: ground node of the augmented Laplacian).
 *  R2  merge of parallel edges (Alg. 3/4, duplicate fill edges): gathered
 *      entries are sorted by the key (u, src, w) with src = -1 for input
 *      edges and the producing pivot's label for fill (w only orders the
 *      repeated draws of one pair in one AC(k) pivot, R18); a run of equal u
 *      is summed by a left fold in key order; its length is the multiplicity
 *      m_u.
 *  R3  sampling order (Alg. 2 sort step): ascending by (w_u, u).
 *  R4  suffix sums of the sorted weights (Alg. 3/4): tiles of 64 sorted
 *      positions starting at position 1; inside a tile Hillis-Steele steps
 *      with offsets 1,2,4,...,32 computed from the previous step's values and
 *      adding only partners inside the tile; tile totals carried right to
 *      left by a sequential fold; S_i = local_i + carry (no add in the last
 *      tile); finally S_i <- max(S_i, S_{i+1}) from the right (exact), which
 *      makes S non-increasing.
 *  R5  D_k = S_1 (the total active weight at k, as in Alg. 3/4).
 *  R6  the draw for slot s (0-based; position p = s+1) of pivot k is
 *      Philox4x64-10 with key (seed, 0) and counter (k, s, 0, 0); the first
 *      output word x gives r = (x >> 11) 2^-53 in [0,1); t = r S_{p+1};
 *      the partner is the first q > p with S_{q+1} <= t (S_{d+1} = 0), so in
 *      exact arithmetic P(q) = w_q / S_{p+1} as Alg. 2 requires.
 *  R7  fill weight c = (S_{p+1} w_p) / D_k, stored at the smaller label of
 *      the sampled pair, with dp[larger]++ (Alg. 3/4).
 *  R8  F(u,k) = -(w_u / D_k) for the merged neighbours, rows ascending.
 *  R9  D_k = 0 for an empty neighbourhood; the apply uses D^+.
 *  R10 apply (§V uses vendor triangular solves, whose summation order is
 *      not given): a row of F y = P r or F^T x = D^+ y with start value s
 *      and products p_1..p_m in ascending column order is the left fold
 *      ((s - p_1) - p_2) - ... - p_m.  Other summation orders (the GPU
 *      library's tree order among them) agree with it to rounding.
 *  R18 AC(k) (§V-B, the variant with k samples per entry): each merged
 *      neighbour u of the pivot enters the sampling as k consecutive slots
 *      of weight w_u / k (so the slot order is (w, u, copy) ascending); R4
 *      to R7 run over the k d slots, D_k being the first suffix sum of the
 *      slot weights; a slot whose drawn partner is a copy of the same
 *      neighbour yields a loop, which adds nothing to a Laplacian and is
 *      dropped (no record, no counter increment).  R8 and the decrements
 *      still use the merged neighbours.  k = 1 is the plain method, bit for
 *      bit.
 *  R17 mixed precision (FP32 preconditioner apply): D^+_i = 1/D_i is
 *      formed in FP64 and rounded to FP32; factor values are rounded to FP32;
 *      r is rounded to FP32 on entry and z widened to FP64 on exit; every
 *      product and difference of the two solves is an FP32 operation.
 */
#include "parac_oracle.h"

#include <float.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

/* ------------------------------------------------------------------------ */
/* Philox4x64-10, from the published description of the generator: ten     */
/* rounds of two 64x64->128 multiplies with a Weyl-sequence key schedule.   */
/* ------------------------------------------------------------------------ */
static void orc_mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2],
                       uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t hi0, lo0, hi1, lo1;
    orc_mulhilo64(M0, c0, &hi0, &lo0);
    orc_mulhilo64(M1, c2, &hi1, &lo1);
    uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += W0; k1 += W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* schedule randomness for the async simulation only (not the method's) */
static uint64_t orc_splitmix64(uint64_t *s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* ------------------------------------------------------------------------ */
/* R1: classification of the input matrix                                   */
/* ------------------------------------------------------------------------ */
static int orc_check_csr(int64_t n, const int64_t *rowptr, const int32_t *col,
                         const double *val) {
  if (n < 0 || n > (int64_t)INT32_MAX - 2) return ORC_EINVAL;
  if (n == 0) return ORC_OK;
  if (!rowptr || rowptr[0] != 0) return ORC_EINVAL;
  for (int64_t i = 0; i < n; ++i) {
    if (rowptr[i + 1] < rowptr[i]) return ORC_EINVAL;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      if (col[e] < 0 || col[e] >= n) return ORC_EINVAL;
      if (e > rowptr[i] && col[e] <= col[e - 1]) return ORC_EINVAL;
      if (!isfinite(val[e])) return ORC_EINVAL;
    }
  }
  return ORC_OK;
}

/* value of a_ji, found by binary search in row j; 0 if absent */
static int orc_find(const int64_t *rowptr, const int32_t *col, int64_t j,
                    int32_t i, int64_t *pos) {
  int64_t lo = rowptr[j], hi = rowptr[j + 1];
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (col[mid] < i) lo = mid + 1; else hi = mid;
  }
  if (lo < rowptr[j + 1] && col[lo] == i) { *pos = lo; return 1; }
  return 0;
}

int orc_classify(int64_t n, const int64_t *rowptr, const int32_t *col,
                 const double *val, int32_t mode_req, int32_t *mode_out,
                 double *excess) {
  int st = orc_check_csr(n, rowptr, col, val);
  if (st) return st;
  if (mode_req < 0 || mode_req > 2) return ORC_EINVAL;
  int any_excess = 0;
  for (int64_t i = 0; i < n; ++i) {
    double diag = 0.0, acc = 0.0;
    int64_t deg = 0;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      int32_t j = col[e];
      double a = val[e];
      if (j == i) { diag = a; continue; }
      if (a == 0.0) continue;              /* explicit zero: no edge       */
      if (a > 0.0) return ORC_ENOTLAP;     /* sign convention (§V)         */
      int64_t pos;
      if (!orc_find(rowptr, col, j, (int32_t)i, &pos) || val[pos] != a)
        return ORC_EINVAL;                 /* not symmetric                */
      acc += -a;
      ++deg;
    }
    double s = diag - acc;
    double tol = 4.0 * (double)(deg + 1) * DBL_EPSILON * fabs(diag);
    if (s < -tol) return ORC_ENOTLAP;
    if (s <= tol) s = 0.0;
    if (s > 0.0) any_excess = 1;
    excess[i] = s;
  }
  int32_t mode = mode_req;
  if (mode == ORC_MODE_AUTO) mode = any_excess ? ORC_MODE_SDDM : ORC_MODE_LAPLACIAN;
  if (mode == ORC_MODE_LAPLACIAN && any_excess) return ORC_ENOTLAP;
  *mode_out = mode;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Elimination state                                                        */
/* ------------------------------------------------------------------------ */
typedef struct { int32_t u; int32_t src; double w; } orc_ent;   /* gathered */
typedef struct { int32_t u; int32_t m; double w; } orc_nbr;     /* merged   */
typedef struct { int32_t other, src; double w; int64_t next; } orc_rec;

enum { OP_INSERT = 1, OP_DEC = 2 };
typedef struct { int32_t kind, a, b, c; double w; } orc_op;

typedef struct {
  orc_op *ops; int64_t n, cap, next;
  int32_t pivot;    /* -1 when idle */
  int64_t slot;     /* next queue slot to poll */
} orc_worker;

typedef struct {
  int64_t ntot;
  /* label-space upper adjacency U (input edges, incl. ground edges) */
  int64_t *uptr; int32_t *uidx; double *uw;
  /* fill records: one linked list per target label */
  orc_rec *rec; int64_t nrec, caprec; int64_t *head;
  int32_t *fill_count;
  /* dependency counters and the ready queue (§III) */
  int64_t *dp; int32_t *q; int64_t tail; uint8_t *enq;
  int32_t *level;
  /* factor columns, in claim order; canonicalised at the end */
  int64_t *colstart; int32_t *colcnt; int32_t *frow; double *fval;
  int64_t ftop, fcap;
  double *D;
  /* sampler */
  uint64_t seed;
  const int32_t *forced; int64_t nforced, iforced; int32_t forced_stride;
  int32_t log_choices;
  int32_t *ch_nopt, *ch_pick; double *ch_prob; int64_t nch, capch;
  /* scratch */
  orc_ent *ent; int64_t capent;
  orc_nbr *nb, *nb_u; double *S, *tmp, *x; int64_t capnb;
  /* trace */
  int32_t want_trace; int64_t *trace; int64_t ntr, captr;
  int32_t debug_flags;
  int32_t samples;  /* R18: sampling slots per merged neighbour (1: plain) */
  int32_t error;
  int64_t n_fill, max_gather, max_deg;
} orc_state;

#define ORC_GROW(ptr, cnt, cap, need, type)                                  \
  do {                                                                       \
    if ((need) > (cap)) {                                                    \
      int64_t nc_ = (cap) ? (cap) : 16;                                      \
      while (nc_ < (need)) nc_ *= 2;                                         \
      type *np_ = (type *)realloc((ptr), (size_t)nc_ * sizeof(type));        \
      if (!np_) return ORC_ENOMEM;                                           \
      (ptr) = np_; (cap) = nc_;                                              \
    }                                                                        \
  } while (0)

static int orc_trace(orc_state *st, int64_t kind, int64_t a, int64_t b,
                     int64_t c) {
  if (!st->want_trace) return ORC_OK;
  ORC_GROW(st->trace, st->ntr, st->captr, 4 * (st->ntr + 1), int64_t);
  int64_t *t = st->trace + 4 * st->ntr;
  t[0] = kind; t[1] = a; t[2] = b; t[3] = c;
  st->ntr++;
  return ORC_OK;
}

static int cmp_ent_usrc(const void *pa, const void *pb) {
  const orc_ent *a = (const orc_ent *)pa, *b = (const orc_ent *)pb;
  if (a->u != b->u) return a->u < b->u ? -1 : 1;
  if (a->src != b->src) return a->src < b->src ? -1 : 1;
  /* equal (u, src): only AC(k) draws the same pair twice in one pivot;
   * their weights order them, and equal weights are interchangeable */
  if (a->w != b->w) return a->w < b->w ? -1 : 1;
  return 0;
}

static int cmp_nbr_wu(const void *pa, const void *pb) {
  const orc_nbr *a = (const orc_nbr *)pa, *b = (const orc_nbr *)pb;
  if (a->w != b->w) return a->w < b->w ? -1 : 1;
  if (a->u != b->u) return a->u < b->u ? -1 : 1;
  return 0;
}

/* R4: suffix sums of x[0..d-1] into S[0..d-1] with the W64 association. */
static void orc_suffix_sums(const double *x, int64_t d, double *S,
                            double *tmp) {
  for (int64_t i = 0; i < d; ++i) S[i] = x[i];
  for (int64_t t0 = 0; t0 < d; t0 += 64) {
    int64_t len = d - t0 < 64 ? d - t0 : 64;
    for (int64_t off = 1; off < 64; off <<= 1) {
      for (int64_t l = 0; l < len; ++l) tmp[l] = S[t0 + l];
      for (int64_t l = 0; l < len; ++l)
        if (l + off < len) S[t0 + l] = tmp[l] + tmp[l + off];
    }
  }
  /* carries: sequential right-to-left fold of the tile totals */
  int64_t ntile = (d + 63) / 64;
  double carry = 0.0;
  for (int64_t t = ntile - 1; t >= 0; --t) {
    int64_t t0 = t * 64, len = d - t0 < 64 ? d - t0 : 64;
    double total = S[t0];
    if (t != ntile - 1)
      for (int64_t l = 0; l < len; ++l) S[t0 + l] = S[t0 + l] + carry;
    carry = (t == ntile - 1) ? total : total + carry;
  }
  for (int64_t i = d - 2; i >= 0; --i)
    if (S[i + 1] > S[i]) S[i] = S[i + 1];
}

/* one draw: offset into the candidate range [s+1, d-1].  Forced choices
 * (test hook): either a sequence consumed draw by draw in this schedule's
 * order, or (forced_stride > 0) a table keyed by pivot label and slot,
 * forced[k * forced_stride + s], where -1 or an absent entry keeps the draw */
static int orc_choose(orc_state *st, int32_t k, int64_t s, int64_t d,
                      const double *xw, const double *S, int64_t *qstar) {
  int64_t off = -1;
  if (st->forced && st->forced_stride > 0) {
    int64_t i = (int64_t)k * st->forced_stride + s;
    if (s < st->forced_stride && i < st->nforced) off = st->forced[i];
  } else if (st->forced) {
    off = st->iforced < st->nforced ? st->forced[st->iforced] : 0;
    st->iforced++;
    if (off < 0) return ORC_EINVAL;
  }
  if (off >= 0) {
    int64_t nopt = d - 1 - s;
    if (off >= nopt) return ORC_EINVAL;
    int64_t q = s + 1 + off;
    if (st->log_choices) {
      int64_t need = st->nch + 1;
      ORC_GROW(st->ch_nopt, st->nch, st->capch, need, int32_t);
      st->ch_pick = (int32_t *)realloc(st->ch_pick, (size_t)st->capch * sizeof(int32_t));
      st->ch_prob = (double *)realloc(st->ch_prob, (size_t)st->capch * sizeof(double));
      if (!st->ch_pick || !st->ch_prob) return ORC_ENOMEM;
      st->ch_nopt[st->nch] = (int32_t)nopt;
      st->ch_pick[st->nch] = (int32_t)off;
      st->ch_prob[st->nch] = xw[q] / S[s + 1];
      st->nch++;
    }
    *qstar = q;
    return ORC_OK;
  }
  uint64_t ctr[4] = {(uint64_t)(uint32_t)k, (uint64_t)s, 0, 0};
  uint64_t key[2] = {st->seed, 0};
  uint64_t out[4];
  orc_philox4x64_10(ctr, key, out);
  double r = (double)(out[0] >> 11) * 0x1.0p-53;
  double t = r * S[s + 1];
  int64_t q = s + 1;
  for (; q < d; ++q) {
    double next = (q + 1 < d) ? S[q + 1] : 0.0;
    if (next <= t) break;
  }
  *qstar = q;
  return ORC_OK;
}

/* grow the per-pivot scratch arrays to hold g entries */
static int orc_scratch(orc_state *st, int64_t g) {
  if (g <= st->capnb) return ORC_OK;
  int64_t c = st->capnb ? st->capnb : 64;
  while (c < g) c *= 2;
  orc_nbr *a = (orc_nbr *)realloc(st->nb, (size_t)c * sizeof(orc_nbr));
  if (a) st->nb = a;
  orc_nbr *b = (orc_nbr *)realloc(st->nb_u, (size_t)c * sizeof(orc_nbr));
  if (b) st->nb_u = b;
  double *S = (double *)realloc(st->S, (size_t)c * sizeof(double));
  if (S) st->S = S;
  double *t = (double *)realloc(st->tmp, (size_t)c * sizeof(double));
  if (t) st->tmp = t;
  double *x = (double *)realloc(st->x, (size_t)c * sizeof(double));
  if (x) st->x = x;
  if (!a || !b || !S || !t || !x) return ORC_ENOMEM;
  st->capnb = c;
  return ORC_OK;
}

/* Eliminate pivot k: gather (U[k] + fill to k), merge, sort, suffix sums,
 * sample, write column k of F and D_k, and queue the micro-operations
 * (insertions, then decrements) on worker wk. */
static int orc_eliminate(orc_state *st, int32_t k, orc_worker *wk) {
  int rc;
  int64_t g = (st->uptr[k + 1] - st->uptr[k]) + st->fill_count[k];
  if (g > st->max_gather) st->max_gather = g;
  ORC_GROW(st->ent, g, st->capent, g, orc_ent);
  int64_t n = 0;
  for (int64_t e = st->uptr[k]; e < st->uptr[k + 1]; ++e) {
    st->ent[n].u = st->uidx[e]; st->ent[n].src = -1; st->ent[n].w = st->uw[e];
    ++n;
  }
  for (int64_t r = st->head[k]; r >= 0; r = st->rec[r].next) {
    if (n >= g) return ORC_EINTERNAL;
    st->ent[n].u = st->rec[r].other; st->ent[n].src = st->rec[r].src;
    st->ent[n].w = st->rec[r].w;
    ++n;
  }
  if (n != g) return ORC_EINTERNAL;
  wk->n = 0; wk->next = 0;
  st->colstart[k] = st->ftop;
  st->colcnt[k] = 0;
  if (g == 0) {           /* Alg. 3/4: empty neighbourhood => D(k,k) = 0 */
    st->D[k] = 0.0;
    return ORC_OK;
  }
  /* R2: merge parallel edges */
  qsort(st->ent, (size_t)g, sizeof(orc_ent), cmp_ent_usrc);
  if ((rc = orc_scratch(st, g))) return rc;
  int64_t d = 0;
  for (int64_t i = 0; i < g;) {
    int64_t j = i;
    double w = st->ent[i].w;
    while (j + 1 < g && st->ent[j + 1].u == st->ent[i].u) { ++j; w = w + st->ent[j].w; }
    st->nb[d].u = st->ent[i].u; st->nb[d].w = w; st->nb[d].m = (int32_t)(j - i + 1);
    ++d;
    i = j + 1;
  }
  if (d > st->max_deg) st->max_deg = d;
  memcpy(st->nb_u, st->nb, (size_t)d * sizeof(orc_nbr)); /* u-ascending */
  /* R3: sampling order */
  qsort(st->nb, (size_t)d, sizeof(orc_nbr), cmp_nbr_wu);
  /* R18: the sampling slots, `ks` per merged neighbour (one: the plain
   * method); slot i belongs to neighbour i / ks */
  const int64_t ks = st->samples > 1 ? st->samples : 1;
  const int64_t ds = d * ks;
  if ((rc = orc_scratch(st, ds))) return rc;
  for (int64_t i = 0; i < ds; ++i) st->x[i] = st->nb[i / ks].w / (double)ks;
  /* R4, R5 */
  orc_suffix_sums(st->x, ds, st->S, st->tmp);
  double Dk = st->S[0];
  st->D[k] = Dk;
  /* R6, R7: one draw per slot p = 1..ds-1 (Alg. 2); a loop is dropped */
  ORC_GROW(wk->ops, wk->n, wk->cap, ds + d, orc_op);
  int64_t ninsert = 0;
  for (int64_t s = 0; s + 1 < ds; ++s) {
    int64_t q;
    rc = orc_choose(st, k, s, ds, st->x, st->S, &q);
    if (rc) return rc;
    int32_t a = st->nb[s / ks].u, b = st->nb[q / ks].u;
    if (a == b) continue;
    double c = (st->S[s + 1] * st->x[s]) / Dk;
    ++ninsert;
    orc_op *op = &wk->ops[wk->n++];
    op->kind = OP_INSERT;
    op->a = a < b ? a : b;     /* target: smaller label */
    op->b = a < b ? b : a;     /* other: larger label   */
    op->c = k;
    op->w = c;
  }
  /* R8: column k of F, rows ascending */
  ORC_GROW(st->frow, st->ftop, st->fcap, st->ftop + d, int32_t);
  st->fval = (double *)realloc(st->fval, (size_t)st->fcap * sizeof(double));
  if (!st->fval) return ORC_ENOMEM;
  for (int64_t i = 0; i < d; ++i) {
    st->frow[st->ftop + i] = st->nb_u[i].u;
    st->fval[st->ftop + i] = -(st->nb_u[i].w / Dk);
  }
  st->ftop += d;
  st->colcnt[k] = (int32_t)d;
  /* pivot-edge removal: dp[u] -= m_u (§III) */
  for (int64_t i = 0; i < d; ++i) {
    orc_op *op = &wk->ops[wk->n++];
    op->kind = OP_DEC; op->a = st->nb_u[i].u; op->b = st->nb_u[i].m; op->c = k;
    op->w = 0.0;
  }
  if (st->debug_flags & ORC_DBG_DELETE_FIRST) {
    /* planted mistake: decrements before insertions */
    orc_op *tmp = (orc_op *)malloc((size_t)wk->n * sizeof(orc_op));
    if (!tmp) return ORC_ENOMEM;
    int64_t ni = ninsert, t = 0;
    for (int64_t i = ni; i < wk->n; ++i) tmp[t++] = wk->ops[i];
    for (int64_t i = 0; i < ni; ++i) tmp[t++] = wk->ops[i];
    memcpy(wk->ops, tmp, (size_t)wk->n * sizeof(orc_op));
    free(tmp);
  }
  return ORC_OK;
}

static int orc_enqueue(orc_state *st, int32_t u) {
  if (st->enq[u]) return ORC_EINTERNAL; /* each vertex is enqueued once */
  st->enq[u] = 1;
  if (st->tail >= st->ntot) return ORC_EINTERNAL;
  st->q[st->tail] = u;
  int rc = orc_trace(st, ORC_EV_ENQ, u, st->tail, 0);
  st->tail++;
  return rc;
}

/* execute one queued micro-operation of worker wk */
static int orc_step(orc_state *st, orc_worker *wk) {
  orc_op *op = &wk->ops[wk->next++];
  if (op->kind == OP_INSERT) {
    ORC_GROW(st->rec, st->nrec, st->caprec, st->nrec + 1, orc_rec);
    orc_rec *r = &st->rec[st->nrec];
    r->other = op->b; r->src = op->c; r->w = op->w; r->next = st->head[op->a];
    st->head[op->a] = st->nrec++;
    st->fill_count[op->a]++;
    st->n_fill++;
    st->dp[op->b] += 1;
    return orc_trace(st, ORC_EV_INSERT, op->a, op->b, st->dp[op->b]);
  } else {
    int32_t u = op->a, m = op->b, k = op->c;
    int64_t prior = st->dp[u];
    st->dp[u] -= m;
    if (st->level[k] + 1 > st->level[u]) st->level[u] = st->level[k] + 1;
    int rc = orc_trace(st, ORC_EV_DEC, u, m, st->dp[u]);
    if (rc) return rc;
    if (st->dp[u] < 0) return ORC_EINTERNAL; /* counter never negative */
    if (prior == m) return orc_enqueue(st, u);
    return ORC_OK;
  }
}

static void orc_state_free(orc_state *st) {
  free(st->uptr); free(st->uidx); free(st->uw); free(st->rec); free(st->head);
  free(st->dp); free(st->q); free(st->enq);
  free(st->colstart); free(st->colcnt); free(st->frow); free(st->fval);
  free(st->ent); free(st->nb); free(st->nb_u); free(st->S); free(st->tmp);
  free(st->x);
  free(st->ch_nopt); free(st->ch_pick); free(st->ch_prob);
  free(st->trace);
}

void orc_factor_free(orc_factor_result *f) {
  if (!f) return;
  free(f->colptr); free(f->rowind); free(f->val); free(f->D); free(f->level);
  free(f->rowptr_f); free(f->colind_f); free(f->val_f);
  free(f->choice_nopt); free(f->choice_pick); free(f->choice_prob);
  free(f->trace); free(f->fill_count);
  free(f);
}

int orc_factor(int64_t n, const int64_t *rowptr, const int32_t *col,
               const double *val, const int32_t *perm, uint64_t seed,
               int32_t mode_req, int32_t schedule, uint64_t sched_seed,
               int32_t nworkers, const int32_t *forced, int64_t nforced,
               int32_t forced_stride, int32_t want_trace, int32_t debug_flags,
               int32_t samples, orc_factor_result **out) {
  *out = NULL;
  orc_factor_result *res = (orc_factor_result *)calloc(1, sizeof(*res));
  if (!res) return ORC_ENOMEM;
  *out = res;
  double *excess = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  if (!excess) return res->status = ORC_ENOMEM;
  int32_t mode = 0;
  int rc = orc_classify(n, rowptr, col, val, mode_req, &mode, excess);
  if (rc) { free(excess); return res->status = rc; }
  /* permutation check */
  int32_t *label = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  uint8_t *seen = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
  if (!label || !seen) { free(excess); free(label); free(seen); return res->status = ORC_ENOMEM; }
  for (int64_t v = 0; v < n; ++v) {
    int32_t l = perm ? perm[v] : (int32_t)v;
    if (l < 0 || l >= n || seen[l]) { free(excess); free(label); free(seen); return res->status = ORC_EINVAL; }
    seen[l] = 1; label[v] = l;
  }
  free(seen);
  int64_t ntot = n + (mode == ORC_MODE_SDDM ? 1 : 0);
  res->mode = mode; res->n = n; res->ntot = ntot;

  orc_state st;
  memset(&st, 0, sizeof(st));
  st.ntot = ntot; st.seed = seed; st.forced = forced; st.nforced = nforced;
  st.forced_stride = forced_stride;
  st.log_choices = forced != NULL; st.want_trace = want_trace;
  st.debug_flags = debug_flags;
  st.samples = samples > 1 ? samples : 1;
  int64_t nt1 = ntot > 0 ? ntot : 1;
  st.uptr = (int64_t *)calloc((size_t)nt1 + 1, sizeof(int64_t));
  st.head = (int64_t *)malloc((size_t)nt1 * sizeof(int64_t));
  st.fill_count = (int32_t *)calloc((size_t)nt1, sizeof(int32_t));
  st.dp = (int64_t *)calloc((size_t)nt1, sizeof(int64_t));
  st.q = (int32_t *)malloc((size_t)nt1 * sizeof(int32_t));
  st.enq = (uint8_t *)calloc((size_t)nt1, 1);
  st.level = (int32_t *)calloc((size_t)nt1, sizeof(int32_t));
  st.colstart = (int64_t *)calloc((size_t)nt1, sizeof(int64_t));
  st.colcnt = (int32_t *)calloc((size_t)nt1, sizeof(int32_t));
  st.D = (double *)calloc((size_t)nt1, sizeof(double));
  if (!st.uptr || !st.head || !st.fill_count || !st.dp || !st.q || !st.enq ||
      !st.level || !st.colstart || !st.colcnt || !st.D) {
    rc = ORC_ENOMEM; goto done;
  }
  for (int64_t v = 0; v < ntot; ++v) st.head[v] = -1;
  /* label-space upper adjacency; dp0[b] = #lower neighbours (§III) */
  for (int64_t i = 0; i < n; ++i) {
    int32_t a = label[i];
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      int32_t j = col[e];
      if (j == i || val[e] == 0.0) continue;
      if (label[j] > a) st.uptr[a + 1]++;
    }
    if (mode == ORC_MODE_SDDM && excess[i] > 0.0) st.uptr[a + 1]++;
  }
  for (int64_t v = 0; v < ntot; ++v) st.uptr[v + 1] += st.uptr[v];
  int64_t ne = st.uptr[ntot];
  st.uidx = (int32_t *)malloc((size_t)(ne > 0 ? ne : 1) * sizeof(int32_t));
  st.uw = (double *)malloc((size_t)(ne > 0 ? ne : 1) * sizeof(double));
  int64_t *fillp = (int64_t *)malloc((size_t)nt1 * sizeof(int64_t));
  if (!st.uidx || !st.uw || !fillp) { free(fillp); rc = ORC_ENOMEM; goto done; }
  for (int64_t v = 0; v < ntot; ++v) fillp[v] = st.uptr[v];
  for (int64_t i = 0; i < n; ++i) {
    int32_t a = label[i];
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      int32_t j = col[e];
      if (j == i || val[e] == 0.0) continue;
      int32_t b = label[j];
      if (b > a) {
        st.uidx[fillp[a]] = b; st.uw[fillp[a]] = -val[e]; fillp[a]++;
        st.dp[b] += 1;
      }
    }
    if (mode == ORC_MODE_SDDM && excess[i] > 0.0) {
      st.uidx[fillp[a]] = (int32_t)n; st.uw[fillp[a]] = excess[i]; fillp[a]++;
      st.dp[n] += 1;
    }
  }
  free(fillp);
  res->n_input_edges = ne;
  for (int64_t v = 0; v < ntot; ++v)
    if ((rc = orc_trace(&st, ORC_EV_INIT_DP, v, st.dp[v], 0))) goto done;
  for (int64_t v = 0; v < ntot; ++v)
    if (st.dp[v] == 0 && (rc = orc_enqueue(&st, (int32_t)v))) goto done;

  if (schedule == ORC_SCHED_LABEL) {
    orc_worker wk;
    memset(&wk, 0, sizeof(wk));
    /* optional progress lines on stderr for long runs (no effect on results) */
    const int progress = getenv("ORC_PROGRESS") != NULL;
    time_t last = time(NULL);
    for (int64_t k = 0; k < ntot && !rc; ++k) {
      if (progress && (k & 1023) == 0 && time(NULL) - last >= 10) {
        last = time(NULL);
        fprintf(stderr, "oracle: %lld of %lld pivots\n", (long long)k, (long long)ntot);
        fflush(stderr);
      }
      if (st.dp[k] != 0 || !st.enq[k]) { rc = ORC_EINTERNAL; break; }
      if ((rc = orc_trace(&st, ORC_EV_CLAIM, k, 0, 0))) break;
      if ((rc = orc_eliminate(&st, (int32_t)k, &wk))) break;
      while (wk.next < wk.n && !rc) rc = orc_step(&st, &wk);
    }
    free(wk.ops);
  } else if (schedule == ORC_SCHED_ASYNC) {
    /* W workers poll queue slots w, w+W, ... (§IV work scheduling); each
     * elimination is split into micro-operations that interleave randomly */
    if (nworkers < 1) { rc = ORC_EINVAL; goto done; }
    orc_worker *wk = (orc_worker *)calloc((size_t)nworkers, sizeof(orc_worker));
    if (!wk) { rc = ORC_ENOMEM; goto done; }
    for (int32_t w = 0; w < nworkers; ++w) { wk[w].pivot = -1; wk[w].slot = w; }
    uint64_t rs = sched_seed;
    int64_t active = nworkers, idle = 0;
    while (active > 0 && !rc) {
      int32_t w = (int32_t)(orc_splitmix64(&rs) % (uint64_t)nworkers);
      orc_worker *x = &wk[w];
      if (x->pivot < 0) {
        if (x->slot >= ntot) continue;
        if (x->slot >= st.tail) {           /* slot not yet written: spin */
          /* every worker spinning with no step taken in between: stuck */
          if (++idle > 64 * (int64_t)nworkers + 100000) rc = ORC_EINTERNAL;
          continue;
        }
        int32_t k = st.q[x->slot];
        if ((rc = orc_trace(&st, ORC_EV_CLAIM, k, 0, 0))) break;
        if ((rc = orc_eliminate(&st, k, x))) break;
        x->pivot = k;
        x->slot += nworkers;
      }
      if (x->next < x->n) { rc = orc_step(&st, x); idle = 0; }
      if (!rc && x->next >= x->n) {
        x->pivot = -1;
        if (x->slot >= ntot) {
          /* worker retires once its remaining slots are past the end */
          active = 0;
          for (int32_t v = 0; v < nworkers; ++v)
            if (wk[v].pivot >= 0 || wk[v].slot < ntot) ++active;
        }
      }
    }
    for (int32_t w = 0; w < nworkers; ++w) free(wk[w].ops);
    free(wk);
    if (!rc && st.tail != ntot) rc = ORC_EINTERNAL;
  } else {
    rc = ORC_EINVAL;
  }
  if (rc) goto done;

  /* canonical CSC of F (label space), CSR transpose, statistics */
  {
    int64_t nnz = st.ftop;
    res->nnz_off = nnz;
    res->colptr = (int64_t *)calloc((size_t)nt1 + 1, sizeof(int64_t));
    res->rowind = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    res->val = (double *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double));
    res->D = (double *)malloc((size_t)nt1 * sizeof(double));
    res->level = (int32_t *)malloc((size_t)nt1 * sizeof(int32_t));
    res->rowptr_f = (int64_t *)calloc((size_t)nt1 + 1, sizeof(int64_t));
    res->colind_f = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    res->val_f = (double *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double));
    res->fill_count = (int32_t *)malloc((size_t)nt1 * sizeof(int32_t));
    if (!res->colptr || !res->rowind || !res->val || !res->D || !res->level ||
        !res->rowptr_f || !res->colind_f || !res->val_f || !res->fill_count) {
      rc = ORC_ENOMEM; goto done;
    }
    for (int64_t k = 0; k < ntot; ++k) res->colptr[k + 1] = res->colptr[k] + st.colcnt[k];
    int64_t depth = 0;
    for (int64_t k = 0; k < ntot; ++k) {
      memcpy(res->rowind + res->colptr[k], st.frow + st.colstart[k], (size_t)st.colcnt[k] * sizeof(int32_t));
      memcpy(res->val + res->colptr[k], st.fval + st.colstart[k], (size_t)st.colcnt[k] * sizeof(double));
      res->D[k] = st.D[k];
      res->level[k] = st.level[k];
      if (st.level[k] + 1 > depth) depth = st.level[k] + 1;
      if (st.D[k] == 0.0) res->n_zero_pivots++;
      res->fill_count[k] = st.fill_count[k];
    }
    for (int64_t e = 0; e < nnz; ++e) res->rowptr_f[res->rowind[e] + 1]++;
    for (int64_t i = 0; i < ntot; ++i) res->rowptr_f[i + 1] += res->rowptr_f[i];
    int64_t *pos = (int64_t *)malloc((size_t)nt1 * sizeof(int64_t));
    if (!pos) { rc = ORC_ENOMEM; goto done; }
    for (int64_t i = 0; i < ntot; ++i) pos[i] = res->rowptr_f[i];
    for (int64_t k = 0; k < ntot; ++k)       /* columns ascending => rows' */
      for (int64_t e = res->colptr[k]; e < res->colptr[k + 1]; ++e) {
        int32_t i = res->rowind[e];
        res->colind_f[pos[i]] = (int32_t)k; res->val_f[pos[i]] = res->val[e];
        pos[i]++;
      }
    free(pos);
    res->n_fill = st.n_fill; res->max_gather = st.max_gather;
    res->max_deg = st.max_deg; res->depth = depth;
    res->n_choice = st.nch;
    res->choice_nopt = st.ch_nopt; res->choice_pick = st.ch_pick; res->choice_prob = st.ch_prob;
    st.ch_nopt = NULL; st.ch_pick = NULL; st.ch_prob = NULL;
  }
done:
  res->n_trace = st.ntr; res->trace = st.trace; st.trace = NULL;
  orc_state_free(&st);
  free(st.level); free(st.D); free(st.fill_count);
  free(excess); free(label);
  res->status = rc;
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Preconditioner apply (R9, R10, R17)                                      */
/* ------------------------------------------------------------------------ */
/* one row of a triangular solve (R10): start from s and subtract the
 * products val[e] * vec[idx[e]] one at a time, e ascending (a left fold in
 * ascending column order, the plain definition of substitution) */
static double orc_row64(double s, int64_t b, int64_t e1, const int32_t *idx,
                        const double *val, const double *vec) {
  double acc = s;
  for (int64_t e = b; e < e1; ++e) acc = acc - val[e] * vec[idx[e]];
  return acc;
}

/* the same in FP32 (R17): each factor value is rounded to FP32 before it is
 * used, every product and every difference is rounded to FP32 */
static float orc_row32(float s, int64_t b, int64_t e1, const int32_t *idx,
                       const double *val, const float *vec) {
  float acc = s;
  for (int64_t e = b; e < e1; ++e) {
    float v = (float)val[e];
    float prod = v * vec[idx[e]];
    acc = acc - prod;
  }
  return acc;
}

/* entries of column i of F without the ground row (the largest row, so the
 * kept entries are a prefix) */
static int64_t orc_col_end(const orc_factor_result *f, int64_t i) {
  int64_t e = f->colptr[i + 1];
  if (e > f->colptr[i] && f->rowind[e - 1] >= f->n) --e; /* SDDM ground (§V) */
  return e;
}

int orc_apply(const orc_factor_result *f, const int32_t *perm, const double *r,
              double *z) {
  if (!f || f->status) return ORC_EINVAL;
  int64_t n = f->n;
  double *y = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  if (!y) return ORC_ENOMEM;
  for (int64_t v = 0; v < n; ++v) y[perm ? perm[v] : v] = r[v];
  /* forward: F y = P r, rows ascending; row i uses row i of F */
  for (int64_t i = 0; i < n; ++i)
    y[i] = orc_row64(y[i], f->rowptr_f[i], f->rowptr_f[i + 1], f->colind_f, f->val_f, y);
  /* diagonal D^+ then backward: F^T x = D^+ y, rows descending; row i uses
   * column i of F */
  for (int64_t i = n - 1; i >= 0; --i) {
    double dinv = f->D[i] > 0.0 ? 1.0 / f->D[i] : 0.0;
    y[i] = orc_row64(dinv * y[i], f->colptr[i], orc_col_end(f, i), f->rowind, f->val, y);
  }
  for (int64_t v = 0; v < n; ++v) z[v] = y[perm ? perm[v] : v];
  free(y);
  return ORC_OK;
}

int orc_apply32(const orc_factor_result *f, const int32_t *perm,
                const double *r, double *z) {
  if (!f || f->status) return ORC_EINVAL;
  int64_t n = f->n;
  float *y = (float *)malloc((size_t)(n > 0 ? n : 1) * sizeof(float));
  if (!y) return ORC_ENOMEM;
  for (int64_t v = 0; v < n; ++v) y[perm ? perm[v] : v] = (float)r[v];
  for (int64_t i = 0; i < n; ++i)
    y[i] = orc_row32(y[i], f->rowptr_f[i], f->rowptr_f[i + 1], f->colind_f, f->val_f, y);
  for (int64_t i = n - 1; i >= 0; --i) {
    float dinv = (float)(f->D[i] > 0.0 ? 1.0 / f->D[i] : 0.0);
    float start = dinv * y[i];
    y[i] = orc_row32(start, f->colptr[i], orc_col_end(f, i), f->rowind, f->val, y);
  }
  for (int64_t v = 0; v < n; ++v) z[v] = (double)y[perm ? perm[v] : v];
  free(y);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Consistency (b orthogonal to each null vector) and PCG                   */
/* ------------------------------------------------------------------------ */
static int64_t orc_uf_find(int64_t *p, int64_t x) {
  while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; }
  return x;
}

int orc_check_consistent(int64_t n, const int64_t *rowptr, const int32_t *col,
                         const double *val, int32_t mode, const double *b) {
  int64_t ng = n + 1; /* slot n is the ground vertex */
  int64_t *p = (int64_t *)malloc((size_t)ng * sizeof(int64_t));
  double *sum = (double *)calloc((size_t)ng, sizeof(double));
  double *sabs = (double *)calloc((size_t)ng, sizeof(double));
  double *excess = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  int rc = ORC_OK;
  if (!p || !sum || !sabs || !excess) { rc = ORC_ENOMEM; goto out; }
  int32_t m = 0;
  rc = orc_classify(n, rowptr, col, val, mode, &m, excess);
  if (rc) goto out;
  for (int64_t i = 0; i < ng; ++i) p[i] = i;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      if (col[e] == i || val[e] == 0.0) continue;
      int64_t a = orc_uf_find(p, i), c = orc_uf_find(p, col[e]);
      if (a != c) p[a] = c;
    }
    if (m == ORC_MODE_SDDM && excess[i] > 0.0) {
      int64_t a = orc_uf_find(p, i), c = orc_uf_find(p, n);
      if (a != c) p[a] = c;
    }
  }
  for (int64_t i = 0; i < n; ++i) {
    int64_t rt = orc_uf_find(p, i);
    sum[rt] += b[i]; sabs[rt] += fabs(b[i]);
  }
  {
    int64_t g = orc_uf_find(p, n);
    for (int64_t i = 0; i < n; ++i) {
      int64_t rt = orc_uf_find(p, i);
      if (rt == i && rt != g && fabs(sum[rt]) > 1e-8 * sabs[rt]) { rc = ORC_EINCONSISTENT; break; }
    }
  }
out:
  free(p); free(sum); free(sabs); free(excess);
  return rc;
}

static double orc_dot(int64_t n, const double *a, const double *b) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s = s + a[i] * b[i];
  return s;
}

static void orc_spmv(int64_t n, const int64_t *rowptr, const int32_t *col,
                     const double *val, const double *x, double *y) {
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) s = s + val[e] * x[col[e]];
    y[i] = s;
  }
}

/* Preconditioned conjugate gradients (the textbook recurrence; the paper
 * cites Saad's book for it and fixes only the stopping rule). */
int orc_pcg(int64_t n, const int64_t *rowptr, const int32_t *col,
            const double *val, const orc_factor_result *f,
            const int32_t *perm, const double *b, double rtol, int32_t maxit,
            int32_t precision, double *x, orc_pcg_stats *st) {
  memset(st, 0, sizeof(*st));
  if (!f || f->status || f->n != n) return st->status = ORC_EINVAL;
  int rc = orc_check_consistent(n, rowptr, col, val, f->mode, b);
  if (rc) return st->status = rc;
  size_t sz = (size_t)(n > 0 ? n : 1) * sizeof(double);
  double *r = (double *)malloc(sz), *z = (double *)malloc(sz);
  double *p = (double *)malloc(sz), *q = (double *)malloc(sz);
  if (!r || !z || !p || !q) { free(r); free(z); free(p); free(q); return st->status = ORC_ENOMEM; }
  int (*apply)(const orc_factor_result *, const int32_t *, const double *, double *) =
      precision ? orc_apply32 : orc_apply;
  for (int64_t i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; }
  double bnorm = sqrt(orc_dot(n, b, b));
  int32_t it = 0;
  double rnorm = bnorm;
  rc = ORC_OK;
  if (bnorm > 0.0) {
    apply(f, perm, r, z);
    for (int64_t i = 0; i < n; ++i) p[i] = z[i];
    double rz = orc_dot(n, r, z);
    rc = ORC_ENOCONV;
    while (it < maxit) {
      orc_spmv(n, rowptr, col, val, p, q);
      double alpha = rz / orc_dot(n, p, q);
      for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
      for (int64_t i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
      ++it;
      rnorm = sqrt(orc_dot(n, r, r));
      if (rnorm <= rtol * bnorm) { rc = ORC_OK; break; }
      apply(f, perm, r, z);
      double rz_new = orc_dot(n, r, z);
      double beta = rz_new / rz;
      for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
      rz = rz_new;
    }
  }
  /* true residual in FP64 */
  orc_spmv(n, rowptr, col, val, x, q);
  for (int64_t i = 0; i < n; ++i) q[i] = b[i] - q[i];
  st->iterations = it;
  st->relres = bnorm > 0.0 ? rnorm / bnorm : 0.0;
  st->true_relres = bnorm > 0.0 ? sqrt(orc_dot(n, q, q)) / bnorm : 0.0;
  free(r); free(z); free(p); free(q);
  return st->status = rc;
}
