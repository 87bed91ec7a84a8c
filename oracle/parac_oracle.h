/*
 * parac_oracle.h -- declarations of the sequential CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY: the oracle exists to check the GPU library.  Only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no source with the GPU library and includes none of
 * its headers.
 *
 * Everything here is plain C11, FP64, built with -O2 -ffp-contract=off and no
 * fast-math, single-threaded.
 */
#ifndef PARAC_ORACLE_H
#define PARAC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes (same numbering as the library's, so results compare) */
enum {
  ORC_OK = 0,
  ORC_EINVAL = -1,        /* malformed CSR / permutation / arguments        */
  ORC_ENOTLAP = -2,       /* positive off-diagonal or negative excess       */
  ORC_ENOMEM = -4,
  ORC_EINCONSISTENT = -7, /* b not orthogonal to a null vector              */
  ORC_ENOCONV = -8,       /* PCG hit maxit                                  */
  ORC_EINTERNAL = -9      /* a scheduler invariant failed (see trace)       */
};

enum { ORC_MODE_AUTO = 0, ORC_MODE_LAPLACIAN = 1, ORC_MODE_SDDM = 2 };

enum {
  ORC_SCHED_LABEL = 0, /* eliminate in label order 0..Ntot-1                */
  ORC_SCHED_ASYNC = 1  /* W virtual workers, random micro-step interleaving */
};

/* debug flags for planted-mistake tests (never used by a product path) */
enum {
  ORC_DBG_DELETE_FIRST = 1 /* apply pivot-edge decrements before the sampled
                              insertions (the order §III forbids)          */
};

/* trace event kinds: (kind, a, b, c) */
enum {
  ORC_EV_INIT_DP = 5, /* (v, dp0[v], 0)            */
  ORC_EV_INIT_Q = 6,  /* (v, queue slot, 0)        */
  ORC_EV_CLAIM = 1,   /* (k, 0, 0)                 */
  ORC_EV_INSERT = 2,  /* (target, other, dp[other] after the increment) */
  ORC_EV_DEC = 3,     /* (u, m, dp[u] after the decrement)              */
  ORC_EV_ENQ = 4      /* (u, queue slot, 0)        */
};

typedef struct {
  int32_t status;
  int32_t mode;            /* ORC_MODE_LAPLACIAN or ORC_MODE_SDDM          */
  int64_t n;               /* original order                               */
  int64_t ntot;            /* n, or n+1 with the ground vertex (label n)   */
  int64_t nnz_off;         /* strictly-lower entries of F                  */
  int64_t *colptr;         /* [ntot+1]  canonical CSC of F, label space    */
  int32_t *rowind;         /* [nnz_off] rows ascending within a column     */
  double *val;             /* [nnz_off]                                    */
  double *D;               /* [ntot]                                       */
  int32_t *level;          /* [ntot] longest dependency chain ending at k  */
  int64_t *rowptr_f;       /* [ntot+1] CSR of F (transpose of the CSC)     */
  int32_t *colind_f;
  double *val_f;
  /* statistics */
  int64_t n_input_edges;   /* undirected edges incl. ground edges          */
  int64_t n_fill;          /* sampled fill records                         */
  int64_t max_gather;      /* largest |U[k]| + |fill[k]|                   */
  int64_t max_deg;         /* largest merged neighbourhood d_k             */
  int64_t depth;           /* 1 + max level                                */
  int64_t n_zero_pivots;   /* D_k == 0                                     */
  /* forced-choice log (only when choices are forced) */
  int64_t n_choice;
  int32_t *choice_nopt;    /* options at each consumed slot                */
  int32_t *choice_pick;    /* offset taken                                 */
  double *choice_prob;     /* w_{n_q} / S_{p+1} of the offset taken        */
  /* event trace (only when requested) */
  int64_t n_trace;
  int64_t *trace;          /* 4 x n_trace                                  */
  /* per-target fill record count (statistic for pool sizing) */
  int32_t *fill_count;     /* [ntot] */
} orc_factor_result;

/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2],
                       uint64_t out[4]);

/* Input classification: Laplacian/SDDM sign convention and excess s_i. */
int orc_classify(int64_t n, const int64_t *rowptr, const int32_t *col,
                 const double *val, int32_t mode_req, int32_t *mode_out,
                 double *excess /* [n] */);

/* The randomized elimination.  perm[v] = elimination label of vertex v
 * (NULL = identity).  forced != NULL switches the sampler to forced choices
 * (offsets into the candidate range) and logs them: with forced_stride <= 0
 * one offset per draw in this schedule's order (0 beyond nforced), with
 * forced_stride > 0 a table keyed by pivot label k and slot s,
 * forced[k * forced_stride + s] (-1 or absent: the draw).  samples > 1 runs
 * AC(k) with k = samples (R18); 0 or 1 the plain method. */
int orc_factor(int64_t n, const int64_t *rowptr, const int32_t *col,
               const double *val, const int32_t *perm, uint64_t seed,
               int32_t mode_req, int32_t schedule, uint64_t sched_seed,
               int32_t nworkers, const int32_t *forced, int64_t nforced,
               int32_t forced_stride, int32_t want_trace, int32_t debug_flags,
               int32_t samples, orc_factor_result **out);

void orc_factor_free(orc_factor_result *f);

/* z = P^T F^-T D^+ F^-1 P r  (SDDM: the ground row/column is dropped). */
int orc_apply(const orc_factor_result *f, const int32_t *perm,
              const double *r, double *z);

/* Same operation in FP32 arithmetic from round-to-nearest copies of F and
 * D^+; r is rounded to FP32 on entry and z widened on exit. */
int orc_apply32(const orc_factor_result *f, const int32_t *perm,
                const double *r, double *z);

/* Per-component consistency of b (components of the augmented graph that do
 * not contain the ground vertex must have zero sum). */
int orc_check_consistent(int64_t n, const int64_t *rowptr, const int32_t *col,
                         const double *val, int32_t mode, const double *b);

typedef struct {
  int32_t status;
  int32_t iterations;   /* number of SpMVs                                 */
  double relres;        /* recursive ||r||/||b|| at exit                  */
  double true_relres;   /* ||b - A x|| / ||b|| recomputed in FP64          */
} orc_pcg_stats;

/* PCG with x0 = 0; stop when ||r_k|| <= rtol ||b||, at most maxit SpMVs.
 * precision 0 = FP64 apply, 1 = FP32 apply. */
int orc_pcg(int64_t n, const int64_t *rowptr, const int32_t *col,
            const double *val, const orc_factor_result *f,
            const int32_t *perm, const double *b, double rtol, int32_t maxit,
            int32_t precision, double *x, orc_pcg_stats *st);

#ifdef __cplusplus
}
#endif
#endif
