/*
 * parac.h -- C ABI of the MI355X (gfx950) ParAC library: randomized
 * approximate-Cholesky preconditioning of graph-Laplacian and SDDM systems,
 * scheduled by dynamic dependency tracking, and the PCG solve that applies it.
 *
 * The method (arXiv 2505.02977):
 *   - the system is L x = b with L a graph Laplacian (eq. (1), Definition of
 *     §II-A) or an SDDM matrix, which is factored through the augmented
 *     Laplacian with a ground vertex (§V methodology);
 *   - the factor is L ~= F D F^T with F unit lower triangular and D diagonal
 *     (§IV), built by the rchol elimination (Alg. 1) whose clique update is
 *     replaced by the sampled spanning tree of Alg. 2;
 *   - pivots are scheduled by the dependency counters d(i) of §III: a vertex
 *     is ready when it has no lower-labelled active neighbour;
 *   - the factor preconditions conjugate gradients to a relative residual
 *     (§V methodology).
 *
 * Environment: PARAC_VERBOSE=1 makes long calls report their progress on
 * stderr (PCG at its host convergence checks, the block-shape tuner per
 * candidate); PARAC_SHAPE_CACHE names the block-shape cache file.
 *
 * Conventions for every call:
 *   - all calls return a parac_status (0 = success, negative = error) and
 *     never abort or throw across the ABI; parac_last_error() returns a
 *     thread-local message describing the last failure;
 *   - "device pointer" means memory on the current HIP device; "host
 *     pointer" means ordinary host memory;
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *     calls are stream-ordered and return after the work they describe has
 *     completed unless stated otherwise;
 *   - vertex labels: perm[v] is the elimination label of original vertex v;
 *     the factor lives in label space.  In SDDM mode the ground vertex takes
 *     the last label n.
 */
#ifndef PARAC_H
#define PARAC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int parac_status;

#define PARAC_OK 0
#define PARAC_EINVAL (-1)        /* malformed CSR, permutation or options   */
#define PARAC_ENOTLAP (-2)       /* positive off-diagonal / negative excess */
#define PARAC_EPOOL (-3)         /* fill pool exhausted (retried inside)    */
#define PARAC_ENOMEM (-4)        /* device allocation failed                */
#define PARAC_ETIMEOUT (-5)      /* elimination watchdog expired            */
#define PARAC_EDEVICE (-6)       /* HIP runtime error                       */
#define PARAC_EINCONSISTENT (-7) /* b has a component along a null vector  */
#define PARAC_ENOCONV (-8)       /* PCG reached maxit                       */
#define PARAC_EINTERNAL (-9)     /* a scheduler invariant failed            */

#define PARAC_MODE_AUTO 0
#define PARAC_MODE_LAPLACIAN 1
#define PARAC_MODE_SDDM 2

#define PARAC_PREC_FP64 0  /* preconditioner apply in FP64               */
#define PARAC_PREC_MIXED 1 /* apply in FP32 from an FP32 copy of F, D^+;
                              SpMV, residuals, dots, alpha/beta in FP64 */

/* A symmetric matrix in CSR form, full (both triangles and the diagonal),
 * columns strictly increasing within each row.  Sign convention of §V:
 * positive diagonal, non-positive off-diagonals; a positive row excess
 * a_ii - sum_{j!=i} |a_ij| makes the matrix SDDM. */
typedef struct {
  int64_t n;              /* order                                          */
  int64_t nnz;            /* stored entries                                 */
  const int64_t *rowptr;  /* [n+1]                                          */
  const int32_t *col;     /* [nnz]                                          */
  const double *val;      /* [nnz]                                          */
  int32_t on_device;      /* 1: the three arrays are device pointers;
                             0: host pointers (copied in by the call)       */
} parac_csr;

typedef struct {
  uint64_t seed;          /* key of the counter-based sampler (Alg. 2 draws) */
  const int32_t *perm;    /* [n] perm[v] = label; NULL = identity.  Device
                             pointer iff the matrix is on the device.      */
  int32_t mode;           /* PARAC_MODE_*                                  */
  double pool_factor;     /* fill-pool capacity in records per stored entry
                             of L (default 4.0, as in §IV-A); doubled and
                             retried automatically on exhaustion            */
  int32_t workers;        /* single-wave workers of the persistent grid
                             (0 = all that fit beside the team workgroups,
                             which take pivots above 128 gathered entries) */
  int32_t keep_fp32;      /* also build the FP32 copy used by MIXED apply   */
  double timeout_s;       /* elimination watchdog (0 = 30 s)                */
  double tail_fraction;   /* share of pivots left to the single-workgroup
                             tail kernel (0 or negative = none; 1 = all)    */
  int32_t samples;        /* AC(k) (§V-B): k sampling slots of weight w/k
                             per merged neighbour, a draw between copies of
                             one neighbour dropped; 0 or 1 = the plain
                             method, at most 16.  A denser factor for fewer
                             iterations.                                    */
} parac_factor_opts;

typedef struct {
  int64_t n, ntot;        /* order; order incl. ground vertex               */
  int32_t mode;           /* resolved mode                                  */
  int64_t nnz_off;        /* strictly-lower entries of F                    */
  int64_t n_input_edges;  /* undirected edges of the (augmented) graph      */
  int64_t n_fill;         /* sampled fill records                           */
  int64_t max_gather;     /* largest gathered neighbourhood                 */
  int64_t max_deg;        /* largest merged neighbourhood d_k               */
  int64_t depth;          /* levels of the elimination dependency DAG       */
  int64_t n_zero_pivots;  /* D_k = 0 (one per connected component)          */
  int32_t workers;        /* single-wave workers used (teams not counted)   */
  int32_t retries;        /* pool-exhaustion retries                        */
  double pool_factor;     /* pool factor of the successful attempt          */
  double ms_setup;        /* relabel, upper adjacency, counters, queue      */
  double ms_eliminate;    /* the persistent elimination kernel              */
  double ms_finalize;     /* canonical CSC, CSR, levels, D^+, FP32 copy     */
  double ms_total;        /* whole call on the stream                       */
  int64_t narrow_levels;  /* final levels the triangular solves take in one
                             workgroup (LDS, a barrier per level) instead of
                             the dependency-driven sweep; 0 = none          */
} parac_factor_stats;

typedef struct parac_factor_s *parac_factor_t;

/* Build L ~= F D F^T (Alg. 1/2 scheduled by §III; scaled form of §IV).
 *   A     matrix, borrowed for the duration of the call
 *   o     options (NULL = defaults)
 *   out   receives a handle that owns all device memory of the factor
 * Errors: EINVAL (bad CSR, asymmetry, bad permutation), ENOTLAP, ENOMEM,
 * ETIMEOUT, EDEVICE, EINTERNAL.  EPOOL is handled by retrying with a larger
 * pool; the factor is identical bit for bit whatever the pool size. */
parac_status parac_factor(const parac_csr *A, const parac_factor_opts *o,
                          void *stream, parac_factor_t *out);

/* Test hook, not for production use: parac_factor with some partners of
 * step 4 of Alg. 2 chosen by the caller instead of drawn, so that a worked
 * example (the dependency trace of §III, Fig. 1) can be reproduced on the
 * device.  forced (host, borrowed) holds `count` entries, `stride` per pivot
 * label k: forced[k * stride + s] >= 0 makes slot s of pivot k take the
 * partner at offset forced[...] in its candidate range (the neighbours after
 * the slot's own in sampling order); -1, or an entry beyond `count` or
 * `stride`, keeps the random draw.  Errors: as parac_factor, plus EINVAL for
 * stride <= 0, count < 0, or an offset past the end of its candidate range. */
parac_status parac_debug_factor_forced(const parac_csr *A, const parac_factor_opts *o,
                                       const int32_t *forced, int32_t stride, int64_t count,
                                       void *stream, parac_factor_t *out);

/* Sizes and statistics of a factor (host struct, caller-owned). */
parac_status parac_factor_info(parac_factor_t f, parac_factor_stats *s);

/* Copy the factor to caller-allocated host arrays: canonical CSC of F in
 * label space (colptr[ntot+1], rowind[nnz_off] rows ascending,
 * val[nnz_off]), D[ntot], and level[ntot] (longest dependency chain ending
 * at each label).  Any pointer may be NULL to skip it. */
parac_status parac_factor_export(parac_factor_t f, int64_t *colptr,
                                 int32_t *rowind, double *val, double *D,
                                 int32_t *level);

/* z = M^+ r with M = P^T F D F^T P (SDDM: ground row/column dropped, §V).
 *   r, z       device pointers, original vertex order, n x nrhs row-major
 *   precision  PARAC_PREC_FP64, or PARAC_PREC_MIXED (needs keep_fp32)
 * The forward solve F y = P r and the backward solve F^T x = D^+ y follow
 * the elimination levels (a row depends only on rows of earlier levels).
 * Two sweeps, each a single launch in which every row starts as soon as the
 * rows it reads are solved.  For one column, the factor's final levels of
 * few rows (parac_factor_stats.narrow_levels) are left to one workgroup
 * (values in LDS, a barrier per level), launched between the two sweeps with
 * a pre-pass; each row's sum keeps the sweeps' association.  With nrhs > 1,
 * chunks of up to 64 columns run as sweep slots of several columns each in
 * the same two launches (the factor read once per slot; see
 * parac_block_shape_set for the shape and how it is chosen).
 * Every column equals, bit for bit, the apply of that column alone.
 * The call returns after the result is complete.  Errors: EINVAL, ETIMEOUT
 * (a sweep's watchdog expired; the factor stays usable). */
parac_status parac_apply(parac_factor_t f, const double *r, double *z,
                         int64_t nrhs, int32_t precision, void *stream);

/* Launch shape of the block apply for chunks of `cols` columns (2..64) in
 * one precision.  The two triangular sweeps run one slot per group of
 * cols_per_sweep columns, all slots in the same two launches; a slot reads
 * each factor row once for all of its columns and sums every column exactly
 * as the single-vector apply does.  Results do not depend on the shape, only
 * speed.
 *   cols_per_sweep  1, 2 or 4 (FP64); 1, 2, 4 or 8 (MIXED)
 *   workgroups      cap on the sweep workgroups of one slot (0 = as many as
 *                   its units need, at most 256; at most 1024)
 *   source          (get) 0 fixed by parac_block_shape_set, 1 timed on first
 *                   use in this process, 2 taken from the shape cache file
 *   ms              (get) time of one block apply with this shape when it was
 *                   timed, else 0
 * Unless fixed, the shape is chosen on first use for (cols, precision): each
 * candidate width is timed on the call's own vectors (a bounded budget of a
 * few seconds) and the fastest kept in the handle and in the JSON file named
 * by the environment variable PARAC_SHAPE_CACHE (default
 * $HOME/.cache/parac_block_shapes.json; empty: no file), keyed by device
 * architecture, precision, columns and the factor's size, depth and entries
 * per row, each to the nearest power of two below. */
typedef struct {
  int32_t cols_per_sweep;
  int32_t workgroups;
  int32_t source;
  float ms;
} parac_block_shape;

/* Fix (shape != NULL) or forget (shape == NULL: the next use takes the cache
 * file's shape or times the candidates again) the shape for (cols,
 * precision).  Errors: EINVAL. */
parac_status parac_block_shape_set(parac_factor_t f, int32_t cols,
                                   int32_t precision,
                                   const parac_block_shape *shape);

/* The shape in use for (cols, precision); EINVAL if none is fixed, timed or
 * cached for this handle yet. */
parac_status parac_block_shape_get(parac_factor_t f, int32_t cols,
                                   int32_t precision,
                                   parac_block_shape *shape);

typedef struct {
  double rtol;            /* stop when ||r_k|| <= rtol ||b|| (default 1e-6) */
  int32_t maxit;          /* SpMV cap (default 10000)                       */
  int32_t precision;      /* PARAC_PREC_*                                   */
  int32_t check_every;    /* iterations between host convergence checks
                             (0 = 8)                                        */
  int32_t timing;         /* 1: time the phases with HIP events on the
                             stream (fills the ms_* fields of the stats)    */
} parac_pcg_opts;

typedef struct {
  int32_t status;         /* per right-hand side                            */
  int32_t iterations;     /* SpMVs performed                                */
  double relres;          /* recursive ||r||/||b|| at exit                  */
  double true_relres;     /* ||b - A x||/||b|| recomputed in FP64           */
  double ms_total;        /* the whole call on the stream                   */
  double ms_apply;        /* preconditioner applies (both triangular solves)
                             when timing = 1, else 0                        */
  int32_t applies;        /* preconditioner applies performed               */
  double ms_fwd;          /* of ms_apply, the forward sweeps (F y = P r) of
                             a single right-hand side; 0 for blocks         */
} parac_pcg_stats;

/* Preconditioned conjugate gradients with x0 = 0 (§V methodology; the
 * textbook recurrence).  With nrhs > 1 the columns run as independent
 * recurrences (own alpha, beta and stopping test) in one block launch
 * sequence per chunk of 64 columns: the matrix is read once per iteration
 * for all columns of a chunk, the factor once per sweep slot of the block
 * shape (parac_block_shape_set); a converged column is frozen while the
 * others go on.
 *   A      the matrix the factor was built from (device arrays)
 *   b, x   device pointers, n x nrhs row-major; x is output only
 *   st     host array of nrhs stats (may be NULL)
 * Errors: EINCONSISTENT (Laplacian component with nonzero sum of b),
 * ENOCONV (x holds the last iterate), EINVAL. */
parac_status parac_pcg(const parac_csr *A, parac_factor_t f, const double *b,
                       double *x, int64_t nrhs, const parac_pcg_opts *o,
                       parac_pcg_stats *st, void *stream);

/* Bytes of the fixed device array behind parac_pcg_static (one copy per GPU,
 * held from library load until the process ends). */
#define PARAC_STATIC_SCRATCH_BYTES ((size_t)128 << 20)

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * single right-hand-side PCG as parac_pcg (same kernels, same launch shapes,
 * so x and the stats are bit for bit those of parac_pcg), but every per-call
 * buffer (the four PCG vectors, partial sums, scalars, flags, launch tables,
 * and the consistency check's sums) lives in a fixed device array of
 * PARAC_STATIC_SCRATCH_BYTES owned by the library; the call makes no device
 * allocation and creates no event.  The caller still passes the inputs and
 * the output, and the factor must have been built with the work vectors of
 * the requested precision (every factor has FP64 ones; MIXED needs
 * keep_fp32).
 *   A, f, b, x, o, stream  as for parac_pcg with nrhs = 1; o->timing is
 *              ignored (ms_* of the stats are 0)
 *   st         one stats struct (may be NULL)
 * Limit: the system may have at most parac_pcg_static_max_rows() rows
 * (ground vertex included), about 4.19 million; a larger one is rejected
 * with EINVAL before any device work.
 * Every call on a GPU uses that GPU's one array, which keeps the previous
 * call's contents (the call clears what it needs): calls that overlap on
 * one GPU (different host threads or streams) race and must be serialised
 * by the caller.
 * Errors: as parac_pcg, plus EINVAL for a system above the limit or a
 * factor without the precision's work vectors. */
parac_status parac_pcg_static(const parac_csr *A, parac_factor_t f,
                              const double *b, double *x,
                              const parac_pcg_opts *o, parac_pcg_stats *st,
                              void *stream);

/* Largest row count (ground vertex included) parac_pcg_static accepts. */
int64_t parac_pcg_static_max_rows(void);

/* One system of a serving stream. */
typedef struct {
  parac_csr A;            /* host arrays                                    */
  const int32_t *perm;    /* host, [n]                                      */
  const double *b;        /* host, [n]                                      */
  double *x;              /* host, [n] output (caller-owned)                */
  uint64_t seed;
  double rtol;
  double arrival_s;       /* arrival time relative to the call's start      */
} parac_request;

typedef struct {
  int32_t status;
  int32_t iterations;
  double true_relres;
  double t_arrive, t_admit, t_done;  /* seconds from the call's start       */
  int64_t bytes_resident;            /* device footprint while admitted     */
} parac_result;

typedef struct {
  size_t hbm_budget;      /* bytes the stream may hold resident (0 = 80% of
                             free device memory)                            */
  int32_t max_slots;      /* systems in flight at once, each on a stream of
                             its own (0 = 4, the device's hardware queues;
                             at most 64)                                    */
  int32_t precision;      /* PARAC_PREC_* for the batched PCG               */
  int32_t maxit;          /* per system (0 = 10000)                         */
  int32_t check_every;    /* batched iterations between convergence checks
                             (0 = 4)                                        */
} parac_serve_opts;

/* Continuous serving loop (not in the paper, which solves one system at a
 * time; each system here is the §III factorisation followed by the §V PCG).
 * Requests are replayed at their arrival times and admitted in arrival order
 * while fewer than max_slots systems are in flight and the budget holds the
 * request's peak footprint (its device copy, the factorisation's peak under
 * the same sizing parac_factor uses, and the PCG vectors); once set up, the
 * reservation shrinks to the bytes actually resident.  Every admitted system
 * runs from upload to result on a worker thread with a HIP stream of its
 * own, so systems in flight overlap on the device and a small system never
 * waits for the launches of a large one.  Each system runs parac_factor's
 * and parac_pcg's own code, so its x is bit for bit the one those calls give
 * for it alone (same seed, permutation and options).  Results go to the
 * caller's x as each system finishes.
 *   reqs, out  host arrays of n entries; request arrays are host memory,
 *              borrowed until the call returns
 * Errors: EINVAL for bad options, EDEVICE/ENOMEM if the device fails the
 * loop itself; per-request failures (ENOMEM for a request larger than the
 * whole budget, EINVAL, ENOTLAP, EINCONSISTENT, ENOCONV) go to
 * out[i].status. */
parac_status parac_serve(const parac_request *reqs, int64_t n,
                         const parac_serve_opts *o, parac_result *out);

/* A factor built on the host CPU by parac_factor_host: canonical CSC of F
 * in label space, D, levels, sizes.  The arrays are malloc'd by the library
 * and released by parac_host_factor_free. */
typedef struct {
  int64_t n, ntot;        /* order; order incl. ground vertex               */
  int32_t mode;           /* resolved mode                                  */
  int32_t threads;        /* worker threads used                            */
  int64_t nnz_off;        /* strictly-lower entries of F                    */
  int64_t n_fill;         /* sampled fill records                           */
  int64_t depth;          /* levels of the elimination dependency DAG       */
  int64_t *colptr;        /* [ntot+1]                                       */
  int32_t *rowind;        /* [nnz_off], rows ascending within a column      */
  double *val;            /* [nnz_off]                                      */
  double *D;              /* [ntot]                                         */
  int32_t *level;         /* [ntot]                                         */
  double ms_total;        /* wall time of the call                          */
} parac_host_factor;

/* The same factorisation on the host's CPU cores: the paper's CPU design
 * (§IV-B, Alg. 3), worker threads that claim ready pivots from a shared
 * queue scheduled by the §III dependency counters.  Same readings and
 * arithmetic as parac_factor, so the result equals parac_factor_export's bit
 * for bit for any thread count.  This is a separate CPU implementation that
 * a caller asks for by name; no GPU entry point calls it.
 *   A        host matrix (on_device must be 0)
 *   o        options (NULL = defaults); perm is a host pointer; workers,
 *            keep_fp32, timeout_s and tail_fraction are ignored; samples
 *            above 1 (AC(k)) is rejected with EINVAL
 *   threads  worker threads (0 = the host's hardware threads)
 *   out      filled on success; release with parac_host_factor_free
 * Errors: EINVAL, ENOTLAP, ENOMEM, EINTERNAL (EPOOL is retried inside);
 * the message is in parac_host_last_error(). */
parac_status parac_factor_host(const parac_csr *A, const parac_factor_opts *o,
                               int32_t threads, parac_host_factor *out);
void parac_host_factor_free(parac_host_factor *f);
const char *parac_host_last_error(void);

#define PARAC_ORDER_RANDOM 0 /* uniformly random permutation             */
#define PARAC_ORDER_NNZ 1    /* ascending stored entries per row        */
#define PARAC_ORDER_MIS 2    /* independent-set rounds, low degree first */

/* An elimination order for parac_factor (perm[v] = label of vertex v),
 * computed on the device.  The paper's ordering study (§V, "Ordering for
 * ParAC") finds that the order sets the depth of the elimination's
 * dependency DAG, on which both the parallel elimination and the triangular
 * solves wait, and recommends NNZ-sorted order for GPUs.
 *   kind   PARAC_ORDER_RANDOM: vertices sorted by h(i);
 *          PARAC_ORDER_NNZ: by (pri(i), i);
 *          PARAC_ORDER_MIS: local-minimum rounds: in round r an unplaced
 *          vertex whose (pri, index) is below that of every neighbour not
 *          placed in an earlier round joins round r (each round is an
 *          independent set of the graph); vertices sorted by (round, pri, i)
 *          where h(i) = the SplitMix64 output for state seed + i and
 *          pri(i) = min(stored entries of row i, 2^20 - 1) << 24 | h(i) >> 40
 *   A      the matrix (device arrays if A->on_device, else host arrays); only
 *          its pattern is read
 *   perm   [n] output, device pointer iff A->on_device
 *   rounds optional host pointer: the number of MIS rounds (0 otherwise)
 * The result depends only on the pattern, kind and seed (integer arithmetic
 * throughout).  Errors: EINVAL. */
parac_status parac_order(const parac_csr *A, int32_t kind, uint64_t seed,
                         int32_t *perm, int32_t *rounds, void *stream);

/* Device memory held by the library (diagnostics): what = 0 the bytes
 * allocated now, 1 the peak since the last reset, 2 reset the peak to the
 * current bytes and return it; -1 for another `what`. */
int64_t parac_device_bytes(int32_t what);

void parac_factor_free(parac_factor_t f);
const char *parac_status_str(parac_status s);
const char *parac_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PARAC_H */
