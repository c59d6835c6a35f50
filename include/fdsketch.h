/*
 * fdsketch.h -- C ABI of libfdsketch.so: the Frequent Directions family of
 * row-streaming matrix sketches on one MI355X (gfx950) GPU.
 *
 * Problem (Section 1.1 of Desai, Ghashami, Phillips, "Improved Practical
 * Matrix Sketching with Guarantees"): rows a_i in R^d of an n x d matrix A
 * arrive as a stream; keep an l x d matrix B such that the covariance error
 * ||A^T A - B^T B||_2 / ||A||_F^2 is small.  The sketch follows the generic
 * iterative scheme of Section 2.3 (Algorithm 1): rows fill free rows of an
 * m-row buffer; when it is full the buffer is factored, its singular values
 * are changed by a ReduceRank rule and the buffer is rebuilt as S'V^T.
 *
 * Rules (sigma_1 >= sigma_2 >= ... the buffer's singular values):
 *   FDSK_FD          delta = sigma_l^2, every sigma'^2 = max(sigma^2 - delta, 0)
 *                    (Section 2.3, Frequent Directions / its fast variant).
 *   FDSK_ISVD        keep sigma_1..sigma_{l-1}, zero the rest (Section 2.3).
 *   FDSK_ALPHA       Algorithm 2 (Section 3.1): the leading l - ceil(alpha*l)
 *                    values untouched, the rest shrunk by delta = sigma_l^2.
 *   FDSK_FAST_ALPHA  Section 3.1, fast parameterized FD: delta = sigma_t^2 with
 *                    t = r + ceil(s/2), s = ceil(alpha*l), r = l - s; the
 *                    trailing s values are shrunk, clamped at zero.
 *   FDSK_SSD         SpaceSaving Directions (Section 3.1, Algorithm 3):
 *                    delta = sigma_{l-1}^2, sigma_{l-1} becomes 0 and sigma_l
 *                    becomes sqrt(sigma_l^2 + delta); the rest untouched.  Needs
 *                    buffer_rows == l and l >= 2 (the rule returns l values).
 *                    When sigma_l^2 <= 1e-12 sigma_1^2 (a direction outside
 *                    the buffer's row space) nothing moves and delta = 0.
 *   FDSK_CFD         Compensative FD (Section 3.1): FD during the stream; at
 *                    finalize B = S^ V^T of the latest reduction, with
 *                    sigma^_j^2 = sigma'_j^2 + Delta (Delta = sum of every
 *                    delta) on the first l directions (rows l..: none); a
 *                    direction with sigma_j^2 <= 1e-12 sigma_1^2 stays zero.
 *                    When rows arrived after the latest reduction, the
 *                    buffer's own factorization (after one more FD reduction
 *                    if more than l rows are occupied) is compensated.
 * Shrunk values are clamped at 0; after a reduction the first t-1 rows are
 * kept (t = l except for the fast variant) and the next rows go after them;
 * SSD's merged direction is kept in row l-1 (1-based).
 *
 * Conventions for every entry point:
 *  - Return 0 on success or a negative FDSK_E* code.  Errors are sticky per
 *    sketch; the message is available from sketch_last_error().  Nothing
 *    throws across the ABI.  A sketch is not thread-safe; distinct sketches
 *    are independent.
 *  - hip_stream is a hipStream_t (NULL = the default stream).  Every device
 *    pointer passed in is read in stream order on that stream; the caller
 *    must not overwrite it until the stream passes the call.  Host pointers
 *    are consumed before the call returns.
 *  - Row-major matrices: element (i, j) of a matrix with leading dimension
 *    ld (in elements) is at p[i*ld + j].
 *  - The library owns all sketch state (buffers, Gram/eigen workspaces, FP64
 *    accumulators); it is allocated in *_create and freed in *_destroy.
 */
#ifndef FDSKETCH_H
#define FDSKETCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdsk_sketch fdsk_sketch;           /* opaque */

typedef enum {
  FDSK_FD = 0,
  FDSK_ISVD = 1,
  FDSK_ALPHA = 2,
  FDSK_FAST_ALPHA = 3,
  FDSK_SSD = 4,
  FDSK_CFD = 5
} fdsk_variant;
typedef enum { FDSK_F64 = 0, FDSK_F32 = 1, FDSK_BF16 = 2 } fdsk_dtype;  /* BF16 = raw uint16 bits */
/* Arithmetic of the Gram and rebuild products.  The eigensolver, the shrink
 * subtraction and every accumulator are FP64 in all modes; the buffer stays
 * FP64.  BF16 (fdsk_gram only; sketch_create and sketch_batch_create return
 * FDSK_EUNSUPPORTED, because one uncompensated pass misses the 1e-3 of
 * ||A||_F^2 covariance-error bar of the reduced-precision sketches): each
 * FP64 operand rounded to bfloat16, products on BF16 matrix cores with FP32
 * accumulation.  BF16X3: operands split as
 * hi = bf16(x), lo = bf16(x - hi) and hi*hi + hi*lo + lo*hi accumulated.
 * FP8X3 (Gram only; the rebuild is BF16X3): each buffer row split as
 * hi = e4m3(x / s), lo = e4m3((x - s hi) / t) with per-row scales s, t (row
 * maximum / 240), and hi*hi + hi*lo + lo*hi on FP8 matrix cores with FP32
 * accumulation, the scales applied in FP64. */
typedef enum { FDSK_P_FP64 = 0, FDSK_P_BF16 = 1, FDSK_P_BF16X3 = 2, FDSK_P_FP8X3 = 3 } fdsk_precision;
typedef enum { FDSK_MEM_HOST = 0, FDSK_MEM_DEVICE = 1 } fdsk_mem;

#define FDSK_FLAG_PROFILE 1u       /* record per-stage HIP events (sketch_profile, sketch_batch_profile) */
#define FDSK_FLAG_EIG_JACOBI 2u    /* always use the Jacobi eigensolver (see fdsk_eigh) */
#define FDSK_FLAG_GRAPH 4u         /* batches: run each append call through HIP graphs captured
                                      per size class (see sketch_batch_append) */

enum {
  FDSK_OK = 0,
  FDSK_EINVAL = -1,       /* bad argument or configuration */
  FDSK_ESTATE = -2,       /* call not allowed in the sketch's state (e.g. append after finalize) */
  FDSK_ENOMEM = -3,       /* device allocation failed */
  FDSK_EDEVICE = -4,      /* a HIP call failed or a kernel reported a fault */
  FDSK_ENONFINITE = -5,   /* NaN/Inf reached the sketch */
  FDSK_EUNSUPPORTED = -6  /* size or dtype/precision combination not supported */
};

typedef struct {
  int64_t d;              /* row length, >= 1 */
  int32_t l;              /* sketch rows, >= 1 */
  int32_t buffer_rows;    /* m: 0 -> 2l; l -> Algorithm 1 literally; any m in [l, 1024] */
  fdsk_variant variant;
  double alpha;           /* (0, 1]; used by FDSK_ALPHA and FDSK_FAST_ALPHA */
  fdsk_precision precision;
  uint32_t flags;         /* FDSK_FLAG_* bits: PROFILE and EIG_JACOBI for single sketches;
                             PROFILE and GRAPH (the same for every sketch) for batches */
} fdsk_config;

typedef struct {
  double cov_err;             /* ||A^T A - B^T B||_2 / ||A||_F^2            (Section 1.1) */
  double proj_err_k;          /* ||A - pi_{B_k}(A)||_F^2 / ||A - A_k||_F^2   (Section 1.1) */
  double proj_full_over_fro2; /* ||A - pi_B(A)||_F^2 / ||A||_F^2 */
  double fro2_A;              /* ||A||_F^2 (FP64 accumulation) */
  double fro2_B;              /* ||B||_F^2 */
  double delta_sum;           /* Delta = sum of delta_i (Section 3.1) */
  double shrink_total;        /* total squared mass removed by the rules (reduced-precision
                                 single sketches other than CFD: measured per reduction as
                                 ||C||_F^2 before minus after, in FP64 from the rows) */
  double lambda_max;          /* largest eigenvalue of A^T A - B^T B */
  double lambda_min;          /* smallest eigenvalue of A^T A - B^T B */
  int64_t n_rows;             /* rows appended */
  int64_t n_reduce;           /* ReduceRank steps run */
  int32_t k;                  /* rank used by proj_err_k */
  int32_t rows_out;           /* rows of the sketch that may be nonzero */
  int32_t eig_unconverged;    /* eigensolves that hit their sweep cap */
  int32_t reserved;
  int64_t eig_sweeps;         /* Jacobi sweeps summed over all eigensolves */
} fdsk_report;

/* Create a sketch (Algorithm 1 state, all rows free).  hip_stream is kept and
 * used by every later call on this sketch.  Sizes: 1 <= l, l <= m <= 1024,
 * d <= 65536.  Errors: EINVAL, EUNSUPPORTED, ENOMEM, EDEVICE. */
int sketch_create(const fdsk_config* cfg, void* hip_stream, fdsk_sketch** out);

/* Append n_rows rows (Algorithm 1, "insert a_i into a zero valued row"); runs
 * every ReduceRank the schedule calls for, asynchronously on the stream.
 * rows: n_rows x d, leading dimension row_stride (elements, >= d), in the
 * given dtype, on the host or on the device.  n_rows = 0 is a no-op.
 * Errors: EINVAL, ESTATE (after finalize), EDEVICE, ENOMEM. */
int sketch_append_rows(fdsk_sketch* s, const void* rows, int64_t n_rows, int64_t row_stride,
                       fdsk_dtype dtype, fdsk_mem mem);

/* Merge: dst absorbs src, so that dst then sketches the concatenation of both
 * streams (dst's rows, then src's).  src's occupied buffer rows are inserted
 * into dst like stream rows (running every ReduceRank dst's schedule calls
 * for) without counting into ||A||_F^2, and src's accumulators (||A||_F^2,
 * delta sum, shrink total, rows, reductions) are added to dst's.  Because
 * each ReduceRank rule satisfies Properties 1-3 of Section 3.1, the merged
 * sketch keeps them for the union with the delta sums added; merges compose
 * into trees (the building block of a sharded stream).  Both sketches must
 * have the same d, l, buffer rows, variant, precision (and alpha for the
 * alpha variants) and must not be finalized; src is left unchanged and stays
 * usable.  Stream-ordered: dst's stream waits for src's stream before reading
 * src, and src's stream waits for dst's reads before any later work on src.
 * Errors: EINVAL (null, dst == src, different configurations, src in an error
 * state), ESTATE (either finalized), EDEVICE. */
int sketch_merge(fdsk_sketch* dst, fdsk_sketch* src);

/* Finish the stream (Algorithm 1, Section 2.3: the sketch returned after the
 * last row): if more than l rows are occupied, one more ReduceRank
 * (FDSK_CFD: then its compensation, see the rules above, *rows_out = l);
 * then write the l x d sketch B (rows beyond *rows_out are zero) to B_out
 * (leading dimension ldb >= d, dtype FDSK_F64 or FDSK_F32).  Synchronises the
 * stream and reports sticky device errors.  Afterwards only sketch_stats,
 * sketch_error, sketch_last_error and sketch_destroy are allowed.
 * Errors: EINVAL, ESTATE (twice), EDEVICE, ENONFINITE. */
int sketch_finalize(fdsk_sketch* s, void* B_out, int64_t ldb, fdsk_dtype out_dtype, fdsk_mem mem,
                    int32_t* rows_out);

/* Error measures of Section 1.1 for the finalized sketch against A (n x d,
 * leading dimension lda): cov-err, proj-err with rank k (the experiments use
 * k = 10) and ||A - pi_B(A)||_F^2/||A||_F^2.  method 0: dense d x d A^T A in
 * FP64 on the device (d <= 8192); method 1: matrix-free (each Lanczos step
 * streams A twice).  cov-err is undefined for ||A||_F = 0 -> EINVAL.
 * Fills *out (also the fields of sketch_stats).  Synchronises the stream. */
int sketch_error(fdsk_sketch* s, const void* A, int64_t n, int64_t lda, fdsk_dtype dtype,
                 fdsk_mem mem, int32_t k, int32_t method, fdsk_report* out);

/* Evaluate the same error measures for an arbitrary B (rows_b x d, ldb)
 * against A, without a sketch object.  Device or host pointers (same mem for
 * both).  Used to score any sketch with the device evaluator. */
int fdsk_evaluate(const void* A, int64_t n, int64_t lda, fdsk_dtype a_dtype,
                  const void* B, int64_t rows_b, int64_t ldb, fdsk_dtype b_dtype,
                  int64_t d, fdsk_mem mem, int32_t k, int32_t method, void* hip_stream,
                  fdsk_report* out);

/* Accumulators so far (Section 3.1: Properties 1-3 are stated in these
 * quantities): ||A||_F^2 (Section 1.1), Delta = sum of the delta_i
 * and the total squared mass removed (the quantities of Properties 1-3,
 * Section 3.1), rows and reductions.  Synchronises the stream. */
int sketch_stats(const fdsk_sketch* s, fdsk_report* out);

/* Return the sketch to its empty state (all rows free, accumulators zero,
 * not finalized) keeping its allocations and stream.  Stream-ordered. */
int sketch_reset(fdsk_sketch* s);

/* Per-stage device time, measured with HIP events on the stream each stage
 * runs on, when the sketch was created with FDSK_FLAG_PROFILE (otherwise
 * zeros).  Totals since create/reset; synchronises the stream.  Resource
 * accounting only: no step of the method.  EIG is the whole eigensolve; with
 * the tridiagonal route its kernels are also timed on their own (TRIDIAG_HEAD
 * + TRIDIAG + DC + BACKTR = EIG up to event overhead; TRIDIAG_HEAD is the
 * packed-triangle part of the reduction of buffers above 208 rows, which
 * single sketches count under TRIDIAG).  work[] is the algorithmic work of
 * the timed launches, computed on the host from the sizes: bytes for INGEST
 * (rows read plus buffer rows written), flops otherwise: Gram m(m+1)d per
 * product pass, Householder tridiagonal reduction 4/3 m^3, divide and conquer
 * 4/3 m^3, back-transformation 2 m^2 per wanted eigenvector, rebuild
 * 2 (t-1) m d per pass, shrink 0 (m = buffer rows, d = row length). */
enum { FDSK_STAGE_INGEST = 0, FDSK_STAGE_GRAM = 1, FDSK_STAGE_EIG = 2, FDSK_STAGE_SHRINK = 3,
       FDSK_STAGE_REBUILD = 4, FDSK_STAGE_TRIDIAG = 5, FDSK_STAGE_DC = 6, FDSK_STAGE_BACKTR = 7,
       FDSK_STAGE_TRIDIAG_HEAD = 8, FDSK_STAGE_COUNT = 9 };
typedef struct {
  double ms[FDSK_STAGE_COUNT];       /* summed stage durations */
  int64_t launches[FDSK_STAGE_COUNT];
  double work[FDSK_STAGE_COUNT];     /* summed algorithmic work (bytes or flops, see above) */
} fdsk_profile;
int sketch_profile(fdsk_sketch* s, fdsk_profile* out);

/* Free everything the sketch owns (waits for its stream first). NULL is ok.
 * Resource management only: no step of the method (the paper's sketches end
 * with the output of finalize, Algorithm 1). */
void sketch_destroy(fdsk_sketch* s);

/* Message of the last error on this sketch ("" if none); valid until the
 * next call on it.  s == NULL gives the last create/evaluate failure. */
const char* sketch_last_error(const fdsk_sketch* s);

/* Kernel-level entry points: the two hot steps of a ReduceRank on their own.
 * Device pointers, FP64, stream-ordered on hip_stream, synchronous on return.
 *
 * fdsk_gram: G = C C^T (rows x rows) for C rows x d (leading dimension ldc),
 *   written to G with leading dimension ldg, with the products in the given
 *   precision (FP64 matrix cores, or BF16 matrix cores with FP32
 *   accumulation, optionally split-bf16 compensated).  This is the Gram
 *   matrix whose eigenvalues are the squared singular values of Algorithm
 *   1's buffer.
 * fdsk_eigh: eigen-decomposition G = V diag(lam) V^T of a symmetric m x m
 *   matrix (m <= 1024); lam unsorted, V's column j (V[i*ldv + j]) belongs to
 *   lam[j].  method FDSK_EIG_AUTO: Householder tridiagonalisation, divide and
 *   conquer and back-transformation at every m; FDSK_EIG_JACOBI: the Jacobi
 *   solvers at every m (cyclic two-sided in
 *   LDS for m <= 100).  Errors: EINVAL, EUNSUPPORTED (m > 1024), ENOMEM,
 *   EDEVICE. */
#define FDSK_EIG_AUTO 0
#define FDSK_EIG_JACOBI 1
int fdsk_gram(const double* C, int32_t rows, int64_t d, int64_t ldc, double* G, int64_t ldg,
              fdsk_precision prec, void* hip_stream);
int fdsk_eigh(const double* G, int32_t m, int64_t ldg, double* lam, double* V, int64_t ldv,
              int32_t method, void* hip_stream);

/* fdsk_eigh_noalloc: fdsk_eigh (method FDSK_EIG_AUTO, the tridiagonal route)
 * for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  It calls
 * no allocating routine; its workspace is a static device array of
 * FDSK_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends.  Sizes: 1 <= m <= FDSK_NOALLOC_EIGH_MAX (else
 * EUNSUPPORTED).  G, lam, V: device pointers as in fdsk_eigh (G m x m,
 * leading dimension ldg; lam m values, any order; V row-major, column j the
 * eigenvector of lam[j]).  Stream-ordered on hip_stream and asynchronous: it
 * returns once the work is enqueued (no synchronisation), so it may be
 * captured into a graph.  Every call on one GPU shares that GPU's scratch
 * and leaves the last call's contents in it (each call clears what it needs
 * first): calls that overlap on one GPU, on different streams or from
 * different threads, race.  Errors (message via sketch_last_error(NULL)):
 * EINVAL, EUNSUPPORTED, EDEVICE. */
#define FDSK_NOALLOC_SCRATCH_BYTES (16u << 20)
#define FDSK_NOALLOC_EIGH_MAX 512
int fdsk_eigh_noalloc(const double* G, int32_t m, int64_t ldg, double* lam, double* V, int64_t ldv,
                      void* hip_stream);

/* ------------------------------------------------------------------------
 * Many independent sketches advanced together (Algorithm 1 for each).
 *
 * The batch owns S sketches, each with its own configuration (buffer rows
 * m <= 256; variants FD, iSVD, alpha and fast alpha; FP64, BF16 or BF16x3; the
 * eigensolver is the tridiagonal route).  Because the schedule of Algorithm 1 does not
 * depend on the data, an append call first lays out, on the host, every
 * sketch's ingests and ReduceRanks for the call; round r then holds at most
 * one ingest and one ReduceRank per sketch, and each stage of a round (ingest,
 * Gram, tridiagonal reduction, divide and conquer, back-transformation,
 * shrink, rebuild) is one launch over all sketches active in it.  Each
 * sketch's arithmetic is exactly that of a single sketch with the same
 * configuration, so results do not depend on how sketches are grouped.
 * grid_size > 0 caps the sketches per launch (0: all active ones).
 * ------------------------------------------------------------------------ */
typedef struct fdsk_batch fdsk_batch;

/* Create S sketches from cfgs[0..S-1] (buffer rows <= 256; flags 0,
 * FDSK_FLAG_PROFILE and/or FDSK_FLAG_GRAPH, the same for every sketch).
 * Errors: EINVAL, EUNSUPPORTED, ENOMEM, EDEVICE. */
int sketch_batch_create(int32_t S, const fdsk_config* cfgs, void* hip_stream, fdsk_batch** out);

/* Append rows[i] (n_rows[i] x d_i, leading dimension strides[i], common
 * dtype) to sketch i for every i.  n_rows[i] may be 0 (rows[i] may then be
 * NULL).  mem FDSK_MEM_DEVICE: device pointers, read in stream order.
 * mem FDSK_MEM_HOST: host pointers, staged through one device buffer holding
 * every sketch's rows of the call (allocated for the call and freed after
 * it).  Returns when the work has completed (the rows may be overwritten
 * afterwards).
 *
 * Launches: each size class of buffer rows runs its rounds on a stream of
 * its own (the classes overlap), ordered after the batch's stream, which
 * then waits for all of them.  With FDSK_FLAG_GRAPH (and without
 * FDSK_FLAG_PROFILE) each class's launches of the call are captured into a
 * HIP graph on its stream, instantiated and launched there; the batch keeps
 * the last graphs with the task lists they read, and a later call whose
 * schedule is identical (the same row pointers, counts and strides, from
 * the same sketch states, e.g. after sketch_batch_reset) replays them
 * without capturing again.  Errors: EINVAL, ESTATE (after finalize), ENOMEM,
 * EDEVICE. */
int sketch_batch_append(fdsk_batch* b, const void* const* rows, const int64_t* n_rows,
                        const int64_t* strides, fdsk_dtype dtype, fdsk_mem mem, int32_t grid_size);

/* Finish every sketch (one more ReduceRank where more than l rows are
 * occupied) and write sketch i (l_i x d_i, leading dimension ldb[i], FDSK_F64 or
 * FDSK_F32) to the device pointer B_out[i]; rows_out[i] (host array, may be
 * NULL) receives the number of rows that may be nonzero.  Synchronises the
 * stream.  Errors: EINVAL, ESTATE (twice), EUNSUPPORTED, EDEVICE, ENONFINITE. */
int sketch_batch_finalize(fdsk_batch* b, void* const* B_out, const int64_t* ldb, fdsk_dtype out_dtype,
                          fdsk_mem mem, int32_t grid_size, int32_t* rows_out);

/* Accumulators of sketch `index` (as sketch_stats).  Synchronises. */
int sketch_batch_stats(const fdsk_batch* b, int32_t index, fdsk_report* out);

/* Return every sketch of the batch to its empty state (all rows free,
 * accumulators zero, not finalized), keeping its allocations, streams and
 * the cached graph.  Stream-ordered.  Errors: EINVAL, EDEVICE. */
int sketch_batch_reset(fdsk_batch* b);

/* Per-stage device time of the batch's launches since create/reset (HIP
 * events recorded on the stream of each size class; the batch must have
 * been created with FDSK_FLAG_PROFILE, which launches rounds directly).
 * Fields as sketch_profile; a launch serves every sketch of its round and
 * class, and work[] sums their algorithmic work.  Synchronises.  Resource
 * accounting only.  Errors: EINVAL, EDEVICE. */
int sketch_batch_profile(fdsk_batch* b, fdsk_profile* out);

/* Free everything the batch owns (waits for its streams first).  NULL is
 * ok.  Resource management only: no step of the method. */
void sketch_batch_destroy(fdsk_batch* b);
/* Message of the batch's last error ("" if none); NULL: the last create
 * failure.  Valid until the next call on the batch. */
const char* sketch_batch_last_error(const fdsk_batch* b);

/* ------------------------------------------------------------------------
 * Hashing and sampling sketches: the paper's fast competitors of the
 * Frequent Directions family, each reading every row once.
 *
 * FDSK_RS_HASH (Section 2.2, "Sparse Random Projections", Hashing): B = S A
 *   with S l x n, one nonzero per column: row i of A is added, with sign
 *   sigma(i), to row h(i) of B.
 * FDSK_RS_OSNAP (same paragraph): s independent such matrices of l/s rows
 *   stacked, each scaled by 1/sqrt(s) (so E[B^T B] = A^T A).
 * FDSK_RS_PRIORITY (Section 3.2, "Priority Sampling"): row i has weight
 *   w_i = ||a_i||^2, u_i ~ Unif(0,1) and priority w_i / u_i; the l rows of
 *   largest priority are kept (ties: earlier rows), each rescaled to squared
 *   norm max(w_i, tau) with tau the (l+1)-th largest priority of the stream
 *   (0 while at most l rows arrived).
 * FDSK_RS_VAROPT (Section 3.2, "VarOpt Sampling"): each append call is one
 *   merge step: the reservoir (adjusted weights w^) and the call's rows
 *   (w^ = w) are the candidates; tau solves sum min(1, w^/tau) = l over
 *   them; candidates with w^ >= tau stay; the others are chosen by
 *   systematic sampling with probabilities w^/tau (positions
 *   (q + u_c) C/(l - t), q < l - t, over the running sum C of those
 *   probabilities in candidate order: the reservoir's rows, then the call's
 *   rows in stream order; u_c the call's uniform) and then carry w^ = tau.
 *   Exactly l rows are kept and sum w^ = ||A||_F^2.  Rows are output as
 *   a_i sqrt(w^_i / w_i).
 * Random numbers (counter-based SplitMix64, Steele, Lea and Flood 2014):
 *   mix(x) = the SplitMix64 output for state x (x + 0x9E3779B97F4A7C15,
 *   then xor-shift 30 / multiply 0xBF58476D1CE4E5B9, xor-shift 27 / multiply
 *   0x94D049BB133111EB, xor-shift 31); r(i, j) = mix(mix(key ^ i) ^ j) for
 *   the stream index i of a row:
 *   h_j(i) = ((r(i, 2j) >> 32) * (l/s)) >> 32 in instance j, sigma_j(i) = -1
 *   when the top bit of r(i, 2j+1) is set, u_i = ((r(i, 0) >> 11) + 1/2)
 *   2^-53, and u_c = the same uniform of index 2^62 + c for the c-th
 *   non-empty append call (from 0).
 * Conventions as for the FD sketches (return codes, stream order, host or
 * device rows with a leading dimension, staging of host rows).
 * ------------------------------------------------------------------------ */
enum { FDSK_RS_HASH = 0, FDSK_RS_OSNAP = 1, FDSK_RS_PRIORITY = 2, FDSK_RS_VAROPT = 3 };
typedef struct fdsk_rsketch fdsk_rsketch;
typedef struct {
  double fro2_A;        /* ||A||_F^2 of the rows appended */
  double tau;           /* current threshold (Priority, VarOpt; 0 otherwise) */
  double weight_sum;    /* sum of the kept rows' adjusted weights (after finalize) */
  int64_t n_rows;
  int32_t rows_kept;    /* rows of B that may be nonzero */
  int32_t reserved;
} fdsk_rs_stats;

/* Create a sketch of kind FDSK_RS_* with l output rows over rows of length
 * d; s is OSNAP's number of stacked instances (1..8, dividing l; ignored
 * otherwise); key seeds the generator.  Errors: EINVAL, EUNSUPPORTED (l
 * above 2^24), ENOMEM. */
int rsketch_create(int32_t kind, int64_t d, int32_t l, int32_t s, uint64_t key, void* hip_stream,
                   fdsk_rsketch** out);
/* Append n rows (n x d, leading dimension stride, dtype, host or device);
 * each call is one step of the stream (one merge step for VarOpt).
 * Errors: EINVAL, ESTATE (after finalize), ENOMEM, EDEVICE, EUNSUPPORTED
 * (more than 2^30 rows in one call). */
int rsketch_append(fdsk_rsketch* s, const void* rows, int64_t n, int64_t stride, fdsk_dtype dtype,
                   fdsk_mem mem);
/* Write B (l x d, leading dimension ldb, F64 or F32, host or device as
 * mem); for the sampling kinds also the stream index of every kept row to
 * index_out (rows_out entries, same memory kind; may be NULL).
 * Synchronises.  Errors: EINVAL, ESTATE, ENOMEM, EDEVICE. */
int rsketch_finalize(fdsk_rsketch* s, void* B_out, int64_t ldb, fdsk_dtype out_dtype, fdsk_mem mem,
                     int64_t* index_out, int32_t* rows_out);
/* ||A||_F^2, tau, the adjusted weight sum and counts (Section 3.2's
 * quantities).  Synchronises. */
int rsketch_stats(const fdsk_rsketch* s, fdsk_rs_stats* out);
/* Free everything the sketch owns (waits for its stream).  NULL is ok.
 * Resource management only. */
void rsketch_destroy(fdsk_rsketch* s);
/* Last error message of the sketch ("" if none); NULL: the last create
 * failure. */
const char* rsketch_last_error(const fdsk_rsketch* s);

/* ------------------------------------------------------------------------
 * Launch-shape tuning of the Gram and rebuild products (the two matrix-core
 * contractions of a ReduceRank, Algorithm 1).  Several launch shapes compute
 * each product: the Gram's number of K slices summed afterwards (split-K) and
 * the rebuild's rows per workgroup (32 or 64).  sketch_create and
 * sketch_batch_create pick the shape per size bucket by timing every
 * candidate once on the new sketch's own (still empty) workspaces; the
 * choice is kept in a per-process table and persisted to a cache file, so
 * later sketches and processes on the same kind of GPU reuse it.
 *
 * Keys name the device ("gfx950/256"), the product, the precision and the
 * bucket:
 *   <dev>|gram|p<P>|m<mp>|d<D>           single sketch, value = split-K count
 *   <dev>|rebuild|p<P>|m<mp>|d<D>        single sketch, value = rows per workgroup
 *   <dev>|bgram|p<P>|m<mp>|d<D>|n<N>     batch size class, value = K slice
 *                                        length (0: one slice; else 256, 512
 *                                        or 1024, raised to d/8 where larger)
 *   <dev>|brebuild|p<P>|m<mp>|d<D>|n<N>  batch size class, rows per workgroup
 * with P = 0 (FP64), 3 (BF16x3) or 8 (FP8x3), mp the buffer rows rounded up
 * to 32 (the class's largest for batches), D the padded row length rounded
 * up to a power of two (the class's largest), N the class's sketch count
 * rounded up to a power of two.
 *
 * Choices change only the order in which partial sums are added; results of
 * different choices differ by rounding (the rebuild's rows per workgroup
 * change nothing).  A batch sketch's slice length is fixed at create, so
 * its results still do not depend on how sketches are grouped into
 * launches.  Mode (fdsk_tune_set_mode, or
 * FDSK_TUNE=off|on|refresh in the environment at first use):
 *   FDSK_TUNE_OFF      fixed defaults, no timing, the table is not read;
 *   FDSK_TUNE_ON       (default) use the table, time on a miss;
 *   FDSK_TUNE_REFRESH  time on every create and overwrite the table.
 * Cache file: FDSK_TUNE_CACHE, else $XDG_CACHE_HOME/fdsketch/tune.tsv, else
 * $HOME/.cache/fdsketch/tune.tsv ("" disables it); lines
 * "key<TAB>value<TAB>candidate:microseconds ...", '#' starts a comment; read
 * at first use, rewritten (temporary file, then rename) after each new
 * choice.  A value set by hand is used only when it is one of the
 * candidates of its key.  The table is process-wide and thread-safe.
 * ------------------------------------------------------------------------ */
#define FDSK_TUNE_OFF 0
#define FDSK_TUNE_ON 1
#define FDSK_TUNE_REFRESH 2
/* Set / read the mode.  Errors: EINVAL (unknown mode). */
int fdsk_tune_set_mode(int32_t mode);
int fdsk_tune_get_mode(void);
/* Value of key: 0 and *value set when present, 1 when absent; EINVAL for
 * NULL arguments. */
int fdsk_tune_lookup(const char* key, int32_t* value);
/* Put key = value in the table (not written to the file until a later
 * choice or fdsk_tune_save).  Errors: EINVAL (NULL/empty key, or a key
 * holding a tab or newline). */
int fdsk_tune_set(const char* key, int32_t value);
/* Empty the table (the file is untouched). */
int fdsk_tune_clear(void);
/* Set the cache file used from now on (NULL or "": none); nothing is read. */
int fdsk_tune_set_path(const char* path);
/* Current cache file path ("" if none); valid until the next tune call. */
const char* fdsk_tune_path(void);
/* Merge the entries of path (NULL: the cache file) into the table.
 * Errors: EINVAL (unreadable). */
int fdsk_tune_load(const char* path);
/* Write the table to path (NULL: the cache file).  Errors: EINVAL (no
 * path), EDEVICE (the file could not be written; message from
 * fdsk_tune_last_error). */
int fdsk_tune_save(const char* path);
/* The table as text (the cache file's lines) into buf (cap bytes, NUL
 * terminated, truncated if short; buf may be NULL); returns the full
 * length. */
int32_t fdsk_tune_dump(char* buf, int64_t cap);
/* Last load/save failure of the tuner ("" if none). */
const char* fdsk_tune_last_error(void);

/* Library build information (static string). */
const char* fdsk_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FDSKETCH_H */
