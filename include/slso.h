/*
 * slso.h -- C ABI of a GPU (AMD MI355X / gfx950) library for sketched
 * leverage scores and leverage-score ordering, after Chin & Liang,
 * "An Empirical Evaluation of Sketched SVD and its Application to Leverage
 * Score Ordering" (ACML 2018).
 *
 * What is computed (paper references are to its sections and algorithms):
 *   - leverage of row i of an n x d matrix A: the i-th diagonal entry of the
 *     hat matrix A (A^T A)^+ A^T, equal to ||U_i||^2 for A = U S V^T (Sec. 2.2);
 *   - the sketched approximation of Algorithm 2, in QR form: sketch S*X
 *     (Sec. 2.1), R of the small sketch (Cholesky-QR on the FP64 matrix
 *     cores: one pass when a condition estimate allows it, two passes
 *     otherwise, Householder QR when neither applies), scores
 *     ||x_i R^{-1} Pi_2||^2 with a second Gaussian projection Pi_2 (d x k),
 *     with the truncation of small singular values of Algorithm 3;
 *   - the "dec" ordering of Sec. 5.2: rows by decreasing score.
 *
 * Conventions shared by every entry point:
 *   - Array pointers marked (device) are device pointers into memory the
 *     caller allocated on the context's device; the library never frees or
 *     retains them past the call's stream work. (host) pointers are read or
 *     written before the call returns.
 *   - ``stream`` is a hipStream_t passed as void* (NULL = the legacy default
 *     stream). Work is enqueued on it; outputs are valid once it has been
 *     synchronised, except where an entry point says it synchronises itself.
 *   - Dense matrices are row-major with a leading dimension ``ld`` (elements
 *     between consecutive rows, ld >= d). CSR matrices use int64 row_ptr[n+1]
 *     and int32 col_idx[nnz], columns sorted and distinct within a row.
 *   - Return value: SLSO_OK (0) or a positive warning on success, a negative
 *     slso_status on failure. On failure no kernel has been enqueued unless
 *     the status is SLSO_EDEVICE, and outputs are unspecified. The text of the
 *     last error of a context is returned by slso_last_error.
 *   - A context is used by one host thread at a time. It owns a device
 *     workspace that grows to the largest problem seen and is reused; after a
 *     first call of a given size, later calls of that size allocate nothing.
 */
#ifndef SLSO_H
#define SLSO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct slso_ctx slso_ctx;

typedef enum {
  SLSO_OK = 0,
  SLSO_RANK_DEFICIENT = 1, /* success; the numerical rank is below d        */
  SLSO_EINVAL = -1,        /* invalid argument (see each entry point)        */
  SLSO_ENOMEM = -2,        /* device workspace could not be allocated        */
  SLSO_ENONFINITE = -3,    /* the input holds Inf or NaN                      */
  SLSO_EDEVICE = -4,       /* a HIP runtime call failed                       */
  SLSO_EUNSUPPORTED = -5   /* combination of format/dtype/kind not provided  */
} slso_status;

typedef enum {
  SLSO_F64 = 0,       /* double                                               */
  SLSO_F32 = 1,       /* float                                                */
  SLSO_BF16 = 2,      /* bfloat16 bit patterns (uint16)                      */
  SLSO_FP8_E4M3 = 3   /* OCP fp8 e4m3fn bytes, dequantised by the scales     */
} slso_dtype;

typedef enum { SLSO_DENSE = 0, SLSO_CSR = 1 } slso_format;

typedef enum {
  SLSO_COUNTSKETCH = 0, /* one signed nonzero per column of S (Sec. 2.1)     */
  SLSO_GAUSSIAN = 1,    /* S = G / sqrt(r), G i.i.d. N(0, 1) (Sec. 2.1)      */
  SLSO_OSNAP = 2,       /* s = nnz_per_col signed nonzeros +-1/sqrt(s) per   */
                        /* column of S, one in each of s blocks of r / s     */
                        /* rows (the sparse embedding of Sec. 2.1, hashed as */
                        /* in Sec. 3.1.2); hash 0 is the CountSketch's, so   */
                        /* s = 1 gives the CountSketch                       */
  SLSO_SRHT = 3         /* S = (1/sqrt(r)) P H D: random signs D, the        */
                        /* Walsh-Hadamard transform H over n' = 2^ceil(log2  */
                        /* n) zero-padded rows, r sampled rows P (Sec. 2.1,  */
                        /* Table 1); dense input, r <= n'                    */
} slso_sketch_kind;

/* An n x d input matrix. Dense: ``values`` (device) holds n rows of ``ld``
 * elements of ``dtype``. CSR: ``values`` (device) holds nnz entries of
 * ``dtype``, with ``row_ptr`` (device, n+1 int64, row_ptr[0] = 0,
 * row_ptr[n] = nnz) and ``col_idx`` (device, nnz int32 in [0, d)).
 * For SLSO_FP8_E4M3 the represented value is q * col_scale[j], with q the
 * e4m3fn value of the code; col_scale (device, d floats) is required for FP8
 * (EUNSUPPORTED without it) and must be NULL for other dtypes (EINVAL).
 * row_scale is reserved and must be NULL (EUNSUPPORTED otherwise).        */
typedef struct {
  int64_t n, d;
  int32_t format; /* slso_format */
  int32_t dtype;  /* slso_dtype  */
  const void* values;
  int64_t ld;
  const int64_t* row_ptr;
  const int32_t* col_idx;
  int64_t nnz;
  const float* col_scale;
  const float* row_scale;
} slso_matrix;

/* Options. Zero-initialised options select: CountSketch, no refinement and
 * the default rank tolerance. */
typedef struct {
  int32_t sketch;   /* slso_sketch_kind                                       */
  int32_t refine;   /* 1: sketch-preconditioned Cholesky-QR refinement of R  */
  double rank_tol;  /* relative threshold of Algorithm 3 step 3; 0 selects   */
                    /* the default 1e-10; a negative value disables          */
                    /* truncation (R^{-1} is used whatever its conditioning) */
  int32_t nnz_per_col; /* OSNAP nonzeros per column of S, 1..16 dividing r;  */
                       /* 0 selects 2; ignored by the other sketches         */
  int32_t flags;       /* SLSO_OPT_* bits; other bits must be 0              */
} slso_options;

/* slso_options.flags bits */
#define SLSO_OPT_SVD_RANK 1 /* decide the rank of Algorithm 3 step 3 by the */
                            /* singular values of R every time (Jacobi SVD), */
                            /* not by the diagonal screen, which can call a  */
                            /* Kahan-type R full rank; with nothing cut the  */
                            /* scores are those of R^{-1}                    */
#define SLSO_OPT_EPS_HAT 2  /* report the realised distortion eps_hat of the */
                            /* sketch on range(X) (Def. 1 / Thm. 1, Sec.     */
                            /* 2.1) in slso_info.eps_hat: with R1 the        */
                            /* refinement's Cholesky factor, R = R1 R_S is   */
                            /* the R of X D, so sigma(S U) = sigma(R_S R^-1) */
                            /* = 1 / sigma(R1), from a Jacobi SVD of R1. The */
                            /* refinement's Gram pass and Cholesky run even  */
                            /* without refine (dense F32 / BF16 / FP8 input  */
                            /* only: EUNSUPPORTED otherwise); the call then  */
                            /* synchronises its stream a few more times      */

#define SLSO_OPT_NO_SYNC 4   /* slso_leverage enqueues the whole job and    */
                             /* returns at once: the QR's passes, the form  */
                             /* of R^{-1} and the rank screen are decided  */
                             /* on the device, no host wait and no other   */
                             /* stream (the call can be captured in a HIP  */
                             /* graph once a call of its size has grown    */
                             /* the workspace). info is filled by          */
                             /* slso_leverage_finish, which the caller     */
                             /* makes before the context's next            */
                             /* slso_leverage call; cases the device path  */
                             /* does not take (a Householder fallback, a   */
                             /* truncation) are rerun there on the         */
                             /* synchronous path. Not with the refinement, */
                             /* SLSO_OPT_EPS_HAT or SLSO_OPT_SVD_RANK      */
                             /* (EUNSUPPORTED). Calls on other streams     */
                             /* that share the context are not ordered     */
                             /* after it: the caller orders them.          */

/* Host-side report of one leverage computation. */
typedef struct {
  int64_t rank;        /* numerical rank used (d when nothing is truncated) */
  int32_t screen_full; /* 1 when the diag(R_D) screen declared full rank    */
  int32_t flags;       /* SLSO_INFO_* bits                                   */
  double diag_min;     /* min |R[j][j]| of the factor used (the refined one  */
  double diag_max;     /* when SLSO_INFO_REFINED is set, else R_D's)         */
  double eps_hat;      /* with SLSO_OPT_EPS_HAT: max(sigma_max(S U)^2 - 1,   */
                       /* 1 - sigma_min(S U)^2), U an orthonormal basis of   */
                       /* range(X); NaN when not asked for or when X D is    */
                       /* numerically rank deficient                         */
} slso_info;

/* slso_info.flags bits */
#define SLSO_INFO_REFINED 1       /* R is the refined factor of X D          */
#define SLSO_INFO_REFINE_FAILED 2 /* refinement asked for but its Cholesky   */
                                  /* met a non-positive pivot (X D is, in    */
                                  /* working precision, rank deficient); the */
                                  /* sketch factor R_D was used instead      */
#define SLSO_INFO_QR_SECOND_CHOLESKY 4 /* the sketch's Cholesky-QR2 needed   */
                                  /* the blocked Cholesky in its second pass */
#define SLSO_INFO_QR_HOUSEHOLDER 8 /* Cholesky-QR2 did not apply to the     */
                                  /* sketch; its R came from the Householder */
                                  /* panel path                              */
#define SLSO_INFO_QR_TREE 16      /* ... and, that failing too, from the     */
                                  /* column-by-column Householder path       */
#define SLSO_INFO_RERUN 64        /* slso_leverage_finish reran the job on   */
                                  /* the synchronous path                    */
#define SLSO_INFO_QR_ONE_PASS 32  /* the sketch's R is the first Cholesky-QR */
                                  /* pass's R1: R1's condition estimate      */
                                  /* kappa bounds the scores' relative error */
                                  /* 4 kappa^2 sqrt(r d) 2^-53 by 1e-7 (by   */
                                  /* 1e-2 with the refinement, where R only  */
                                  /* preconditions); Algorithm 2 step 2      */
                                  /* needs only R^T R of the sketch. Tried   */
                                  /* only when 2 r d^2 >= 2^31, where the    */
                                  /* second pass costs more than the estimate*/

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device ``device``. workspace_bytes = 0: the
 * context's device workspace grows on demand (a call that needs more than
 * the context holds waits for the context's earlier work, frees the old
 * buffer and allocates a larger one). workspace_bytes > 0: that much is
 * allocated here (rounded up to 2 MiB) and never again; a call that needs
 * more (slso_workspace_size) fails with SLSO_ENOMEM and enqueues nothing,
 * so no call of the context allocates device memory. EINVAL: ctx NULL or
 * no such device; ENOMEM: the workspace allocation failed; EDEVICE: HIP
 * failure. */
int slso_create(slso_ctx** ctx, int device, size_t workspace_bytes);

/* Release the context and its workspace (synchronises the device first). */
int slso_destroy(slso_ctx* ctx);

/* Static text for a status code; the last error text of a context (never
 * NULL; empty when no error has occurred). */
const char* slso_status_string(int status);
const char* slso_last_error(const slso_ctx* ctx);

/* ---- the hot path -------------------------------------------------------- */

/* Sketch S*X (Algorithm 2 step 1; Sec. 2.1; Sec. 3.1.2 "pair of hash
 * functions" for CountSketch).
 *   X      matrix as above (dense F64/F32/BF16/FP8 or CSR F32 for CountSketch;
 *          dense BF16/F32/FP8 for Gaussian).
 *   seed   64-bit seed; the bucket hash, sign hash and Gaussian entries are
 *          derived from it per row index (0-based global row i).
 *   r      sketch rows, r >= d (EINVAL otherwise).
 *   sx     (device) r x d doubles, row-major, overwritten with S*X (without
 *          column equilibration).
 * CountSketch: sx[h(i)] += s(i) x_i, summed in FP64 in ascending i within
 * each bucket (deterministic). Gaussian: S = G/sqrt(r) with G[j][i] the
 * FP32 generator value of slso_gaussian_sketch_entries for F32 input, the
 * quantile-form value of slso_gaussian_sketch_entries_q (BF16 or e4m3
 * table) for BF16 and FP8 input; products on MFMA, sums in FP32 within
 * slices of rows (at most 65536 rows for F32 input, 2^18 for BF16 and FP8)
 * and in FP64 across slices, in a fixed order (deterministic); the
 * 1/sqrt(r) (and for FP8 the column scale) is applied once to the FP64 sum. OSNAP (same inputs as CountSketch): for every hash
 * j < s, sx[h_j(i)] += s_j(i) x_i in ascending i (each sketch row belongs to
 * one hash's block), then every sum is multiplied once by 1/sqrt(s) in FP64.
 * SRHT (dense input): D_ii = +1 if the polynomial hash of stream 7 is even
 * at i, else -1; rows past n are zero up to n' = 2^ceil(log2 n); H is applied
 * as Sylvester-order stages t = 0, 1, ..., each replacing rows a and
 * a + 2^t (bit t of a clear) by their FP64 sum and difference; P takes the r
 * rows i < n' with the smallest words w0 of the Philox block with counter
 * (lo32(i), hi32(i), 0, 8) and key (lo32(seed), hi32(seed)), ties by
 * ascending i, in that order; the result is multiplied once by 1/sqrt(r).
 * EUNSUPPORTED: Gaussian with F64 or CSR input, SRHT with CSR input. EINVAL:
 * OSNAP with nnz_per_col outside 1..16 or not dividing r; SRHT with r > n'. */
int slso_sketch(slso_ctx* ctx, const slso_matrix* X, uint64_t seed, int64_t r,
                const slso_options* opt, double* sx, void* stream);

/* The sketched SVD S X = U Sigma V^T of Algorithm 2 step 2 (the object the
 * paper evaluates): S X by slso_sketch (same seed and options), R = the R of
 * S X by slso_qr_r (Cholesky-QR2, else Householder), then the one-sided
 * Jacobi SVD of R, whose singular values and right singular vectors are
 * those of S X.
 *   sx     (device) r x d doubles of caller scratch (overwritten).
 *   sigma  (device) d doubles: the singular values, descending.
 *   v      (device) d x d doubles, row-major: column j is the right singular
 *          vector of sigma[j], its largest-magnitude entry made positive
 *          (the first such entry when several tie).
 * Errors as slso_sketch and slso_qr_r; the call synchronises the stream
 * (the Jacobi sweeps stop when a sweep rotates nothing). */
int slso_sketch_svd(slso_ctx* ctx, const slso_matrix* X, uint64_t seed,
                    int64_t r, const slso_options* opt, double* sx,
                    double* sigma, double* v, void* stream);

/* Sketched leverage scores (Algorithms 2 and 3, QR form, with Pi_2).
 *   k       columns of Pi_2 (k >= 0; k = 0 means Pi_2 = I, exact sketched
 *           scores ||x_i R^{-1}||^2).
 *   scores  (device) n floats, overwritten with l_i = ||x_i M||^2, where
 *           M = D pinv_rank(R_D) Pi_2, D the power-of-two column
 *           equilibration of X and R_D the R factor (non-negative diagonal)
 *           of the equilibrated sketch.
 *   opt     (host, may be NULL) sketch kind, refinement, rank tolerance.
 *           refine = 1 (dense F32/BF16/FP8 input only, EUNSUPPORTED
 *           otherwise): one more pass over X forms G = (X D)^T (X D) on MFMA
 *           (FP32 accumulation within row chunks, FP64 across them); then
 *           in FP64, G' = R_D^{-T} G R_D^{-1}, R1 = chol(G') and R = R1 R_D,
 *           the R factor of X D itself (a Cholesky-QR step preconditioned by
 *           the sketch; the sketch only needs to make G' well conditioned).
 *           R replaces R_D below (info.flags reports which was used).
 *   info    (host, may be NULL) filled with the rank decision.
 * Synchronises ``stream`` once (to read the rank screen). Returns
 * SLSO_RANK_DEFICIENT when the rank used is below d. ENONFINITE when X holds
 * Inf/NaN; EINVAL for n < 1, d < 1, r < d, k < 0 or a malformed matrix. */
int slso_leverage(slso_ctx* ctx, const slso_matrix* X, uint64_t seed,
                  int64_t r, int64_t k, const slso_options* opt,
                  float* scores, slso_info* info, void* stream);

/* Completes the context's last call made with SLSO_OPT_NO_SYNC (Algorithm
 * 2 steps 2-4 on the device), or the last execution of a graph that
 * captured it (the caller has waited for it): waits for that call's stream,
 * fills info (host, may be NULL) and returns its status; when the device
 * path did not apply (see SLSO_OPT_NO_SYNC) the job is rerun on the
 * synchronous path into the same scores, info->flags then has
 * SLSO_INFO_RERUN and the call's stream holds the rerun's work (that stream
 * must still exist; its input and output buffers too). EINVAL when the
 * context made no such call. */
int slso_leverage_finish(slso_ctx* ctx, slso_info* info);

/* ---- tuned launch shapes ---------------------------------------------------
 * Two passes of slso_leverage have launch shapes whose best choice depends on
 * d, the input type and the device; every choice sums the same terms in the
 * same order, so results are bit-identical whatever is chosen. A table shared
 * by all contexts of the process holds the choice per (pass, d, dtype); a
 * launch without an entry takes the default.
 *   SLSO_TUNE_SCORE: scoring of dense BF16 / FP8 input (d a multiple of 16 up
 *     to 512, k <= 64), rows taken through a ring of 2, 4 or 8 register
 *     buffers per 32-row block (choices 0, 1, 2; default 0).
 *   SLSO_TUNE_COUNTSKETCH: the CountSketch / OSNAP gather of dense F32, BF16
 *     or FP8 input with rows on 4-element boundaries, rows in flight per
 *     bucket wave (choice 0 fewer, 1 more; default 1). */
#define SLSO_TUNE_SCORE 0
#define SLSO_TUNE_COUNTSKETCH 1

/* Times every choice of each tunable pass that X takes with these arguments
 * (one untimed and three timed runs each, on `stream`, which the call
 * synchronises) on X itself, and records the fastest for (pass, X->d,
 * X->dtype). Arguments as for slso_leverage; nothing is written that the
 * caller owns. Calls that overlap with this one on the same context are
 * ordered after it. */
int slso_tune(slso_ctx* ctx, const slso_matrix* X, int64_t r, int64_t k,
              const slso_options* opt, void* stream);
/* The recorded choice (-1: none); record one by hand (-1 removes it). EINVAL:
 * unknown pass, d < 1, choice out of range, choice NULL. Host only. */
int slso_tune_get(int pass, int64_t d, int dtype, int* choice);
int slso_tune_set(int pass, int64_t d, int dtype, int choice);

/* "dec" ordering (Sec. 5.2): perm[0] is the row of the largest score; equal
 * scores keep ascending row index (stable). scores (device) n floats,
 * perm (device) n int32. EINVAL for n < 1 or n >= 2^31. */
int slso_order(slso_ctx* ctx, const float* scores, int64_t n, int32_t* perm,
               void* stream);

/* Orderings for one training epoch by a sampling policy of Algorithm 4
 * step 4 (policies of Sec. 5.2), from P_i = L_i / sum_j L_j (step 3); a
 * score that is not a positive finite number has P_i = 0.
 *   scores  (device) n floats (1 <= n < 2^31).
 *   policy  SLSO_ORDER_DEC: the "dec" order of slso_order (seed and epoch
 *           unused). SLSO_ORDER_SWR ("dec, swr"): out[t], t < n, are n draws
 *           with replacement, in draw order: with integer weights
 *           w_i = floor(L_i 2^(30 - e)), 2^(e-1) <= max L < 2^e, cumulative
 *           C_i and W = C_{n-1}, draw t is the smallest i with
 *           C_i > floor(m_t W / 2^53). SLSO_ORDER_SWOR ("dec, swor"): the
 *           permutation of weighted sampling without replacement, in draw
 *           order: rows by ascending key E_i / L_i (FP32), E_i = 0 - ln u_i,
 *           ties by ascending row, P_i = 0 rows last.
 *   seed, epoch  the draws' stream: item t of an epoch takes one
 *           Philox4x32-10 block, counter (lo32(t), hi32(t), epoch, 5 for swr
 *           or 6 for swor), key (lo32(seed), hi32(seed)); swr uses
 *           m_t = ((w0 << 32) | w1) >> 11, swor u_t = ((w0 >> 8) + 1) 2^-24
 *           and ln u_t by the FP32 logarithm of the Gaussian sketch
 *           generator (see slso_gaussian_sketch_entries).
 *   out     (device) n int32 row indices.
 * EINVAL: bad arguments, an unknown policy, or SLSO_ORDER_SWR without a
 * positive score (the call then synchronises the stream to check W). */
typedef enum {
  SLSO_ORDER_DEC = 0,
  SLSO_ORDER_SWR = 1,
  SLSO_ORDER_SWOR = 2
} slso_order_policy;
int slso_order_sample(slso_ctx* ctx, const float* scores, int64_t n,
                      int32_t policy, uint64_t seed, uint32_t epoch,
                      int32_t* out, void* stream);

/* Device workspace (bytes) a context allocates to run slso_leverage and then
 * slso_order on X with these arguments; nothing is enqueued. Same argument
 * checks and error codes as slso_leverage. */
int slso_workspace_size(const slso_matrix* X, int64_t r, int64_t k,
                        const slso_options* opt, size_t* bytes);

/* ---- serving --------------------------------------------------------------- */
/* A server runs leverage-score jobs that arrive at any time.
 *   - Slots: it has ``slots`` of them, each a context with its own stream and
 *     worker thread; jobs on different slots overlap on the device.
 *   - Admission: a queued job starts when a slot is idle and the workspaces
 *     all slots then hold (slso_workspace_size of their jobs) stay within
 *     ``hbm_budget`` bytes. Idle slots release their workspaces when the head
 *     of the queue waits for memory.
 *   - Order: first in, first out, with backfilling of later jobs that fit,
 *     at most 2 * slots times past a waiting head.
 *   - Results: a job's result equals that of the same slso_leverage
 *     (+ slso_order) call made alone.
 * The caller keeps X, scores and perm allocated until the job has completed,
 * and X must hold its final values when the job is submitted (synchronise the
 * stream that produced it). */
typedef struct slso_server slso_server;

typedef struct {
  slso_matrix X;       /* input, as for slso_leverage                       */
  uint64_t seed;
  int64_t r, k;
  slso_options opt;
  float* scores;       /* (device) n floats                                  */
  int32_t* perm;       /* (device) n int32 "dec" ordering, or NULL          */
} slso_job;

typedef struct {
  int32_t status;      /* slso_leverage / slso_order status of the job       */
  int32_t slot;        /* slot that ran it                                   */
  slso_info info;
  double submit_ms;    /* host steady clock, ms since the server was created */
  double start_ms;     /* admitted to a slot                                 */
  double end_ms;       /* outputs resident (the slot's stream synchronised)  */
} slso_job_result;

typedef struct {
  int64_t queued, running, max_running, completed;
  size_t allocated_bytes, budget_bytes;
} slso_server_counters;

/* EINVAL: out NULL, slots outside [1, 64], hbm_budget 0, or no such device. */
int slso_server_create(slso_server** server, int device, int slots,
                       size_t hbm_budget);
/* Queue a job (the descriptor is copied); *ticket identifies it. Argument
 * errors as slso_leverage; ENOMEM when the job alone exceeds the budget. */
int slso_server_submit(slso_server* server, const slso_job* job,
                       int64_t* ticket);
/* 1 and *result filled when the job has completed (the ticket is then
 * retired), 0 while it is queued or running, EINVAL for an unknown ticket. */
int slso_server_poll(slso_server* server, int64_t ticket,
                     slso_job_result* result);
/* Block until the job completes; fills *result and retires the ticket. */
int slso_server_wait(slso_server* server, int64_t ticket,
                     slso_job_result* result);
int slso_server_stats(slso_server* server, slso_server_counters* stats);
/* Run every queued job to completion, then release the slots. */
int slso_server_destroy(slso_server* server);

/* ---- stages, exposed for verification and composition -------------------- */

/* CountSketch bucket and sign of rows row0 .. row0+n-1 (Sec. 3.1.2):
 * bucket (device) n int32 in [0, r), sign (device) n int8 in {+1, -1}. */
int slso_hash(uint64_t seed, int64_t r, int64_t row0, int64_t n,
              int32_t* bucket, int8_t* sign, void* stream);

/* Gaussian stream entries z(a, b) for a in [0, rows), b in [0, cols)
 * (stream_id 3: sketch entries with a = row of X, b = sketch row;
 * stream_id 4: Pi_2 before its 1/sqrt(k) scale). out (device) rows x cols
 * doubles, row-major. */
int slso_gaussian(uint64_t seed, int32_t stream_id, int64_t rows, int64_t cols,
                  double* out, void* stream);

/* FP32 Gaussian sketch entries G[j][row0 + i] for j in [0, r), i in
 * [0, n): out (device) r x n floats, row-major. Definition (Sec. 2.1 asks
 * for i.i.d. N(0,1) entries; this is the counter-based form used): with
 * (w0, w1, w2, w3) = Philox4x32-10(counter (lo32(q), hi32(q), j, 3),
 * key (lo32(seed), hi32(seed))), q = floor(c / 4) for column c = row0 + i,
 * the pair (wa, wb) = (w0, w1) for c mod 4 in {0, 1} and (w2, w3) otherwise;
 * u1 = ((wa >> 8) + 1) 2^-24, u2 = (wb >> 8) 2^-24, and the value is
 * sqrt(-2 ln u1) cos(2 pi u2) for even c, sin(2 pi u2) for odd c (Box-Muller),
 * evaluated in a fixed sequence of separately rounded FP32 operations
 * (degree-7 polynomial logarithm, Newton reciprocal square root, Taylor
 * cosine and sine by quadrant), so every value is reproducible bit for bit.
 * EINVAL for negative sizes. */
int slso_gaussian_sketch_entries(uint64_t seed, int64_t r, int64_t row0,
                                 int64_t n, float* out, void* stream);

/* Quantile-form Gaussian sketch entries G[j][row0 + i] of the BF16
 * (dtype SLSO_BF16) or FP8 (dtype SLSO_FP8_E4M3) input path, j in [0, r),
 * i in [0, n): out (device) r x n floats, row-major (each value a BF16 or
 * e4m3 number). Definition (Sec. 2.1 asks for i.i.d. N(0,1) entries; these
 * are N(0,1) quantiles on 2^16 equiprobable signed cells, rounded to the
 * input's format): with (w0, w1, w2, w3) = Philox4x32-10(counter (lo32(q),
 * hi32(q), j, 9), key (lo32(seed), hi32(seed))), q = floor(c / 8) for
 * column c = row0 + i, v = the 16-bit half (c & 1 ? high : low) of word
 * w[(c >> 1) & 3]; the value is (-1)^(v >> 15) T[v & 0x7FFF] with
 * T[m] = sqrt(2) erfinv((2 m + 1) / 65536) rounded to nearest even in BF16
 * (SLSO_BF16) or e4m3 (SLSO_FP8_E4M3). The tables are computed once per
 * device. EINVAL for negative sizes or another dtype; EDEVICE when the
 * tables cannot be copied to the current device. */
int slso_gaussian_sketch_entries_q(uint64_t seed, int32_t dtype, int64_t r,
                                   int64_t row0, int64_t n, float* out,
                                   void* stream);

/* R factor of a QR factorisation (Algorithm 2 step 2, QR form) of the m x d
 * matrix a (device, row-major, lda = d, m >= d), which is overwritten.
 * r_out (device) d x d doubles: upper triangle of R with a non-negative
 * diagonal, zeros below (R is unique up to the signs of its rows when a has
 * full column rank; past a zero pivot any valid R may be returned).
 * Path: Cholesky-QR2 over the whole matrix; when its checks fail (the first
 * Gram matrix is not numerically positive definite, or the first pass leaves
 * Q1 too far from orthonormal), Householder QR with 64-column panels; when a
 * panel is too ill-conditioned for that, Householder QR column by column.
 * The call synchronises the stream once per path tried. */
int slso_qr_r(slso_ctx* ctx, double* a, int64_t m, int64_t d, double* r_out,
              void* stream);

/* QR paths (slso_qr_r_path) */
#define SLSO_QR_AUTO 0          /* the cascade of slso_qr_r                  */
#define SLSO_QR_PANEL 1         /* Householder, 64-column panels (then tree) */
#define SLSO_QR_TREE 2          /* Householder, column by column             */
#define SLSO_QR_CHOLQR2 3       /* reported: Cholesky-QR2, one-launch R2     */
#define SLSO_QR_CHOLQR2_FULL 4  /* reported: Cholesky-QR2, blocked R2        */

/* slso_qr_r starting from a given path (SLSO_QR_AUTO, SLSO_QR_PANEL or
 * SLSO_QR_TREE; EINVAL otherwise); *path_used (host, nullable) receives the
 * path that produced r_out (SLSO_QR_CHOLQR2, SLSO_QR_CHOLQR2_FULL,
 * SLSO_QR_PANEL or SLSO_QR_TREE). */
int slso_qr_r_path(slso_ctx* ctx, double* a, int64_t m, int64_t d,
                   double* r_out, int path, int32_t* path_used, void* stream);

/* Solve R X = B in place for upper-triangular R (device, d x d, row-major)
 * and B (device, d x k, row-major) -- the R^{-1} Pi_2 of Algorithm 2 step 3. */
int slso_solve_upper(slso_ctx* ctx, const double* r, int64_t d, double* b,
                     int64_t k, void* stream);

/* Row scores l_i = ||x_i M||^2 for a given M (device, d x k doubles,
 * row-major), Algorithm 2 step 4; scores (device) n floats. The same pass
 * scores rows in slso_leverage. Dense input with k <= 64 runs on the MFMA:
 * M is cut into three BF16 parts (Mh + Mm + Ml within 2^-24 |M|); BF16 and
 * FP8 X multiply all three; FP32 X (d a multiple of 8, 16-byte aligned) is
 * cut the same way as it is read and the six products of parts whose orders
 * add to at most four are taken (split-BF16 emulation of the FP32 product),
 * else the FP32 MFMA multiplies X and M rounded to FP32. Every product is
 * summed in FP32 over 32-column chunks and the chunks in FP64. FP64 input,
 * CSR input and k > 64 use FP64 or FP32 vector arithmetic. */
int slso_scores(slso_ctx* ctx, const slso_matrix* X, const double* m,
                int64_t k, float* scores, void* stream);

/* slso_scores without any device allocation, for callers that cannot
 * allocate: work under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc. Same arguments, kernels and results (bit-identical to
 * slso_scores on the same input). Instead of the context's workspace it uses
 * one fixed device array per GPU of 16 MiB (SLSO_NOALLOC_SCRATCH_BYTES),
 * which holds, 256-byte aligned, d FP64 column factors, M as d x k FP64 and
 * FP32, and for dense non-FP64 input with k <= 64 the three BF16 parts of M
 * (3 x 64 x d x 2 bytes), or for dense input with k > 64 ceil(k / 64) x n
 * FP64 partial sums: dense FP32 / BF16 / FP8 input with k <= 64 fits up to
 * d of about 14000. A call whose buffers exceed the array returns
 * SLSO_EINVAL (nothing is enqueued). The array is set up by slso_create
 * (once per device) and kept until the process ends; it keeps the last
 * call's contents, and every call on one GPU shares it, so calls that
 * overlap on one GPU (other streams, other contexts, other threads) race:
 * order them on one stream or with events. */
#define SLSO_NOALLOC_SCRATCH_BYTES (16ll << 20)
int slso_scores_noalloc(slso_ctx* ctx, const slso_matrix* X, const double* m,
                        int64_t k, float* scores, void* stream);

/* ---- measurement ---------------------------------------------------------- */

/* Process-wide launch profiler. While enabled, HIP events are recorded on
 * the launch stream around every launch of the library's kernels (grouped by
 * kernel id). slso_profile_read synchronises the current device, adds the
 * elapsed milliseconds and launch counts of kernel ids 0 .. n-1 into ms and
 * launches (host arrays of n entries, each may be NULL), resets the totals
 * and returns the number of kernel ids; slso_profile_name gives the name of
 * an id ("" when out of range). */
int slso_profile_enable(int on);
int slso_profile_read(double* ms, int64_t* launches, int n);
const char* slso_profile_name(int id);
/* Restrict recording to kernel id ``id`` (-1: every kernel, the default), so
 * that timing one kernel adds two events per launch of that kernel only.
 * EINVAL for an id out of range. */
int slso_profile_only(int id);

#ifdef __cplusplus
}
#endif
#endif /* SLSO_H */
