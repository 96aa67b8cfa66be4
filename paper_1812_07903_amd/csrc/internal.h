// Host-side launch interfaces between the kernel translation units and the
// C ABI layer. Every launcher enqueues on the given stream and never
// synchronises.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.h"

struct slso_ctx;

namespace slso {

// ---- launch profiler (slso_capi.hip) ----------------------------------------
// When enabled (slso_profile_enable), HIP events are recorded on the launch
// stream around every launch of the listed kernels and resolved on read.
enum KernelId : int {
  kKHash = 0,
  kKSortHist,
  kKSortScan,
  kKSortScatter,
  kKOffsets,
  kKColmax,
  kKSketch,
  kKQrNode,
  kKQrUpdate,
  kKQrExtract,
  kKTrsm,
  kKScore,
  kKGauss,
  kKGaussSketch,
  kKGram,
  kKChol,
  kKCqGram,
  kKCqSum,
  kKCqChol,
  kKCqQ1,
  kKCqZ,
  kKCqRecon,
  kKCqW,
  kKCqUpdate,
  kKCq2Gram,
  kKCq2GramEdge,
  kKCq2GramSum,
  kKCq2Chol,
  kKCq2Solve,
  kKCq2R,
  kKCount
};
void prof_begin(int kid, hipStream_t s);
void prof_end(int kid, hipStream_t s);

// ---- tuned launch shapes (slso_capi.hip) -------------------------------------
// Passes with launch shapes chosen per (d, dtype) by slso_tune (the values
// of SLSO_TUNE_*); every choice gives bit-identical results.
constexpr int kTuneScore = 0;        // score_q register ring: 2, 4, 8 units
constexpr int kScoreRingChoices = 3;
constexpr int kTuneCountSketch = 1;  // CountSketch rows in flight: less, more
constexpr int kCsChoices = 2;
// The recorded choice for (pass, d, dtype), or -1. Thread-safe.
int tune_choice(int pass, int64_t d, int dtype);

// ---- context internals used by the serving loop (slso_capi.hip) -------------
// Wait for the context's last use of its workspace and free it.
int ctx_release_workspace(::slso_ctx* c);
int ctx_reserve_workspace(::slso_ctx* c, size_t bytes);

// ---- streams / ordering (k_sort.hip) ----------------------------------------
// keys[i] = bucket h(row0+i), vals[i] = i | (sign bit << 31).
void launch_hash_pack(const HashCoeffs& hb, const HashCoeffs& hs, int64_t r,
                      int64_t row0, int64_t n, uint32_t* keys, uint32_t* vals,
                      hipStream_t s);
// OSNAP entries, nnz per row: entry e = j n + i (hash j, row i) gets
// keys[e] = j (r / nnz) + (P_1j(i) mod (r / nnz)), vals[e] = i | (sign << 31).
void launch_hash_pack_osnap(const OsnapCoeffs& h, int nnz, int64_t r,
                            int64_t n, uint32_t* keys, uint32_t* vals,
                            hipStream_t s);
void launch_hash_out(const HashCoeffs& hb, const HashCoeffs& hs, int64_t r,
                     int64_t row0, int64_t n, int32_t* bucket, int8_t* sign,
                     hipStream_t s);
// out[a * cols + b] = z(a, b) / divisor
void launch_gaussian(uint64_t seed, uint32_t stream_id, int64_t rows,
                     int64_t cols, double divisor, double* out, hipStream_t s);
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
// Order-preserving descending keys of FP32 scores.
void launch_score_keys(const float* scores, int64_t n, uint32_t* keys,
                       hipStream_t s);
// Stable LSD radix sort of (key, value) pairs on bits [0, nbits); vals_in may
// be NULL (values = input positions). Results land in keys_out / vals_out.
size_t radix_sort_scratch_bytes(int64_t n);
void radix_sort_pairs(const uint32_t* keys_in, const uint32_t* vals_in,
                      uint32_t* keys_out, uint32_t* vals_out,
                      uint32_t* keys_tmp, uint32_t* vals_tmp, int64_t n,
                      int nbits, void* scratch, hipStream_t s);
// offsets[b] = first sorted position with key >= b, b in [0, r]
void launch_bucket_offsets(const uint32_t* sorted_keys, int64_t n, int64_t r,
                           int32_t* offsets, hipStream_t s);

// ---- SRHT sketch (k_srht.hip) -------------------------------------------------
// n' = the power of two >= n; scratch: srht_scratch_bytes(n, d).
// sx = (1/sqrt(r)) P H D X times colfac[j] per column (nullable); dense input
// (dtype 0 F64, 1 F32, 2 BF16, 3 FP8 codes). -1 when r > n'.
int64_t srht_rows_padded(int64_t n);
size_t srht_scratch_bytes(int64_t n, int64_t d);
int launch_srht(const void* x, int dtype, int64_t n, int64_t d, int64_t ld,
                uint64_t seed, int64_t r, const double* colfac, void* scratch,
                double* sx, hipStream_t s);

// ---- sampling policies (k_sample.hip) ---------------------------------------
// dec-swor: keys[i] = bits of E_i / L_i (FP32, +inf for probability 0), to be
// sorted ascending with the row index as the value.
void launch_swor_keys(const float* scores, int64_t n, uint64_t seed,
                      uint32_t epoch, uint32_t* keys, hipStream_t s);
// dec-swr: the exact cumulative integer weights (first n int64 of scratch,
// swr_scratch_bytes(n) in all), then the n draws from them.
size_t swr_scratch_bytes(int64_t n);
void launch_swr_prefix(const float* scores, int64_t n, void* scratch,
                       hipStream_t s);
void launch_swr_draws(const void* scratch, int64_t n, uint64_t seed,
                      uint32_t epoch, int32_t* out, hipStream_t s);

// ---- sketch (k_sketch.hip) ---------------------------------------------------
void launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s);
// colmax_bits: d u64 (bit patterns of non-negative doubles), zero-filled by
// the caller; nonfinite: int flag set to 1 on Inf/NaN.
void launch_colmax(const void* x, int dtype, int format, int64_t n, int64_t d,
                   int64_t ld, const int64_t* row_ptr, const int32_t* col_idx,
                   int64_t nnz, const float* col_scale, const float* row_scale,
                   uint64_t* colmax_bits, int* nonfinite, hipStream_t s);
void launch_colscale(const uint64_t* colmax_bits, int64_t d, double* dscale,
                     hipStream_t s);
// out[j] = a[j] * b[j] (a NULL: 1)
void launch_mul_scale(const double* a, const float* b, int64_t d, double* out,
                      hipStream_t s);
// sx[b] = (sum_{entries of bucket b, ascending row} sign * x_row) * sscale *
// dscale (FP8: codes; the caller folds the column scales into dscale;
// sscale: 1 for CountSketch, 1/sqrt(nnz) for OSNAP)
void launch_countsketch(const void* x, int dtype, int format, int64_t n,
                        int64_t d, int64_t ld, const int64_t* row_ptr,
                        const int32_t* col_idx, const float* col_scale,
                        const float* row_scale, const uint32_t* sorted_vals,
                        const int32_t* offsets, int64_t r,
                        const double* dscale, double* sx, hipStream_t s,
                        double sscale = 1.0);

// CountSketch and column equilibration in one pass over dense F32 / BF16 /
// FP8 input (ld and the base address multiples of 4 elements): sx[b] =
// (sum_{entries of bucket b, ascending row} sign * x_row) * sscale * cs (cs:
// the FP8 column scales, else 1) WITHOUT the equilibration D, which the consumer applies (qr_factor's
// dsc), and dscale = D from the column max-abs values (times |cs|), as
// launch_colmax + launch_colscale would give. parts: countsketch_colmax_groups(r)
// * d floats of scratch. False, with nothing launched, when the input does
// not qualify.
int64_t countsketch_colmax_groups(int64_t r);
bool countsketch_colmax_ok(const void* x, int dtype, int format, int64_t ld);
// choice: the launch shape (rows in flight per bucket wave, see
// kTuneCountSketch); -1 takes the tuned choice for (d, dtype), else the
// default.
bool launch_countsketch_colmax(const void* x, int dtype, int64_t d, int64_t ld,
                               const float* col_scale,
                               const uint32_t* sorted_vals,
                               const int32_t* offsets, int64_t r, float* parts,
                               int* nonfinite, double* dscale, double* sx,
                               hipStream_t s, double sscale = 1.0,
                               int choice = -1);

// ---- QR (k_qr.hip) -----------------------------------------------------------
// A second stream and two events that let the QR overlap one panel's
// trailing update with the next panel's factorisation (side == nullptr:
// everything on the calling stream).
struct QrStreams {
  hipStream_t side = nullptr;
  hipEvent_t factored = nullptr;
  hipEvent_t bulk_done = nullptr;
};

size_t qr_scratch_bytes(int64_t m, int64_t d);
// R factor of a (m x d, lda = d, m >= d) into r_out (d x d, positive
// diagonal, zeros below it) by Cholesky-QR2 (k_cholqr.hip); a is overwritten
// by the first-pass Q1 (left as it was when R is not wanted and m d <= 2^24:
// Q1 is then formed out of place). *status (device int): 0 done; 2: r_out not yet
// written, call qr_factor_finish; 1: Cholesky-QR2 does not apply (a too
// ill-conditioned or rank deficient): a and r_out are unusable, the caller
// factors the original matrix with qr_factor_panel; 3: one pass taken (R =
// R1, see one_pass). dsc (nullable): powers of two that scale a's columns
// as they are read; the factorisation is then that of a diag(dsc), with the
// same rounding as if a had been scaled first. one_pass: 0 two passes; 2
// one when the condition estimate of R1 bounds the score error far below
// the gate; 1 the same with the looser bound of a preconditioner (both only
// where 2 m d^2 >= 2^31: smaller factorisations always take two passes).
void qr_factor(double* a, int64_t m, int64_t d, double* r_out, void* scratch,
               int* status, const QrStreams& qs, hipStream_t s,
               bool want_r = true, double* dstat = nullptr,
               const double* dsc = nullptr, int one_pass = 0);
// After status 2: the second pass's blocked Cholesky and R = R2 R1 (status
// set again, 0 or 1).
void qr_factor_finish(int64_t m, int64_t d, double* r_out, void* scratch,
                      int* status, hipStream_t s, bool want_r = true,
                      double* dstat = nullptr);
// want_r = false: R is not formed; dstat[0..1] receive min and max |R_jj|, and
// the scratch keeps R^{-1} in factored form for qr_apply_rinv (and the factors
// for qr_write_r) until the scratch is reused. form: 0 two passes ending in
// status 0, 1 two passes through status 2, 2 one pass (status 3).
void qr_apply_rinv(int64_t m, int64_t d, void* scratch, int form, double* b,
                   int64_t k, hipStream_t s);  // b (d x k) <- R^{-1} b
void qr_write_r(int64_t m, int64_t d, double* r_out, void* scratch, int form,
                hipStream_t s);
// no-sync forms of qr_factor_finish and qr_apply_rinv (see cholqr2_*_dev)
void qr_finish_dev(int64_t m, int64_t d, void* scratch, const int* status,
                   int* p2, double* dstat, hipStream_t s);
void qr_apply_rinv_dev(int64_t m, int64_t d, void* scratch, const int* f,
                       double* b, int64_t k, hipStream_t s);
// Householder QR of a in place, r_out as above. 64-column panels by
// Cholesky-QR2 with Householder reconstruction (k_cqr.hip), the remaining
// columns by the tree path. *fail (device int) is set to 1 when a panel is
// too ill-conditioned for Cholesky-QR: a and r_out are then unusable and the
// caller reruns qr_factor_robust on the original matrix.
void qr_factor_panel(double* a, int64_t m, int64_t d, double* r_out,
                     void* scratch, int* fail, const QrStreams& qs,
                     hipStream_t s);
// The same factorisation by the tree path alone (every column).
void qr_factor_robust(double* a, int64_t m, int64_t d, double* r_out,
                      void* scratch, hipStream_t s);
// whole-matrix Cholesky-QR2 (k_cholqr.hip)
size_t cholqr2_scratch_bytes(int64_t m, int64_t d);
// (qs is reserved for overlapping parts of the factorisation)
void cholqr2_factor(double* a, int64_t m, int64_t d, double* r_out,
                    void* scratch, int* status, const QrStreams& qs,
                    hipStream_t s, bool want_r, double* dstat,
                    const double* dsc, int one_pass);
void cholqr2_finish(int64_t m, int64_t d, double* r_out, void* scratch,
                    int* status, hipStream_t s, bool want_r, double* dstat);
void cholqr2_write_r(int64_t m, int64_t d, double* r_out, void* scratch,
                     int form, hipStream_t s);
// The no-sync forms (every decision on the device): the second pass's
// Cholesky when *status = 2 (p2 receives its exit flag, set on failure), the
// choice of R^{-1}'s form and of the synchronous fallback (f[0..3]), and
// the conditional product b <- R^{-1} b.
void cholqr2_finish_dev(int64_t m, int64_t d, void* scratch, const int* status,
                        int* p2, double* dstat, hipStream_t s);
void cholqr2_decide_dev(const int* status, const int* p2, const double* dstat,
                        double tol, const int* nonfinite, int* f,
                        hipStream_t s);
void cholqr2_apply_rinv_dev(int64_t m, int64_t d, void* scratch, const int* f,
                            double* b, int64_t kk, hipStream_t s);
void cholqr2_apply_rinv(int64_t m, int64_t d, void* scratch, int form,
                        double* b, int64_t k, hipStream_t s);
// 64-column panel path (k_cqr.hip)
size_t cqr_scratch_bytes(int64_t m, int64_t d);
int64_t cqr_panels(int64_t m, int64_t d);
// all 64-column panels (d / 64 of them), overlapped as described above
void cqr_factor(double* a, int64_t m, int64_t d, void* scratch, int* flag,
                const QrStreams& qs, hipStream_t s);
// diag stats of upper-triangular r (d x d): out[0] = min |r_jj|, out[1] = max
void launch_diag_stats(const double* r, int64_t d, double* out, hipStream_t s);

// ---- triangular solve / Jacobi (k_solve.hip) --------------------------------------
// Solve R X = B in place (R upper triangular d x d, B d x k row-major).
// With scratch (trsm_blocked_scratch(d, k) bytes) the blocked solver with
// 64 x 64 diagonal inverses on MFMA runs (k_cqr.hip); without it, 64-row
// blocks with one wave per right-hand side.
void solve_upper(const double* r, int64_t d, double* b, int64_t k,
                 hipStream_t s, double* scratch = nullptr);
size_t trsm_blocked_scratch(int64_t d, int64_t k);
// R X = B (transposed = false) or R^T X = B (true), in place
void trsm_blocked(const double* r, int64_t d, double* b, int64_t k,
                  bool transposed, void* scratch, hipStream_t s);
// pinv of the rank-`rank` truncation of r applied to b: out = V' S'^-1 U'^T b.
// Works on copies; sigma (host) receives the d singular values, descending.
size_t jacobi_scratch_bytes(int64_t d, int64_t k);
// SVD of an upper-triangular d x d R (row-major) by one-sided Jacobi:
// sigma (device, d, descending) and v (device, d x d row-major, column j the
// right singular vector of sigma[j], largest-magnitude entry positive). r may
// alias v. Synchronises the stream. 0 on success.
size_t jacobi_svd_scratch_bytes(int64_t d);
int jacobi_svd(const double* r, int64_t d, double* sigma, double* v,
               void* scratch, hipStream_t s);
int jacobi_truncated_apply(const double* r, int64_t d, const double* b,
                           int64_t k, double rank_tol, double* out,
                           int64_t* rank_out, void* scratch, hipStream_t s);
// out = I (d x d)
void launch_eye(double* out, int64_t d, hipStream_t s);
// m_out[j][c] = scale_row[j] * m[j][c] as float (m_out32) and/or double
void launch_scale_rows(const double* m, const double* scale_row, int64_t d,
                       int64_t k, double* out64, float* out32, hipStream_t s);

// ---- Gaussian sketch, quantile form (k_gauss_q.hip) ----------------------------
// Copy the quantile tables (BF16 and e4m3 magnitudes) to the current device;
// 0 on success. Idempotent per device.
int init_quantile_tables(int device);
bool gauss_q_dtype(int dtype);
size_t gauss_q_partial_bytes(int64_t n, int64_t r, int64_t d);
// partial[s][j][c] = FP32 sums of G[j][i] x[i][c] over slice s of the rows
// (BF16 input: dtype 2; FP8 codes: dtype 3, without their column scales);
// *splits = the number of slices. With colmax (zero-filled by the caller),
// the column max-abs values (times |col_scale| for FP8) are folded into it
// as FP64 bit patterns and *nonfinite is set on Inf / NaN.
void launch_gauss_q_sketch(const void* x, int dtype, int64_t n, int64_t d,
                           int64_t ld, uint64_t seed, int64_t r,
                           float* partial, int64_t* splits,
                           const float* col_scale, uint64_t* colmax,
                           int* nonfinite, hipStream_t s);
// partial[s][i][j] = FP32 sums of x[.][i] x[.][j] over slice s of the rows,
// for i, j in 256-column blocks A <= B (BF16 / FP8 input, as above)
size_t gram_q_partial_bytes(int64_t n, int64_t d);
void launch_gram_q(const void* x, int dtype, int64_t n, int64_t d, int64_t ld,
                   float* partial, int64_t* splits, hipStream_t s);
// out[j * n + i] = quantile-form entry G[j][row0 + i] (fmt 0: BF16, 1: e4m3)
void launch_gauss_q_entries(uint64_t seed, int64_t r, int64_t n, int64_t row0,
                            int fmt, float* out, hipStream_t s);

// ---- Gaussian sketch and Gram matrix (k_gauss.hip) -------------------------
// dtype: slso_dtype of a dense X (F32, BF16 or FP8-e4m3 with col_scale)
size_t gauss_partial_bytes(int64_t n, int64_t r, int64_t d, int dtype);
// sx = G X / sqrt(r) (times col_scale for FP8 and dscale when given); BF16
// and FP8 input take the quantile form of the entries (k_gauss_q.hip), F32
// input the FP32 Box-Muller generator
void launch_gauss_sketch(const void* x, int dtype, int64_t n, int64_t d,
                         int64_t ld, const float* col_scale, uint64_t seed,
                         int64_t r, const double* dscale, float* partial,
                         double* sx, hipStream_t s);
// BF16 / FP8 input: the sketch and the column equilibration in one pass over
// X. colmax_bits (d u64) is zero-filled here, dscale_out = D from the column
// max-abs values (times |col_scale| for FP8, as launch_colmax +
// launch_colscale give), sx = G X D / sqrt(r) (times col_scale for FP8);
// *nonfinite is set on Inf / NaN.
void launch_gauss_sketch_eq(const void* x, int dtype, int64_t n, int64_t d,
                            int64_t ld, const float* col_scale, uint64_t seed,
                            int64_t r, uint64_t* colmax_bits, int* nonfinite,
                            double* dscale_out, float* partial, double* sx,
                            hipStream_t s);
size_t gram_partial_bytes(int64_t n, int64_t d, int dtype);
// g (d x d) = Dc X^T X Dc with Dc = diag(col_scale (FP8) * dscale); FP32
// input on the FP64 MFMA (exact products, FP64 sums), BF16/FP8 on the BF16
// MFMA (exact products, FP32 sums within row chunks, FP64 across them)
void launch_gram(const void* x, int dtype, int64_t n, int64_t d, int64_t ld,
                 const float* col_scale, const double* dscale, void* scratch,
                 double* g, hipStream_t s);
// out[j * n + i] = FP32 Gaussian sketch entry G[j][row0 + i]
void launch_gauss_entries(uint64_t seed, int64_t r, int64_t n, int64_t row0,
                          float* out, hipStream_t s);

// ---- Cholesky refinement (k_chol.hip) ----------------------------------------
// Solve R^T X = B in place (R upper triangular d x d, B d x k).
void solve_upper_trans(const double* r, int64_t d, double* b, int64_t k,
                       hipStream_t s, double* scratch = nullptr);
void launch_transpose(const double* a, int64_t d, double* out, hipStream_t s);
// Upper Cholesky factor of symmetric positive definite g (d x d row-major,
// upper triangle read, not modified) into r (zeros below the diagonal) by
// the tiled blocked Cholesky of the sketch's QR (k_cholqr.hip: 64 x 64
// tiles, one launch per block step, MFMA products); *flag (device int, 0 on
// entry) set to 1 when a pivot falls to 1e-13 of its diagonal entry.
// scratch: chol_tiled_scratch_bytes(d) bytes of device memory.
size_t chol_tiled_scratch_bytes(int64_t d);
void chol_tiled(const double* g, int64_t d, double* r, void* scratch,
                int* flag, hipStream_t s);
// c = a b for upper-triangular a, b (d x d)
void launch_trmm_upper(const double* a, const double* b, int64_t d, double* c,
                       hipStream_t s);

// ---- scoring, BF16 / FP8 input with M resident in LDS (k_score_q.hip) ---------
// applies to dense BF16 (dtype 2) / FP8 (3) input with d % 16 == 0,
// d <= 512, k <= 64, rows on 16-byte (BF16) or 8-byte (FP8) boundaries
bool score_q_ok(const void* x, int dtype, int format, int64_t d, int64_t ld,
                int64_t k);
size_t score_q_scratch_bytes(int64_t d);
// scores[i] = ||x_i M||^2 with M = m64 (d x k FP64, row-major; FP8: the
// column scales already folded into its rows); scratch: score_q_scratch_bytes
// choice: the register ring (kTuneScore); -1 takes the tuned choice for
// (d, dtype), else the default
void launch_score_q(const void* x, int dtype, int64_t n, int64_t d, int64_t ld,
                    const double* m64, int64_t k, void* scratch, float* scores,
                    hipStream_t s, int choice = -1);

// ---- scoring (k_score.hip) ---------------------------------------------------
void launch_scores(const void* x, int dtype, int format, int64_t n, int64_t d,
                   int64_t ld, const int64_t* row_ptr, const int32_t* col_idx,
                   const float* col_scale, const float* row_scale,
                   const double* m64, const float* m32, int64_t k,
                   float* scores, hipStream_t s, double* partial);
// bytes of the FP64 partial-sum buffer needed by launch_scores (0 if none)
size_t scores_partial_bytes(int64_t n, int64_t d, int64_t k, int format,
                            int dtype);

}  // namespace slso
