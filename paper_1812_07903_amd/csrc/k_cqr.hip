// Blocked Householder QR of the sketch with 64-column panels (Algorithm 2
// step 2 in QR form; only R is kept).
//
// Panel factorisation. A panel P (the m' = m - j0 active rows of 64 columns)
// is factored by Cholesky-QR twice over all its rows:
//   G1 = P^T P = R1^T R1,   Q1 = P R1^{-1},   G2 = Q1^T Q1 = R2^T R2,
//   Q = Q1 R2^{-1},         R = R2 R1.
// The Gram matrices are summed over row blocks on the FP64 MFMA; the 64 x 64
// Cholesky factorisations and triangular inverses run in one workgroup.
// Householder reconstruction (Ballard, Demmel, Grigori, Jacquelin, Knight &
// Nguyen, "Reconstructing Householder vectors from tall-skinny QR", 2014)
// turns Q into the Householder vectors of the panel:
//   - a sign-choosing LU without pivoting of the top block, Q_top - S = L U,
//     with every pivot of magnitude >= 1;
//   - Y = [L; Q_bottom U^{-1}] and T = -U S L^{-T}, so that
//     I - Y T Y^T = H_1 ... H_64;
//   - the panel's Householder R is S R.
//
// Trailing update. C <- (I - Y T Y^T)^T C = C - Y T^T (Y^T C) with
//   Y^T C = L^T C_top + M2^T (Q1^T C - Q1_top^T C_top),  M2 = R2^{-1} U^{-1},
//   Y_bottom T^T W = Q1_bottom (M2 T^T W).
// Q1^T C is summed over row blocks, like the Gram matrices. The bottom part of
// Y is never formed, because Q is not needed.
//
// Robustness. A Cholesky pivot below 1e-10 of its column's squared norm (or,
// in the second pass, below 1e-10) means the panel is too ill-conditioned for
// Cholesky-QR. It raises a device flag; every later kernel of this path then
// returns at once, and the caller reruns the whole factorisation with the
// column-by-column tree path of k_qr.hip on the original matrix. Columns
// beyond the last full 64-column panel are always factored by that path.
//
// MFMA operand layout (v_mfma_f64_16x16x4f64): A operand lane l = A[l%16][l/16],
// B operand lane l = B[l/16][l%16], result register v of lane l =
// D[4v + l/16][l%16]. 64 x 64 tiles in LDS have a row stride of 65 doubles;
// wave w of a 256-thread workgroup owns tile rows 16w .. 16w + 15.
#include "internal.h"
#include "tile64.h"

namespace slso {
namespace {

constexpr int kRG = 128;   // rows per workgroup: Gram and Q1 passes
constexpr int kRZ = 512;   // rows per part: Q1^T C
constexpr int kRU = 256;   // rows per workgroup: trailing update
constexpr double kTol1 = 1e-10;  // pivot / column squared norm, first pass
constexpr double kTol2 = 1e-10;  // pivot, second pass (G2 ~ I)

// ---- K1: partial Gram matrices P^T P of row blocks ----------------------------
__global__ void __launch_bounds__(256)
    cq_gram_kernel(const double* __restrict__ A, int64_t lda, int64_t m,
                   int64_t j0, double* __restrict__ gpart,
                   const int* __restrict__ flag) {
  __shared__ double T[kTile];
  if (*flag) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t r0 = j0 + static_cast<int64_t>(blockIdx.x) * kRG;
  dbl4 acc[4];
  zero4(acc);
  Stage v;
  stage_load(v, A + r0 * lda + j0, lda, m - r0, kP, t);
  for (int c = 0; c < kRG / kP; ++c) {
    const int64_t rb = r0 + c * kP;
    if (rb >= m) break;
    __syncthreads();
    stage_store(T, v, t);
    __syncthreads();
    if (c + 1 < kRG / kP && rb + kP < m)
      stage_load(v, A + (rb + kP) * lda + j0, lda, m - rb - kP, kP, t);
    mm64<true>(T, T, acc, lane, w);
  }
  store_acc_global(gpart + static_cast<int64_t>(blockIdx.x) * kP * kP, kP, acc,
                   1.0, lane, w);
}

// ---- sum of partial 64 x 64 matrices (fixed order) ------------------------------
__global__ void __launch_bounds__(256)
    cq_sum_kernel(const double* __restrict__ parts, int64_t nparts,
                  double* __restrict__ out, const int* __restrict__ flag) {
  if (*flag) return;
  const int e = blockIdx.x * 256 + threadIdx.x;
  out[e] = sum_parts(parts, nparts, kP * kP, e);
}

// ---- K2: R1 = chol(G1), R1^{-1} ------------------------------------------------
__global__ void __launch_bounds__(256)
    cq_chol1_kernel(const double* __restrict__ g, double* __restrict__ r1,
                    double* __restrict__ r1i, int* __restrict__ flag) {
  __shared__ double T0[kTile];
  __shared__ double T1[kTile];
  __shared__ double lim[kP];
  __shared__ double tmp[4][16][17];
  __shared__ int bad;
  if (*flag) return;
  const int t = threadIdx.x;
  load_tile(T0, g, kP, kP, kP, t);
  __syncthreads();
  if (t < kP) lim[t] = kTol1 * T0[t * kS + t];
  __syncthreads();
  if (!chol64b(T0, T1, lim, &bad, tmp, t)) {
    if (t == 0) *flag = 1;
    return;
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u;
    r1[e] = T0[(e >> 6) * kS + (e & 63)];
    r1i[e] = T1[(e >> 6) * kS + (e & 63)];
  }
}

// ---- K3: Q1 = P R1^{-1} in place, partial G2 = Q1^T Q1 --------------------------
__global__ void __launch_bounds__(256)
    cq_q1_kernel(double* __restrict__ A, int64_t lda, int64_t m, int64_t j0,
                 const double* __restrict__ r1i, double* __restrict__ gpart,
                 const int* __restrict__ flag) {
  __shared__ double T[kTile];
  __shared__ double Ri[kTile];
  if (*flag) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int p = lane & 15, q = lane >> 4;
  const int64_t r0 = j0 + static_cast<int64_t>(blockIdx.x) * kRG;
  Stage v;
  stage_load(v, A + r0 * lda + j0, lda, m - r0, kP, t);
  load_tile(Ri, r1i, kP, kP, kP, t);
  dbl4 g2[4];
  zero4(g2);
  for (int c = 0; c < kRG / kP; ++c) {
    const int64_t rb = r0 + c * kP;
    if (rb >= m) break;
    __syncthreads();
    stage_store(T, v, t);
    __syncthreads();
    if (c + 1 < kRG / kP && rb + kP < m)
      stage_load(v, A + (rb + kP) * lda + j0, lda, m - rb - kP, kP, t);
    dbl4 acc[4];
    zero4(acc);
    mm64<false>(T, Ri, acc, lane, w);
    __syncthreads();
    store_acc(T, acc, 1.0, lane, w);
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) {
        const int64_t row = rb + 16 * w + 4 * vv + q;
        if (row < m) A[row * lda + j0 + 16 * bj + p] = acc[bj][vv];
      }
    __syncthreads();
    mm64<true>(T, T, g2, lane, w);
  }
  store_acc_global(gpart + static_cast<int64_t>(blockIdx.x) * kP * kP, kP, g2,
                   1.0, lane, w);
}

// ---- K4: partial Z = Q1^T C over row parts x 64-column blocks -------------------
__global__ void __launch_bounds__(256)
    cq_z_kernel(const double* __restrict__ A, int64_t lda, int64_t m, int64_t j0,
                int64_t ncols, int64_t cb0, const double* __restrict__ q1top,
                double* __restrict__ zpart, int64_t ldz,
                const int* __restrict__ flag) {
  __shared__ double TQ[kTile];
  __shared__ double TC[kTile];
  if (*flag) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int p = lane & 15, q = lane >> 4;
  const int64_t r0 = j0 + static_cast<int64_t>(blockIdx.x) * kRZ;
  const int64_t c0 = (cb0 + blockIdx.y) * kP;  // trailing column
  const int64_t nc = ncols - c0 < kP ? ncols - c0 : kP;
  const int64_t cc = j0 + kP + c0;
  dbl4 acc[4];
  zero4(acc);
  // the panel's top 64 rows hold its R by now: their Q1 comes from the copy
  Stage vq, vc;
  if (r0 == j0)
    stage_load(vq, q1top, kP, kP, kP, t);
  else
    stage_load(vq, A + r0 * lda + j0, lda, m - r0, kP, t);
  stage_load(vc, A + r0 * lda + cc, lda, m - r0, nc, t);
  for (int c = 0; c < kRZ / kP; ++c) {
    const int64_t rb = r0 + c * kP;
    if (rb >= m) break;
    __syncthreads();
    stage_store(TQ, vq, t);
    stage_store(TC, vc, t);
    __syncthreads();
    if (c + 1 < kRZ / kP && rb + kP < m) {
      stage_load(vq, A + (rb + kP) * lda + j0, lda, m - rb - kP, kP, t);
      stage_load(vc, A + (rb + kP) * lda + cc, lda, m - rb - kP, nc, t);
    }
    mm64<true>(TQ, TC, acc, lane, w);
  }
  double* Z = zpart + static_cast<int64_t>(blockIdx.x) * kP * ldz + c0;
#pragma unroll
  for (int bj = 0; bj < 4; ++bj)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int col = 16 * bj + p;
      if (col < nc) Z[(16 * w + 4 * v + q) * ldz + col] = acc[bj][v];
    }
}

// Z summed over the row parts (fixed order): zsum[i][c], c_lo <= c < c_hi
__global__ void __launch_bounds__(256)
    cq_zsum_kernel(const double* __restrict__ zpart, int64_t nz, int64_t ldz,
                   int64_t c_lo, int64_t c_hi, double* __restrict__ zsum,
                   const int* __restrict__ flag) {
  if (*flag) return;
  const int64_t w = c_hi - c_lo;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (e >= kP * w) return;
  const int64_t i = e / w, c = c_lo + e % w;
  zsum[i * ldz + c] = sum_parts(zpart, nz, kP * ldz, i * ldz + c);
}

// ---- K5: second Cholesky, reconstruction, T, M2, the panel's R ----------------
struct ReconLds {
  double T0[kTile], T1[kTile], T2[kTile], T3[kTile];
  double lim[kP], Sg[kP];
  double tmp[4][16][17];
  int bad;
};

// R2 = chol(G2) and R2^{-1} for G2 = I + E with small E (after one
// Cholesky-QR pass E is of the order of the unit roundoff times the panel's
// squared condition number): R2 = I + F with F upper triangular solving
// F + F^T = E - F^T F, by the fixed-point iteration F <- up(E - F^T F)
// (up: strict upper part plus half the diagonal; three steps from F = up(E)
// reach rounding level when |E| <= 1e-7 elementwise), and
// R2^{-1} = I - F + F^2 - F^3 (the next term is below rounding).
// G in T0 on entry; R2 in T0 and R2^{-1} in T1 on return; T2 is scratch.
__device__ __forceinline__ void chol_near_identity(double* T0, double* T1,
                                                   double* T2, int t) {
  const int lane = t & 63, w = t >> 6;
  // T2 <- E = G - I (full), T0 <- F0 = up(E)
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u;
    const int i = e >> 6, j = e & 63;
    const double ev = T0[i * kS + j] - (i == j ? 1.0 : 0.0);
    T2[i * kS + j] = ev;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u;
    const int i = e >> 6, j = e & 63;
    const double ev = T2[i * kS + j];
    T0[i * kS + j] = i < j ? ev : (i == j ? 0.5 * ev : 0.0);
  }
  __syncthreads();
  for (int it = 0; it < 3; ++it) {
    dbl4 acc[4];
    zero4(acc);
    mm64<true>(T0, T0, acc, lane, w);  // F^T F
    __syncthreads();
    const int p = lane & 15, q = lane >> 4;
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * w + 4 * v + q, j = 16 * bj + p;
        const double m = T2[i * kS + j] - acc[bj][v];
        T0[i * kS + j] = i < j ? m : (i == j ? 0.5 * m : 0.0);
      }
    __syncthreads();
  }
  // R2^{-1} = I - F + F^2 - F^3 = I - F (I - F (I - F))
  {
    const int p = lane & 15, q = lane >> 4;
    // T1 <- I - F
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = t + 256 * u;
      const int i = e >> 6, j = e & 63;
      T1[i * kS + j] = (i == j ? 1.0 : 0.0) - T0[i * kS + j];
    }
    __syncthreads();
    for (int it = 0; it < 2; ++it) {
      dbl4 acc[4];
      zero4(acc);
      mm64<false>(T0, T1, acc, lane, w);  // F X
      __syncthreads();
#pragma unroll
      for (int bj = 0; bj < 4; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * w + 4 * v + q, j = 16 * bj + p;
          T1[i * kS + j] = (i == j ? 1.0 : 0.0) - acc[bj][v];
        }
      __syncthreads();
    }
  }
  // T0 <- R2 = I + F
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u;
    const int i = e >> 6, j = e & 63;
    if (i == j) T0[i * kS + j] += 1.0;
  }
  __syncthreads();
}

// max |G - I| over a 64 x 64 tile, the same value in every thread
__device__ __forceinline__ double dist_identity(const double* T, double* red,
                                                int t) {
  double em = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u;
    const int i = e >> 6, j = e & 63;
    const double v = fabs(T[i * kS + j] - (i == j ? 1.0 : 0.0));
    em = (v > em || v != v) ? v : em;  // NaN propagates
  }
  red[t] = em;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      const double a = red[t], b = red[t + o];
      red[t] = (b > a || b != b) ? b : a;
    }
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

constexpr double kNearIdentity = 1e-7;

// K5f: the blocked Cholesky of G2 when G2 is not within kNearIdentity of I
// (status = 1, R2 and R2^{-1} to global); otherwise status = 0 and nothing
// else (the near-identity form is evaluated by K5a).
__global__ void __launch_bounds__(256)
    cq_chol2_kernel(const double* __restrict__ g2, double* __restrict__ r2,
                    double* __restrict__ r2i, int* __restrict__ status,
                    int* __restrict__ flag) {
  __shared__ double T0[kTile];
  __shared__ double T1[kTile];
  __shared__ double red[256];
  __shared__ double lim[kP];
  __shared__ double tmp[4][16][17];
  __shared__ int bad;
  if (*flag) return;
  const int t = threadIdx.x;
  load_tile(T0, g2, kP, kP, kP, t);
  __syncthreads();
  const double em = dist_identity(T0, red, t);
  if (em <= kNearIdentity) {
    if (t == 0) *status = 0;
    return;
  }
  if (t == 0) *status = 1;
  if (t < kP) lim[t] = kTol2;
  __syncthreads();
  if (!chol64b(T0, T1, lim, &bad, tmp, t)) {
    if (t == 0) *flag = 1;
    return;
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u;
    r2[e] = T0[(e >> 6) * kS + (e & 63)];
    r2i[e] = T1[(e >> 6) * kS + (e & 63)];
  }
}

// K5a: R2 and R2^{-1} (near-identity form, or the blocked result of K5f),
// R = R2 R1 (unsigned, into the panel's top block), Q1_top (saved),
// Q_top = Q1_top R2^{-1} (to global).
__global__ void __launch_bounds__(256)
    cq_recon_a_kernel(double* __restrict__ A, int64_t lda, int64_t j0,
                      const double* __restrict__ g2, const double* __restrict__ r1,
                      double* __restrict__ q1top, double* __restrict__ qtop,
                      double* __restrict__ r2, double* __restrict__ r2i,
                      const int* __restrict__ status,
                      const int* __restrict__ flag) {
  __shared__ ReconLds sh;
  if (*flag) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int p = lane & 15, q = lane >> 4;
  if (*status == 0) {
    load_tile(sh.T0, g2, kP, kP, kP, t);
    __syncthreads();
    chol_near_identity(sh.T0, sh.T1, sh.T2, t);
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = t + 256 * u;
      r2i[e] = sh.T1[(e >> 6) * kS + (e & 63)];
    }
  } else {
    load_tile(sh.T0, r2, kP, kP, kP, t);
    load_tile(sh.T1, r2i, kP, kP, kP, t);
  }
  // R = R2 R1 into the panel's top block (signs applied later)
  load_tile(sh.T2, r1, kP, kP, kP, t);
  load_tile(sh.T3, A + j0 * lda + j0, lda, kP, kP, t);  // Q1_top
  __syncthreads();
  {
    dbl4 acc[4];
    zero4(acc);
    mm64<false>(sh.T0, sh.T2, acc, lane, w);
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * w + 4 * v + q, j = 16 * bj + p;
        A[(j0 + i) * lda + j0 + j] = j >= i ? acc[bj][v] : 0.0;
      }
  }
  {
    dbl4 acc[4];
    zero4(acc);
    mm64<false>(sh.T3, sh.T1, acc, lane, w);
    store_acc_global(qtop, kP, acc, 1.0, lane, w);
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u;
    q1top[e] = sh.T3[(e >> 6) * kS + (e & 63)];
  }
}

// K5b: Q_top - S = L U, T = -U S L^{-T}, M2 = R2^{-1} U^{-1}, L to global,
// the panel's Householder R = S R.
__global__ void __launch_bounds__(256)
    cq_recon_b_kernel(double* __restrict__ A, int64_t lda, int64_t j0,
                      const double* __restrict__ qtop,
                      const double* __restrict__ r2i, double* __restrict__ lbuf,
                      double* __restrict__ tbuf, double* __restrict__ m2buf,
                      const int* __restrict__ flag) {
  __shared__ ReconLds sh;
  if (*flag) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  load_tile(sh.T0, qtop, kP, kP, kP, t);
  zero_tile(sh.T2, t);
  zero_tile(sh.T3, t);
  __syncthreads();
  // T0 <- U / L, T2 <- diagonal blocks of L^{-1}, T3 <- those of U^{-1}
  lu64b(sh.T0, sh.T2, sh.T3, sh.Sg, &sh.tmp[0][0][0], t);
  inv_offdiag(sh.T0, sh.T3, sh.tmp, t);  // T3 = U^{-1}
  load_tile(sh.T1, r2i, kP, kP, kP, t);
  __syncthreads();
  {
    // M2 = R2^{-1} U^{-1}
    dbl4 acc[4];
    zero4(acc);
    mm64<false>(sh.T1, sh.T3, acc, lane, w);
    store_acc_global(m2buf, kP, acc, 1.0, lane, w);
  }
  __syncthreads();
  // L to global; T1 <- L^T (unit upper); T2 <- transposed diagonal blocks of
  // L^{-1} (zeros elsewhere), i.e. the diagonal blocks of L^{-T}
  {
    double dv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = t + 256 * u;
      const int r = e >> 6, c = e & 63;
      const double lv = r > c ? sh.T0[r * kS + c] : (r == c ? 1.0 : 0.0);
      lbuf[e] = lv;
      sh.T1[c * kS + r] = lv;
      dv[u] = (r >> 4) == (c >> 4) ? sh.T2[r * kS + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = t + 256 * u;
      const int r = e >> 6, c = e & 63;
      sh.T2[c * kS + r] = dv[u];
    }
  }
  __syncthreads();
  inv_offdiag(sh.T1, sh.T2, sh.tmp, t);  // T2 = L^{-T}
  // T3 <- U S; T = -(U S) L^{-T}
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u;
    const int r = e >> 6, c = e & 63;
    sh.T3[r * kS + c] = r <= c ? sh.T0[r * kS + c] * sh.Sg[c] : 0.0;
  }
  __syncthreads();
  {
    dbl4 acc[4];
    zero4(acc);
    mm64<false>(sh.T3, sh.T2, acc, lane, w);
    store_acc_global(tbuf, kP, acc, -1.0, lane, w);
  }
  // the panel's Householder R = S R
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u;
    const int i = e >> 6, j = e & 63;
    double* ap = A + (j0 + i) * lda + j0 + j;
    *ap = sh.Sg[i] * *ap;
  }
}

// ---- K6: W' = T^T (L^T C_top + M2^T (Z - Q1_top^T C_top)), K = M2 W' ----------
__global__ void __launch_bounds__(256)
    cq_w_kernel(const double* __restrict__ A, int64_t lda, int64_t j0,
                int64_t ncols, int64_t cb0, const double* __restrict__ zsum,
                int64_t ldz,
                const double* __restrict__ q1top, const double* __restrict__ lbuf,
                const double* __restrict__ tbuf, const double* __restrict__ m2buf,
                double* __restrict__ wp, double* __restrict__ kb,
                const int* __restrict__ flag) {
  __shared__ double TZ[kTile];
  __shared__ double TC[kTile];
  __shared__ double TQ[kTile];
  __shared__ double TM[kTile];
  if (*flag) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int p = lane & 15, q = lane >> 4;
  const int64_t c0 = (cb0 + blockIdx.x) * kP;
  const int64_t nc = ncols - c0 < kP ? ncols - c0 : kP;
  load_tile(TZ, zsum + c0, ldz, kP, nc, t);
  load_tile(TC, A + j0 * lda + j0 + kP + c0, lda, kP, nc, t);
  load_tile(TQ, q1top, kP, kP, kP, t);
  load_tile(TM, m2buf, kP, kP, kP, t);
  __syncthreads();
  {
    dbl4 acc[4];
    zero4(acc);
    mm64<true>(TQ, TC, acc, lane, w);  // Q1_top^T C_top
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        TZ[(16 * w + 4 * v + q) * kS + 16 * bj + p] -= acc[bj][v];
  }
  __syncthreads();
  load_tile(TQ, lbuf, kP, kP, kP, t);  // L (unit lower)
  __syncthreads();
  {
    dbl4 acc[4];
    zero4(acc);
    mm64<true>(TM, TZ, acc, lane, w);  // M2^T (Z - Q1_top^T C_top)
    mm64<true>(TQ, TC, acc, lane, w);  // + L^T C_top
    __syncthreads();
    store_acc(TZ, acc, 1.0, lane, w);  // W
  }
  load_tile(TC, tbuf, kP, kP, kP, t);  // T
  __syncthreads();
  {
    dbl4 acc[4];
    zero4(acc);
    mm64<true>(TC, TZ, acc, lane, w);  // W' = T^T W
    store_acc(TQ, acc, 1.0, lane, w);
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = 16 * bj + p;
        if (col < nc) wp[(16 * w + 4 * v + q) * ldz + c0 + col] = acc[bj][v];
      }
  }
  __syncthreads();
  {
    dbl4 acc[4];
    zero4(acc);
    mm64<false>(TM, TQ, acc, lane, w);  // K = M2 W'
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = 16 * bj + p;
        if (col < nc) kb[(16 * w + 4 * v + q) * ldz + c0 + col] = acc[bj][v];
      }
  }
}

// ---- K7: C -= L W' (top 64 rows), C -= Q1 K (rows below) -----------------------
__global__ void __launch_bounds__(256)
    cq_update_kernel(double* __restrict__ A, int64_t lda, int64_t m, int64_t j0,
                     int64_t ncols, int64_t cb0, const double* __restrict__ lbuf,
                     const double* __restrict__ wp, const double* __restrict__ kb,
                     int64_t ldz, const int* __restrict__ flag) {
  __shared__ double TA[kTile];
  __shared__ double TB[kTile];
  if (*flag) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int p = lane & 15, q = lane >> 4;
  const int64_t r0 = j0 + static_cast<int64_t>(blockIdx.x) * kRU;
  const int64_t c0 = (cb0 + blockIdx.y) * kP;
  const int64_t nc = ncols - c0 < kP ? ncols - c0 : kP;
  const int64_t ccol = j0 + kP + c0;  // first column of this block in A
  // A-operand rows of the first chunk: L for the panel's top rows, else Q1
  Stage va;
  if (r0 == j0)
    stage_load(va, lbuf, kP, kP, kP, t);
  else
    stage_load(va, A + r0 * lda + j0, lda, m - r0, kP, t);
  bool b_is_k = false;
  for (int c = 0; c < kRU / kP; ++c) {
    const int64_t rb = r0 + c * kP;
    if (rb >= m) break;
    const bool top = rb == j0;
    __syncthreads();
    stage_store(TA, va, t);
    if (top) {
      load_tile(TB, wp + c0, ldz, kP, nc, t);
    } else if (!b_is_k) {
      load_tile(TB, kb + c0, ldz, kP, nc, t);
      b_is_k = true;
    }
    dbl4 acc[4];
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = rb + 16 * w + 4 * v + q;
        const int col = 16 * bj + p;
        acc[bj][v] = (row < m && col < nc) ? A[row * lda + ccol + col] : 0.0;
      }
    __syncthreads();
    if (c + 1 < kRU / kP && rb + kP < m)
      stage_load(va, A + (rb + kP) * lda + j0, lda, m - rb - kP, kP, t);
    // acc -= A-tile B-tile (the A operand negated)
#pragma unroll 4
    for (int kk = 0; kk < 16; ++kk) {
      const int k = 4 * kk + q;
      const double a = -TA[(16 * w + p) * kS + k];
#pragma unroll
      for (int bj = 0; bj < 4; ++bj)
        acc[bj] = mfma(a, TB[k * kS + 16 * bj + p], acc[bj]);
    }
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = rb + 16 * w + 4 * v + q;
        const int col = 16 * bj + p;
        if (row < m && col < nc) A[row * lda + ccol + col] = acc[bj][v];
      }
  }
}

// ---- blocked triangular solves with 64 x 64 diagonal inverses -----------------
// Inverse of each 64 x 64 diagonal block of the upper-triangular R (d x d),
// the block past d padded with the identity: wave w inverts the 16 x 16
// diagonal block w by substitution, inv_offdiag fills the rest.
__global__ void __launch_bounds__(256)
    trinv_diag_kernel(const double* __restrict__ R, int64_t d,
                      double* __restrict__ rinv) {
  __shared__ double T[kTile];
  __shared__ double X[kTile];
  __shared__ double idg[kP];
  __shared__ double tmp[4][16][17];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t o = static_cast<int64_t>(blockIdx.x) * kP;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u;
    const int i = e >> 6, j = e & 63;
    double v;
    if (o + i < d && o + j < d)
      v = j >= i ? R[(o + i) * d + o + j] : 0.0;
    else
      v = i == j ? 1.0 : 0.0;
    T[i * kS + j] = v;
    X[i * kS + j] = 0.0;
  }
  __syncthreads();
  if (t < kP) idg[t] = 1.0 / T[t * kS + t];
  __syncthreads();
  tri_inv16(&T[16 * w * kS + 16 * w], nullptr, &X[16 * w * kS + 16 * w],
            idg + 16 * w, lane);
  __syncthreads();
  inv_offdiag(T, X, tmp, t);
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u;
    rinv[blockIdx.x * kP * kP + e] = X[(e >> 6) * kS + (e & 63)];
  }
}

// One block step of R X = B (back, blocks from the last) or R^T X = B
// (forward, from the first): X_J = inv(J) B_J, with inv(J) = R_JJ^{-1} (back)
// or R_JJ^{-T} (forward), written to X by the workgroups of block row J;
// every other block row I still to be solved takes B_I -= C_IJ X_J with
// C_IJ = R_IJ (back) or R_JI^T (forward), computing X_J itself. Grid:
// (block rows, 64-column blocks of B).
template <bool BACK>
__global__ void __launch_bounds__(256)
    trsm_step_kernel(const double* __restrict__ R, const double* __restrict__ rinv,
                     int64_t d, double* __restrict__ B, double* __restrict__ X,
                     int64_t k, int64_t J) {
  __shared__ double TI[kTile];
  __shared__ double TB[kTile];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int p = lane & 15, q = lane >> 4;
  const int64_t I = BACK ? static_cast<int64_t>(blockIdx.x)
                         : J + static_cast<int64_t>(blockIdx.x);
  const int64_t c0 = static_cast<int64_t>(blockIdx.y) * kP;
  const int64_t nc = k - c0 < kP ? k - c0 : kP;
  const int64_t oJ = J * kP, oI = I * kP;
  const int64_t nrJ = d - oJ < kP ? d - oJ : kP;
  load_tile(TI, rinv + J * kP * kP, kP, kP, kP, t);
  load_tile(TB, B + oJ * k + c0, k, nrJ, nc, t);
  __syncthreads();
  dbl4 acc[4];
  zero4(acc);
  if (BACK)
    mm64<false>(TI, TB, acc, lane, w);
  else
    mm64<true>(TI, TB, acc, lane, w);
  if (I == J) {
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = oJ + 16 * w + 4 * v + q;
        const int64_t col = 16 * bj + p;
        if (r < d && col < nc) X[r * k + c0 + col] = acc[bj][v];
      }
    return;
  }
  __syncthreads();
  store_acc(TB, acc, 1.0, lane, w);  // X_J
  // C_IJ: rows of block I, columns of block J of R (back), or the transpose
  // of R_JI (forward); the block past d is zero
  const int64_t nrI = d - oI < kP ? d - oI : kP;
  if (BACK)
    load_tile(TI, R + oI * d + oJ, d, nrI, nrJ, t);
  else
    load_tile(TI, R + oJ * d + oI, d, nrJ, nrI, t);
  __syncthreads();
#pragma unroll
  for (int bj = 0; bj < 4; ++bj)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = oI + 16 * w + 4 * v + q;
      const int64_t col = 16 * bj + p;
      acc[bj][v] = (r < d && col < nc) ? B[r * k + c0 + col] : 0.0;
    }
  // acc -= C_IJ X_J
#pragma unroll 4
  for (int kk = 0; kk < 16; ++kk) {
    const int kx = 4 * kk + q;
    const double a = BACK ? -TI[(16 * w + p) * kS + kx] : -TI[kx * kS + 16 * w + p];
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc[bj] = mfma(a, TB[kx * kS + 16 * bj + p], acc[bj]);
  }
#pragma unroll
  for (int bj = 0; bj < 4; ++bj)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = oI + 16 * w + 4 * v + q;
      const int64_t col = 16 * bj + p;
      if (r < d && col < nc) B[r * k + c0 + col] = acc[bj][v];
    }
}

inline unsigned cdiv(int64_t a, int64_t b) {
  return static_cast<unsigned>((a + b - 1) / b);
}

struct CqrScratch {
  double *gpart, *g, *r1, *r1i, *qtop, *r2, *r2i, *zpart, *zsum, *wp, *kb;
  // read by a panel's trailing update while the next panel is factored:
  // one set per panel parity
  double *q1top[2], *l[2], *t[2], *m2[2];
  int* status;
};

CqrScratch carve(void* base, int64_t m, int64_t d) {
  double* p = static_cast<double*>(base);
  CqrScratch c{};
  const int64_t ng = (m + kRG - 1) / kRG;
  const int64_t nz = (m + kRZ - 1) / kRZ;
  c.gpart = p;   p += ng * kP * kP;
  c.g = p;       p += kP * kP;
  c.r1 = p;      p += kP * kP;
  c.r1i = p;     p += kP * kP;
  c.qtop = p;    p += kP * kP;
  c.r2 = p;      p += kP * kP;
  c.r2i = p;     p += kP * kP;
  for (int b = 0; b < 2; ++b) {
    c.q1top[b] = p; p += kP * kP;
    c.l[b] = p;     p += kP * kP;
    c.t[b] = p;     p += kP * kP;
    c.m2[b] = p;    p += kP * kP;
  }
  c.zpart = p;   p += nz * kP * d;
  c.zsum = p;    p += kP * d;
  c.wp = p;      p += kP * d;
  c.kb = p;      p += kP * d;
  c.status = reinterpret_cast<int*>(p);
  return c;
}

// Trailing update of panel j0 restricted to the 64-column blocks
// [cb0, cb1) of its trailing columns, on stream s.
void cqr_trailing(double* a, int64_t m, int64_t d, int64_t j0,
                  const CqrScratch& c, int par, int64_t cb0, int64_t cb1,
                  int* flag, hipStream_t s) {
  const int64_t mp = m - j0;
  const int64_t ncols = d - j0 - kP;
  const int64_t c_hi = cb1 * kP < ncols ? cb1 * kP : ncols;
  const unsigned nb = static_cast<unsigned>(cb1 - cb0);
  const unsigned nz = cdiv(mp, kRZ);
  if (nb == 0) return;
  prof_begin(kKCqZ, s);
  cq_z_kernel<<<dim3(nz, nb), 256, 0, s>>>(a, d, m, j0, ncols, cb0,
                                           c.q1top[par], c.zpart, d, flag);
  prof_end(kKCqZ, s);
  prof_begin(kKCqW, s);
  cq_zsum_kernel<<<cdiv(kP * (c_hi - cb0 * kP), 256), 256, 0, s>>>(
      c.zpart, nz, d, cb0 * kP, c_hi, c.zsum, flag);
  cq_w_kernel<<<nb, 256, 0, s>>>(a, d, j0, ncols, cb0, c.zsum, d, c.q1top[par],
                                 c.l[par], c.t[par], c.m2[par], c.wp, c.kb,
                                 flag);
  prof_end(kKCqW, s);
  prof_begin(kKCqUpdate, s);
  cq_update_kernel<<<dim3(cdiv(mp, kRU), nb), 256, 0, s>>>(
      a, d, m, j0, ncols, cb0, c.l[par], c.wp, c.kb, d, flag);
  prof_end(kKCqUpdate, s);
}

// Factorisation chain of panel j0 on stream s (ends with its Householder R,
// Y and T in place / in the parity set).
void cqr_chain(double* a, int64_t m, int64_t d, int64_t j0, const CqrScratch& c,
               int par, int* flag, hipStream_t s) {
  const int64_t mp = m - j0;
  const unsigned ng = cdiv(mp, kRG);
  constexpr unsigned kSumGrid = kP * kP / 256;
  prof_begin(kKCqGram, s);
  cq_gram_kernel<<<ng, 256, 0, s>>>(a, d, m, j0, c.gpart, flag);
  prof_end(kKCqGram, s);
  prof_begin(kKCqSum, s);
  cq_sum_kernel<<<kSumGrid, 256, 0, s>>>(c.gpart, ng, c.g, flag);
  prof_end(kKCqSum, s);
  prof_begin(kKCqChol, s);
  cq_chol1_kernel<<<1, 256, 0, s>>>(c.g, c.r1, c.r1i, flag);
  prof_end(kKCqChol, s);
  prof_begin(kKCqQ1, s);
  cq_q1_kernel<<<ng, 256, 0, s>>>(a, d, m, j0, c.r1i, c.gpart, flag);
  prof_end(kKCqQ1, s);
  prof_begin(kKCqSum, s);
  cq_sum_kernel<<<kSumGrid, 256, 0, s>>>(c.gpart, ng, c.g, flag);
  prof_end(kKCqSum, s);
  prof_begin(kKCqRecon, s);
  cq_chol2_kernel<<<1, 256, 0, s>>>(c.g, c.r2, c.r2i, c.status, flag);
  cq_recon_a_kernel<<<1, 256, 0, s>>>(a, d, j0, c.g, c.r1, c.q1top[par], c.qtop,
                                      c.r2, c.r2i, c.status, flag);
  cq_recon_b_kernel<<<1, 256, 0, s>>>(a, d, j0, c.qtop, c.r2i, c.l[par],
                                      c.t[par], c.m2[par], flag);
  prof_end(kKCqRecon, s);
}

}  // namespace

size_t cqr_scratch_bytes(int64_t m, int64_t d) {
  const int64_t ng = (m + kRG - 1) / kRG;
  const int64_t nz = (m + kRZ - 1) / kRZ;
  return static_cast<size_t>(ng * kP * kP + 14 * kP * kP + nz * kP * d +
                             3 * kP * d + 1) * sizeof(double);
}

int64_t cqr_panels(int64_t m, int64_t d) {
  (void)m;
  return d / kP;
}

void cqr_factor(double* a, int64_t m, int64_t d, void* scratch, int* flag,
                const QrStreams& qs, hipStream_t s) {
  const int64_t np = d / kP;
  if (np == 0) return;
  const CqrScratch c = carve(scratch, m, d);
  hipStream_t side = qs.side ? qs.side : s;
  for (int64_t p = 0; p < np; ++p) {
    const int64_t j0 = p * kP;
    const int par = static_cast<int>(p & 1);
    const int64_t nblk = (d - j0 - kP + kP - 1) / kP;  // trailing blocks
    cqr_chain(a, m, d, j0, c, par, flag, s);
    if (nblk == 0) continue;
    // block 0 (the next panel's columns; all of them for the last panel)
    // on the main stream, after the previous panel's bulk update
    const int64_t next_end = p + 1 < np ? 1 : nblk;
    if (qs.side && p > 0) (void)hipStreamWaitEvent(s, qs.bulk_done, 0);
    if (qs.side && next_end < nblk)
      (void)hipEventRecord(qs.factored, s);
    cqr_trailing(a, m, d, j0, c, par, 0, next_end, flag, s);
    // the remaining blocks on the side stream, overlapping the next panel's
    // factorisation
    if (next_end < nblk) {
      if (qs.side) (void)hipStreamWaitEvent(side, qs.factored, 0);
      cqr_trailing(a, m, d, j0, c, par, next_end, nblk, flag, side);
      if (qs.side) (void)hipEventRecord(qs.bulk_done, side);
    }
  }
  if (qs.side) (void)hipStreamWaitEvent(s, qs.bulk_done, 0);
}

size_t trsm_blocked_scratch(int64_t d, int64_t k) {
  const int64_t nb = (d + kP - 1) / kP;
  return static_cast<size_t>(nb * kP * kP + d * k) * sizeof(double);
}

void trsm_blocked(const double* r, int64_t d, double* b, int64_t k,
                  bool transposed, void* scratch, hipStream_t s) {
  if (d <= 0 || k <= 0) return;
  const int64_t nb = (d + kP - 1) / kP;
  double* rinv = static_cast<double*>(scratch);
  double* x = rinv + nb * kP * kP;
  const unsigned ncb = cdiv(k, kP);
  prof_begin(kKTrsm, s);
  trinv_diag_kernel<<<static_cast<unsigned>(nb), 256, 0, s>>>(r, d, rinv);
  for (int64_t i = 0; i < nb; ++i) {
    const int64_t J = transposed ? i : nb - 1 - i;
    if (transposed)
      trsm_step_kernel<false><<<dim3(static_cast<unsigned>(nb - J), ncb), 256, 0,
                                s>>>(r, rinv, d, b, x, k, J);
    else
      trsm_step_kernel<true><<<dim3(static_cast<unsigned>(J + 1), ncb), 256, 0,
                               s>>>(r, rinv, d, b, x, k, J);
  }
  (void)hipMemcpyAsync(b, x, static_cast<size_t>(d * k) * sizeof(double),
                       hipMemcpyDeviceToDevice, s);
  prof_end(kKTrsm, s);
}

}  // namespace slso
