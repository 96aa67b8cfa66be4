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

namespace slso {
namespace {

constexpr int kP = 64;     // panel width
constexpr int kS = 65;     // LDS row stride of a 64 x 64 tile
constexpr int kTile = kP * kS;
constexpr int kRG = 128;   // rows per workgroup: Gram and Q1 passes
constexpr int kRZ = 512;   // rows per part: Q1^T C
constexpr int kRU = 256;   // rows per workgroup: trailing update
constexpr double kTol1 = 1e-10;  // pivot / column squared norm, first pass
constexpr double kTol2 = 1e-10;  // pivot, second pass (G2 ~ I)

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dbl4 mfma(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void zero4(dbl4 (&acc)[4]) {
#pragma unroll
  for (int bj = 0; bj < 4; ++bj) acc[bj] = dbl4{0.0, 0.0, 0.0, 0.0};
}

// acc[bj] += A(16w + i, k) B(k, 16bj + j) over k < 64, both from LDS tiles;
// A(i, k) = A[i][k], or A[k][i] when AT.
template <bool AT>
__device__ __forceinline__ void mm64(const double* A, const double* B,
                                     dbl4 (&acc)[4], int lane, int w) {
  const int p = lane & 15, q = lane >> 4;
#pragma unroll 4
  for (int kk = 0; kk < 16; ++kk) {
    const int k = 4 * kk + q;
    const double a = AT ? A[k * kS + 16 * w + p] : A[(16 * w + p) * kS + k];
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc[bj] = mfma(a, B[k * kS + 16 * bj + p], acc[bj]);
  }
}

// tile[16w + 4v + l/16][16bj + l%16] = sc * acc[bj][v]
__device__ __forceinline__ void store_acc(double* tile, const dbl4 (&acc)[4],
                                          double sc, int lane, int w) {
  const int p = lane & 15, q = lane >> 4;
#pragma unroll
  for (int bj = 0; bj < 4; ++bj)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      tile[(16 * w + 4 * v + q) * kS + 16 * bj + p] = sc * acc[bj][v];
}

__device__ __forceinline__ void store_acc_global(double* g, int64_t ldg,
                                                 const dbl4 (&acc)[4], double sc,
                                                 int lane, int w) {
  const int p = lane & 15, q = lane >> 4;
#pragma unroll
  for (int bj = 0; bj < 4; ++bj)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      g[(16 * w + 4 * v + q) * ldg + 16 * bj + p] = sc * acc[bj][v];
}

// 64 x 64 block of a row-major matrix: v[u] = a[i][j] for element
// e = t + 256 u (i = e / 64, j = e % 64); rows >= nr and columns >= nc read as
// zero. All sixteen loads are issued before any is used.
__device__ __forceinline__ void load_regs(double (&v)[16], const double* a,
                                          int64_t lda, int64_t nr, int64_t nc,
                                          int t) {
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u;
    const int i = e >> 6, j = e & 63;
    v[u] = (i < nr && j < nc) ? a[i * lda + j] : 0.0;
  }
}

__device__ __forceinline__ void store_regs(double* tile, const double (&v)[16],
                                           int t) {
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u;
    tile[(e >> 6) * kS + (e & 63)] = v[u];
  }
}

__device__ __forceinline__ void load_tile(double* tile, const double* a,
                                          int64_t lda, int64_t nr, int64_t nc,
                                          int t) {
  double v[16];
  load_regs(v, a, lda, nr, nc, t);
  store_regs(tile, v, t);
}

// 16 x 16 products on one wave, acc += A B with A(i, k) = A[i lda + k]
// (mm16) or A[k lda + i] (mm16t), B(k, j) = B[k ldb + j].
__device__ __forceinline__ dbl4 mm16(const double* A, int lda, const double* B,
                                     int ldb, dbl4 acc, int lane) {
  const int p = lane & 15, q = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk)
    acc = mfma(A[p * lda + 4 * kk + q], B[(4 * kk + q) * ldb + p], acc);
  return acc;
}
__device__ __forceinline__ dbl4 mm16t(const double* A, int lda, const double* B,
                                      int ldb, dbl4 acc, int lane) {
  const int p = lane & 15, q = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk)
    acc = mfma(A[(4 * kk + q) * lda + p], B[(4 * kk + q) * ldb + p], acc);
  return acc;
}

// 16 x 16 block in result layout: element (4v + l/16, l%16)
__device__ __forceinline__ dbl4 ld16(const double* B, int lane) {
  const int p = lane & 15, q = lane >> 4;
  dbl4 r;
#pragma unroll
  for (int v = 0; v < 4; ++v) r[v] = B[(4 * v + q) * kS + p];
  return r;
}
__device__ __forceinline__ void st16(double* B, dbl4 x, int lane) {
  const int p = lane & 15, q = lane >> 4;
#pragma unroll
  for (int v = 0; v < 4; ++v) B[(4 * v + q) * kS + p] = x[v];
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ double readlane_d(double x, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                          __builtin_amdgcn_readlane(__double2loint(x), l));
}

// 1/x and 1/sqrt(x) from the hardware approximations refined by two Newton
// steps (full double precision, shorter chains than the library sequences).
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}

// ---- 16 x 16 factorisations on one wave (lane l < 16 owns column l) ----------
// Triangular inverses of a 16 x 16 block B by substitution: lanes 0..15
// compute column l of L^{-1} for the unit lower triangle L held below B's
// diagonal (when Li is given); lanes 16..31 compute column l - 16 of U^{-1}
// for the upper triangle U on and above it (inv[i] = 1 / U_ii). The U lanes
// hold their column reversed (b[r] = X[15 - r][c]), so both substitutions
// advance together: step s finalises entry s and updates the entries after
// it. One step's coefficients are loaded while the previous step computes.
__device__ __forceinline__ void tri_inv16(const double* B, double* Li, double* Ui,
                                          const double* inv, int l) {
  const bool isL = l < 16 && Li != nullptr;
  const bool isU = l >= 16 && l < 32;
  const int c = l & 15;
  // coefficient (r, s), r > s: L[r][s] = B[r][s] for the L lanes,
  // U[15 - r][15 - s] = B[15 - r][15 - s] for the U lanes
  const int base = l >= 16 ? 15 * kS + 15 : 0;
  const int sgn = l >= 16 ? -1 : 1;
  const double* Bb = B + base;
  double b[16];
#pragma unroll
  for (int r = 0; r < 16; ++r)
    b[r] = (isL && r == c) || (isU && 15 - r == c) ? 1.0 : 0.0;
  double m[16];
#pragma unroll
  for (int r = 1; r < 16; ++r) m[r] = Bb[sgn * (r * kS)];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const double x = isU ? b[s] * inv[15 - s] : b[s];
    b[s] = x;
    double mn[16];
#pragma unroll
    for (int r = s + 2; r < 16; ++r) mn[r] = Bb[sgn * (r * kS + s + 1)];
#pragma unroll
    for (int r = s + 1; r < 16; ++r) b[r] -= m[r] * x;
#pragma unroll
    for (int r = s + 2; r < 16; ++r) m[r] = mn[r];
    __builtin_amdgcn_sched_barrier(0);
  }
  if (isL) {
#pragma unroll
    for (int r = 0; r < 16; ++r) Li[r * kS + c] = b[r];
  }
  if (isU) {
#pragma unroll
    for (int r = 0; r < 16; ++r) Ui[(15 - r) * kS + c] = b[r];
  }
}

// Cholesky of the symmetric block B (upper triangle read): B <- R (zeros
// below), Xi <- R^{-1}; s16 (16 doubles of LDS) is scratch. False (the same
// in every lane) when a pivot is not above lim[j].
__device__ __forceinline__ bool chol16w(double* B, double* Xi, const double* lim,
                                        double* s16, int lane) {
  const int l = lane;
  bool ok = true;
  {
    double gc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i)
      gc[i] = l < 16 ? (i <= l ? B[i * kS + l] : B[l * kS + i]) : 0.0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const double piv = readlane_d(gc[j], j);
      ok = ok && (piv > lim[j]);
      const double pv = ok ? piv : 1.0;
      const double ir = rsq_nr(pv);
      if (l == 0) s16[j] = ir;
      const double rjl = l > j ? gc[j] * ir : (l == j ? pv * ir : 0.0);
      gc[j] = rjl;  // row j of R from here on
#pragma unroll
      for (int i = j + 1; i < 16; ++i) gc[i] -= readlane_d(rjl, i) * rjl;
    }
    wave_sync();
    if (l < 16) {
#pragma unroll
      for (int i = 0; i < 16; ++i) B[i * kS + l] = gc[i];
    }
  }
  wave_sync();
  tri_inv16(B, nullptr, Xi, s16, l);
  wave_sync();
  return ok;
}

// Sign-choosing LU without pivoting of the block B: B - diag(sg) = L U with
// sg_i = -sign(current pivot), so |U_ii| >= 1. B <- U on and above the
// diagonal and the multipliers of L below; Li <- L^{-1}; Ui <- U^{-1}; s16
// (16 doubles of LDS) is scratch.
__device__ __forceinline__ void lu16w(double* B, double* Li, double* Ui,
                                      double* sg, double* s16, int lane) {
  const int l = lane;
  {
    double wc[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) wc[r] = l < 16 ? B[r * kS + l] : 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const double pv = readlane_d(wc[i], i);
      const double sgi = pv >= 0.0 ? -1.0 : 1.0;
      const double piv = pv - sgi;
      const double ip = rcp_nr(piv);
      if (l == 0) {
        sg[i] = sgi;
        s16[i] = ip;
      }
      if (l == i) {
        wc[i] = piv;
#pragma unroll
        for (int r = i + 1; r < 16; ++r) wc[r] *= ip;
      }
      const double uil = wc[i];
#pragma unroll
      for (int r = i + 1; r < 16; ++r) {
        const double mr = readlane_d(wc[r], i);
        if (l > i) wc[r] -= mr * uil;
      }
    }
    // lane l: wc[r] = U[r][l] for r <= l, L[r][l] for r > l
    wave_sync();
    if (l < 16) {
#pragma unroll
      for (int r = 0; r < 16; ++r) B[r * kS + l] = wc[r];
    }
  }
  wave_sync();
  tri_inv16(B, Li, Ui, s16, l);
  wave_sync();
}

// Off-diagonal blocks of X = R^{-1} for upper-triangular R, given X's
// diagonal blocks (and zeros below them): X_ij = -X_ii sum_{k=i+1..j} R_ik X_kj.
__device__ __forceinline__ void inv_offdiag(const double* R, double* X, double (*tmp)[16][17],
                            int t) {
  const int lane = t & 63, w = t >> 6, p = lane & 15, q = lane >> 4;
#pragma unroll 1
  for (int dist = 1; dist < 4; ++dist) {
    const int i = w, j = w + dist;
    if (j < 4) {
      dbl4 acc = {0.0, 0.0, 0.0, 0.0};
      for (int k = i + 1; k <= j; ++k)
        acc = mm16(&R[16 * i * kS + 16 * k], kS, &X[16 * k * kS + 16 * j], kS,
                   acc, lane);
#pragma unroll
      for (int v = 0; v < 4; ++v) tmp[w][4 * v + q][p] = acc[v];
      wave_sync();
      dbl4 acc2 = {0.0, 0.0, 0.0, 0.0};
      acc2 = mm16(&X[16 * i * kS + 16 * i], kS, &tmp[w][0][0], 17, acc2, lane);
#pragma unroll
      for (int v = 0; v < 4; ++v) X[(16 * i + 4 * v + q) * kS + 16 * j + p] = -acc2[v];
      wave_sync();
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void zero_tile(double* X, int t) {
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u;
    X[(e >> 6) * kS + (e & 63)] = 0.0;
  }
}

// Blocked upper Cholesky of the symmetric tile G (upper triangle read) with
// 16 x 16 diagonal factorisations on wave 0 and MFMA block updates. On
// success G holds R (zeros below) and X holds R^{-1}. False, in every
// thread, when a pivot is not above lim[j].
__device__ __forceinline__ bool chol64b(double* G, double* X, const double* lim, int* bad,
                        double (*tmp)[16][17], int t) {
  const int lane = t & 63, w = t >> 6;
  zero_tile(X, t);
  if (t == 0) *bad = 0;
  __syncthreads();
#pragma unroll 1
  for (int k = 0; k < 4; ++k) {
    const int o = 16 * k;
    if (w == 0) {
      const bool ok = chol16w(&G[o * kS + o], &X[o * kS + o], lim + o,
                              &tmp[0][0][0], lane);
      if (!ok && lane == 0) *bad = 1;
    }
    __syncthreads();
    if (*bad) return false;
    // row block k: R_kj = R_kk^{-T} G_kj
    if (w < 3 - k) {
      const int j = k + 1 + w;
      dbl4 acc = {0.0, 0.0, 0.0, 0.0};
      acc = mm16t(&X[o * kS + o], kS, &G[o * kS + 16 * j], kS, acc, lane);
      st16(&G[o * kS + 16 * j], acc, lane);
    }
    __syncthreads();
    // trailing blocks G_ij -= R_ki^T R_kj, k < i <= j
    int idx = 0;
    for (int i = k + 1; i < 4; ++i)
      for (int j = i; j < 4; ++j, ++idx) {
        if ((idx & 3) != w) continue;
        dbl4 acc = ld16(&G[16 * i * kS + 16 * j], lane);
        dbl4 sub = {0.0, 0.0, 0.0, 0.0};
        sub = mm16t(&G[o * kS + 16 * i], kS, &G[o * kS + 16 * j], kS, sub, lane);
        st16(&G[16 * i * kS + 16 * j], acc - sub, lane);
      }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u;
    const int i = e >> 6, c = e & 63;
    if (i > c) G[i * kS + c] = 0.0;
  }
  __syncthreads();
  inv_offdiag(G, X, tmp, t);
  return true;
}

// Blocked sign-choosing LU of the tile Q (see lu16w): Q <- U on and above
// the diagonal, L's multipliers below; Li and Ui receive the inverses of L's
// and U's diagonal blocks (the caller zeroes them first); sg the signs.
__device__ __forceinline__ void lu64b(double* Q, double* Li, double* Ui, double* sg, double* s16,
                      int t) {
  const int lane = t & 63, w = t >> 6;
#pragma unroll 1
  for (int k = 0; k < 4; ++k) {
    const int o = 16 * k;
    if (w == 0) lu16w(&Q[o * kS + o], &Li[o * kS + o], &Ui[o * kS + o], sg + o,
                      s16, lane);
    __syncthreads();
    // U_kj = L_kk^{-1} Q_kj (j > k) and L_ik = Q_ik U_kk^{-1} (i > k)
    const int nb = 3 - k;
    for (int idx = w; idx < 2 * nb; idx += 4) {
      dbl4 acc = {0.0, 0.0, 0.0, 0.0};
      if (idx < nb) {
        const int j = k + 1 + idx;
        acc = mm16(&Li[o * kS + o], kS, &Q[o * kS + 16 * j], kS, acc, lane);
        st16(&Q[o * kS + 16 * j], acc, lane);
      } else {
        const int i = k + 1 + idx - nb;
        acc = mm16(&Q[16 * i * kS + o], kS, &Ui[o * kS + o], kS, acc, lane);
        st16(&Q[16 * i * kS + o], acc, lane);
      }
    }
    __syncthreads();
    // trailing Q_ij -= L_ik U_kj, i, j > k
    for (int idx = w; idx < nb * nb; idx += 4) {
      const int i = k + 1 + idx / nb, j = k + 1 + idx % nb;
      dbl4 acc = ld16(&Q[16 * i * kS + 16 * j], lane);
      dbl4 sub = {0.0, 0.0, 0.0, 0.0};
      sub = mm16(&Q[16 * i * kS + o], kS, &Q[o * kS + 16 * j], kS, sub, lane);
      st16(&Q[16 * i * kS + 16 * j], acc - sub, lane);
    }
    __syncthreads();
  }
}

// sum of nparts 64 x 64 matrices (fixed order), element e; sixteen loads in
// flight
__device__ __forceinline__ double sum_parts(const double* parts, int64_t nparts,
                                            int64_t stride, int64_t e) {
  double s = 0.0;
  int64_t pp = 0;
  for (; pp + 16 <= nparts; pp += 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = parts[(pp + u) * stride + e];
#pragma unroll
    for (int u = 0; u < 16; ++u) s += v[u];
  }
  for (; pp < nparts; ++pp) s += parts[pp * stride + e];
  return s;
}

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
  double v[16];
  load_regs(v, A + r0 * lda + j0, lda, m - r0, kP, t);
  for (int c = 0; c < kRG / kP; ++c) {
    const int64_t rb = r0 + c * kP;
    if (rb >= m) break;
    __syncthreads();
    store_regs(T, v, t);
    __syncthreads();
    if (c + 1 < kRG / kP && rb + kP < m)
      load_regs(v, A + (rb + kP) * lda + j0, lda, m - rb - kP, kP, t);
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
  double v[16];
  load_regs(v, A + r0 * lda + j0, lda, m - r0, kP, t);
  load_tile(Ri, r1i, kP, kP, kP, t);
  dbl4 g2[4];
  zero4(g2);
  for (int c = 0; c < kRG / kP; ++c) {
    const int64_t rb = r0 + c * kP;
    if (rb >= m) break;
    __syncthreads();
    store_regs(T, v, t);
    __syncthreads();
    if (c + 1 < kRG / kP && rb + kP < m)
      load_regs(v, A + (rb + kP) * lda + j0, lda, m - rb - kP, kP, t);
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
  double vq[16], vc[16];
  if (r0 == j0)
    load_regs(vq, q1top, kP, kP, kP, t);
  else
    load_regs(vq, A + r0 * lda + j0, lda, m - r0, kP, t);
  load_regs(vc, A + r0 * lda + cc, lda, m - r0, nc, t);
  for (int c = 0; c < kRZ / kP; ++c) {
    const int64_t rb = r0 + c * kP;
    if (rb >= m) break;
    __syncthreads();
    store_regs(TQ, vq, t);
    store_regs(TC, vc, t);
    __syncthreads();
    if (c + 1 < kRZ / kP && rb + kP < m) {
      load_regs(vq, A + (rb + kP) * lda + j0, lda, m - rb - kP, kP, t);
      load_regs(vc, A + (rb + kP) * lda + cc, lda, m - rb - kP, nc, t);
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
  double va[16];
  if (r0 == j0)
    load_regs(va, lbuf, kP, kP, kP, t);
  else
    load_regs(va, A + r0 * lda + j0, lda, m - r0, kP, t);
  bool b_is_k = false;
  for (int c = 0; c < kRU / kP; ++c) {
    const int64_t rb = r0 + c * kP;
    if (rb >= m) break;
    const bool top = rb == j0;
    __syncthreads();
    store_regs(TA, va, t);
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
      load_regs(va, A + (rb + kP) * lda + j0, lda, m - rb - kP, kP, t);
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
