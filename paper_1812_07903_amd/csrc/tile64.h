// 64 x 64 FP64 tile helpers on the MFMA (v_mfma_f64_16x16x4f64) and the
// one-workgroup factorisations built on them: products of LDS tiles,
// 16 x 16 Cholesky / LU / triangular inverses on one wave, blocked 64 x 64
// Cholesky and LU, and the inverse's off-diagonal blocks.
//
// Operand layout: A operand lane l = A[l%16][l/16], B operand lane l =
// B[l/16][l%16], result register v of lane l = D[4v + l/16][l%16]. Tiles in
// LDS have a row stride of 65 doubles; wave w of a 256-thread workgroup owns
// tile rows 16w .. 16w + 15.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace slso {
namespace {

constexpr int kP = 64;     // tile width
constexpr int kS = 65;     // LDS row stride of a 64 x 64 tile
constexpr int kTile = kP * kS;
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
  // four steps' operands per LDS round trip (sixteen MFMAs)
#pragma unroll
  for (int k0 = 0; k0 < 16; k0 += 4) {
    double a[4], b[4][4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int k = 4 * (k0 + kk) + q;
      a[kk] = AT ? A[k * kS + 16 * w + p] : A[(16 * w + p) * kS + k];
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) b[kk][bj] = B[k * kS + 16 * bj + p];
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) acc[bj] = mfma(a[kk], b[kk][bj], acc[bj]);
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
// A 64 x 64 tile staged in registers: thread t holds elements e = t + 256 u
// (row e / 64, column e % 64). stage_load reads the rows < nr and columns
// < nc of a (row stride lda) without branches -- an element outside reads a
// clamped address inside that rectangle -- and records which elements are
// inside; stage_store writes the tile to LDS with zeros outside. The loaded
// values are not used before stage_store, so loads issued ahead of a
// multiplication stay in flight during it.
struct Stage {
  double v[16];
  uint32_t ok;
};

__device__ __forceinline__ void stage_load(Stage& s, const double* a,
                                           int64_t lda, int64_t nr, int64_t nc,
                                           int t) {
  s.ok = 0u;
  if (nr <= 0 || nc <= 0) {
#pragma unroll
    for (int u = 0; u < 16; ++u) s.v[u] = 0.0;
    return;
  }
  const int64_t r1 = nr - 1, c1 = nc - 1;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u;
    const int64_t i = e >> 6, j = e & 63;
    s.ok |= (i < nr && j < nc) ? (1u << u) : 0u;
    s.v[u] = a[(i < r1 ? i : r1) * lda + (j < c1 ? j : c1)];
  }
}

__device__ __forceinline__ void stage_store(double* tile, const Stage& s,
                                            int t) {
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u;
    tile[(e >> 6) * kS + (e & 63)] = ((s.ok >> u) & 1u) ? s.v[u] : 0.0;
  }
}

__device__ __forceinline__ void load_tile(double* tile, const double* a,
                                          int64_t lda, int64_t nr, int64_t nc,
                                          int t) {
  Stage v;
  stage_load(v, a, lda, nr, nc, t);
  stage_store(tile, v, t);
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

// 1/x from the hardware approximation refined by two Newton steps (full
// double precision, a shorter chain than the library sequence).
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
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

// Cholesky of the symmetric block B (upper triangle read) on one wave, with
// R^{-1} from the same eliminations: lane l < 16 holds column l of B, lane
// 16 + c column c of the identity. Pivot j scales row j by 1/sqrt(pivot) and
// subtracts multiples of it from the rows below; on the identity columns
// these steps are forward substitution with R^T, so lane 16 + c ends with
// column c of R^{-T}, which is row c of R^{-1}. B <- R (zeros below),
// Xi <- R^{-1}. False (the same in every lane) when a pivot is not above
// lim[j]; the outputs are then meaningless.
__device__ __forceinline__ bool chol16x(double* B, double* Xi, const double* lim,
                                        int lane) {
  const int l = lane, lc = lane & 15, c = lane - 16;
  double gc[16], lm[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const double bv = B[i <= lc ? i * kS + lc : lc * kS + i];
    gc[i] = l < 16 ? bv : (i == c ? 1.0 : 0.0);
    lm[i] = lim[i];
  }
  bool ok = true;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const double piv = readlane_d(gc[j], j);
    ok = ok && piv > lm[j];
    // 1/sqrt(piv) = y0 (1 - e)^{-1/2} with e = 1 - piv y0^2 for the hardware
    // estimate y0; |e| < 1e-7, so the series to e^2 leaves a remainder far
    // below rounding. Row j of R (or of the substitution) is g (1 + e/2 +
    // 3e^2/8) with g = gc[j] y0.
    const double y0 = __builtin_amdgcn_rsq(piv);
    const double e = fma(-piv * y0, y0, 1.0);
    const double g = l < j ? 0.0 : gc[j] * y0;
    const double rjl = fma(g * e, fma(e, 0.375, 0.5), g);
    gc[j] = rjl;
    // row j of R: all its lane reads first (each into registers of its own),
    // then the updates; read and use interleaved, the reads queue behind one
    // another on a shared scalar register pair
    double rb[16];
#pragma unroll
    for (int i = j + 1; i < 16; ++i) rb[i] = readlane_d(rjl, i);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = j + 1; i < 16; ++i) gc[i] -= rb[i] * rjl;
  }
  wave_sync();
  if (l < 16) {
#pragma unroll
    for (int i = 0; i < 16; ++i) B[i * kS + l] = gc[i];
  } else if (l < 32) {
#pragma unroll
    for (int i = 0; i < 16; ++i) Xi[c * kS + i] = gc[i];
  }
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
// 16 x 16 diagonal factorisations (and their inverses) on wave 0 and MFMA
// block updates. On success G holds R (zeros below) and X holds R^{-1}.
// False, in every thread, when a pivot is not above lim[j].
//
// X's off-diagonal blocks follow from X R = I by block rows:
// X_rj = -(sum_{m=r}^{j-1} X_rm R_mj) X_jj, r < j. Wave r + 1 keeps the
// running sums P_rj in registers and, while wave 0 factors diagonal block k,
// finishes X_r,k-1 and adds the terms m = k - 1 (block row k - 1 of R is
// final by then), so the inverse costs no step of its own.
// nblk < 4: the diagonal blocks from nblk on are padding (identity in G,
// untouched by the updates, since the rows above them are zero there), so
// their Cholesky is the identity and is written, not computed.
__device__ __forceinline__ bool chol64b(double* G, double* X, const double* lim, int* bad,
                        double (*tmp)[16][17], int t, int nblk = 4) {
  const int lane = t & 63, w = t >> 6, p = lane & 15, q = lane >> 4;
  const int r = w - 1;
  zero_tile(X, t);
  if (t == 0) *bad = 0;
  __syncthreads();
  dbl4 pacc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) pacc[j] = dbl4{0.0, 0.0, 0.0, 0.0};
  // X_rm = -P_rm X_mm, through the wave's LDS scratch
  auto finish = [&](int m, const dbl4& pm) {
#pragma unroll
    for (int v = 0; v < 4; ++v) tmp[w][4 * v + q][p] = pm[v];
    wave_sync();
    dbl4 x = {0.0, 0.0, 0.0, 0.0};
    x = mm16(&tmp[w][0][0], 17, &X[16 * m * kS + 16 * m], kS, x, lane);
#pragma unroll
    for (int v = 0; v < 4; ++v) X[(16 * r + 4 * v + q) * kS + 16 * m + p] = -x[v];
    wave_sync();
  };
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int o = 16 * k;
    if (w == 0) {
      if (k < nblk) {
        const bool ok = chol16x(&G[o * kS + o], &X[o * kS + o], lim + o, lane);
        if (!ok && lane == 0) *bad = 1;
      } else if (lane < 16) {
        X[(o + lane) * kS + o + lane] = 1.0;
      }
    } else if (k > 0 && r <= k - 1) {
      const int m = k - 1;
      if (r < m) finish(m, pacc[m]);
#pragma unroll
      for (int j = m + 1; j < 4; ++j)
        pacc[j] = mm16(&X[16 * r * kS + 16 * m], kS, &G[16 * m * kS + 16 * j], kS,
                       pacc[j], lane);
    }
    __syncthreads();
    if (*bad) return false;
    if (k == 3) break;
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
#pragma unroll
    for (int i = k + 1; i < 4; ++i)
#pragma unroll
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
  if (w > 0) finish(3, pacc[3]);
  __syncthreads();
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


}  // namespace
}  // namespace slso
