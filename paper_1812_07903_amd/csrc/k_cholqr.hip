// R factor of the sketch by Cholesky-QR2 over the whole matrix (Algorithm 2
// step 2 in QR form; only R is kept):
//   G1 = A^T A = R1^T R1,   Q1 = A R1^{-1} (in place over A),
//   G2 = Q1^T Q1 = R2^T R2, R = R2 R1.
// R has a positive diagonal and equals the R of a Householder QR of A up to
// the signs of its rows (Fukaya, Nakatsukasa, Yanagisawa & Yamamoto,
// "CholeskyQR2: a simple and communication-avoiding algorithm for computing a
// tall-skinny QR factorization", 2014). All the O(m d^2) work is in three
// passes over the rows on the FP64 MFMA: the two Gram matrices (upper 64 x 64
// tiles, rows split into chunks, partial tiles summed in a fixed order) and
// the blocked forward substitution that forms Q1.
//
// Validity. Cholesky-QR2 reaches the accuracy of Householder QR when the first
// pass leaves Q1 well conditioned, i.e. when kappa(A)^2 u is well below one.
// This is checked a posteriori: with E = G2 - I and e = max |E_ij|,
//   e <= 1e-9      R2 = I + up(E) (strict upper part plus half the diagonal;
//                  the neglected F^T F term is below d e^2 <= 1e-15 for
//                  d <= 1000) and R = R1 + up(E) R1 in one launch;
//   e <= 0.25 / d  status 2: the caller runs cholqr2_finish, the blocked
//                  Cholesky of G2 and R = R2 R1;
//   otherwise, or when a Cholesky pivot of G1 falls to 1e-13 of its diagonal
//   entry, status 1: the caller factors the (re-formed) matrix with the
//   Householder paths.
//
// Data layout. d x d matrices are kept as nb x nb tiles of 64 x 64 (tile
// (I, J) at (I nb + J) 4096, row-major inside), padded past d with the
// identity on the diagonal and zeros elsewhere; only tiles on and above the
// diagonal are used. The Cholesky of a tiled matrix is right-looking by 64-row
// block steps, one launch per step: the workgroup of tile (i, j) forms
// X_i = R_kk^{-T} G_ki and X_j, updates G_ij -= X_i^T X_j, writes R_kj when
// i = k + 1, and the workgroup of the next diagonal tile factors it at once
// (Cholesky and inverse in one workgroup), so a step costs one launch.
#include "internal.h"
#include "tile64.h"

namespace slso {
namespace {

constexpr int64_t kT2 = kP * kP;        // elements of a tile
constexpr double kPivotTol = 1e-13;     // Cholesky pivot / diagonal entry
constexpr double kNearId = 1e-9;        // max |G2 - I| for the one-launch R2

inline unsigned cdivu(int64_t a, int64_t b) {
  return static_cast<unsigned>((a + b - 1) / b);
}

__host__ __device__ inline int64_t tix(int64_t i, int64_t j, int64_t nb) {
  return (i * nb + j) * kT2;
}

// t-th tile on or above the diagonal of an n x n tile grid, row by row
__device__ __forceinline__ void upper_tile(int64_t t, int64_t n, int64_t& i,
                                           int64_t& j) {
  int64_t r = 0;
  while (t >= n - r) {
    t -= n - r;
    ++r;
  }
  i = r;
  j = r + t;
}

// index of tile (i, j), i <= j, in the enumeration of upper_tile
__host__ __device__ inline int64_t upper_index(int64_t i, int64_t j, int64_t n) {
  return i * n - i * (i - 1) / 2 + (j - i);
}

// acc -= A B (AT: A^T B) for LDS tiles, see mm64
template <bool AT>
__device__ __forceinline__ void mm64_sub(const double* A, const double* B,
                                         dbl4 (&acc)[4], int lane, int w) {
  const int p = lane & 15, q = lane >> 4;
#pragma unroll 4
  for (int kk = 0; kk < 16; ++kk) {
    const int k = 4 * kk + q;
    const double a = AT ? -A[k * kS + 16 * w + p] : -A[(16 * w + p) * kS + k];
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc[bj] = mfma(a, B[k * kS + 16 * bj + p], acc[bj]);
  }
}

// 64 x 64 tile (row-major, ld 64) from global memory in result layout
__device__ __forceinline__ void ld_acc(dbl4 (&acc)[4], const double* g, int lane,
                                       int w) {
  const int p = lane & 15, q = lane >> 4;
#pragma unroll
  for (int bj = 0; bj < 4; ++bj)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[bj][v] = g[(16 * w + 4 * v + q) * kP + 16 * bj + p];
}

__device__ __forceinline__ void tile_to_global(double* g, const double* T,
                                               int t) {
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u;
    g[e] = T[(e >> 6) * kS + (e & 63)];
  }
}

// ---- Gram tiles: partial sums over row chunks ----------------------------------
// A workgroup forms one 128 x 128 block of the Gram matrix (a pair of
// 128-column blocks I2 <= J2 of A) over one chunk of rows. Wave w owns the
// 32-row strip 32 w .. 32 w + 31 of the block and all its columns, so the four
// waves carry equal work (on diagonal blocks the lower half is formed too and
// ignored). Rows advance in steps of 16 through two LDS buffers (one barrier
// per step); the next step's rows are loaded into registers while the current
// step multiplies. Blocks made of full 128-column blocks of A are formed by
// one launch with about two workgroups per CU; the blocks that touch a last,
// partial column block (little work) by a second launch with predicates.
// Partial blocks are stored 128 x 128 row-major (edge blocks: only their
// columns inside the matrix): full block t, chunk s at
// part[(t S + s) 16384], edge block e, chunk s after all of those at
// [(nfull S + e S_e + s) 16384].
constexpr int kGK = 16;    // rows per step
constexpr int kGS = 144;   // LDS row stride: rows 4 apart fall on the other
                           // half of the banks
constexpr int64_t kB2 = 128 * 128;

template <bool EDGE>
__global__ void __launch_bounds__(256, 2)
    gram_block_kernel(const double* __restrict__ A, int64_t lda, int64_t m,
                      int64_t d, int64_t S, int64_t chunk, int64_t part0,
                      double* __restrict__ part, const int* __restrict__ flag) {
  __shared__ double X[2][2][kGK * kGS];
  if (*flag) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int p = lane & 15, q = lane >> 4;
  const int64_t g = blockIdx.x, s = g % S, tt = g / S;
  const int64_t nf = d / 128;  // full 128-column blocks
  int64_t I2, J2;
  if (EDGE) {
    I2 = tt;
    J2 = nf;
  } else {
    upper_tile(tt, nf, I2, J2);
  }
  const bool diag = I2 == J2;
  const int64_t cA = I2 * 128, cB = J2 * 128;
  const int64_t nA = d - cA < 128 ? d - cA : 128;
  const int64_t nB = d - cB < 128 ? d - cB : 128;
  // 16-row / 16-column sub-blocks of this wave's strip inside the matrix
  const int64_t rw = nA - 32 * w;
  const int nrow = EDGE ? (rw <= 0 ? 0 : (rw >= 32 ? 2 : (rw > 16 ? 2 : 1))) : 2;
  const int ncol = EDGE ? static_cast<int>((nB + 15) / 16) : 8;
  const int64_t r0 = s * chunk;
  const int64_t r1 = m < r0 + chunk ? m : r0 + chunk;
  dbl4 acc[2][8];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 8; ++y) acc[x][y] = dbl4{0.0, 0.0, 0.0, 0.0};
  const int c = t & 127, rr = t >> 7;
  double v[16];
  // loads without branches (an entry outside the matrix reads A[0]); the
  // zeros are put in when the values go to LDS
  auto gload = [&](int64_t r) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t row = r + rr + 2 * u;
      const bool oka = row < r1 && c < nA;
      v[u] = A[oka ? row * lda + cA + c : 0];
      if (!diag) {
        const bool okb = row < r1 && c < nB;
        v[8 + u] = A[okb ? row * lda + cB + c : 0];
      }
    }
  };
  auto lstore = [&](int buf, int64_t r) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t row = r + rr + 2 * u;
      X[buf][0][(rr + 2 * u) * kGS + c] = (row < r1 && c < nA) ? v[u] : 0.0;
      if (!diag)
        X[buf][1][(rr + 2 * u) * kGS + c] = (row < r1 && c < nB) ? v[8 + u] : 0.0;
    }
  };
  if (r0 < r1) {
    gload(r0);
    lstore(0, r0);
    __syncthreads();
    int buf = 0;
    for (int64_t r = r0; r < r1; r += kGK) {
      const bool more = r + kGK < r1;
      if (more) gload(r + kGK);
      const double* XA = X[buf][0];
      const double* XB = diag ? X[buf][0] : X[buf][1];
#pragma unroll
      for (int kk = 0; kk < kGK / 4; ++kk) {
        const int k = 4 * kk + q;
        double a[2], b[8];
#pragma unroll
        for (int x = 0; x < 2; ++x) a[x] = XA[k * kGS + 32 * w + 16 * x + p];
#pragma unroll
        for (int y = 0; y < 8; ++y) b[y] = XB[k * kGS + 16 * y + p];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 8; ++y)
            if (!EDGE || (x < nrow && y < ncol))
              acc[x][y] = mfma(a[x], b[y], acc[x][y]);
      }
      if (more) lstore(buf ^ 1, r + kGK);
      __syncthreads();
      buf ^= 1;
    }
  }
  double* out = part + (part0 + g) * kB2;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 8; ++y)
      if (!EDGE || y < ncol) {
#pragma unroll
        for (int vv = 0; vv < 4; ++vv)
          out[(32 * w + 16 * x + 4 * vv + q) * 128 + 16 * y + p] = acc[x][y][vv];
      }
}

// G tile = sum of its partial blocks (fixed order); the padding is the
// identity; gdiag receives the diagonal. With emax, emax[workgroup] = max
// |G - I| over the workgroup's valid entries (bit patterns of non-negative
// doubles order like the values, a NaN above every number).
__global__ void __launch_bounds__(256)
    gram_reduce_kernel(const double* __restrict__ part, int64_t S, int64_t Se,
                       int64_t nb, int64_t d, double* __restrict__ G,
                       double* __restrict__ gdiag, unsigned long long* emax,
                       const int* __restrict__ flag) {
  __shared__ unsigned long long red[4];
  if (*flag) return;
  const int64_t tt = blockIdx.x >> 4;
  const int e = static_cast<int>((blockIdx.x & 15) << 8) + threadIdx.x;
  int64_t I0, J0;
  upper_tile(tt, nb, I0, J0);
  // the 128 x 128 partial block holding 64-tile (I0, J0), and the offset of
  // this element inside it
  const int64_t nf = d / 128;
  const int64_t I2 = I0 >> 1, J2 = J0 >> 1;
  const int64_t off = ((I0 & 1) * 64 + (e >> 6)) * 128 + (J0 & 1) * 64 + (e & 63);
  const int64_t gi = I0 * kP + (e >> 6), gj = J0 * kP + (e & 63);
  double v = 0.0;
  if (gi >= d || gj >= d) {
    // padding: the identity (partial edge blocks hold nothing there)
    v = gi == gj ? 1.0 : 0.0;
  } else if (J2 < nf) {
    const int64_t blk = upper_index(I2, J2, nf) * S;
    v = sum_parts(part + blk * kB2 + off, S, kB2, 0);
  } else {
    const int64_t blk = nf * (nf + 1) / 2 * S + I2 * Se;
    v = sum_parts(part + blk * kB2 + off, Se, kB2, 0);
  }
  G[tix(I0, J0, nb) + e] = v;
  if (gi == gj) gdiag[gi] = v;
  if (emax) {
    double dev = 0.0;
    if (gi < d && gj < d) dev = fabs(v - (gi == gj ? 1.0 : 0.0));
    unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(dev));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long ob = __shfl_xor(b, o);
      b = ob > b ? ob : b;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long m = red[0];
      for (int k = 1; k < 4; ++k) m = red[k] > m ? red[k] : m;
      emax[blockIdx.x] = m;
    }
  }
}

// ---- blocked Cholesky of a tiled SPD matrix ------------------------------------
__global__ void __launch_bounds__(256)
    bchol_first_kernel(const double* __restrict__ G, const double* __restrict__ gdiag,
                       double tol, double* __restrict__ R,
                       double* __restrict__ Dinv, int* __restrict__ flag) {
  __shared__ double TC[kTile];
  __shared__ double TX[kTile];
  __shared__ double tmp[4][16][17];
  __shared__ double lim[kP];
  __shared__ int bad;
  if (*flag) return;
  const int t = threadIdx.x;
  load_tile(TC, G, kP, kP, kP, t);
  if (t < kP) lim[t] = tol * gdiag[t];
  __syncthreads();
  if (!chol64b(TC, TX, lim, &bad, tmp, t)) {
    if (t == 0) *flag = 1;
    return;
  }
  tile_to_global(R, TC, t);
  tile_to_global(Dinv, TX, t);
}

// Step k: tiles (i, j), k < i <= j, one workgroup each (see the header).
__global__ void __launch_bounds__(256)
    bchol_step_kernel(double* __restrict__ G, int64_t nb, int64_t k,
                      const double* __restrict__ gdiag, double tol,
                      double* __restrict__ R, double* __restrict__ Dinv,
                      int* __restrict__ flag) {
  __shared__ double TI[kTile];
  __shared__ double TA[kTile];
  __shared__ double TB[kTile];
  __shared__ double TC[kTile];
  __shared__ double tmp[4][16][17];
  __shared__ double lim[kP];
  __shared__ int bad;
  if (*flag) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int64_t i, j;
  upper_tile(blockIdx.x, nb - k - 1, i, j);
  i += k + 1;
  j += k + 1;
  const bool diag = i == j;
  load_tile(TI, Dinv + k * kT2, kP, kP, kP, t);
  load_tile(TA, G + tix(k, i, nb), kP, kP, kP, t);
  if (!diag) load_tile(TB, G + tix(k, j, nb), kP, kP, kP, t);
  dbl4 acc[4];
  ld_acc(acc, G + tix(i, j, nb), lane, w);
  __syncthreads();
  dbl4 xa[4], xb[4];
  zero4(xa);
  mm64<true>(TI, TA, xa, lane, w);  // X_i = R_kk^{-T} G_ki = R_ki
  if (!diag) {
    zero4(xb);
    mm64<true>(TI, TB, xb, lane, w);
  }
  __syncthreads();
  store_acc(TA, xa, 1.0, lane, w);
  if (!diag) store_acc(TB, xb, 1.0, lane, w);
  if (i == k + 1) {
    if (diag)
      store_acc_global(R + tix(k, j, nb), kP, xa, 1.0, lane, w);
    else
      store_acc_global(R + tix(k, j, nb), kP, xb, 1.0, lane, w);
  }
  __syncthreads();
  mm64_sub<true>(TA, diag ? TA : TB, acc, lane, w);  // G_ij -= X_i^T X_j
  if (diag && i == k + 1) {
    store_acc(TC, acc, 1.0, lane, w);
    if (t < kP) lim[t] = tol * gdiag[i * kP + t];
    __syncthreads();
    if (!chol64b(TC, TI, lim, &bad, tmp, t)) {
      if (t == 0) *flag = 1;
      return;
    }
    tile_to_global(R + tix(i, i, nb), TC, t);
    tile_to_global(Dinv + i * kT2, TI, t);
  } else {
    store_acc_global(G + tix(i, j, nb), kP, acc, 1.0, lane, w);
  }
}

// ---- Q1 = A R^{-1} in place, by 64-row stripes ---------------------------------
// Stripe rows are independent: column block J of the stripe becomes
// (A_J - sum_{I<J} Q1_I R_IJ) R_JJ^{-1}, blocks in increasing J, each written
// over A_J once A_J has been read. Eight waves per stripe, two per SIMD:
// wave w owns rows 16 (w & 3) .. + 15 and columns 32 (w >> 2) .. + 31 of each
// 64 x 64 product, so one wave's LDS reads overlap the other's products.
constexpr int kSW = 512;  // threads of a stripe workgroup

struct Stage8 {
  double v[8];
  uint32_t ok;
};
// tile element e = t + 512 u (row e / 64, column e % 64), as stage_load
__device__ __forceinline__ void stage8_load(Stage8& s, const double* a,
                                            int64_t lda, int64_t nr, int64_t nc,
                                            int t) {
  s.ok = 0u;
  const int64_t r1 = nr - 1, c1 = nc - 1;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int e = t + kSW * u;
    const int64_t i = e >> 6, j = e & 63;
    s.ok |= (i < nr && j < nc) ? (1u << u) : 0u;
    s.v[u] = a[(i < r1 ? i : r1) * lda + (j < c1 ? j : c1)];
  }
}
__device__ __forceinline__ void stage8_store(double* tile, const Stage8& s,
                                             int t) {
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int e = t + kSW * u;
    tile[(e >> 6) * kS + (e & 63)] = ((s.ok >> u) & 1u) ? s.v[u] : 0.0;
  }
}
// acc (+)= A B on the wave's 16 x 32 part
template <bool SUB>
__device__ __forceinline__ void mm64x8(const double* A, const double* B,
                                       dbl4 (&acc)[2], int lane, int w) {
  const int p = lane & 15, q = lane >> 4, wr = w & 3, wc = w >> 2;
#pragma unroll 4
  for (int kk = 0; kk < 16; ++kk) {
    const int k = 4 * kk + q;
    const double a = SUB ? -A[(16 * wr + p) * kS + k] : A[(16 * wr + p) * kS + k];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
      acc[bj] = mfma(a, B[k * kS + 32 * wc + 16 * bj + p], acc[bj]);
  }
}

__global__ void __launch_bounds__(kSW)
    stripe_solve_kernel(double* __restrict__ A, int64_t lda, int64_t m,
                        int64_t d, int64_t nb, const double* __restrict__ R,
                        const double* __restrict__ Dinv,
                        const int* __restrict__ flag) {
  __shared__ double TA[kTile];
  __shared__ double TB[kTile];
  if (*flag) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wr = w & 3, wc = w >> 2;
  const int p = lane & 15, q = lane >> 4;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kP;
  const int64_t nr = m - r0 < kP ? m - r0 : kP;
  double* As = A + r0 * lda;
  for (int64_t J = 0; J < nb; ++J) {
    const int64_t cJ = J * kP;
    const int64_t nc = d - cJ < kP ? d - cJ : kP;
    dbl4 acc[2];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * wr + 4 * v + q, col = 32 * wc + 16 * bj + p;
        acc[bj][v] = (row < nr && col < nc) ? As[row * lda + cJ + col] : 0.0;
      }
    // blocks I < J are complete (only the last block can be partial)
    Stage8 va, vb;
    if (J > 0) {
      stage8_load(va, As, lda, nr, kP, t);
      stage8_load(vb, R + tix(0, J, nb), kP, kP, kP, t);
    }
    for (int64_t I = 0; I < J; ++I) {
      __syncthreads();
      stage8_store(TA, va, t);
      stage8_store(TB, vb, t);
      __syncthreads();
      if (I + 1 < J) {
        stage8_load(va, As + (I + 1) * kP, lda, nr, kP, t);
        stage8_load(vb, R + tix(I + 1, J, nb), kP, kP, kP, t);
      }
      mm64x8<true>(TA, TB, acc, lane, w);
    }
    stage8_load(vb, Dinv + J * kT2, kP, kP, kP, t);
    __syncthreads();
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        TA[(16 * wr + 4 * v + q) * kS + 32 * wc + 16 * bj + p] = acc[bj][v];
    stage8_store(TB, vb, t);
    __syncthreads();
    dbl4 res[2];
    res[0] = res[1] = dbl4{0.0, 0.0, 0.0, 0.0};
    mm64x8<false>(TA, TB, res, lane, w);
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * wr + 4 * v + q, col = 32 * wc + 16 * bj + p;
        if (row < nr && col < nc) As[row * lda + cJ + col] = res[bj][v];
      }
    // Q1_J is read back by other threads of the workgroup for later blocks
    __syncthreads();
  }
}

// ---- R = R2 R1 into r_out (d x d row-major) ------------------------------------
// NEAR: F = G2 holds the second Gram matrix; after the checks of the header,
// R_ij = R1_ij + sum_{i<=l<=j} up(E)_il R1_lj. Otherwise F holds R2 (tiled,
// from the blocked Cholesky) and R_ij = sum_{i<=l<=j} R2_il R1_lj.
template <bool NEAR>
__global__ void __launch_bounds__(256)
    r_final_kernel(const double* __restrict__ R1, const double* __restrict__ F,
                   int64_t nb, int64_t d, const unsigned long long* __restrict__ emax,
                   int* __restrict__ status, double* __restrict__ r_out) {
  __shared__ double TA[kTile];
  __shared__ double TB[kTile];
  if (*status) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int p = lane & 15, q = lane >> 4;
  const int64_t i = blockIdx.x / nb, j = blockIdx.x % nb;
  if (NEAR) {
    __shared__ unsigned long long red[256];
    const int64_t ne = nb * (nb + 1) / 2 * 16;
    unsigned long long b = 0ull;
    for (int64_t e = t; e < ne; e += 256) b = emax[e] > b ? emax[e] : b;
    red[t] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (t < o) red[t] = red[t + o] > red[t] ? red[t + o] : red[t];
      __syncthreads();
    }
    const double em = __longlong_as_double(static_cast<long long>(red[0]));
    const bool ok = em <= 0.25 / static_cast<double>(d);  // false for NaN
    if (!ok || em > kNearId) {
      if (blockIdx.x == 0 && t == 0) *status = ok ? 2 : 1;
      return;
    }
  }
  dbl4 acc[4];
  zero4(acc);
  if (i <= j) {
    if (NEAR) ld_acc(acc, R1 + tix(i, j, nb), lane, w);
    // tiles of term l + 1 load while term l multiplies
    Stage vf, vr;
    auto issue = [&](int64_t l) {
      stage_load(vf, F + tix(i, l, nb), kP, kP, kP, t);
      stage_load(vr, R1 + tix(l, j, nb), kP, kP, kP, t);
    };
    issue(i);
    for (int64_t l = i; l <= j; ++l) {
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = t + 256 * u;
        const int a = e >> 6, b = e & 63;
        double v = vf.v[u];
        if (NEAR) {
          // up(E): strict upper part of G2 - I and half its diagonal
          const int64_t gi = i * kP + a, gl = l * kP + b;
          v = gi < gl ? v : (gi == gl ? 0.5 * (v - 1.0) : 0.0);
        }
        TA[a * kS + b] = v;
      }
      stage_store(TB, vr, t);
      __syncthreads();
      if (l < j) issue(l + 1);
      mm64<false>(TA, TB, acc, lane, w);
    }
  }
#pragma unroll
  for (int bj = 0; bj < 4; ++bj)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t gi = i * kP + 16 * w + 4 * v + q, gj = j * kP + 16 * bj + p;
      if (gi < d && gj < d) r_out[gi * d + gj] = gi <= gj ? acc[bj][v] : 0.0;
    }
}

struct Cq2 {
  int64_t nb, nt, S, chunk, Se, chunk_e, nfull, nedge;
  double *part, *G, *R1, *R2, *Dinv, *gdiag;
  unsigned long long* emax;
};

Cq2 cq2_shape(int64_t m, int64_t d) {
  Cq2 c{};
  c.nb = (d + kP - 1) / kP;
  c.nt = c.nb * (c.nb + 1) / 2;
  // Gram row chunks: blocks of full 128-column blocks take at most 512
  // workgroups in all (two per CU: one round), the edge blocks (thin: their
  // time is load latency, so they get many short chunks) at most 512;
  // chunks of at least 256 rows
  const int64_t nf = d / 128;
  c.nfull = nf * (nf + 1) / 2;
  c.nedge = d % 128 ? nf + 1 : 0;
  const int64_t steps = (m + kGK - 1) / kGK;
  const int64_t smax = (m + 255) / 256 > 1 ? (m + 255) / 256 : 1;
  auto pick = [&](int64_t slots, int64_t blocks, int64_t& S, int64_t& chunk) {
    S = blocks > 0 ? slots / blocks : 1;
    if (S > smax) S = smax;
    if (S < 1) S = 1;
    chunk = (steps + S - 1) / S * kGK;
  };
  pick(512, c.nfull, c.S, c.chunk);
  pick(512, c.nedge, c.Se, c.chunk_e);
  return c;
}

Cq2 cq2_carve(void* base, int64_t m, int64_t d) {
  Cq2 c = cq2_shape(m, d);
  double* p = static_cast<double*>(base);
  c.part = p;  p += (c.nfull * c.S + c.nedge * c.Se) * kB2;
  c.G = p;     p += c.nb * c.nb * kT2;
  c.R1 = p;    p += c.nb * c.nb * kT2;
  c.R2 = p;    p += c.nb * c.nb * kT2;
  c.Dinv = p;  p += c.nb * kT2;
  c.gdiag = p; p += c.nb * kP;
  c.emax = reinterpret_cast<unsigned long long*>(p);  // nt * 16 entries
  return c;
}

void gram_tiles(const double* a, int64_t m, int64_t d, const Cq2& c,
                bool with_emax, int* flag, hipStream_t s) {
  unsigned long long* em = with_emax ? c.emax : nullptr;
  prof_begin(kKCq2Gram, s);
  if (c.nfull > 0)
    gram_block_kernel<false><<<static_cast<unsigned>(c.nfull * c.S), 256, 0, s>>>(
        a, d, m, d, c.S, c.chunk, 0, c.part, flag);
  prof_end(kKCq2Gram, s);
  prof_begin(kKCq2GramEdge, s);
  if (c.nedge > 0)
    gram_block_kernel<true><<<static_cast<unsigned>(c.nedge * c.Se), 256, 0, s>>>(
        a, d, m, d, c.Se, c.chunk_e, c.nfull * c.S, c.part, flag);
  gram_reduce_kernel<<<static_cast<unsigned>(c.nt * 16), 256, 0, s>>>(
      c.part, c.S, c.Se, c.nb, d, c.G, c.gdiag, em, flag);
  prof_end(kKCq2GramEdge, s);
}

void bchol(const Cq2& c, double* R, int* flag, hipStream_t s) {
  prof_begin(kKCq2Chol, s);
  bchol_first_kernel<<<1, 256, 0, s>>>(c.G, c.gdiag, kPivotTol, R, c.Dinv, flag);
  for (int64_t k = 0; k + 1 < c.nb; ++k) {
    const int64_t n = c.nb - k - 1;
    bchol_step_kernel<<<static_cast<unsigned>(n * (n + 1) / 2), 256, 0, s>>>(
        c.G, c.nb, k, c.gdiag, kPivotTol, R, c.Dinv, flag);
  }
  prof_end(kKCq2Chol, s);
}

}  // namespace

size_t cholqr2_scratch_bytes(int64_t m, int64_t d) {
  const Cq2 c = cq2_shape(m, d);
  return static_cast<size_t>((c.nfull * c.S + c.nedge * c.Se) * kB2 +
                             3 * c.nb * c.nb * kT2 +
                             c.nb * kT2 + c.nb * kP + c.nt * 16 + 8) *
         sizeof(double);
}

void cholqr2_factor(double* a, int64_t m, int64_t d, double* r_out,
                    void* scratch, int* status, hipStream_t s) {
  const Cq2 c = cq2_carve(scratch, m, d);
  launch_fill_i32(status, 1, 0, s);
  gram_tiles(a, m, d, c, false, status, s);
  bchol(c, c.R1, status, s);
  prof_begin(kKCq2Solve, s);
  stripe_solve_kernel<<<cdivu(m, kP), kSW, 0, s>>>(a, d, m, d, c.nb, c.R1,
                                                    c.Dinv, status);
  prof_end(kKCq2Solve, s);
  gram_tiles(a, m, d, c, true, status, s);
  prof_begin(kKCq2R, s);
  r_final_kernel<true><<<static_cast<unsigned>(c.nb * c.nb), 256, 0, s>>>(
      c.R1, c.G, c.nb, d, c.emax, status, r_out);
  prof_end(kKCq2R, s);
}

void cholqr2_finish(int64_t m, int64_t d, double* r_out, void* scratch,
                    int* status, hipStream_t s) {
  const Cq2 c = cq2_carve(scratch, m, d);
  launch_fill_i32(status, 1, 0, s);
  bchol(c, c.R2, status, s);
  prof_begin(kKCq2R, s);
  r_final_kernel<false><<<static_cast<unsigned>(c.nb * c.nb), 256, 0, s>>>(
      c.R1, c.R2, c.nb, d, c.emax, status, r_out);
  prof_end(kKCq2R, s);
}

}  // namespace slso
