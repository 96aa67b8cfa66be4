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
//   e <= e_near(d) R2 = I + up(E) (strict upper part plus half the diagonal)
//                  and R = R1 + up(E) R1 in one launch. With R2 = I + F,
//                  F + F^T = E - F^T F, so the neglected term is at most
//                  d e^2 per entry; e_near(d) = min(1e-9, sqrt(1e-15 / d))
//                  keeps it below 1e-15 (about 9 units of FP64 rounding) at
//                  every d: 1e-9 up to d = 1000, 4.9e-10 at d = 4096;
//   e <= 0.25 / d  status 2: the caller runs cholqr2_finish, the blocked
//                  Cholesky of G2 and R = R2 R1;
//   otherwise, or when a Cholesky pivot of G1 falls to 1e-13 of its diagonal
//   entry, status 1: the caller factors the (re-formed) matrix with the
//   Householder paths.
//
// One pass (CholeskyQR). For the scores only R^T R matters: the first
// pass's R1 has R1^T R1 = A^T A + E with |E| about sqrt(m d) u |A|^2 under
// the usual model of rounding errors that add like random ones, which moves
// every score by a relative amount up to |E| / sigma_min(A)^2 =
// sqrt(m d) u kappa(A)^2. With one_pass = 2 the passes stop after R1 when
// 4 kappa_est^2 sqrt(m d) u <= 1e-7 (two orders below the FP32 gate of
// the scores), kappa_est = |R1 x| |R1^{-1} y| from six power iterations on
// R1 and on R1^{-1} (a lower bound of kappa, hence the factor 4 = 2^2):
// status 3, R = R1. With one_pass = 1 (the sketch factor only preconditions
// the refinement, which needs R^{-T} A^T A R^{-1} near I, not R itself) the
// bound is 1e-2. The estimate is a chain of about 17 small launches (about
// 0.1 ms at d = 256 to 512); it is only tried when the second pass's two
// m d^2 products (its Gram and Q1 = A R1^{-1}) reach 2^31 flop each, where
// they take longer than the estimate: below that both passes always run.
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
// max |G2 - I| for the one-launch R2 (see above)
__host__ __device__ inline double near_id(int64_t d) {
  const double b = sqrt(1e-15 / static_cast<double>(d));
  return b < 1e-9 ? b : 1e-9;
}

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
      for (int bj = 0; bj < 4; ++bj) acc[bj] = mfma(-a[kk], b[kk][bj], acc[bj]);
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
// FE (a last column block of at most 16 columns): no second launch. On a
// diagonal block the lower-left 64 x 64 quadrant is the transpose of the
// upper-right one, so waves 2 and 3 skip it and form the edge products
// A_I2^T A_e instead (8 + 4 MFMA blocks against the 16 of waves 0 and 1),
// and wave 2 of block (0, 0) also the corner A_e^T A_e; S_e = S.
constexpr int kGK = 16;    // rows per step
constexpr int64_t kGMin = 64;  // fewest rows of a workgroup's chunk
// Q1 out of place (q1_gemm_kernel) up to this many entries (128 MB): the
// sketches of the dense and serving workloads; above it the stripe solve
// works in place
constexpr int64_t kQ1Max = int64_t{1} << 24;
constexpr int kGS = 144;   // LDS row stride: rows 4 apart fall on the other
                           // half of the banks
constexpr int64_t kB2 = 128 * 128;

template <bool EDGE, bool FE>
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
  // FE: edge products on this diagonal block (waves 2, 3), the corner on (0, 0)
  const bool fe = FE && diag;
  const bool fw = fe && w >= 2;
  const bool corner = fe && I2 == 0 && w == 2;
  const int64_t cE = nf * 128, nE = d - cE;
  const int er = t >> 4, ec = t & 15;  // this thread's element of the edge rows
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
    if (fe) {
      const int64_t row = r + er;
      v[8] = A[(row < r1 && ec < nE) ? row * lda + cE + ec : 0];
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
    if (fe)
      X[buf][1][er * kGS + ec] = (r + er < r1 && ec < nE) ? v[8] : 0.0;
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
      if (!fw) {
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
      } else if (FE) {
        // acc[x][y], y >= 4: the upper-right quadrant as above; acc[0][y],
        // y < 4: edge block rows 64 (w - 2) + 16 y ..; acc[1][0]: corner
        const double* XE = X[buf][1];
#pragma unroll
        for (int kk = 0; kk < kGK / 4; ++kk) {
          const int k = 4 * kk + q;
          double a[2], b[4], ea[4];
#pragma unroll
          for (int x = 0; x < 2; ++x) a[x] = XA[k * kGS + 32 * w + 16 * x + p];
#pragma unroll
          for (int y = 0; y < 4; ++y) {
            b[y] = XA[k * kGS + 64 + 16 * y + p];
            ea[y] = XA[k * kGS + 64 * (w - 2) + 16 * y + p];
          }
          const double eb = XE[k * kGS + p];
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][4 + y] = mfma(a[x], b[y], acc[x][4 + y]);
#pragma unroll
          for (int y = 0; y < 4; ++y) acc[0][y] = mfma(ea[y], eb, acc[0][y]);
          if (corner) acc[1][0] = mfma(eb, eb, acc[1][0]);
        }
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
      if ((!EDGE || y < ncol) && !(fw && y < 4)) {
#pragma unroll
        for (int vv = 0; vv < 4; ++vv)
          out[(32 * w + 16 * x + 4 * vv + q) * 128 + 16 * y + p] = acc[x][y][vv];
      }
  if (FE && fw) {
    const int64_t nfull = nf * (nf + 1) / 2;
    double* oe = part + ((nfull + I2) * S + s) * kB2;
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int vv = 0; vv < 4; ++vv)
        oe[(64 * (w - 2) + 16 * y + 4 * vv + q) * 128 + p] = acc[0][y][vv];
    if (corner) {
      double* oc = part + ((nfull + nf) * S + s) * kB2;
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) oc[(4 * vv + q) * 128 + p] = acc[1][0][vv];
    }
  }
}

// Stream-K form of the full blocks (used when the last column block is not
// folded into the diagonal blocks): the work is cut into units of one block
// over one chunk of rows, C units per block in row order, blocks in
// upper_tile order, and workgroup g takes units g Q .. g Q + Q - 1, so every
// workgroup carries the same work whatever the number of blocks (528 blocks
// at d = 4096 would otherwise take two rounds of 512 slots, the second
// nearly empty). A run of a workgroup's units inside one block (a segment)
// is summed into partial block s of that block, s = the number of workgroup
// boundaries inside the block before the run, at part[(blk NS + s) 16384].
// one segment: block (I2, J2) over rows r0 .. r1 - 1 into out
__device__ __attribute__((noinline)) void gram_segment(
    const double* __restrict__ A, int64_t lda, int64_t I2, int64_t J2,
    int64_t r0, int64_t r1, double (*X)[2][kGK * kGS],
    double* __restrict__ out) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int p = lane & 15, q = lane >> 4;
  const bool diag = I2 == J2;
  const int c = t & 127, rr = t >> 7;
  const double* pa = A + I2 * 128 + c;
  const double* pb = A + J2 * 128 + c;
  dbl4 acc[2][8];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 8; ++y) acc[x][y] = dbl4{0.0, 0.0, 0.0, 0.0};
  double v[16];
  // loads without branches (rows past r1 read row r0); zeros put in when
  // the values go to LDS
  auto gload = [&](int64_t r) {
#pragma unroll
    for (int uu = 0; uu < 8; ++uu) {
      const int64_t row = r + rr + 2 * uu;
      const int64_t ro = (row < r1 ? row : r0) * lda;
      v[uu] = pa[ro];
      if (!diag) v[8 + uu] = pb[ro];
    }
  };
  auto lstore = [&](int buf, int64_t r) {
#pragma unroll
    for (int uu = 0; uu < 8; ++uu) {
      const int64_t row = r + rr + 2 * uu;
      X[buf][0][(rr + 2 * uu) * kGS + c] = row < r1 ? v[uu] : 0.0;
      if (!diag) X[buf][1][(rr + 2 * uu) * kGS + c] = row < r1 ? v[8 + uu] : 0.0;
    }
  };
  __syncthreads();  // the previous segment's last reads of X
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
        for (int y = 0; y < 8; ++y) acc[x][y] = mfma(a[x], b[y], acc[x][y]);
    }
    if (more) lstore(buf ^ 1, r + kGK);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 8; ++y)
#pragma unroll
      for (int vv = 0; vv < 4; ++vv)
        out[(32 * w + 16 * x + 4 * vv + q) * 128 + 16 * y + p] = acc[x][y][vv];
}

__global__ void __launch_bounds__(256, 2)
    gram_sk_kernel(const double* __restrict__ A, int64_t lda, int64_t m,
                   int64_t d, int64_t C, int64_t chunk, int64_t Q, int64_t NS,
                   double* __restrict__ part, const int* __restrict__ flag) {
  __shared__ double X[2][2][kGK * kGS];
  if (*flag) return;
  const int64_t nf = d / 128;
  const int64_t U = nf * (nf + 1) / 2 * C;
  int64_t u = static_cast<int64_t>(blockIdx.x) * Q;
  const int64_t uend = u + Q < U ? u + Q : U;
  while (u < uend) {
    const int64_t blk = u / C, c0 = u % C;
    const int64_t c1 = C < c0 + (uend - u) ? C : c0 + (uend - u);
    const int64_t seg = c0 == 0 ? 0 : u / Q - (blk * C) / Q;
    int64_t I2, J2;
    upper_tile(blk, nf, I2, J2);
    const int64_t r0 = c0 * chunk;
    const int64_t r1 = m < c1 * chunk ? m : c1 * chunk;
    // (r0 < m always: units past the last row are never made)
    gram_segment(A, lda, I2, J2, r0, r1, X, part + (blk * NS + seg) * kB2);
    u += c1 - c0;
  }
}

// G tile = sum of its partial blocks (fixed order); the padding is the
// identity; gdiag receives the diagonal. With emax, emax[workgroup] = max
// |G - I| over the workgroup's valid entries (bit patterns of non-negative
// doubles order like the values, a NaN above every number).
// Q > 0: the full blocks are in the stream-K form (C units per block, Q per
// workgroup, NS = S partial slots per block, the first nseg of them used).
__global__ void __launch_bounds__(256)
    gram_reduce_kernel(const double* __restrict__ part, int64_t S, int64_t Se,
                       int64_t C, int64_t Q, int64_t nb, int64_t d,
                       const double* __restrict__ dsc, double* __restrict__ G,
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
    const int64_t b = upper_index(I2, J2, nf);
    // partial blocks of this block: S of them, or in the stream-K form one
    // per workgroup boundary inside its units plus one
    const int64_t np = Q > 0 ? 1 + (b * C + C - 1) / Q - (b * C) / Q : S;
    v = sum_parts(part + b * S * kB2 + off, np, kB2, 0);
  } else {
    const int64_t blk = nf * (nf + 1) / 2 * S + I2 * Se;
    v = sum_parts(part + blk * kB2 + off, Se, kB2, 0);
  }
  // (A diag(dsc))^T (A diag(dsc)): exact scaling by powers of two
  if (dsc && gi < d && gj < d) v *= dsc[gi] * dsc[gj];
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
                       double* __restrict__ Dinv, double* __restrict__ X,
                       int* __restrict__ flag) {
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
  if (X) tile_to_global(X, TX, t);
}

// X = R^{-1} block column by block column from X R = I:
//   X_ik = -(sum_{l=i}^{k-1} X_il R_lk) R_kk^{-1},  i < k.
// Each term needs block column l of X and block row l of R, which the step
// launches produce at step l. So the terms are added as they become
// available: at step k every pair (i, j), i < k < j, takes the term
// l = k - 1 into a running sum P_ij (one product per workgroup), and block
// column k is finished from P_ik and its last term (two products). No
// workgroup of a step then does more than the diagonal one.
__device__ __forceinline__ void two_tiles(double* TA, double* TB,
                                          const double* a, const double* b,
                                          int t) {
  load_tile(TA, a, kP, kP, kP, t);
  load_tile(TB, b, kP, kP, kP, t);
}

// X_ik = -(P_ik + X_{i,k-1} R_{k-1,k}) R_kk^{-1} (P_ik holds the terms
// l <= k - 2 when i <= k - 2)
__device__ __forceinline__ void xinv_finish(int64_t i, int64_t k, int64_t nb,
                                            const double* __restrict__ R,
                                            const double* __restrict__ Dinv,
                                            double* __restrict__ X,
                                            const double* __restrict__ P,
                                            double* TA, double* TB, int t) {
  const int lane = t & 63, w = t >> 6;
  dbl4 acc[4];
  if (i + 2 <= k)
    ld_acc(acc, P + tix(i, k, nb), lane, w);
  else
    zero4(acc);
  two_tiles(TA, TB, X + tix(i, k - 1, nb), R + tix(k - 1, k, nb), t);
  __syncthreads();
  mm64<false>(TA, TB, acc, lane, w);
  __syncthreads();
  store_acc(TA, acc, -1.0, lane, w);
  load_tile(TB, Dinv + k * kT2, kP, kP, kP, t);
  __syncthreads();
  dbl4 res[4];
  zero4(res);
  mm64<false>(TA, TB, res, lane, w);
  store_acc_global(X + tix(i, k, nb), kP, res, 1.0, lane, w);
}

// P_ij (+)= X_{i,k-1} R_{k-1,j}: the first term when i = k - 1
__device__ __forceinline__ void xinv_term(int64_t i, int64_t j, int64_t k,
                                          int64_t nb, const double* __restrict__ R,
                                          const double* __restrict__ X,
                                          double* __restrict__ P, double* TA,
                                          double* TB, int t) {
  const int lane = t & 63, w = t >> 6;
  dbl4 acc[4];
  if (i + 1 < k)
    ld_acc(acc, P + tix(i, j, nb), lane, w);
  else
    zero4(acc);
  two_tiles(TA, TB, X + tix(i, k - 1, nb), R + tix(k - 1, j, nb), t);
  __syncthreads();
  mm64<false>(TA, TB, acc, lane, w);
  store_acc_global(P + tix(i, j, nb), kP, acc, 1.0, lane, w);
}

// Block column k of X (tiles i < k); used for the last block column, which
// the step launches do not reach.
__global__ void __launch_bounds__(256)
    binv_col_kernel(int64_t nb, int64_t k, const double* __restrict__ R,
                    const double* __restrict__ Dinv, double* __restrict__ X,
                    const double* __restrict__ P, const int* __restrict__ flag) {
  __shared__ double TA[kTile];
  __shared__ double TB[kTile];
  if (*flag) return;
  xinv_finish(blockIdx.x, k, nb, R, Dinv, X, P, TA, TB, threadIdx.x);
}

// The step's diagonal workgroup (tile (k + 1, k + 1)), which the next step
// waits for: X = R_kk^{-T} G_k,k+1 by column strips (wave w forms columns
// 16 w .. 16 w + 15; row block rb of R_kk^{-T} is zero past column block rb,
// so each wave does 40 of the 64 MFMA blocks), then G_k+1,k+1 - X^T X on the
// upper 16 x 16 blocks only (the factorisation reads no others): three or
// two blocks per wave. TI holds R_kk^{-1}, TA G_k,k+1; TC receives the
// updated tile (lower blocks undefined) and may be TI, which is read only
// before the first barrier.
__device__ __forceinline__ void bchol_lead(const double* TI, double* TA, double* TC,
                                           const double* __restrict__ Gd,
                                           double* __restrict__ Rg, int lane, int w) {
  const int p = lane & 15, q = lane >> 4;
  // the tile's own blocks: upper block w + 4 u of the wave
  // (rb, cb) of upper block b in row order: (0,0) .. (0,3), (1,1) .. (3,3)
  auto up_r = [](int b) { return b < 4 ? 0 : b < 7 ? 1 : b < 9 ? 2 : 3; };
  auto up_c = [](int b) { return b < 4 ? b : b < 7 ? b - 3 : b < 9 ? b - 5 : 3; };
  dbl4 g[3];
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int b = w + 4 * u < 10 ? w + 4 * u : 9;
#pragma unroll
    for (int v = 0; v < 4; ++v)
      g[u][v] = Gd[(16 * up_r(b) + 4 * v + q) * kP + 16 * up_c(b) + p];
  }
  dbl4 x[4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) x[rb] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k0 = 0; k0 < 4; ++k0) {
    // column block k0 of R_kk^{-T} feeds row blocks rb >= k0
    double b[4], a[4][4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int k = 16 * k0 + 4 * kk + q;
      b[kk] = TA[k * kS + 16 * w + p];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
        if (rb >= k0) a[kk][rb] = TI[k * kS + 16 * rb + p];
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
        if (rb >= k0) x[rb] = mfma(a[kk][rb], b[kk], x[rb]);
  }
  __syncthreads();  // every wave is done reading TA
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      TA[(16 * rb + 4 * v + q) * kS + 16 * w + p] = x[rb][v];
      Rg[(16 * rb + 4 * v + q) * kP + 16 * w + p] = x[rb][v];
    }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    if (w + 4 * u >= 10) break;
    const int rb = up_r(w + 4 * u), cb = up_c(w + 4 * u);
#pragma unroll
    for (int k0 = 0; k0 < 16; k0 += 8) {
      double a[8], b[8];
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        const int k = 4 * (k0 + kk) + q;
        a[kk] = TA[k * kS + 16 * rb + p];
        b[kk] = TA[k * kS + 16 * cb + p];
      }
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) g[u] = mfma(-a[kk], b[kk], g[u]);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) TC[(16 * rb + 4 * v + q) * kS + 16 * cb + p] = g[u][v];
  }
}

// Step k: tiles (i, j), k < i <= j, one workgroup each (see the header).
// With X, k more workgroups finish block column k of X = R^{-1}, and
// k (nb - k - 1) more add the term l = k - 1 to the running sums P_ij.
__global__ void __launch_bounds__(256)
    bchol_step_kernel(double* __restrict__ G, int64_t nb, int64_t k, int64_t d,
                      const double* __restrict__ gdiag, double tol,
                      double* __restrict__ R, double* __restrict__ Dinv,
                      double* __restrict__ X, double* __restrict__ P,
                      int* __restrict__ flag) {
  // two tiles of LDS (76 KB with the factorisation's scratch), so two
  // workgroups share a CU
  __shared__ double T0[kTile];
  __shared__ double T1[kTile];
  __shared__ double tmp[4][16][17];
  __shared__ double lim[kP];
  __shared__ int bad;
  if (*flag) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t n = nb - k - 1;
  const int64_t ntile = n * (n + 1) / 2;
  if (blockIdx.x >= ntile) {
    const int64_t b = blockIdx.x - ntile;
    if (b < k)
      xinv_finish(b, k, nb, R, Dinv, X, P, T0, T1, t);
    else
      xinv_term((b - k) / n, k + 1 + (b - k) % n, k, nb, R, X, P, T0, T1, t);
    return;
  }
  int64_t i, j;
  upper_tile(blockIdx.x, n, i, j);
  i += k + 1;
  j += k + 1;
  const bool diag = i == j;
  if (diag && i == k + 1) {
    // T0 = R_kk^{-1}, then the updated tile (R after the factorisation);
    // T1 = G_k,k+1, then X, then R^{-1} of the tile
    load_tile(T0, Dinv + k * kT2, kP, kP, kP, t);
    load_tile(T1, G + tix(k, i, nb), kP, kP, kP, t);
    if (t < kP) lim[t] = tol * gdiag[i * kP + t];
    __syncthreads();
    bchol_lead(T0, T1, T0, G + tix(i, i, nb), R + tix(k, i, nb), lane, w);
    __syncthreads();
    const int64_t nv = d - i * kP;  // columns of the tile inside the matrix
    const int nblk = nv >= kP ? 4 : static_cast<int>((nv + 15) / 16);
    if (!chol64b(T0, T1, lim, &bad, tmp, t, nblk)) {
      if (t == 0) *flag = 1;
      return;
    }
    tile_to_global(R + tix(i, i, nb), T0, t);
    tile_to_global(Dinv + i * kT2, T1, t);
    if (X) tile_to_global(X + tix(i, i, nb), T1, t);
    return;
  }
  // G_kj staged in registers while X_i = R_kk^-T G_ki is formed; T1 then
  // takes it for X_j
  Stage sb;
  if (!diag) stage_load(sb, G + tix(k, j, nb), kP, kP, kP, t);
  load_tile(T0, Dinv + k * kT2, kP, kP, kP, t);
  load_tile(T1, G + tix(k, i, nb), kP, kP, kP, t);
  dbl4 acc[4];
  ld_acc(acc, G + tix(i, j, nb), lane, w);
  __syncthreads();
  dbl4 xa[4], xb[4];
  zero4(xa);
  mm64<true>(T0, T1, xa, lane, w);  // X_i = R_kk^{-T} G_ki = R_ki
  if (!diag) {
    __syncthreads();
    stage_store(T1, sb, t);
    __syncthreads();
    zero4(xb);
    mm64<true>(T0, T1, xb, lane, w);
  }
  __syncthreads();
  store_acc(T0, xa, 1.0, lane, w);
  if (!diag) store_acc(T1, xb, 1.0, lane, w);
  if (i == k + 1) {
    if (diag)
      store_acc_global(R + tix(k, j, nb), kP, xa, 1.0, lane, w);
    else
      store_acc_global(R + tix(k, j, nb), kP, xb, 1.0, lane, w);
  }
  __syncthreads();
  mm64_sub<true>(T0, diag ? T0 : T1, acc, lane, w);  // G_ij -= X_i^T X_j
  store_acc_global(G + tix(i, j, nb), kP, acc, 1.0, lane, w);
}

// ---- Q1 = A R^{-1} in place, by row stripes -------------------------------------
// Stripe rows are independent: column block J of the stripe becomes
// (A_J - sum_{I<J} Q1_I R_IJ) R_JJ^{-1}, blocks in increasing J, each written
// over A_J once A_J has been read. A stripe of kR rows has kR / 8 waves
// (kR / 16 row groups x 2 column halves): wave w owns rows
// 16 (w % (kR / 16)) .. + 15 and columns 32 (w / (kR / 16)) .. + 31 of each
// kR x 64 product. 64-row stripes (eight waves, two per SIMD) measured
// faster than 32-row ones (two workgroups of four waves per CU).
constexpr int kStripeRows = 64;

template <int N>
struct StageN {
  double v[N];
  uint32_t ok;
};
// element e = t + kT u (row e / 64, column e % 64) of a tile, loaded without
// branches (clamped addresses, validity bits), as stage_load
template <int N, int kT>
__device__ __forceinline__ void stagen_load(StageN<N>& s, const double* a,
                                            int64_t lda, int64_t nr, int64_t nc,
                                            int t) {
  s.ok = 0u;
  const int64_t r1 = nr - 1, c1 = nc - 1;
#pragma unroll
  for (int u = 0; u < N; ++u) {
    const int e = t + kT * u;
    const int64_t i = e >> 6, j = e & 63;
    s.ok |= (i < nr && j < nc) ? (1u << u) : 0u;
    s.v[u] = a[(i < r1 ? i : r1) * lda + (j < c1 ? j : c1)];
  }
}
template <int N, int kT>
__device__ __forceinline__ void stagen_store(double* tile, const StageN<N>& s,
                                             int t) {
#pragma unroll
  for (int u = 0; u < N; ++u) {
    const int e = t + kT * u;
    tile[(e >> 6) * kS + (e & 63)] = ((s.ok >> u) & 1u) ? s.v[u] : 0.0;
  }
}
// acc (+)= A B on the wave's 16 x 32 part (kWR row groups); NBJ < 2: only
// its first NBJ 16-column blocks (the others lie past the matrix)
template <bool SUB, int kWR, int NBJ = 2>
__device__ __forceinline__ void mm_stripe(const double* A, const double* B,
                                          dbl4 (&acc)[2], int lane, int w) {
  const int p = lane & 15, q = lane >> 4, wr = w % kWR, wc = w / kWR;
  // the operands of eight steps are read before their products: one LDS
  // round trip per sixteen MFMAs
#pragma unroll
  for (int k0 = 0; k0 < 16; k0 += 8) {
    double a[8], b[8][2];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const int k = 4 * (k0 + kk) + q;
      a[kk] = A[(16 * wr + p) * kS + k];
#pragma unroll
      for (int bj = 0; bj < NBJ; ++bj) b[kk][bj] = B[k * kS + 32 * wc + 16 * bj + p];
    }
#pragma unroll
    for (int kk = 0; kk < 8; ++kk)
#pragma unroll
      for (int bj = 0; bj < NBJ; ++bj)
        acc[bj] = mfma(SUB ? -a[kk] : a[kk], b[kk][bj], acc[bj]);
  }
}
// the product on the columns below nc only (whole-wave choice)
template <bool SUB, int kWR>
__device__ __forceinline__ void mm_stripe_nc(const double* A, const double* B,
                                             dbl4 (&acc)[2], int lane, int w,
                                             int64_t nc) {
  const int wc = w / kWR;
  if (32 * wc + 16 < nc)
    mm_stripe<SUB, kWR, 2>(A, B, acc, lane, w);
  else if (32 * wc < nc)
    mm_stripe<SUB, kWR, 1>(A, B, acc, lane, w);
}

// The products of a stripe form one sequence of phases: for each J the terms
// I = 0 .. J - 1 (operands Q1_I and R_IJ), then the diagonal one (the
// accumulated block times R_JJ^{-1}). The phase operands go through two LDS
// buffers, so one barrier per phase separates the stores into one buffer from
// the products on the other, and each phase's loads (the next block's A_J
// included) are issued before the previous phase multiplies. The one load that
// would read a block stored by the phase before it (Q1_0, right after the
// diagonal phase of J = 0) is issued after that store and a barrier instead.
template <int kR>
__global__ void __launch_bounds__(8 * kR)
    stripe_solve_kernel(double* __restrict__ A, int64_t lda, int64_t m,
                        int64_t d, int64_t nb, const double* __restrict__ R,
                        const double* __restrict__ Dinv,
                        const double* __restrict__ dsc,
                        const int* __restrict__ flag) {
  constexpr int kT = 8 * kR, kWR = kR / 16;
  constexpr int kNA = kR * 64 / kT, kNB = 4096 / kT;  // staged per thread
  __shared__ double TA[2][kR * kS];
  __shared__ double TB[2][kTile];
  if (*flag) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wr = w % kWR, wc = w / kWR;
  const int p = lane & 15, q = lane >> 4;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kR;
  const int64_t nr = m - r0 < kR ? m - r0 : kR;
  double* As = A + r0 * lda;
  // A_J (times dsc) in this thread's accumulator layout; branch-free loads
  // (an entry outside the matrix reads a clamped address and becomes zero)
  auto load_aj = [&](dbl4 (&x)[2], int64_t J) {
    const int64_t cJ = J * kP;
    const int64_t nc = d - cJ < kP ? d - cJ : kP;
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * wr + 4 * v + q, col = 32 * wc + 16 * bj + p;
        const bool ok = row < nr && col < nc;
        const double av = As[ok ? row * lda + cJ + col : 0];
        x[bj][v] = ok ? av : 0.0;
      }
    if (dsc) {
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        const int col = 32 * wc + 16 * bj + p;
        const double sc = dsc[col < nc ? cJ + col : 0];
#pragma unroll
        for (int v = 0; v < 4; ++v) x[bj][v] *= sc;
      }
    }
  };
  StageN<kNA> va;
  StageN<kNB> vb;
  // phase (I, J): I < J a term, I == J the diagonal phase
  auto issue = [&](int64_t I, int64_t J) {
    if (I < J) {
      stagen_load<kNA, kT>(va, As + I * kP, lda, nr, kP, t);
      stagen_load<kNB, kT>(vb, R + tix(I, J, nb), kP, kP, kP, t);
    } else {
      stagen_load<kNB, kT>(vb, Dinv + J * kT2, kP, kP, kP, t);
    }
  };
  dbl4 acc[2], nacc[2];
  load_aj(acc, 0);
  issue(0, 0);
  int buf = 0;
  int64_t I = 0, J = 0;
  while (J < nb) {
    const int64_t nc = d - J * kP < kP ? d - J * kP : kP;
    const bool dg = I == J;
    if (dg) {
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          TA[buf][(16 * wr + 4 * v + q) * kS + 32 * wc + 16 * bj + p] = acc[bj][v];
    } else {
      stagen_store<kNA, kT>(TA[buf], va, t);
    }
    stagen_store<kNB, kT>(TB[buf], vb, t);
    __syncthreads();
    // the next phase
    const int64_t nI = dg ? 0 : I + 1, nJ = dg ? J + 1 : J;
    const bool more = nJ < nb;
    const bool late = dg && J == 0 && more && nI < nJ;  // reads Q1_0
    if (more && !late) issue(nI, nJ);
    if (dg && more) load_aj(nacc, nJ);
    if (dg) {
      dbl4 res[2];
      res[0] = res[1] = dbl4{0.0, 0.0, 0.0, 0.0};
      mm_stripe_nc<false, kWR>(TA[buf], TB[buf], res, lane, w, nc);
      const int64_t cJ = J * kP;
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * wr + 4 * v + q, col = 32 * wc + 16 * bj + p;
          if (row < nr && col < nc) As[row * lda + cJ + col] = res[bj][v];
        }
      if (late) {
        // Q1_0 is read back by other threads of the workgroup
        __syncthreads();
        issue(nI, nJ);
      }
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) acc[bj] = nacc[bj];
    } else {
      mm_stripe_nc<true, kWR>(TA[buf], TB[buf], acc, lane, w, nc);
    }
    buf ^= 1;
    I = nI;
    J = nJ;
  }
}

// ---- Q1 = (A diag(dsc)) X1 out of place, by 64 x 64 tiles --------------------
// When R^{-1} is kept in factored form (no R wanted), the second pass may take
// Q1 as A times the tiled X1 = R1^{-1} that the blocked Cholesky built, not as
// a triangular solve: the second Gram is then that of exactly this product,
// and R^{-1} = X1 R2^{-1} (or X1 (I - F)) is applied with the same X1, so X1's
// own rounding cancels. Tile (R, J) of Q1 = sum over I <= J of A_RI X1_IJ,
// one workgroup each (blockIdx.x the row block, blockIdx.y = J), the K loop
// through one pair of LDS tiles (66 KB: two workgroups per CU) with the next
// term's tiles loaded into registers while the current one multiplies.
// Unlike the stripe solve the terms do not depend on each other, so every
// tile of Q1 runs at once.
__global__ void __launch_bounds__(256)
    q1_gemm_kernel(const double* __restrict__ A, int64_t m, int64_t d,
                   int64_t nb, const double* __restrict__ X,
                   const double* __restrict__ dsc, double* __restrict__ Q,
                   const int* __restrict__ flag) {
  __shared__ double TA[kTile];
  __shared__ double TB[kTile];
  if (*flag) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t R = blockIdx.x, J = blockIdx.y;
  const int64_t r0 = R * kP;
  const int64_t nr = m - r0 < kP ? m - r0 : kP;
  dbl4 acc[4];
  zero4(acc);
  Stage va, vb;
  auto issue = [&](int64_t I) {
    const int64_t c0 = I * kP;
    const int64_t nc = d - c0 < kP ? d - c0 : kP;
    stage_load(va, A + r0 * d + c0, d, nr, nc, t);
    stage_load(vb, X + tix(I, J, nb), kP, kP, kP, t);
  };
  issue(0);
  for (int64_t I = 0; I <= J; ++I) {
    if (dsc) {
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int64_t col = I * kP + ((t + 256 * u) & 63);
        va.v[u] *= dsc[col < d ? col : 0];
      }
    }
    if (I > 0) __syncthreads();  // every wave is done with the last term
    stage_store(TA, va, t);
    stage_store(TB, vb, t);
    __syncthreads();
    if (I < J) issue(I + 1);
    mm64<false>(TA, TB, acc, lane, w);
  }
  const int p = lane & 15, q = lane >> 4;
  const int64_t c0 = J * kP;
#pragma unroll
  for (int bj = 0; bj < 4; ++bj)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = 16 * w + 4 * v + q, col = 16 * bj + p;
      if (row < nr && c0 + col < d) Q[(r0 + row) * d + c0 + col] = acc[bj][v];
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
  if (status && *status) return;
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
    if (!ok || em > near_id(d)) {
      if (status && blockIdx.x == 0 && t == 0) *status = ok ? 2 : 1;
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

// ---- R^{-1} B through the tiled inverse ---------------------------------------
// out = T B for an upper-triangular tiled T (d x d) and B (d x kk row-major):
// row block I of out sums T_IJ B_J over J >= I; the sum is split into chunks
// of kCH tile columns (one workgroup each, partial 64 x 64 blocks), then the
// chunks are added in order. MODE 0 takes T's tiles as stored; MODE 1 forms
// T = I - up(G - I) from the tiles of a Gram matrix G close to I (the first
// two terms of (I + up(G - I))^{-1}; the next is below d max|G - I|^2).
constexpr int64_t kCH = 1;  // one tile product per workgroup: the products
                            // are latency bound, so more workgroups win

__host__ __device__ inline int64_t tri_chunks(int64_t nb, int64_t I) {
  return (nb - I + kCH - 1) / kCH;
}
__host__ __device__ inline int64_t tri_parts(int64_t nb) {
  int64_t n = 0;
  for (int64_t I = 0; I < nb; ++I) n += tri_chunks(nb, I);
  return n;
}

template <int MODE>
__global__ void __launch_bounds__(256)
    tri_part_kernel(const double* __restrict__ T, int64_t nb, int64_t d,
                    const double* __restrict__ B, int64_t kk, int64_t cb0,
                    int64_t ncb, double* __restrict__ part,
                    const int* __restrict__ flag) {
  __shared__ double TA[kTile];
  __shared__ double TB[kTile];
  if (flag && *flag) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int64_t pidx = blockIdx.x, I = 0, rest = blockIdx.x;
  while (rest >= tri_chunks(nb, I)) {
    rest -= tri_chunks(nb, I);
    ++I;
  }
  const int64_t J0 = I + rest * kCH;
  const int64_t J1 = J0 + kCH < nb ? J0 + kCH : nb;
  const int64_t cb = cb0 + blockIdx.y;
  const int64_t c0 = cb * kP;
  dbl4 acc[4];
  zero4(acc);
  // the next pair of tiles is loaded while this one multiplies
  Stage vt, vb;
  stage_load(vt, T + tix(I, J0, nb), kP, kP, kP, t);
  stage_load(vb, B + J0 * kP * kk + c0, kk, d - J0 * kP, kk - c0, t);
  for (int64_t J = J0; J < J1; ++J) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = t + 256 * u;
      const int a = e >> 6, b = e & 63;
      double v = vt.v[u];
      if (MODE == 1) {
        const int64_t gi = I * kP + a, gj = J * kP + b;
        v = gi < gj ? -v : (gi == gj ? 1.0 - 0.5 * (v - 1.0) : 0.0);
      }
      TA[a * kS + b] = v;
    }
    stage_store(TB, vb, t);
    __syncthreads();
    if (J + 1 < J1) {
      stage_load(vt, T + tix(I, J + 1, nb), kP, kP, kP, t);
      stage_load(vb, B + (J + 1) * kP * kk + c0, kk, d - (J + 1) * kP, kk - c0, t);
    }
    mm64<false>(TA, TB, acc, lane, w);
  }
  store_acc_global(part + (pidx * ncb + blockIdx.y) * kT2, kP, acc, 1.0, lane,
                   w);
}

__global__ void __launch_bounds__(256)
    tri_sum_kernel(const double* __restrict__ part, int64_t nb, int64_t d,
                   int64_t kk, int64_t cb0, int64_t ncb,
                   double* __restrict__ out, const int* __restrict__ flag) {
  if (flag && *flag) return;
  const int64_t I = blockIdx.x, cbl = blockIdx.y;
  const int e = static_cast<int>(blockIdx.z) * 256 + threadIdx.x;
  int64_t p0 = 0;
  for (int64_t i = 0; i < I; ++i) p0 += tri_chunks(nb, i);
  double v = 0.0;
  for (int64_t ch = 0; ch < tri_chunks(nb, I); ++ch)
    v += part[((p0 + ch) * ncb + cbl) * kT2 + e];
  const int64_t row = I * kP + (e >> 6), col = (cb0 + cbl) * kP + (e & 63);
  if (row < d && col < kk) out[row * kk + col] = v;
}

// min and max |R_jj| without forming R: R_jj = (1 + F_jj) R1_jj with
// F_jj = (G2_jj - 1) / 2 (NEAR, after the checks of r_final_kernel), or
// R2_jj R1_jj.
template <bool NEAR>
__global__ void __launch_bounds__(256)
    r_diag_kernel(const double* __restrict__ R1, const double* __restrict__ R2,
                  const double* __restrict__ gdiag, int64_t nb, int64_t d,
                  const unsigned long long* __restrict__ emax,
                  int* __restrict__ status, double* __restrict__ dstat) {
  __shared__ unsigned long long redu[256];
  __shared__ double rmin[256], rmax[256];
  if (*status) return;
  const int t = threadIdx.x;
  if (NEAR) {
    const int64_t ne = nb * (nb + 1) / 2 * 16;
    unsigned long long b = 0ull;
    for (int64_t e = t; e < ne; e += 256) b = emax[e] > b ? emax[e] : b;
    redu[t] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (t < o) redu[t] = redu[t + o] > redu[t] ? redu[t + o] : redu[t];
      __syncthreads();
    }
    const double em = __longlong_as_double(static_cast<long long>(redu[0]));
    const bool ok = em <= 0.25 / static_cast<double>(d);
    if (!ok || em > near_id(d)) {
      if (t == 0) *status = ok ? 2 : 1;
      return;
    }
  }
  double lo = 1.0 / 0.0, hi = 0.0;
  for (int64_t j = t; j < d; j += 256) {
    const int64_t I = j / kP, o = (j % kP) * kP + j % kP;
    const double r1 = R1[tix(I, I, nb) + o];
    const double f = NEAR ? 1.0 + 0.5 * (gdiag[j] - 1.0) : R2[tix(I, I, nb) + o];
    const double v = fabs(f * r1);
    lo = v < lo ? v : lo;
    hi = v > hi ? v : hi;
  }
  rmin[t] = lo;
  rmax[t] = hi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      rmin[t] = rmin[t + o] < rmin[t] ? rmin[t + o] : rmin[t];
      rmax[t] = rmax[t + o] > rmax[t] ? rmax[t + o] : rmax[t];
    }
    __syncthreads();
  }
  if (t == 0) {
    dstat[0] = rmin[0];
    dstat[1] = rmax[0];
  }
}

// ---- condition estimate of R1 (one-pass acceptance) -------------------------
// Power iteration on R1 and X1 = R1^{-1} together (blockIdx.y = 0, 1): the
// vectors live in v[mat][nb 64] (zero past d, where the tiles hold the
// identity). Every workgroup forms the norm of its input vector itself, in
// the same order, so the iteration is deterministic.
constexpr int kPowIters = 6;

// Cheap lower bounds of kappa(R1) = sigma_max(R1) sigma_max(X1): for a
// triangular matrix max |R1_jj| / min |R1_jj|, and the largest column norm
// of R1 (that of A: sqrt(G_jj)) times the largest row norm of X1. When one
// of them already breaks the one-pass bound, *skip = 1 and the power
// iterations do not run. xrow[I] receives the largest squared row norm of
// row block I of X1 (one workgroup each).
__global__ void __launch_bounds__(256)
    x_rownorm_kernel(const double* __restrict__ X1, int64_t nb,
                     const int* __restrict__ status, double* __restrict__ xrow) {
  __shared__ double red[256];
  if (*status) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t I = blockIdx.x;
  // lane b, rows w + 4 u: row sums of squares over the tiles J >= I
  double acc[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) acc[u] = 0.0;
  for (int64_t J = I; J < nb; ++J) {
    const double* tile = X1 + tix(I, J, nb);
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const double e = tile[(w + 4 * u) * kP + lane];
      acc[u] += e * e;
    }
  }
  double mx = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    double a = acc[u];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    mx = a > mx ? a : mx;
  }
  red[t] = mx;
  __syncthreads();
  if (t == 0) {
    const double m01 = red[0] > red[64] ? red[0] : red[64];
    const double m23 = red[128] > red[192] ? red[128] : red[192];
    xrow[I] = m01 > m23 ? m01 : m23;
  }
}

__global__ void __launch_bounds__(256)
    cq1_precheck_kernel(const double* __restrict__ R1,
                        const double* __restrict__ gdiag,
                        const double* __restrict__ xrow, int64_t nb, int64_t m,
                        int64_t d, double bound, const int* __restrict__ status,
                        int* __restrict__ skip) {
  __shared__ double red[3][256];
  const int t = threadIdx.x;
  if (*status) {
    if (t == 0) *skip = 1;
    return;
  }
  // red[0]: min |R1_jj|, red[1]: max |R1_jj|, red[2]: max G_jj, and then
  // max of xrow
  double lo = 1.0 / 0.0, hi = 0.0, gm = 0.0, xm = 0.0;
  for (int64_t j = t; j < d; j += 256) {
    const int64_t I = j / kP, o = (j % kP) * kP + j % kP;
    const double r = fabs(R1[tix(I, I, nb) + o]);
    lo = r < lo ? r : lo;
    hi = r > hi ? r : hi;
    gm = gdiag[j] > gm ? gdiag[j] : gm;
  }
  for (int64_t I = t; I < nb; I += 256) xm = xrow[I] > xm ? xrow[I] : xm;
  red[0][t] = lo;
  red[1][t] = hi;
  red[2][t] = gm;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      red[0][t] = red[0][t + o] < red[0][t] ? red[0][t + o] : red[0][t];
      red[1][t] = red[1][t + o] > red[1][t] ? red[1][t + o] : red[1][t];
      red[2][t] = red[2][t + o] > red[2][t] ? red[2][t + o] : red[2][t];
    }
    __syncthreads();
  }
  const double rlo = red[0][0], rhi = red[1][0], gmax = red[2][0];
  __syncthreads();
  red[0][t] = xm;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) red[0][t] = red[0][t + o] > red[0][t] ? red[0][t + o] : red[0][t];
    __syncthreads();
  }
  if (t == 0) {
    const double k1 = rhi / rlo;
    const double k2 = sqrt(gmax * red[0][0]);
    const double kl = k1 > k2 ? k1 : k2;
    const bool ok = 4.0 * kl * kl * sqrt(static_cast<double>(m) * d) *
                        0x1p-53 <= bound;  // false for NaN
    *skip = ok ? 0 : 1;
  }
}

__global__ void __launch_bounds__(256)
    pow_init_kernel(int64_t nb, int64_t d, double* __restrict__ v,
                    const int* __restrict__ skip) {
  if (*skip) return;
  const int64_t n = nb * kP;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < 2 * n; i += gridDim.x * 256) {
    const int64_t j = i % n;
    // signs and sizes from a multiplicative hash of the index
    const uint32_t hsh = static_cast<uint32_t>(j) * 0x9E3779B9u;
    const double val = (1.0 + static_cast<double>(hsh >> 22) / 1024.0) *
                       ((hsh >> 21) & 1u ? -1.0 : 1.0);
    v[i] = j < d ? val : 0.0;
  }
}

// 1 / |x| of x[0 .. n), the same value in every workgroup
__device__ double inv_norm(const double* __restrict__ x, int64_t n,
                           double* red) {
  const int t = threadIdx.x;
  double acc = 0.0;
  for (int64_t i = t; i < n; i += 256) acc += x[i] * x[i];
  red[t] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r > 0.0 ? 1.0 / sqrt(r) : 0.0;
}

// y = T (x / |x|) (TRANS: T^T (x / |x|)) for T = R1 (y 0) or X1 (y 1);
// workgroup blockIdx.x forms the 64 entries of row block I (TRANS: column
// block J). One launch per product: the form for nb <= kPowOne, where the
// longest row of tiles is short.
template <bool TRANS>
__global__ void __launch_bounds__(256)
    pow_step_kernel(const double* __restrict__ R1, const double* __restrict__ X1,
                    int64_t nb, const double* __restrict__ xin,
                    double* __restrict__ yout, const int* __restrict__ skip) {
  __shared__ double red[256];
  __shared__ double xs[kP];
  if (*skip) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t n = nb * kP;
  const int mat = blockIdx.y;
  const double* T = mat ? X1 : R1;
  const double* x = xin + mat * n;
  double* y = yout + mat * n;
  const double inv = inv_norm(x, n, red);
  const int64_t B = blockIdx.x;
  if (!TRANS) {
    // y_B[a] = sum_{J >= B} sum_b T_BJ[a][b] x_J[b]; lane b, rows w + 4 u
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0;
    for (int64_t J = B; J < nb; ++J) {
      const double* tile = T + tix(B, J, nb);
      const double xb = x[J * kP + lane];
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[u] += tile[(w + 4 * u) * kP + lane] * xb;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      double a = acc[u];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
      if (lane == 0) y[B * kP + w + 4 * u] = a * inv;
    }
  } else {
    // y_B[b] = sum_{I <= B} sum_a T_IB[a][b] x_I[a]; lane b, rows w + 4 u
    double acc = 0.0;
    for (int64_t I = 0; I <= B; ++I) {
      const double* tile = T + tix(I, B, nb);
      __syncthreads();
      if (t < kP) xs[t] = x[I * kP + t];
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 16; ++u)
        acc += tile[(w + 4 * u) * kP + lane] * xs[w + 4 * u];
    }
    red[t] = acc;
    __syncthreads();
    if (t < kP) y[B * kP + t] = (red[t] + red[t + 64] + red[t + 128] + red[t + 192]) * inv;
  }
}

// y = T (x / |x|) (TRANS: T^T (x / |x|)) for T = R1 (y 0) or X1 (y 1), in
// two launches so that every tile product has a workgroup of its own (nb >
// kPowOne: a row of up to nb tiles on one workgroup would take most of the
// step): the
// products of row block B (TRANS: column block B) are cut into chunks of
// kPowC tiles, one workgroup each (blockIdx.x over all chunks, blockIdx.y the
// matrix), writing 64 partial sums of T x; pow_fin_kernel then adds a
// block's chunks in order and scales by 1 / |x|.
constexpr int64_t kPowC = 4;
constexpr int64_t kPowOne = 16;

__host__ __device__ inline int64_t pow_chunks(int64_t len) {
  return (len + kPowC - 1) / kPowC;
}
// chunks of all blocks (the same for both orientations)
__host__ __device__ inline int64_t pow_chunks_total(int64_t nb) {
  int64_t n = 0;
  for (int64_t B = 0; B < nb; ++B) n += pow_chunks(nb - B);
  return n;
}

template <bool TRANS>
__global__ void __launch_bounds__(256)
    pow_part_kernel(const double* __restrict__ R1, const double* __restrict__ X1,
                    int64_t nb, const double* __restrict__ xin,
                    double* __restrict__ part, const int* __restrict__ skip) {
  __shared__ double red[4][kP];
  if (*skip) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t n = nb * kP;
  const int mat = blockIdx.y;
  const double* T = mat ? X1 : R1;
  const double* x = xin + mat * n;
  // chunk blockIdx.x -> block B, chunk c of its products
  int64_t B = 0, c = blockIdx.x;
  for (;;) {
    const int64_t len = TRANS ? B + 1 : nb - B;
    if (c < pow_chunks(len)) break;
    c -= pow_chunks(len);
    ++B;
  }
  const int64_t maxc = pow_chunks(nb);
  double* out = part + ((mat * nb + B) * maxc + c) * kP;
  if (!TRANS) {
    // y_B[a] += sum_b T_BJ[a][b] x_J[b] over J = B + kPowC c ..; lane b,
    // rows w + 4 u
    const int64_t J0 = B + kPowC * c;
    const int64_t J1 = J0 + kPowC < nb ? J0 + kPowC : nb;
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0;
    for (int64_t J = J0; J < J1; ++J) {
      const double* tile = T + tix(B, J, nb);
      const double xb = x[J * kP + lane];
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[u] += tile[(w + 4 * u) * kP + lane] * xb;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      double a = acc[u];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
      if (lane == 0) out[w + 4 * u] = a;
    }
  } else {
    // y_B[b] += sum_a T_IB[a][b] x_I[a] over I = kPowC c ..; lane b, rows
    // w + 4 u
    const int64_t I0 = kPowC * c;
    const int64_t I1 = I0 + kPowC < B + 1 ? I0 + kPowC : B + 1;
    double acc = 0.0;
    for (int64_t I = I0; I < I1; ++I) {
      const double* tile = T + tix(I, B, nb);
#pragma unroll
      for (int u = 0; u < 16; ++u)
        acc += tile[(w + 4 * u) * kP + lane] * x[I * kP + w + 4 * u];
    }
    red[w][lane] = acc;
    __syncthreads();
    if (t < kP) out[t] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
  }
}

// y_B = (sum of block B's chunks, in order) / |x|; one workgroup per block
// and matrix
template <bool TRANS>
__global__ void __launch_bounds__(256)
    pow_fin_kernel(int64_t nb, const double* __restrict__ xin,
                   const double* __restrict__ part, double* __restrict__ yout,
                   const int* __restrict__ skip) {
  __shared__ double red[256];
  if (*skip) return;
  const int t = threadIdx.x;
  const int64_t n = nb * kP;
  const int mat = blockIdx.y;
  const int64_t B = blockIdx.x;
  const double inv = inv_norm(xin + mat * n, n, red);
  const int64_t len = TRANS ? B + 1 : nb - B;
  const int64_t maxc = pow_chunks(nb);
  if (t < kP) {
    const double* pp = part + (mat * nb + B) * maxc * kP + t;
    double y = 0.0;
    for (int64_t c = 0; c < pow_chunks(len); ++c) y += pp[c * kP];
    yout[mat * n + B * kP + t] = y * inv;
  }
}

// one workgroup: kappa_est = |R1 x^| |X1 y^| from the last forward products
// (v holds R1 x^ and X1 y^ for unit x^, y^); when the one-pass bound holds,
// min and max |R1_jj| into dstat and status 3
__global__ void __launch_bounds__(256)
    cq1_decide_kernel(const double* __restrict__ R1, int64_t nb, int64_t m,
                      int64_t d, const double* __restrict__ v, double bound,
                      const int* __restrict__ skip, double* __restrict__ dstat,
                      double* __restrict__ kest, int* __restrict__ status) {
  __shared__ double red[256];
  __shared__ double rmin[256], rmax[256];
  if (*status || *skip) return;
  const int t = threadIdx.x;
  const int64_t n = nb * kP;
  const double sr = 1.0 / inv_norm(v, n, red);
  const double sx = 1.0 / inv_norm(v + n, n, red);
  const double kap = sr * sx;
  if (kest && t == 0) *kest = kap;
  const double u = 0x1p-53;
  const bool ok = 4.0 * kap * kap * sqrt(static_cast<double>(m) * d) * u <= bound;
  if (!ok) return;  // (false for NaN too)
  double lo = 1.0 / 0.0, hi = 0.0;
  for (int64_t j = t; j < d; j += 256) {
    const int64_t I = j / kP, o = (j % kP) * kP + j % kP;
    const double r = fabs(R1[tix(I, I, nb) + o]);
    lo = r < lo ? r : lo;
    hi = r > hi ? r : hi;
  }
  rmin[t] = lo;
  rmax[t] = hi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      rmin[t] = rmin[t + o] < rmin[t] ? rmin[t + o] : rmin[t];
      rmax[t] = rmax[t + o] > rmax[t] ? rmax[t + o] : rmax[t];
    }
    __syncthreads();
  }
  if (t == 0) {
    if (dstat) {
      dstat[0] = rmin[0];
      dstat[1] = rmax[0];
    }
    *status = 3;
  }
}

// R1 (tiled) into r_out (d x d row-major, zeros below the diagonal); with
// status, only when *status = 3
__global__ void __launch_bounds__(256)
    r_copy_kernel(const double* __restrict__ R1, int64_t nb, int64_t d,
                  const int* __restrict__ status, double* __restrict__ r_out) {
  if (status && *status != 3) return;
  const int64_t i = blockIdx.x / nb, j = blockIdx.x % nb;
  const double* tile = R1 + tix(i, j, nb);
  for (int e = threadIdx.x; e < kP * kP; e += 256) {
    const int64_t gi = i * kP + e / kP, gj = j * kP + e % kP;
    if (gi < d && gj < d) r_out[gi * d + gj] = gi <= gj && i <= j ? tile[e] : 0.0;
  }
}

// ---- a job without host decisions (the no-sync leverage path) --------------
// out = 0 when *status == value, else 1 (the exit flag of a conditional pass)
__global__ void status_select_kernel(const int* __restrict__ status, int value,
                                     int* __restrict__ out) {
  if (threadIdx.x == 0) *out = *status == value ? 0 : 1;
}

// After the first pass (status 0, 2, 3 or 1) and the conditional second
// Cholesky (p2 = 0 when it ran and succeeded): which factored form of R^{-1}
// applies, and whether the rank screen calls R full rank (min |R_jj| >
// sqrt(tol) max |R_jj|, dstat of the path taken). f[0]: exit flag of the
// (I - F) correction, f[1]: of R2^{-1}, f[2]: of R1^{-1} (0: apply);
// f[3] = 1 when the job needs the synchronous path (a Householder fallback,
// a failed second pass, a truncation, or non-finite input: nonfinite).
__global__ void nosync_decide_kernel(const int* __restrict__ status,
                                     const int* __restrict__ p2,
                                     const double* __restrict__ dstat,
                                     double tol,
                                     const int* __restrict__ nonfinite,
                                     int* __restrict__ f) {
  if (threadIdx.x != 0) return;
  const int st = *status;
  const bool second = st == 2 && *p2 == 0;
  const bool ok = st == 0 || st == 3 || second;
  const double lo = dstat[0], hi = dstat[1];
  const bool full = tol < 0.0 || (hi > 0.0 && lo > sqrt(tol) * hi);
  const bool run = ok && full && *nonfinite == 0;
  f[0] = run && st == 0 ? 0 : 1;
  f[1] = run && second ? 0 : 1;
  f[2] = run ? 0 : 1;
  f[3] = run ? 0 : 1;
}

struct Cq2 {
  int64_t d, nb, nt, S, chunk, Se, chunk_e, nfull, nedge;
  int64_t C, Q, nwg;  // stream-K full blocks (Q > 0): units per block and
                      // per workgroup, workgroups; S: slots per block
  bool fe;  // edge products formed by the diagonal blocks (no edge launch)
  double *part, *G, *R1, *R2, *X1, *X2, *P, *Dinv, *gdiag, *apart, *pv, *kest,
      *pp, *qo;  // qo: Q1 out of place (nullptr above kQ1Max entries)
  unsigned long long* emax;
};

Cq2 cq2_shape(int64_t m, int64_t d) {
  Cq2 c{};
  c.d = d;
  c.nb = (d + kP - 1) / kP;
  c.nt = c.nb * (c.nb + 1) / 2;
  // Gram row chunks: blocks of full 128-column blocks take at most 512
  // workgroups in all (two per CU: one round), the edge blocks (thin: their
  // time is load latency, so they get many short chunks) at most 512;
  // chunks of at least kGMin rows (a workgroup's chain of 16-row steps is
  // latency bound: a short matrix is split into short chains)
  const int64_t nf = d / 128;
  c.nfull = nf * (nf + 1) / 2;
  c.nedge = d % 128 ? nf + 1 : 0;
  const int64_t steps = (m + kGK - 1) / kGK;
  const int64_t smax = (m + kGMin - 1) / kGMin > 1 ? (m + kGMin - 1) / kGMin : 1;
  auto pick = [&](int64_t slots, int64_t blocks, int64_t& S, int64_t& chunk) {
    S = blocks > 0 ? slots / blocks : 1;
    if (S > smax) S = smax;
    if (S < 1) S = 1;
    chunk = (steps + S - 1) / S * kGK;
  };
  pick(512, c.nfull, c.S, c.chunk);
  pick(512, c.nedge, c.Se, c.chunk_e);
  c.fe = nf > 0 && d % 128 != 0 && d % 128 <= 16;
  if (c.fe) {
    c.Se = c.S;
    c.chunk_e = c.chunk;
  } else if (c.nfull > 0 &&
             8 * c.nfull * c.S < 7 * 512 * ((c.nfull * c.S + 511) / 512)) {
    // the rounds of the 512 slots less than seven eighths busy (528 blocks
    // at d = 4096: two rounds, the second nearly empty): the stream-K form,
    // with at least kGMin rows per unit and 32 units per block where the
    // rows allow, one round of at most 512 equal workgroups
    c.C = 32;
    const int64_t rows = (m + c.C - 1) / c.C;
    if (rows < kGMin) c.C = smax;
    c.chunk = ((m + c.C - 1) / c.C + kGK - 1) / kGK * kGK;
    c.C = (m + c.chunk - 1) / c.chunk;
    const int64_t U = c.nfull * c.C;
    c.Q = (U + 511) / 512;
    c.nwg = (U + c.Q - 1) / c.Q;
    c.S = (c.C - 1) / c.Q + 2;
  }
  return c;
}

Cq2 cq2_carve(void* base, int64_t m, int64_t d) {
  Cq2 c = cq2_shape(m, d);
  double* p = static_cast<double*>(base);
  c.part = p;  p += (c.nfull * c.S + c.nedge * c.Se) * kB2;
  c.G = p;     p += c.nb * c.nb * kT2;
  c.R1 = p;    p += c.nb * c.nb * kT2;
  c.R2 = p;    p += c.nb * c.nb * kT2;
  c.X1 = p;    p += c.nb * c.nb * kT2;
  c.X2 = p;    p += c.nb * c.nb * kT2;
  c.P = p;     p += c.nb * c.nb * kT2;
  c.apart = p; p += tri_parts(c.nb) * c.nb * kT2;
  c.Dinv = p;  p += c.nb * kT2;
  c.gdiag = p; p += c.nb * kP;
  c.emax = reinterpret_cast<unsigned long long*>(p);  // nt * 16 entries
  p += c.nt * 16;
  c.pv = p;    p += 4 * c.nb * kP;  // power-iteration vectors, two per matrix
  c.kest = p;  p += 8;
  c.pp = p;    p += 2 * c.nb * pow_chunks(c.nb) * kP;  // their partial products
  c.qo = m * d <= kQ1Max ? p : nullptr;
  return c;
}

void gram_tiles(const double* a, int64_t m, int64_t d, const Cq2& c,
                bool with_emax, const double* dsc, int* flag, hipStream_t s) {
  unsigned long long* em = with_emax ? c.emax : nullptr;
  // (the thin blocks gain nothing on a second stream: the main blocks hold
  // every slot until their last round ends)
  prof_begin(kKCq2Gram, s);
  if (c.Q > 0)
    gram_sk_kernel<<<static_cast<unsigned>(c.nwg), 256, 0, s>>>(
        a, d, m, d, c.C, c.chunk, c.Q, c.S, c.part, flag);
  else if (c.fe)
    gram_block_kernel<false, true><<<static_cast<unsigned>(c.nfull * c.S), 256, 0, s>>>(
        a, d, m, d, c.S, c.chunk, 0, c.part, flag);
  else if (c.nfull > 0)
    gram_block_kernel<false, false><<<static_cast<unsigned>(c.nfull * c.S), 256, 0, s>>>(
        a, d, m, d, c.S, c.chunk, 0, c.part, flag);
  prof_end(kKCq2Gram, s);
  prof_begin(kKCq2GramEdge, s);
  if (c.nedge > 0 && !c.fe)
    gram_block_kernel<true, false><<<static_cast<unsigned>(c.nedge * c.Se), 256, 0, s>>>(
        a, d, m, d, c.Se, c.chunk_e, c.nfull * c.S, c.part, flag);
  prof_end(kKCq2GramEdge, s);
  prof_begin(kKCq2GramSum, s);
  gram_reduce_kernel<<<static_cast<unsigned>(c.nt * 16), 256, 0, s>>>(
      c.part, c.S, c.Se, c.C, c.Q, c.nb, d, dsc, c.G, c.gdiag, em, flag);
  prof_end(kKCq2GramSum, s);
}

// Blocked Cholesky of c.G into the tiles R (and, with X, R^{-1} into X)
void bchol(const Cq2& c, double* R, double* X, int* flag, hipStream_t s) {
  prof_begin(kKCq2Chol, s);
  bchol_first_kernel<<<1, 256, 0, s>>>(c.G, c.gdiag, kPivotTol, R, c.Dinv, X,
                                       flag);
  for (int64_t k = 0; k + 1 < c.nb; ++k) {
    const int64_t n = c.nb - k - 1;
    const int64_t grid = n * (n + 1) / 2 + (X ? k + k * n : 0);
    bchol_step_kernel<<<static_cast<unsigned>(grid), 256, 0, s>>>(
        c.G, c.nb, k, c.d, c.gdiag, kPivotTol, R, c.Dinv, X, c.P, flag);
  }
  if (X && c.nb > 1)
    binv_col_kernel<<<static_cast<unsigned>(c.nb - 1), 256, 0, s>>>(
        c.nb, c.nb - 1, R, c.Dinv, X, c.P, flag);
  prof_end(kKCq2Chol, s);
}

// G's upper triangle (row-major d x d) into tiles (I, J), I <= J, one
// workgroup each (blockIdx.x in the order of upper_tile), padded with the
// identity past d; gdiag receives the diagonal
__global__ void __launch_bounds__(256)
    tile_pack_kernel(const double* __restrict__ g, int64_t d, int64_t nb,
                     double* __restrict__ G, double* __restrict__ gdiag) {
  int64_t I, J;
  upper_tile(blockIdx.x, nb, I, J);
  for (int e = threadIdx.x; e < kT2; e += 256) {
    const int64_t gi = I * kP + e / kP, gj = J * kP + e % kP;
    double v = gi == gj ? 1.0 : 0.0;
    if (gi < d && gj < d) v = gi <= gj ? g[gi * d + gj] : g[gj * d + gi];
    G[tix(I, J, nb) + e] = v;
    if (gi == gj) gdiag[gi] = v;
  }
}

}  // namespace

size_t chol_tiled_scratch_bytes(int64_t d) {
  const int64_t nb = (d + kP - 1) / kP;
  return static_cast<size_t>(2 * nb * nb * kT2 + nb * kT2 + nb * kP) *
         sizeof(double);
}

void chol_tiled(const double* g, int64_t d, double* r, void* scratch,
                int* flag, hipStream_t s) {
  Cq2 c{};
  c.d = d;
  c.nb = (d + kP - 1) / kP;
  double* p = static_cast<double*>(scratch);
  c.G = p;     p += c.nb * c.nb * kT2;
  c.R1 = p;    p += c.nb * c.nb * kT2;
  c.Dinv = p;  p += c.nb * kT2;
  c.gdiag = p;
  const unsigned nb = static_cast<unsigned>(c.nb);
  tile_pack_kernel<<<nb * (nb + 1) / 2, 256, 0, s>>>(g, d, c.nb, c.G, c.gdiag);
  bchol(c, c.R1, nullptr, flag, s);
  r_copy_kernel<<<nb * nb, 256, 0, s>>>(c.R1, c.nb, d, nullptr, r);
}

size_t cholqr2_scratch_bytes(int64_t m, int64_t d) {
  const Cq2 c = cq2_shape(m, d);
  return static_cast<size_t>((c.nfull * c.S + c.nedge * c.Se) * kB2 +
                             6 * c.nb * c.nb * kT2 +
                             tri_parts(c.nb) * c.nb * kT2 +
                             c.nb * kT2 + c.nb * kP + c.nt * 16 +
                             4 * c.nb * kP + 8 +
                             2 * c.nb * pow_chunks(c.nb) * kP +
                             (m * d <= kQ1Max ? m * d : 0)) *
         sizeof(double);
}

namespace {
// out = T B (see tri_part_kernel); out may be B
template <int MODE>
void tri_apply(const Cq2& c, const double* T, int64_t d, const double* B,
               int64_t kk, double* out, const int* flag, hipStream_t s) {
  const int64_t ncb_all = (kk + kP - 1) / kP;
  const unsigned np = static_cast<unsigned>(tri_parts(c.nb));
  for (int64_t cb0 = 0; cb0 < ncb_all; cb0 += c.nb) {
    const int64_t ncb = ncb_all - cb0 < c.nb ? ncb_all - cb0 : c.nb;
    tri_part_kernel<MODE><<<dim3(np, static_cast<unsigned>(ncb)), 256, 0, s>>>(
        T, c.nb, d, B, kk, cb0, ncb, c.apart, flag);
    tri_sum_kernel<<<dim3(static_cast<unsigned>(c.nb),
                          static_cast<unsigned>(ncb), 16),
                     256, 0, s>>>(c.apart, c.nb, d, kk, cb0, ncb, out, flag);
  }
}
}  // namespace

void cholqr2_factor(double* a, int64_t m, int64_t d, double* r_out,
                    void* scratch, int* status, const QrStreams& qs,
                    hipStream_t s, bool want_r, double* dstat,
                    const double* dsc, int one_pass) {
  (void)qs;
  if (2.0 * static_cast<double>(m) * static_cast<double>(d) * d < 0x1p31)
    one_pass = 0;
  const Cq2 c = cq2_carve(scratch, m, d);
  launch_fill_i32(status, 1, 0, s);
  gram_tiles(a, m, d, c, false, dsc, status, s);
  bchol(c, c.R1, want_r && one_pass == 0 ? nullptr : c.X1, status, s);
  // the one-pass forms (status 3 stops every later launch of this pass)
  if (one_pass != 0) {
    prof_begin(kKCq2R, s);
    const unsigned nb = static_cast<unsigned>(c.nb);
    const double bound = one_pass == 1 ? 1e-2 : 1e-7;
    double* va = c.pv;
    double* vb = c.pv + 2 * c.nb * kP;
    int* skip = reinterpret_cast<int*>(c.kest + 1);
    x_rownorm_kernel<<<nb, 256, 0, s>>>(c.X1, c.nb, status, va);
    cq1_precheck_kernel<<<1, 256, 0, s>>>(c.R1, c.gdiag, va, c.nb, m, d, bound,
                                          status, skip);
    pow_init_kernel<<<8, 256, 0, s>>>(c.nb, d, va, skip);
    const unsigned nch = static_cast<unsigned>(pow_chunks_total(c.nb));
    auto step = [&](bool trans, const double* xi, double* yo) {
      if (c.nb <= kPowOne) {
        if (trans)
          pow_step_kernel<true><<<dim3(nb, 2), 256, 0, s>>>(c.R1, c.X1, c.nb,
                                                            xi, yo, skip);
        else
          pow_step_kernel<false><<<dim3(nb, 2), 256, 0, s>>>(c.R1, c.X1, c.nb,
                                                             xi, yo, skip);
      } else if (trans) {
        pow_part_kernel<true><<<dim3(nch, 2), 256, 0, s>>>(c.R1, c.X1, c.nb,
                                                           xi, c.pp, skip);
        pow_fin_kernel<true><<<dim3(nb, 2), 256, 0, s>>>(c.nb, xi, c.pp, yo,
                                                         skip);
      } else {
        pow_part_kernel<false><<<dim3(nch, 2), 256, 0, s>>>(c.R1, c.X1, c.nb,
                                                            xi, c.pp, skip);
        pow_fin_kernel<false><<<dim3(nb, 2), 256, 0, s>>>(c.nb, xi, c.pp, yo,
                                                          skip);
      }
    };
    for (int it = 0; it < kPowIters; ++it) {
      step(false, va, vb);
      step(true, vb, va);
    }
    step(false, va, vb);
    cq1_decide_kernel<<<1, 256, 0, s>>>(c.R1, c.nb, m, d, vb, bound, skip,
                                        want_r ? nullptr : dstat, c.kest,
                                        status);
    if (want_r)
      r_copy_kernel<<<static_cast<unsigned>(c.nb * c.nb), 256, 0, s>>>(
          c.R1, c.nb, d, status, r_out);
    prof_end(kKCq2R, s);
  }
  // Q1: with R^{-1} kept factored (X1 built, no R wanted), the product with
  // X1 out of place when the buffer exists; otherwise the stripe solve
  const bool gemm = !want_r && c.qo != nullptr;
  prof_begin(kKCq2Solve, s);
  if (gemm)
    q1_gemm_kernel<<<dim3(cdivu(m, kP), static_cast<unsigned>(c.nb)), 256, 0,
                     s>>>(a, m, d, c.nb, c.X1, dsc, c.qo, status);
  else
    stripe_solve_kernel<kStripeRows><<<cdivu(m, kStripeRows), 8 * kStripeRows,
                                       0, s>>>(a, d, m, d, c.nb, c.R1, c.Dinv,
                                               dsc, status);
  prof_end(kKCq2Solve, s);
  gram_tiles(gemm ? c.qo : a, m, d, c, true, nullptr, status, s);
  prof_begin(kKCq2R, s);
  if (want_r)
    r_final_kernel<true><<<static_cast<unsigned>(c.nb * c.nb), 256, 0, s>>>(
        c.R1, c.G, c.nb, d, c.emax, status, r_out);
  else
    r_diag_kernel<true><<<1, 256, 0, s>>>(c.R1, nullptr, c.gdiag, c.nb, d,
                                          c.emax, status, dstat);
  prof_end(kKCq2R, s);
}

void cholqr2_finish(int64_t m, int64_t d, double* r_out, void* scratch,
                    int* status, hipStream_t s, bool want_r, double* dstat) {
  const Cq2 c = cq2_carve(scratch, m, d);
  launch_fill_i32(status, 1, 0, s);
  bchol(c, c.R2, want_r ? nullptr : c.X2, status, s);
  prof_begin(kKCq2R, s);
  if (want_r)
    r_final_kernel<false><<<static_cast<unsigned>(c.nb * c.nb), 256, 0, s>>>(
        c.R1, c.R2, c.nb, d, c.emax, status, r_out);
  else
    r_diag_kernel<false><<<1, 256, 0, s>>>(c.R1, c.R2, c.gdiag, c.nb, d,
                                           c.emax, status, dstat);
  prof_end(kKCq2R, s);
}

void cholqr2_write_r(int64_t m, int64_t d, double* r_out, void* scratch,
                     int form, hipStream_t s) {
  const Cq2 c = cq2_carve(scratch, m, d);
  prof_begin(kKCq2R, s);
  if (form == 2)
    r_copy_kernel<<<static_cast<unsigned>(c.nb * c.nb), 256, 0, s>>>(
        c.R1, c.nb, d, nullptr, r_out);
  else if (form == 1)
    r_final_kernel<false><<<static_cast<unsigned>(c.nb * c.nb), 256, 0, s>>>(
        c.R1, c.R2, c.nb, d, c.emax, nullptr, r_out);
  else
    r_final_kernel<true><<<static_cast<unsigned>(c.nb * c.nb), 256, 0, s>>>(
        c.R1, c.G, c.nb, d, c.emax, nullptr, r_out);
  prof_end(kKCq2R, s);
}

void cholqr2_apply_rinv(int64_t m, int64_t d, void* scratch, int form,
                        double* b, int64_t kk, hipStream_t s) {
  const Cq2 c = cq2_carve(scratch, m, d);
  prof_begin(kKTrsm, s);
  // R^{-1} = R1^{-1} (I + F)^{-1} = X1 (I - F) to rounding (form 0), or
  // X1 R2^{-1} (form 1), or X1 (form 2: one pass)
  if (form == 1)
    tri_apply<0>(c, c.X2, d, b, kk, b, nullptr, s);
  else if (form == 0)
    tri_apply<1>(c, c.G, d, b, kk, b, nullptr, s);
  tri_apply<0>(c, c.X1, d, b, kk, b, nullptr, s);
  prof_end(kKTrsm, s);
}

void cholqr2_finish_dev(int64_t m, int64_t d, void* scratch, const int* status,
                        int* p2, double* dstat, hipStream_t s) {
  const Cq2 c = cq2_carve(scratch, m, d);
  status_select_kernel<<<1, 64, 0, s>>>(status, 2, p2);
  bchol(c, c.R2, c.X2, p2, s);
  prof_begin(kKCq2R, s);
  r_diag_kernel<false><<<1, 256, 0, s>>>(c.R1, c.R2, c.gdiag, c.nb, d, c.emax,
                                         p2, dstat);
  prof_end(kKCq2R, s);
}

void cholqr2_decide_dev(const int* status, const int* p2, const double* dstat,
                        double tol, const int* nonfinite, int* f,
                        hipStream_t s) {
  nosync_decide_kernel<<<1, 64, 0, s>>>(status, p2, dstat, tol, nonfinite, f);
}

void cholqr2_apply_rinv_dev(int64_t m, int64_t d, void* scratch, const int* f,
                            double* b, int64_t kk, hipStream_t s) {
  const Cq2 c = cq2_carve(scratch, m, d);
  prof_begin(kKTrsm, s);
  tri_apply<1>(c, c.G, d, b, kk, b, f + 0, s);
  tri_apply<0>(c, c.X2, d, b, kk, b, f + 1, s);
  tri_apply<0>(c, c.X1, d, b, kk, b, f + 2, s);
  prof_end(kKTrsm, s);
}

}  // namespace slso
