// FP64 pieces of the sketch-preconditioned Cholesky-QR refinement of R:
// with R_S the R factor of the (reduced-precision) sketch and G = (X D)^T (X D),
//   G' = R_S^{-T} G R_S^{-1},  G' = R1^T R1 (Cholesky),  R = R1 R_S,
// which is the R factor of X D (the R of a Householder QR of X D up to row
// signs, here with a positive diagonal) computed in one pass over X.
//
// solve_upper_trans: blocked forward substitution R^T X = B (64-row blocks,
// one wave per right-hand side for the diagonal block, lane = row). The
// Cholesky of G' is the tiled blocked Cholesky of the sketch's QR
// (chol_tiled, k_cholqr.hip).
#include "internal.h"

namespace slso {
namespace {

constexpr int kB = 64;

__global__ void __launch_bounds__(256)
    trsm_t_diag_kernel(const double* __restrict__ R, int64_t d, int64_t r0,
                       int bs, double* __restrict__ B, int64_t k) {
  __shared__ double Rs[kB][kB + 1];
  const int t = threadIdx.x;
  const int lane = t & 63;
  for (int e = t; e < kB * kB; e += 256) {
    const int i = e / kB, j = e % kB;
    double v = 0.0;
    if (i < bs && j < bs && j >= i) v = R[(r0 + i) * d + r0 + j];
    Rs[i][j] = v;
  }
  __syncthreads();
  const int64_t c = static_cast<int64_t>(blockIdx.x) * 4 + (t >> 6);
  if (c >= k) return;
  double b = lane < bs ? B[(r0 + lane) * k + c] : 0.0;
  double x = 0.0;
  for (int l = 0; l < bs; ++l) {
    const double bl = __shfl(b, l, 64);
    const double xl = bl / Rs[l][l];
    if (lane == l) x = xl;
    b -= Rs[l][lane] * xl;  // (R^T)[lane][l] = R[l][lane], zero for lane < l
  }
  if (lane < bs) B[(r0 + lane) * k + c] = x;
}

// B[i][c] -= sum_l R[r0 + l][i] X[l][c] for rows i >= r0 + bs
__global__ void __launch_bounds__(256)
    trsm_t_update_kernel(const double* __restrict__ R, int64_t d, int64_t r0,
                         int bs, double* __restrict__ B, int64_t k) {
  __shared__ double Xs[kB][64];
  const int t = threadIdx.x;
  const int lc = t & 63;
  const int64_t c = static_cast<int64_t>(blockIdx.y) * 64 + lc;
  for (int e = t; e < bs * 64; e += 256) {
    const int l = e / 64, cc = e % 64;
    const int64_t col = static_cast<int64_t>(blockIdx.y) * 64 + cc;
    Xs[l][cc] = col < k ? B[(r0 + l) * k + col] : 0.0;
  }
  __syncthreads();
  const int64_t i = r0 + bs + static_cast<int64_t>(blockIdx.x) * 4 + (t >> 6);
  if (i >= d || c >= k) return;
  double s = 0.0;
  for (int l = 0; l < bs; ++l) s += R[(r0 + l) * d + i] * Xs[l][lc];
  B[i * k + c] -= s;
}

__global__ void transpose_kernel(const double* __restrict__ a, int64_t d,
                                 double* __restrict__ out) {
  __shared__ double tile[32][33];
  const int64_t bx = static_cast<int64_t>(blockIdx.x) * 32;
  const int64_t by = static_cast<int64_t>(blockIdx.y) * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t i = by + yy, j = bx + tx;
    tile[yy][tx] = (i < d && j < d) ? a[i * d + j] : 0.0;
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t i = bx + yy, j = by + tx;
    if (i < d && j < d) out[i * d + j] = tile[tx][yy];
  }
}

__global__ void trmm_upper_kernel(const double* __restrict__ a,
                                  const double* __restrict__ b, int64_t d,
                                  double* __restrict__ c) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= d * d) return;
  const int64_t i = e / d, j = e % d;
  double s = 0.0;
  for (int64_t k = i; k <= j; ++k) s += a[i * d + k] * b[k * d + j];
  c[e] = j >= i ? s : 0.0;
}

inline unsigned grid1(int64_t n, int t) {
  return static_cast<unsigned>((n + t - 1) / t);
}

}  // namespace

void solve_upper_trans(const double* r, int64_t d, double* b, int64_t k,
                       hipStream_t s, double* scratch) {
  if (d <= 0 || k <= 0) return;
  if (scratch) {
    trsm_blocked(r, d, b, k, true, scratch, s);
    return;
  }
  const unsigned cgrid = static_cast<unsigned>((k + 63) / 64);
  const int64_t nb = (d + kB - 1) / kB;
  for (int64_t bi = 0; bi < nb; ++bi) {
    const int64_t r0 = bi * kB;
    const int bs = static_cast<int>(d - r0 < kB ? d - r0 : kB);
    prof_begin(kKTrsm, s);
    trsm_t_diag_kernel<<<static_cast<unsigned>((k + 3) / 4), 256, 0, s>>>(
        r, d, r0, bs, b, k);
    prof_end(kKTrsm, s);
    const int64_t rest = d - r0 - bs;
    if (rest > 0) {
      dim3 grid(static_cast<unsigned>((rest + 3) / 4), cgrid);
      prof_begin(kKTrsm, s);
      trsm_t_update_kernel<<<grid, 256, 0, s>>>(r, d, r0, bs, b, k);
      prof_end(kKTrsm, s);
    }
  }
}

void launch_transpose(const double* a, int64_t d, double* out, hipStream_t s) {
  dim3 grid(static_cast<unsigned>((d + 31) / 32), static_cast<unsigned>((d + 31) / 32));
  transpose_kernel<<<grid, 256, 0, s>>>(a, d, out);
}

void launch_trmm_upper(const double* a, const double* b, int64_t d, double* c,
                       hipStream_t s) {
  trmm_upper_kernel<<<grid1(d * d, 256), 256, 0, s>>>(a, b, d, c);
}

}  // namespace slso
