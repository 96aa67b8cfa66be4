// FP64 pieces of the sketch-preconditioned Cholesky-QR refinement of R:
// with R_S the R factor of the (reduced-precision) sketch and G = (X D)^T (X D),
//   G' = R_S^{-T} G R_S^{-1},  G' = R1^T R1 (Cholesky),  R = R1 R_S,
// which is the R factor of X D (the R of a Householder QR of X D up to row
// signs, here with a positive diagonal) computed in one pass over X.
//
// solve_upper_trans: blocked forward substitution R^T X = B (64-row blocks,
// one wave per right-hand side for the diagonal block, lane = row).
// cholesky: right-looking, 16-column panels: the diagonal block by one wave
// with columns in registers and pivots/rows broadcast by readlane, the panel
// row by a forward substitution per column, the trailing matrix by a rank-16
// update of its upper triangle.
#include "internal.h"

namespace slso {
namespace {

constexpr int kB = 64;
constexpr int kP = 16;

__device__ __forceinline__ double readlane_d(double x, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                          __builtin_amdgcn_readlane(__double2loint(x), l));
}

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

// Cholesky of the bs x bs diagonal block at j0 (upper triangle of g), one
// wave, lane l < 16 owning column l; result rows into r.
__global__ void __launch_bounds__(64)
    chol_diag_kernel(const double* __restrict__ g, int64_t d, int64_t j0,
                     int bs, double* __restrict__ r, int* __restrict__ flag) {
  const int l = threadIdx.x;
  double gc[kP];
#pragma unroll
  for (int i = 0; i < kP; ++i) {
    double v = (l == i) ? 1.0 : 0.0;  // identity padding beyond bs
    if (l < bs && i < bs) v = i <= l ? g[(j0 + i) * d + j0 + l] : g[(j0 + l) * d + j0 + i];
    gc[i] = v;
  }
  bool ok = true;
#pragma unroll
  for (int j = 0; j < kP; ++j) {
    const double piv = readlane_d(gc[j], j);
    ok = ok && piv > 0.0;
    const double rjj = sqrt(piv > 0.0 ? piv : 1.0);
    const double rjl = l > j ? gc[j] / rjj : (l == j ? rjj : 0.0);
    if (l < bs && j < bs) r[(j0 + j) * d + j0 + l] = rjl;
#pragma unroll
    for (int i = j + 1; i < kP; ++i) gc[i] -= readlane_d(rjl, i) * rjl;
  }
  if (!ok && l == 0) atomicExch(flag, 1);
}

// R[j0 + i][c] for c >= j0 + bs: forward substitution with R_jj^T per column
__global__ void __launch_bounds__(256)
    chol_panel_kernel(const double* __restrict__ g, int64_t d, int64_t j0,
                      int bs, double* __restrict__ r) {
  __shared__ double Rd[kP][kP];
  const int t = threadIdx.x;
  {
    const int i = t / kP, j = t % kP;
    Rd[i][j] = (i < bs && j < bs && j >= i) ? r[(j0 + i) * d + j0 + j] : 0.0;
  }
  __syncthreads();
  const int64_t c = j0 + bs + static_cast<int64_t>(blockIdx.x) * 256 + t;
  if (c >= d) return;
  double y[kP];
#pragma unroll
  for (int i = 0; i < kP; ++i) {
    if (i < bs) {
      double s = g[(j0 + i) * d + c];
#pragma unroll
      for (int l = 0; l < i; ++l) s -= Rd[l][i] * y[l];
      y[i] = s / Rd[i][i];
      r[(j0 + i) * d + c] = y[i];
    } else {
      y[i] = 0.0;
    }
  }
}

// g[i][c] -= sum_l R[j0 + l][i] R[j0 + l][c] for j1 <= i <= c
__global__ void __launch_bounds__(256)
    chol_update_kernel(double* __restrict__ g, int64_t d, int64_t j0, int bs,
                       const double* __restrict__ r) {
  const int64_t j1 = j0 + bs;
  const int64_t i = j1 + static_cast<int64_t>(blockIdx.y) * 16 + (threadIdx.x >> 4);
  const int64_t c = j1 + static_cast<int64_t>(blockIdx.x) * 16 + (threadIdx.x & 15);
  if (i >= d || c >= d || c < i) return;
  double s = 0.0;
  for (int l = 0; l < bs; ++l) s += r[(j0 + l) * d + i] * r[(j0 + l) * d + c];
  g[i * d + c] -= s;
}

__global__ void zero_lower_kernel(double* __restrict__ r, int64_t d) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= d * d) return;
  if (e / d > e % d) r[e] = 0.0;
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

void cholesky(double* g, int64_t d, double* r, int* flag, hipStream_t s) {
  zero_lower_kernel<<<grid1(d * d, 256), 256, 0, s>>>(r, d);
  for (int64_t j0 = 0; j0 < d; j0 += kP) {
    const int bs = static_cast<int>(d - j0 < kP ? d - j0 : kP);
    prof_begin(kKChol, s);
    chol_diag_kernel<<<1, 64, 0, s>>>(g, d, j0, bs, r, flag);
    const int64_t rest = d - j0 - bs;
    if (rest > 0) {
      chol_panel_kernel<<<grid1(rest, 256), 256, 0, s>>>(g, d, j0, bs, r);
      dim3 grid(static_cast<unsigned>((rest + 15) / 16),
                static_cast<unsigned>((rest + 15) / 16));
      chol_update_kernel<<<grid, 256, 0, s>>>(g, d, j0, bs, r);
    }
    prof_end(kKChol, s);
  }
}

void launch_trmm_upper(const double* a, const double* b, int64_t d, double* c,
                       hipStream_t s) {
  trmm_upper_kernel<<<grid1(d * d, 256), 256, 0, s>>>(a, b, d, c);
}

}  // namespace slso
