// R^{-1} Pi_2 (Algorithm 2 step 3 in QR form) and the truncated pseudo-inverse
// of Algorithm 3 step 3, both in FP64.
//
// solve_upper: blocked back substitution, 64-row blocks from the bottom: the
// diagonal block is solved by one workgroup (one thread per right-hand
// side, the block of R in LDS), then the rows above are updated with a
// rank-64 product, B[0:r0] -= R[0:r0, blk] X_blk.
//
// jacobi_truncated_apply: one-sided (Hestenes) Jacobi SVD of R: column pairs
// of A = R are rotated until mutually orthogonal, A V = U Sigma; the rank is
// #{sigma_j > tau sigma_1}; out = V' Sigma'^{-1} U'^T B over the kept
// columns. Each sweep is d-1 rounds of a round-robin tournament (every round
// pairs all columns disjointly, one wave per pair, one launch per round).
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "internal.h"

namespace slso {
namespace {

constexpr int kB = 64;

// One wave per right-hand side, lane i = row i of the diagonal block:
// x_l = b_l / R_ll is broadcast from lane l, then b_i -= R_il x_l for i < l.
__global__ void __launch_bounds__(256)
    trsm_diag_kernel(const double* __restrict__ R, int64_t d, int64_t r0,
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
  for (int l = bs - 1; l >= 0; --l) {
    const double bl = __shfl(b, l, 64);
    const double xl = bl / Rs[l][l];
    if (lane == l) x = xl;
    b -= Rs[lane][l] * xl;
  }
  if (lane < bs) B[(r0 + lane) * k + c] = x;
}

// B[0:r0, :] -= R[0:r0, r0:r0+bs] X, X = B[r0:r0+bs, :]; 4 rows x 64 columns
// per workgroup.
__global__ void __launch_bounds__(256)
    trsm_update_kernel(const double* __restrict__ R, int64_t d, int64_t r0,
                       int bs, double* __restrict__ B, int64_t k) {
  __shared__ double Xs[kB][64];
  const int t = threadIdx.x;
  const int lc = t & 63;
  const int64_t c = static_cast<int64_t>(blockIdx.y) * 64 + lc;
  const bool cok = c < k;
  for (int e = t; e < bs * 64; e += 256) {
    const int l = e / 64, cc = e % 64;
    const int64_t col = static_cast<int64_t>(blockIdx.y) * 64 + cc;
    Xs[l][cc] = col < k ? B[(r0 + l) * k + col] : 0.0;
  }
  __syncthreads();
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 4 + (t >> 6);
  if (i >= r0 || !cok) return;
  const double* Ri = R + i * d + r0;
  double s = 0.0;
  for (int l = 0; l < bs; ++l) s += Ri[l] * Xs[l][lc];
  B[i * k + c] -= s;
}

__global__ void eye_kernel(double* __restrict__ out, int64_t d) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= d * d) return;
  out[e] = (e / d) == (e % d) ? 1.0 : 0.0;
}

__global__ void scale_rows_kernel(const double* __restrict__ m,
                                  const double* __restrict__ sc, int64_t d,
                                  int64_t k, double* __restrict__ o64,
                                  float* __restrict__ o32) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= d * k) return;
  const int64_t j = e / k;
  const double v = (sc ? sc[j] : 1.0) * m[e];
  if (o64) o64[e] = v;
  if (o32) o32[e] = static_cast<float>(v);
}

// ---- one-sided Jacobi on column-major copies -------------------------------
// A: d x d column-major (column j contiguous), V: d x d column-major.
__global__ void __launch_bounds__(256)
    jacobi_round_kernel(double* __restrict__ A, double* __restrict__ V,
                        int64_t d, int64_t dpad, int64_t round, double tol,
                        int* __restrict__ rotated) {
  const int lane = threadIdx.x & 63;
  const int64_t pair = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int64_t npairs = dpad / 2;
  if (pair >= npairs) return;
  // round-robin tournament: position 0 fixed, others rotate
  const int64_t nm1 = dpad - 1;
  int64_t p, q;
  if (pair == 0) {
    p = 0;
    q = 1 + (round % nm1);
  } else {
    p = 1 + ((round + pair) % nm1);
    q = 1 + ((round + nm1 - pair) % nm1);
  }
  if (p > q) {
    const int64_t tmp = p;
    p = q;
    q = tmp;
  }
  if (q >= d) return;  // padding column
  double* ap = A + p * d;
  double* aq = A + q * d;
  double alpha = 0.0, beta = 0.0, gamma = 0.0;
  for (int64_t i = lane; i < d; i += 64) {
    const double x = ap[i], y = aq[i];
    alpha += x * x;
    beta += y * y;
    gamma += x * y;
  }
  alpha = wave_sum_d(alpha);
  beta = wave_sum_d(beta);
  gamma = wave_sum_d(gamma);
  if (gamma == 0.0 || fabs(gamma) <= tol * sqrt(alpha * beta)) return;
  const double zeta = (beta - alpha) / (2.0 * gamma);
  const double tt = (zeta >= 0.0 ? 1.0 : -1.0) /
                    (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double cs = 1.0 / sqrt(1.0 + tt * tt);
  const double sn = cs * tt;
  for (int64_t i = lane; i < d; i += 64) {
    const double x = ap[i], y = aq[i];
    ap[i] = cs * x - sn * y;
    aq[i] = sn * x + cs * y;
  }
  double* vp = V + p * d;
  double* vq = V + q * d;
  for (int64_t i = lane; i < d; i += 64) {
    const double x = vp[i], y = vq[i];
    vp[i] = cs * x - sn * y;
    vq[i] = sn * x + cs * y;
  }
  if (lane == 0) atomicExch(rotated, 1);
}

__global__ void transpose_init_kernel(const double* __restrict__ R, int64_t d,
                                      double* __restrict__ A,
                                      double* __restrict__ V) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= d * d) return;
  const int64_t i = e / d, j = e - i * d;  // R[i][j] -> A column j, row i
  A[j * d + i] = R[e];
  V[e] = i == j ? 1.0 : 0.0;
}

__global__ void col_norms_kernel(const double* __restrict__ A, int64_t d,
                                 double* __restrict__ sig) {
  const int lane = threadIdx.x & 63;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (j >= d) return;
  double s = 0.0;
  for (int64_t i = lane; i < d; i += 64) s += A[j * d + i] * A[j * d + i];
  s = wave_sum_d(s);
  if (lane == 0) sig[j] = sqrt(s);
}

// out[i][c] = sum over kept columns j of V[i][j] (u_j . b_c) / sigma_j,
// u_j = A[:, j] / sigma_j; one workgroup per row i of out, 64 columns.
__global__ void __launch_bounds__(64)
    pinv_apply_kernel(const double* __restrict__ A, const double* __restrict__ V,
                      const double* __restrict__ sig, const int* __restrict__ keep,
                      int nkeep, int64_t d, const double* __restrict__ UtB,
                      int64_t k, double* __restrict__ out) {
  const int64_t i = blockIdx.x;
  const int64_t c = static_cast<int64_t>(blockIdx.y) * 64 + threadIdx.x;
  if (c >= k) return;
  (void)A;
  double s = 0.0;
  for (int jj = 0; jj < nkeep; ++jj) {
    const int j = keep[jj];
    s += V[static_cast<int64_t>(j) * d + i] * UtB[jj * k + c] / sig[j];
  }
  out[i * k + c] = s;
}

// UtB[jj][c] = (A[:, j] / sigma_j) . B[:, c] for kept column j = keep[jj]
__global__ void __launch_bounds__(64)
    utb_kernel(const double* __restrict__ A, const double* __restrict__ sig,
               const int* __restrict__ keep, int64_t d,
               const double* __restrict__ B, int64_t k,
               double* __restrict__ UtB) {
  const int jj = blockIdx.x;
  const int64_t c = static_cast<int64_t>(blockIdx.y) * 64 + threadIdx.x;
  if (c >= k) return;
  const int j = keep[jj];
  const double* aj = A + static_cast<int64_t>(j) * d;
  double s = 0.0;
  for (int64_t i = 0; i < d; ++i) s += aj[i] * B[i * k + c];
  UtB[static_cast<int64_t>(jj) * k + c] = s / sig[j];
}

// out column k: the right singular vector V[:, idx[k]] with its
// largest-magnitude entry (the first on ties) made positive; sigma_out[k]
__global__ void __launch_bounds__(64)
    svd_out_kernel(const double* __restrict__ V, const double* __restrict__ sig,
                   const int* __restrict__ idx, int64_t d,
                   double* __restrict__ sigma_out, double* __restrict__ v_out) {
  const int64_t k = blockIdx.x;
  const int lane = threadIdx.x;
  const int j = idx[k];
  const double* vj = V + static_cast<int64_t>(j) * d;
  double best = -1.0;
  int64_t bi = d;
  for (int64_t i = lane; i < d; i += 64) {
    const double a = fabs(vj[i]);
    if (a > best) {
      best = a;
      bi = i;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o, 64);
    const int64_t oi = __shfl_xor(bi, o, 64);
    if (ob > best || (ob == best && oi < bi)) {
      best = ob;
      bi = oi;
    }
  }
  const double sg = vj[bi] < 0.0 ? -1.0 : 1.0;
  for (int64_t i = lane; i < d; i += 64) v_out[i * d + k] = sg * vj[i];
  if (lane == 0) sigma_out[k] = sig[j];
}

}  // namespace

size_t jacobi_svd_scratch_bytes(int64_t d) {
  return static_cast<size_t>(2 * d * d + d) * sizeof(double) +
         static_cast<size_t>(d + 64) * sizeof(int);
}

int jacobi_svd(const double* r, int64_t d, double* sigma, double* v,
               void* scratch, hipStream_t s) {
  if (d <= 0) return 0;
  double* A = static_cast<double*>(scratch);
  double* V = A + d * d;
  double* sig = V + d * d;
  int* idx_d = reinterpret_cast<int*>(sig + d);
  int* rotated = idx_d + d;
  const int64_t dd = d * d;
  transpose_init_kernel<<<static_cast<unsigned>((dd + 255) / 256), 256, 0, s>>>(
      r, d, A, V);
  const int64_t dpad = d + (d & 1);
  const int64_t rounds = dpad - 1 > 0 ? dpad - 1 : 1;
  const unsigned pgrid = static_cast<unsigned>((dpad / 2 + 3) / 4);
  int host_rot = 1;
  for (int sweep = 0; sweep < 40 && host_rot && d > 1; ++sweep) {
    if (hipMemsetAsync(rotated, 0, sizeof(int), s) != hipSuccess) return -1;
    for (int64_t rd = 0; rd < rounds; ++rd)
      jacobi_round_kernel<<<pgrid, 256, 0, s>>>(A, V, d, dpad, rd, 1e-15, rotated);
    if (hipMemcpyAsync(&host_rot, rotated, sizeof(int), hipMemcpyDeviceToHost,
                       s) != hipSuccess)
      return -1;
    if (hipStreamSynchronize(s) != hipSuccess) return -1;
  }
  col_norms_kernel<<<static_cast<unsigned>((d + 3) / 4), 256, 0, s>>>(A, d, sig);
  std::vector<double> hs(static_cast<size_t>(d));
  if (hipMemcpyAsync(hs.data(), sig, d * sizeof(double), hipMemcpyDeviceToHost,
                     s) != hipSuccess)
    return -1;
  if (hipStreamSynchronize(s) != hipSuccess) return -1;
  std::vector<int> idx(static_cast<size_t>(d));
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(),
                   [&](int x, int y) { return hs[x] > hs[y]; });
  if (hipMemcpyAsync(idx_d, idx.data(), d * sizeof(int), hipMemcpyHostToDevice,
                     s) != hipSuccess)
    return -1;
  svd_out_kernel<<<static_cast<unsigned>(d), 64, 0, s>>>(V, sig, idx_d, d, sigma,
                                                         v);
  // keep the host index buffer alive until the copy has been consumed
  if (hipStreamSynchronize(s) != hipSuccess) return -1;
  return 0;
}

void solve_upper(const double* r, int64_t d, double* b, int64_t k,
                 hipStream_t s, double* scratch) {
  if (d <= 0 || k <= 0) return;
  if (scratch) {
    trsm_blocked(r, d, b, k, false, scratch, s);
    return;
  }
  const unsigned cgrid = static_cast<unsigned>((k + 63) / 64);
  const int64_t nb = (d + kB - 1) / kB;
  for (int64_t bi = nb - 1; bi >= 0; --bi) {
    const int64_t r0 = bi * kB;
    const int bs = static_cast<int>(d - r0 < kB ? d - r0 : kB);
    prof_begin(kKTrsm, s);
    trsm_diag_kernel<<<static_cast<unsigned>((k + 3) / 4), 256, 0, s>>>(
        r, d, r0, bs, b, k);
    prof_end(kKTrsm, s);
    if (r0 > 0) {
      dim3 grid(static_cast<unsigned>((r0 + 3) / 4), cgrid);
      prof_begin(kKTrsm, s);
      trsm_update_kernel<<<grid, 256, 0, s>>>(r, d, r0, bs, b, k);
      prof_end(kKTrsm, s);
    }
  }
}

void launch_eye(double* out, int64_t d, hipStream_t s) {
  const int64_t n = d * d;
  if (n <= 0) return;
  eye_kernel<<<static_cast<unsigned>((n + 255) / 256), 256, 0, s>>>(out, d);
}

void launch_scale_rows(const double* m, const double* scale_row, int64_t d,
                       int64_t k, double* out64, float* out32, hipStream_t s) {
  const int64_t n = d * k;
  if (n <= 0) return;
  scale_rows_kernel<<<static_cast<unsigned>((n + 255) / 256), 256, 0, s>>>(
      m, scale_row, d, k, out64, out32);
}

size_t jacobi_scratch_bytes(int64_t d, int64_t k) {
  return static_cast<size_t>(2 * d * d + d + d * k) * sizeof(double) +
         static_cast<size_t>(d + 64) * sizeof(int);
}

int jacobi_truncated_apply(const double* r, int64_t d, const double* b,
                           int64_t k, double rank_tol, double* out,
                           int64_t* rank_out, void* scratch, hipStream_t s) {
  double* A = static_cast<double*>(scratch);
  double* V = A + d * d;
  double* sig = V + d * d;
  double* UtB = sig + d;
  int* keep = reinterpret_cast<int*>(UtB + d * k);
  int* rotated = keep + d;
  const int64_t dd = d * d;
  transpose_init_kernel<<<static_cast<unsigned>((dd + 255) / 256), 256, 0, s>>>(
      r, d, A, V);
  const int64_t dpad = d + (d & 1);
  const int64_t rounds = dpad - 1 > 0 ? dpad - 1 : 1;
  const unsigned pgrid = static_cast<unsigned>((dpad / 2 + 3) / 4);
  const double tol = 1e-15;
  int host_rot = 1;
  for (int sweep = 0; sweep < 40 && host_rot && d > 1; ++sweep) {
    if (hipMemsetAsync(rotated, 0, sizeof(int), s) != hipSuccess) return -1;
    for (int64_t rd = 0; rd < rounds; ++rd)
      jacobi_round_kernel<<<pgrid, 256, 0, s>>>(A, V, d, dpad, rd, tol, rotated);
    if (hipMemcpyAsync(&host_rot, rotated, sizeof(int), hipMemcpyDeviceToHost,
                       s) != hipSuccess)
      return -1;
    if (hipStreamSynchronize(s) != hipSuccess) return -1;
  }
  col_norms_kernel<<<static_cast<unsigned>((d + 3) / 4), 256, 0, s>>>(A, d, sig);
  std::vector<double> hs(static_cast<size_t>(d));
  if (hipMemcpyAsync(hs.data(), sig, d * sizeof(double), hipMemcpyDeviceToHost,
                     s) != hipSuccess)
    return -1;
  if (hipStreamSynchronize(s) != hipSuccess) return -1;
  std::vector<int> idx(static_cast<size_t>(d));
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(),
                   [&](int x, int y) { return hs[x] > hs[y]; });
  const double smax = hs[idx[0]];
  int nkeep = 0;
  if (smax > 0.0)
    while (nkeep < d && hs[idx[nkeep]] > rank_tol * smax) ++nkeep;
  *rank_out = nkeep;
  if (nkeep == 0) {
    if (hipMemsetAsync(out, 0, d * k * sizeof(double), s) != hipSuccess)
      return -1;
    return 0;
  }
  if (hipMemcpyAsync(keep, idx.data(), nkeep * sizeof(int),
                     hipMemcpyHostToDevice, s) != hipSuccess)
    return -1;
  const unsigned cgrid = static_cast<unsigned>((k + 63) / 64);
  utb_kernel<<<dim3(static_cast<unsigned>(nkeep), cgrid), 64, 0, s>>>(
      A, sig, keep, d, b, k, UtB);
  pinv_apply_kernel<<<dim3(static_cast<unsigned>(d), cgrid), 64, 0, s>>>(
      A, V, sig, keep, nkeep, d, UtB, k, out);
  // keep the host index buffer alive until the copy has been consumed
  if (hipStreamSynchronize(s) != hipSuccess) return -1;
  return 0;
}

}  // namespace slso
