// Blocked Householder QR of the r x d sketch in FP64 (Algorithm 2 step 2 in
// QR form; only R is kept).
//
// Right-looking, panels of W = 16 columns. Each panel is reduced by a tree of
// Householder factorisations (the communication-avoiding ordering of
// tall-skinny QR): the active rows are cut into leaves of L = 256 rows; a node
// factors its <= 256 rows x W panel columns, keeps its reflectors in
// compact-WY form (Y, T: Q = I - Y T Y^T) and leaves its triangle in its first
// W rows (its "head"); a parent stacks the heads of up to F = L / W = 16
// children. Every node is a Householder factorisation, so R is the R of a
// Householder QR (rows normalised to a non-negative diagonal at the end). One
// launch per tree level: kernel boundaries order the levels, no inter-block
// synchronisation.
//
// Node factorisation (four waves, one row per thread). Fast path, used when
// the node's Gram matrix is numerically well conditioned: Cholesky-QR twice
// (the Gram matrix on FP64 MFMA, Cholesky and the triangular solves in FP64)
// gives an orthonormal Q and R; Householder reconstruction (Ballard, Demmel,
// Grigori, Jacquelin, Knight & Nguyen, "Reconstructing Householder vectors
// from tall-skinny QR", 2014) then yields the Householder vectors exactly:
// a sign-choosing LU without pivoting, Q - [S; 0] = Y U with every pivot of
// magnitude >= 1, T = -U S Y1^{-T}, and the Householder R is S R. Otherwise
// (a Cholesky pivot below 1e-10 of its column's squared norm, fewer than W
// rows, or a ragged last panel) wave 0 factors the node column by column:
// per column one wave-wide reduction of the 16-vector g_j = sum_{t > c}
// a_tc a_tj (norm and all dots) plus z_j = y_j . y_{c-1} for the T recurrence
// T[0:i, i] = -tau_i T[0:i, 0:i] (Y[:, 0:i]^T y_i).
//
// Trailing update: one workgroup of four waves per (node, 64 columns), each
// wave a 16-column strip held in registers, on FP64 MFMA
// (v_mfma_f64_16x16x4f64: A operand lane l = A[l%16][l/16], B operand
// B[l/16][l%16], result register v of lane l = D[4v + l/16][l%16]). The result
// layout of W1 = Y^T C is the B-operand layout of T^T W1 and of C - Y W2, so
// the 16 x 16 intermediates never leave registers.
#include <algorithm>

#include "internal.h"

namespace slso {
namespace {

constexpr int kW = 16;       // panel width
constexpr int kR = 4;        // rows per lane (wave-0 fallback layout)
constexpr int kL = 64 * kR;  // rows per tree node
constexpr int kF = kL / kW;  // fan-in
constexpr int kMaxLevels = 8;
constexpr int kYP = kW + 1;  // padded LDS row of a W-wide block
#ifndef SLSO_QR_PIVOT_TOL
#define SLSO_QR_PIVOT_TOL 1e-10
#endif
#ifndef SLSO_QR_FORCE_FALLBACK
#define SLSO_QR_FORCE_FALLBACK 0
#endif
constexpr double kPivotTol = SLSO_QR_PIVOT_TOL;

typedef double dbl4 __attribute__((ext_vector_type(4)));

struct Panel {
  int64_t m, j0;
  int w;                        // panel width (<= kW)
  int nlev;                     // tree levels
  int64_t nodes[kMaxLevels];    // nodes per level
  int64_t off[kMaxLevels];      // first node id of a level
  int64_t span[kMaxLevels];     // leaves per node of a level
};

__device__ __forceinline__ int64_t leaf_rows(const Panel& P, int64_t leaf) {
  const int64_t rem = P.m - P.j0 - leaf * kL;
  return rem < kL ? rem : kL;
}

// Global row of local row t of node (level, q) (-1 when absent), and the
// node's row count.
__device__ __forceinline__ int64_t node_row(const Panel& P, int level,
                                            int64_t q, int t, int* cnt_out) {
  int64_t row = -1;
  if (level == 0) {
    const int cnt = static_cast<int>(leaf_rows(P, q));
    if (t < cnt) row = P.j0 + q * kL + t;
    *cnt_out = cnt;
    return row;
  }
  const int64_t cs = P.span[level - 1];
  int pre = 0;
#pragma unroll
  for (int c = 0; c < kF; ++c) {
    const int64_t cq = kF * q + c;
    if (cq < P.nodes[level - 1]) {
      const int64_t lc = leaf_rows(P, cq * cs);
      const int h = static_cast<int>(lc < P.w ? lc : P.w);
      if (t >= pre && t < pre + h) row = P.j0 + cq * cs * kL + (t - pre);
      pre += h;
    }
  }
  *cnt_out = pre;
  return row;
}

// LDS ordering among the lanes of one wave (no block barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Cross-lane moves of doubles: DPP (within rows of 16 lanes), ds_swizzle
// (within 32 lanes) and ds_bpermute (across the 32-lane halves).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, 0xf, 0xf, false),
                          __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xf, 0xf, false));
}
template <int PAT>
__device__ __forceinline__ double swz_d(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  return __hiloint2double(__builtin_amdgcn_ds_swizzle(hi, PAT),
                          __builtin_amdgcn_ds_swizzle(lo, PAT));
}
constexpr int kDppRowMirror = 0x140;      // lane i <-> 15 - i within 16
constexpr int kDppRowHalfMirror = 0x141;  // lane i <-> 7 - i within 8
constexpr int kDppQuadSwap2 = 0x4E;       // quad_perm [2,3,0,1]
constexpr int kDppQuadSwap1 = 0xB1;       // quad_perm [1,0,3,2]
constexpr int kSwzXor16 = (16 << 10) | 0x1f;

// Recursive halving of 16 values over 64 lanes: on return every lane holds in
// v[0] the wave sum of entry (lane >> 2) & 15. Each stage pairs every lane
// with a partner whose deciding bit differs (xor 32, xor 16, mirror within 16,
// mirror within 8), so the kept halves of the 16 entries line up; the lanes
// merged into one partial sum are l ^ {0,7,8,15,...,63}, and the last two
// quad exchanges add the four disjoint partials of each entry.
__device__ __forceinline__ void reduce16(double (&v)[kW], int lane) {
  {
    const bool hi = lane & 32;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const double send = hi ? v[i] : v[i + 8];
      const double keep = hi ? v[i + 8] : v[i];
      v[i] = keep + __shfl_xor(send, 32, 64);
    }
  }
  {
    const bool hi = lane & 16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double send = hi ? v[i] : v[i + 4];
      const double keep = hi ? v[i + 4] : v[i];
      v[i] = keep + swz_d<kSwzXor16>(send);
    }
  }
  {
    const bool hi = lane & 8;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const double send = hi ? v[i] : v[i + 2];
      const double keep = hi ? v[i + 2] : v[i];
      v[i] = keep + dpp_d<kDppRowMirror>(send);
    }
  }
  {
    const bool hi = lane & 4;
    const double send = hi ? v[0] : v[1];
    const double keep = hi ? v[1] : v[0];
    v[0] = keep + dpp_d<kDppRowHalfMirror>(send);
  }
  v[0] += dpp_d<kDppQuadSwap2>(v[0]);
  v[0] += dpp_d<kDppQuadSwap1>(v[0]);
}

struct FactorLds {
  double gsum[kW];
  double rowc[kW];
  double T[kW][kW + 1];
  double taus[kW];
};

template <int C>
__device__ __forceinline__ void fstep(double (&a)[kR][kW], FactorLds& sh,
                                      int lane, int nsteps) {
  if (C > nsteps) return;  // wave-uniform
  constexpr int cm1 = C > 0 ? C - 1 : 0;
  constexpr int cc = C < kW ? C : kW - 1;
  const bool piv = C < nsteps;
  // Rows in register slots r >= 1 have t = lane + 64 r > every column index,
  // so only slot 0 needs the position tests below/at/above the diagonal.
  double v[kW];
#pragma unroll
  for (int j = 0; j < kW; ++j) v[j] = 0.0;
  if (C >= 2) {
    const double yp0 = lane > cm1 ? a[0][cm1] : (lane == cm1 ? 1.0 : 0.0);
#pragma unroll
    for (int j = 0; j + 1 < C; ++j) {
      const double yj = lane > j ? a[0][j] : (lane == j ? 1.0 : 0.0);
      v[j] = yj * yp0;
#pragma unroll
      for (int r = 1; r < kR; ++r) v[j] += a[r][j] * a[r][cm1];
    }
  }
  if (piv) {
    const double ac0 = lane > C ? a[0][cc] : 0.0;
#pragma unroll
    for (int j = cc; j < kW; ++j) {
      v[j] += ac0 * a[0][j];
#pragma unroll
      for (int r = 1; r < kR; ++r) v[j] += a[r][cc] * a[r][j];
    }
  }
  reduce16(v, lane);
  if ((lane & 3) == 0) sh.gsum[lane >> 2] = v[0];
  if (piv && lane == C) {
#pragma unroll
    for (int j = 0; j < kW; ++j) sh.rowc[j] = a[0][j];
  }
  wave_sync();
  if (C >= 1 && lane < C) {
    // column C-1 of T: T[i][C-1] = -tau_{C-1} sum_{l=i}^{C-2} T[i][l] z[l]
    const int i = lane;
    if (i == cm1) {
      sh.T[cm1][cm1] = sh.taus[cm1];
    } else {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < cm1; ++l)
        if (l >= i) s += sh.T[i][l] * sh.gsum[l];
      sh.T[i][cm1] = -sh.taus[cm1] * s;
    }
  }
  if (piv) {
    const double s2 = sh.gsum[cc];
    const double alpha = sh.rowc[cc];
    double tau = 0.0, beta = alpha, scal = 0.0;
    if (s2 > 0.0) {
      const double nrm = sqrt(alpha * alpha + s2);
      beta = alpha >= 0.0 ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    double p[kW];
#pragma unroll
    for (int j = cc + 1; j < kW; ++j) p[j] = sh.rowc[j] + scal * sh.gsum[j];
    {
      const double vt = lane > C ? a[0][cc] * scal : (lane == C ? 1.0 : 0.0);
      const double f = tau * vt;
#pragma unroll
      for (int j = cc + 1; j < kW; ++j) a[0][j] -= f * p[j];
      a[0][cc] = lane > C ? vt : (lane == C ? beta : a[0][cc]);
    }
#pragma unroll
    for (int r = 1; r < kR; ++r) {
      const double vt = a[r][cc] * scal;
      const double f = tau * vt;
#pragma unroll
      for (int j = cc + 1; j < kW; ++j) a[r][j] -= f * p[j];
      a[r][cc] = vt;
    }
    if (lane == 0) sh.taus[cc] = tau;
  }
  wave_sync();
}

template <int C>
__device__ __forceinline__ void fsteps(double (&a)[kR][kW], FactorLds& sh,
                                       int lane, int nsteps) {
  fstep<C>(a, sh, lane, nsteps);
  if constexpr (C < kW) fsteps<C + 1>(a, sh, lane, nsteps);
}


struct NodeLds {
  int64_t rows[kL];
  double Ash[kL * kYP];        // staged rows of the node (A, then Q1)
  double Gp[4][kW * kW];       // per-wave partial Gram matrices
  double G[kW][kYP];
  double Gd[kW];               // diagonal of the first Gram matrix
  double R1[kW][kYP];
  double R2[kW][kYP];
  double Rf[kW][kYP];
  double Wl[kW][kYP];          // sign-choosing LU of the top block of Q
  double Z[kW][kYP];           // Y1^{-T}
  double Tm[kW][kYP];
  double inv1[kW], inv2[kW], invu[kW], sgn[kW];
  int flag;
  FactorLds fb;
};

// G = X^T X of the staged rows (256 x 16) on MFMA, four waves x 64 rows.
__device__ __forceinline__ void gram(NodeLds& sh, int t) {
  const int lane = t & 63, wv = t >> 6, p = lane & 15, qd = lane >> 4;
  dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const double x = sh.Ash[(64 * wv + 4 * kk + qd) * kYP + p];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, x, acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) sh.Gp[wv][(4 * v + qd) * kW + p] = acc[v];
  __syncthreads();
  {
    const int i = t / kW, j = t % kW;
    sh.G[i][j] = sh.Gp[0][t] + sh.Gp[1][t] + sh.Gp[2][t] + sh.Gp[3][t];
  }
  __syncthreads();
}

// 1/x and sqrt(x) from the hardware approximations refined by Newton steps
// (two steps take the approximations to full double precision), shorter
// dependency chains than the correctly rounded library sequences.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ __forceinline__ double rsq_nr(double x) {  // 1/sqrt(x), x > 0
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}

__device__ __forceinline__ double readlane_d(double x, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                          __builtin_amdgcn_readlane(__double2loint(x), l));
}

// Cholesky G = R^T R by wave 0 with lane l < 16 owning column l of G in
// registers (pivots and rows of R broadcast by readlane). Writes R and the
// inverse diagonal to LDS; sets the fallback flag when a pivot falls below
// kPivotTol times its reference (the column's squared norm; 1 when ref is
// NULL).
__device__ void cholesky16(NodeLds& sh, double (*R)[kYP], double* inv,
                           const double* ref, int lane) {
  const int l = lane;
  double gc[kW], rc[kW];
#pragma unroll
  for (int i = 0; i < kW; ++i) {
    gc[i] = l < kW ? sh.G[i][l] : 0.0;
    rc[i] = 0.0;
  }
  bool ok = true;
#pragma unroll
  for (int j = 0; j < kW; ++j) {
    const double piv = readlane_d(gc[j], j);
    ok = ok && (piv > kPivotTol * (ref ? ref[j] : 1.0));
    const double ir = rsq_nr(ok ? piv : 1.0);
    const double rjj = (ok ? piv : 1.0) * ir;
    const double rjl = l > j ? gc[j] * ir : (l == j ? rjj : 0.0);
    rc[j] = rjl;
    if (l == j) inv[j] = ir;
#pragma unroll
    for (int i = j + 1; i < kW; ++i) gc[i] -= readlane_d(rjl, i) * rjl;
  }
  if (!ok) {
    if (lane == 0) sh.flag = 1;
    return;
  }
  if (l < kW) {
#pragma unroll
    for (int i = 0; i < kW; ++i) R[i][l] = rc[i];
  }
}

// x = a R^{-1} for one row (R upper triangular, inverse diagonal given)
__device__ __forceinline__ void row_solve(const double (&a)[kW], double (&x)[kW],
                                          const double (*R)[kYP],
                                          const double* inv) {
#pragma unroll
  for (int j = 0; j < kW; ++j) {
    double s = a[j];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= x[k] * R[k][j];
    x[j] = s * inv[j];
  }
}

__global__ void __launch_bounds__(256)
    qr_node_kernel(double* __restrict__ A, int64_t lda, Panel P, int level,
                   double* __restrict__ Yws, double* __restrict__ Tws) {
  __shared__ NodeLds sh;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wv = t >> 6;
  const int64_t q = blockIdx.x;
  int cnt;
  const int64_t row = node_row(P, level, q, t, &cnt);
  sh.rows[t] = row;
  const int nsteps = cnt < P.w ? cnt : P.w;
  __syncthreads();
  // coalesced load: 16 consecutive threads read one row's 16 panel entries;
  // all loads are issued before any LDS store waits on them
  {
    const int j = t & 15;
    double ld[kW];
#pragma unroll
    for (int k = 0; k < kW; ++k) {
      const int64_t rr = sh.rows[16 * k + (t >> 4)];
      ld[k] = (rr >= 0 && j < P.w) ? A[rr * lda + P.j0 + j] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kW; ++k) sh.Ash[(16 * k + (t >> 4)) * kYP + j] = ld[k];
  }
  __syncthreads();
  double a[kW];
#pragma unroll
  for (int j = 0; j < kW; ++j) a[j] = sh.Ash[t * kYP + j];
  if (t == 0)
    sh.flag = (SLSO_QR_FORCE_FALLBACK || P.w != kW || cnt < kW) ? 1 : 0;
  __syncthreads();
  const int64_t nid = P.off[level] + q;
  double* Y = Yws + nid * (kL * kW);
  double* Tn = Tws + nid * (kW * kW);

  double x[kW];
  if (!sh.flag) {
    // ---- Cholesky-QR, first pass: R1, x = a R1^{-1} -------------------------
    gram(sh, t);
    if (t < kW) sh.Gd[t] = sh.G[t][t];
    __syncthreads();
    if (wv == 0) cholesky16(sh, sh.R1, sh.inv1, sh.Gd, lane);
    __syncthreads();
  }
  if (!sh.flag) {
    row_solve(a, x, sh.R1, sh.inv1);
#pragma unroll
    for (int j = 0; j < kW; ++j) sh.Ash[t * kYP + j] = x[j];
    __syncthreads();
    // ---- second pass: R2, q = x R2^{-1} -----------------------------------
    gram(sh, t);
    if (wv == 0) cholesky16(sh, sh.R2, sh.inv2, nullptr, lane);  // G2 ~ I
    __syncthreads();
  }
  if (!sh.flag) {
    double qv[kW];
    row_solve(x, qv, sh.R2, sh.inv2);
    {
      // R = R2 R1
      const int i = t / kW, j = t % kW;
      double sres = 0.0;
#pragma unroll
      for (int k = 0; k < kW; ++k)
        if (k >= i && k <= j) sres += sh.R2[i][k] * sh.R1[k][j];
      sh.Rf[i][j] = sres;
    }
    if (t < kW) {
#pragma unroll
      for (int j = 0; j < kW; ++j) sh.Wl[t][j] = qv[j];
    }
    __syncthreads();
    // ---- Householder reconstruction: sign-choosing LU of the top block ------
    // wave 0, lane l < 16 owning column l of the top 16 x 16 block of Q
    if (wv == 0) {
      const int l = lane;
      double wc[kW], z[kW];
#pragma unroll
      for (int r = 0; r < kW; ++r) wc[r] = l < kW ? sh.Wl[r][l] : 0.0;
#pragma unroll
      for (int i = 0; i < kW; ++i) {
        const double pv = readlane_d(wc[i], i);
        const double sg = pv >= 0.0 ? -1.0 : 1.0;
        const double piv = pv - sg;  // |piv| >= 1
        const double ip = rcp_nr(piv);
        if (l == i) {
          wc[i] = piv;
#pragma unroll
          for (int r = i + 1; r < kW; ++r) wc[r] *= ip;
        }
        if (lane == 0) {
          sh.sgn[i] = sg;
          sh.invu[i] = ip;
        }
        const double wil = wc[i];
#pragma unroll
        for (int r = i + 1; r < kW; ++r) {
          const double mr = readlane_d(wc[r], i);
          if (l > i) wc[r] -= mr * wil;
        }
      }
      // lane c: column c of Y1^{-1} (Y1 unit lower, multipliers of the LU)
#pragma unroll
      for (int i = 0; i < kW; ++i) z[i] = (i == l) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < kW; ++k)
#pragma unroll
        for (int i = k + 1; i < kW; ++i) z[i] -= readlane_d(wc[i], k) * z[k];
      if (l < kW) {
#pragma unroll
        for (int r = 0; r < kW; ++r) {
          sh.Wl[r][l] = wc[r];   // U on and above the diagonal, L below
          sh.Z[l][r] = z[r];     // Z = Y1^{-T}: row l of Z = column l of Y1^{-1}
        }
      }
    }
    __syncthreads();
    {
      // T = -U S Z (upper triangular)
      const int i = t / kW, j = t % kW;
      double st = 0.0;
#pragma unroll
      for (int k = 0; k < kW; ++k)
        if (k >= i && k <= j) st += sh.Wl[i][k] * sh.sgn[k] * sh.Z[k][j];
      Tn[t] = i <= j ? -st : 0.0;
    }
    // Y rows: top block from the LU, the rest y = q U^{-1}
    double yv[kW];
    if (t < kW) {
#pragma unroll
      for (int j = 0; j < kW; ++j)
        yv[j] = j < t ? sh.Wl[t][j] : (j == t ? 1.0 : 0.0);
    } else {
#pragma unroll
      for (int j = 0; j < kW; ++j) {
        double sy = qv[j];
#pragma unroll
        for (int k = 0; k < j; ++k) sy -= yv[k] * sh.Wl[k][j];
        yv[j] = sy * sh.invu[j];
      }
    }
#pragma unroll
    for (int j = 0; j < kW; ++j) Y[t * kW + j] = t < cnt ? yv[j] : 0.0;
    // Householder R = S R in the head rows, zeros in the rest of the panel
    if (row >= 0) {
#pragma unroll
      for (int j = 0; j < kW; ++j)
        A[row * lda + P.j0 + j] =
            (t < kW && j >= t) ? sh.sgn[t] * sh.Rf[t][j] : 0.0;
    }
    return;
  }

  // ---- fallback: column-by-column Householder by wave 0 ----------------------
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kW; ++j) sh.Ash[t * kYP + j] = a[j];
  __syncthreads();
  if (wv != 0) return;
  FactorLds& fb = sh.fb;
  double a4[kR][kW];
#pragma unroll
  for (int r = 0; r < kR; ++r)
#pragma unroll
    for (int j = 0; j < kW; ++j) a4[r][j] = sh.Ash[(lane + 64 * r) * kYP + j];
  for (int e = lane; e < kW * (kW + 1); e += 64) (&fb.T[0][0])[e] = 0.0;
  if (lane < kW) fb.taus[lane] = 0.0;
  wave_sync();
  fsteps<0>(a4, fb, lane, nsteps);
#pragma unroll
  for (int r = 0; r < kR; ++r) {
    const int tt = lane + 64 * r;
#pragma unroll
    for (int j = 0; j < kW; ++j) {
      double y = 0.0;
      if (j < nsteps && tt < cnt) y = tt > j ? a4[r][j] : (tt == j ? 1.0 : 0.0);
      Y[tt * kW + j] = y;
    }
    const int64_t rr = sh.rows[tt];
    if (rr >= 0) {
#pragma unroll
      for (int j = 0; j < kW; ++j)
        if (j < P.w)
          A[rr * lda + P.j0 + j] = (tt < nsteps && j >= tt) ? a4[r][j] : 0.0;
    }
  }
  for (int e = lane; e < kW * kW; e += 64) {
    const int i = e / kW, j = e % kW;
    Tn[e] = (i < nsteps && j < nsteps) ? fb.T[i][j] : 0.0;
  }
}

// Q^T of the nodes of one tree level applied to the trailing matrix: one
// workgroup of four waves per (node, 64 columns), each wave a 16-column strip
// of the node's rows held in registers (rows t = 4 m + l/16).
__global__ void __launch_bounds__(256)
    qr_update_kernel(double* __restrict__ A, int64_t lda, Panel P, int level,
                     const double* __restrict__ Yws,
                     const double* __restrict__ Tws, int64_t col0,
                     int64_t ncols) {
  __shared__ int64_t rows[kL];
  __shared__ double Ys[kL * kYP];
  __shared__ double Ts[kW * kW];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int p = lane & 15;
  const int qd = lane >> 4;
  const int64_t q = blockIdx.x;
  const int64_t col = col0 + static_cast<int64_t>(blockIdx.y) * 64 + wave * 16 + p;
  const bool cok = col < col0 + ncols;
  int cnt;
  rows[t] = node_row(P, level, q, t, &cnt);
  const int64_t nid = P.off[level] + q;
  const double* Y = Yws + nid * (kL * kW);
  for (int e = t; e < kL * kW; e += 256) Ys[(e / kW) * kYP + (e % kW)] = Y[e];
  Ts[t] = Tws[nid * (kW * kW) + t];
  __syncthreads();

  double creg[kL / 4];
#pragma unroll
  for (int m = 0; m < kL / 4; ++m) {
    const int tt = 4 * m + qd;
    creg[m] = (tt < cnt && cok) ? A[rows[tt] * lda + col] : 0.0;
  }
  // W1 = Y^T C
  dbl4 w1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int m = 0; m < kL / 4; ++m)
    if (4 * m < cnt)
      w1 = __builtin_amdgcn_mfma_f64_16x16x4f64(Ys[(4 * m + qd) * kYP + p],
                                                creg[m], w1, 0, 0, 0);
  // W2 = T^T W1 (W1 in result layout is the B operand of k-steps 0..3)
  dbl4 w2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < 4; ++kk)
    w2 = __builtin_amdgcn_mfma_f64_16x16x4f64(Ts[(4 * kk + qd) * kW + p],
                                              w1[kk], w2, 0, 0, 0);
  // C = C - Y W2, 16 rows at a time with the C tile as accumulator
#pragma unroll
  for (int rt = 0; rt < kL / 16; ++rt) {
    if (16 * rt < cnt) {
      dbl4 acc = {creg[4 * rt], creg[4 * rt + 1], creg[4 * rt + 2],
                  creg[4 * rt + 3]};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(
            Ys[(16 * rt + p) * kYP + 4 * kk + qd], -w2[kk], acc, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) creg[4 * rt + v] = acc[v];
    }
  }
#pragma unroll
  for (int m = 0; m < kL / 4; ++m) {
    const int tt = 4 * m + qd;
    if (tt < cnt && cok) A[rows[tt] * lda + col] = creg[m];
  }
}

Panel make_panel(int64_t m, int64_t d, int64_t j0) {
  Panel P{};
  P.m = m;
  P.j0 = j0;
  P.w = static_cast<int>(d - j0 < kW ? d - j0 : kW);
  int64_t nodes = (m - j0 + kL - 1) / kL;
  int64_t off = 0, span = 1;
  int lev = 0;
  for (;;) {
    P.nodes[lev] = nodes;
    P.off[lev] = off;
    P.span[lev] = span;
    off += nodes;
    ++lev;
    if (nodes == 1) break;
    nodes = (nodes + kF - 1) / kF;
    span *= kF;
  }
  P.nlev = lev;
  return P;
}

int64_t total_nodes(int64_t m) {
  int64_t nodes = (m + kL - 1) / kL, tot = 0;
  for (;;) {
    tot += nodes;
    if (nodes == 1) break;
    nodes = (nodes + kF - 1) / kF;
  }
  return tot;
}

__global__ void extract_r_kernel(const double* __restrict__ A, int64_t lda,
                                 int64_t d, double* __restrict__ R) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= d * d) return;
  const int64_t i = e / d, j = e - i * d;
  const double s = A[i * lda + i] < 0.0 ? -1.0 : 1.0;
  R[e] = j >= i ? s * A[i * lda + j] : 0.0;
}

__global__ void __launch_bounds__(256)
    diag_stats_kernel(const double* __restrict__ R, int64_t d,
                      double* __restrict__ out) {
  __shared__ double smin[256], smax[256];
  const int t = threadIdx.x;
  double mn = INFINITY, mx = 0.0;
  for (int64_t j = t; j < d; j += 256) {
    const double v = fabs(R[j * d + j]);
    mn = fmin(mn, v);
    mx = fmax(mx, v);
  }
  smin[t] = mn;
  smax[t] = mx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      smin[t] = fmin(smin[t], smin[t + o]);
      smax[t] = fmax(smax[t], smax[t + o]);
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = smin[0];
    out[1] = smax[0];
  }
}

}  // namespace

namespace {

size_t tree_scratch_bytes(int64_t m) {
  const int64_t tn = total_nodes(m);
  return static_cast<size_t>(tn) * (kL * kW + kW * kW) * sizeof(double);
}

// Tree-path panels of columns [j_start, d)
void tree_panels(double* a, int64_t m, int64_t d, int64_t j_start,
                 void* scratch, hipStream_t s) {
  const int64_t tn = total_nodes(m);
  double* Yws = static_cast<double*>(scratch);
  double* Tws = Yws + tn * (kL * kW);
  for (int64_t j0 = j_start; j0 < d; j0 += kW) {
    const Panel P = make_panel(m, d, j0);
    const int64_t tc0 = j0 + P.w;
    const int64_t tcols = d - tc0;
    const unsigned groups = static_cast<unsigned>((tcols + 63) / 64);
    for (int lev = 0; lev < P.nlev; ++lev) {
      prof_begin(kKQrNode, s);
      qr_node_kernel<<<static_cast<unsigned>(P.nodes[lev]), 256, 0, s>>>(
          a, d, P, lev, Yws, Tws);
      prof_end(kKQrNode, s);
    }
    if (tcols > 0) {
      for (int lev = 0; lev < P.nlev; ++lev) {
        prof_begin(kKQrUpdate, s);
        qr_update_kernel<<<dim3(static_cast<unsigned>(P.nodes[lev]), groups),
                           256, 0, s>>>(a, d, P, lev, Yws, Tws, tc0, tcols);
        prof_end(kKQrUpdate, s);
      }
    }
  }
}

void extract_r(const double* a, int64_t d, double* r_out, hipStream_t s) {
  const int64_t dd = d * d;
  prof_begin(kKQrExtract, s);
  extract_r_kernel<<<static_cast<unsigned>((dd + 255) / 256), 256, 0, s>>>(
      a, d, d, r_out);
  prof_end(kKQrExtract, s);
}

size_t tree_part(int64_t m) {
  return (tree_scratch_bytes(m) + 255) / 256 * 256;
}

}  // namespace

size_t qr_scratch_bytes(int64_t m, int64_t d) {
  return tree_part(m) +
         std::max(cqr_scratch_bytes(m, d), cholqr2_scratch_bytes(m, d)) + 512;
}
void qr_factor(double* a, int64_t m, int64_t d, double* r_out, void* scratch,
               int* status, const QrStreams& qs, hipStream_t s, bool want_r,
               double* dstat, const double* dsc, int one_pass) {
  cholqr2_factor(a, m, d, r_out, static_cast<char*>(scratch) + tree_part(m),
                 status, qs, s, want_r, dstat, dsc, one_pass);
}
void qr_factor_finish(int64_t m, int64_t d, double* r_out, void* scratch,
                      int* status, hipStream_t s, bool want_r, double* dstat) {
  cholqr2_finish(m, d, r_out, static_cast<char*>(scratch) + tree_part(m),
                 status, s, want_r, dstat);
}
void qr_apply_rinv(int64_t m, int64_t d, void* scratch, int form, double* b,
                   int64_t k, hipStream_t s) {
  cholqr2_apply_rinv(m, d, static_cast<char*>(scratch) + tree_part(m), form,
                     b, k, s);
}
void qr_finish_dev(int64_t m, int64_t d, void* scratch, const int* status,
                   int* p2, double* dstat, hipStream_t s) {
  cholqr2_finish_dev(m, d, static_cast<char*>(scratch) + tree_part(m), status,
                     p2, dstat, s);
}
void qr_apply_rinv_dev(int64_t m, int64_t d, void* scratch, const int* f,
                       double* b, int64_t k, hipStream_t s) {
  cholqr2_apply_rinv_dev(m, d, static_cast<char*>(scratch) + tree_part(m), f,
                         b, k, s);
}
void qr_write_r(int64_t m, int64_t d, double* r_out, void* scratch, int form,
                hipStream_t s) {
  cholqr2_write_r(m, d, r_out, static_cast<char*>(scratch) + tree_part(m),
                  form, s);
}
void qr_factor_panel(double* a, int64_t m, int64_t d, double* r_out,
                     void* scratch, int* fail, const QrStreams& qs,
                     hipStream_t s) {
  launch_fill_i32(fail, 1, 0, s);
  void* cws = static_cast<char*>(scratch) + tree_part(m);
  const int64_t np = cqr_panels(m, d);
  cqr_factor(a, m, d, cws, fail, qs, s);
  tree_panels(a, m, d, 64 * np, scratch, s);
  extract_r(a, d, r_out, s);
}
void qr_factor_robust(double* a, int64_t m, int64_t d, double* r_out,
                      void* scratch, hipStream_t s) {
  tree_panels(a, m, d, 0, scratch, s);
  extract_r(a, d, r_out, s);
}

void launch_diag_stats(const double* r, int64_t d, double* out,
                       hipStream_t s) {
  diag_stats_kernel<<<1, 256, 0, s>>>(r, d, out);
}

}  // namespace slso
