// Blocked Householder QR of the r x d sketch in FP64 (Algorithm 2 step 2 in
// QR form; only R is kept).
//
// The factorisation is right-looking with panels of W = 32 columns. Each
// panel is reduced by a tree of Householder factorisations (the
// communication-avoiding ordering of tall-skinny QR): the active rows are
// cut into leaves of L = 256 rows; every tree node factors its <= 256 rows x
// W panel columns in registers (one workgroup, one row per thread), stores
// its reflectors in compact-WY form (Y, T with Q = I - Y T Y^T) and leaves
// its triangle in its first rows (its "head"); the parent stacks the heads of
// up to F = L / W = 8 children and repeats, until one node remains, whose
// head holds the panel's rows of R. After every node level, Q^T = I - Y T^T
// Y^T is applied to the trailing columns of the node's rows. All reflectors
// are Householder reflectors, so R is the R of a Householder QR (rows differ
// from LAPACK's only by sign, which is normalised to a non-negative
// diagonal at the end).
//
// Node kernel, one column step c: a single block-wide reduction of the
// 32-vector  g_j = sum_{t > c} a_tc a_tj  (j >= c) gives the column norm
// (g_c) and, with the broadcast pivot row, the dots v^T a_j; the same
// reduction carries z_j = y_j^T y_{c-1} (j < c-1) for the T recurrence
// T[0:i, i] = -tau_i T[0:i, 0:i] (Y[:, 0:i]^T y_i). Each wave reduces its 32
// values by recursive halving (31 shuffles instead of 6 x 32), the four waves
// combine through LDS.
#include "internal.h"

namespace slso {
namespace {

constexpr int kW = 32;    // panel width
constexpr int kL = 256;   // rows per tree node (threads per workgroup)
constexpr int kF = kL / kW;

struct NodeGeom {
  int64_t m, j0;
  int w;
  int level;
  int64_t child_span;     // rows spanned by a node of level-1 (level >= 1)
  int64_t child_leaves;   // leaves per node of level-1
  int64_t nchild;         // number of nodes at level-1
  int64_t nleaves;
};

__device__ __forceinline__ int64_t leaf_count(const NodeGeom& g, int64_t leaf) {
  const int64_t rem = g.m - g.j0 - leaf * kL;
  return rem < kL ? rem : kL;
}

// Fills rows[0..255] (global row of local row t, -1 when absent) and returns
// the node's row count. All threads of the block call it; uses a barrier.
__device__ int node_rows(const NodeGeom& g, int64_t q, int64_t* rows) {
  const int t = threadIdx.x;
  if (g.level == 0) {
    const int64_t cnt = leaf_count(g, q);
    rows[t] = t < cnt ? g.j0 + q * kL + t : -1;
    __syncthreads();
    return static_cast<int>(cnt);
  }
  int64_t start[kF];
  int pre[kF + 1];
  pre[0] = 0;
#pragma unroll
  for (int c = 0; c < kF; ++c) {
    const int64_t cq = kF * q + c;
    int h = 0;
    if (cq < g.nchild) {
      const int64_t lc = leaf_count(g, cq * g.child_leaves);
      h = static_cast<int>(lc < g.w ? lc : g.w);
      start[c] = g.j0 + cq * g.child_span;
    } else {
      start[c] = 0;
    }
    pre[c + 1] = pre[c] + h;
  }
  int64_t row = -1;
#pragma unroll
  for (int c = 0; c < kF; ++c)
    if (t >= pre[c] && t < pre[c + 1]) row = start[c] + (t - pre[c]);
  rows[t] = row;
  __syncthreads();
  return pre[kF];
}

// Recursive-halving reduction of 32 values over the 64 lanes of a wave: on
// return lane l holds in v[0] the wave sum of entry (l >> 1).
__device__ __forceinline__ void wave_reduce32(double (&v)[kW], int lane) {
  {
    const bool hi = lane & 32;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const double send = hi ? v[i] : v[i + 16];
      const double keep = hi ? v[i + 16] : v[i];
      v[i] = keep + __shfl_xor(send, 32, 64);
    }
  }
  {
    const bool hi = lane & 16;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const double send = hi ? v[i] : v[i + 8];
      const double keep = hi ? v[i + 8] : v[i];
      v[i] = keep + __shfl_xor(send, 16, 64);
    }
  }
  {
    const bool hi = lane & 8;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double send = hi ? v[i] : v[i + 4];
      const double keep = hi ? v[i + 4] : v[i];
      v[i] = keep + __shfl_xor(send, 8, 64);
    }
  }
  {
    const bool hi = lane & 4;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const double send = hi ? v[i] : v[i + 2];
      const double keep = hi ? v[i + 2] : v[i];
      v[i] = keep + __shfl_xor(send, 4, 64);
    }
  }
  {
    const bool hi = lane & 2;
    const double send = hi ? v[0] : v[1];
    const double keep = hi ? v[1] : v[0];
    v[0] = keep + __shfl_xor(send, 2, 64);
  }
  v[0] += __shfl_xor(v[0], 1, 64);
}

__global__ void __launch_bounds__(kL)
    qr_node_kernel(double* __restrict__ A, int64_t lda, NodeGeom g,
                   double* __restrict__ Yws, double* __restrict__ Tws) {
  __shared__ int64_t rows[kL];
  __shared__ double red[4][kW];
  __shared__ double gsum[kW];
  __shared__ double rowc[kW];
  __shared__ double T[kW][kW + 1];
  __shared__ double taus[kW];

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int64_t q = blockIdx.x;
  const int cnt = node_rows(g, q, rows);
  const int nsteps = cnt < g.w ? cnt : g.w;
  const int64_t row = rows[t];

  double a[kW];
#pragma unroll
  for (int j = 0; j < kW; ++j)
    a[j] = (row >= 0 && j < g.w) ? A[row * lda + g.j0 + j] : 0.0;
  for (int j = t; j < kW * (kW + 1); j += kL) (&T[0][0])[j] = 0.0;
  if (t < kW) taus[t] = 0.0;
  __syncthreads();

#pragma unroll
  for (int c = 0; c <= kW; ++c) {
    if (c <= nsteps) {
      // static indices clamped for the first and the closing step
      const int cm1 = c > 0 ? c - 1 : 0;
      const int cc0 = c < kW ? c : kW - 1;
      const double yprev = t > cm1 ? a[cm1] : (t == cm1 ? 1.0 : 0.0);
      double v[kW];
#pragma unroll
      for (int j = 0; j < kW; ++j) {
        double val = 0.0;
        if (j + 1 < c) {
          // z_{c-1}[j] = y_j . y_{c-1}, y_t[j] = (t>j ? a_j : t==j ? 1 : 0)
          const double yj = t > j ? a[j] : (t == j ? 1.0 : 0.0);
          val = yj * yprev;
        } else if (j >= c && c < nsteps) {
          val = t > c ? a[cc0] * a[j] : 0.0;
        }
        v[j] = val;
      }
      wave_reduce32(v, lane);
      if ((lane & 1) == 0) red[wave][lane >> 1] = v[0];
      __syncthreads();
      if (t < kW) gsum[t] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
      if (c < nsteps && t == c) {
#pragma unroll
        for (int j = 0; j < kW; ++j) rowc[j] = a[j];
      }
      __syncthreads();
      if (c >= 1 && t < c) {
        // column c-1 of T
        const int i = t;
        const int cc = c - 1;
        if (i == cc) {
          T[cc][cc] = taus[cc];
        } else {
          double s = 0.0;
          for (int l = i; l < cc; ++l) s += T[i][l] * gsum[l];
          T[i][cc] = -taus[cc] * s;
        }
      }
      if (c < nsteps) {
        const double s2 = gsum[cc0];
        const double alpha = rowc[cc0];
        double tau = 0.0, beta = alpha, scal = 0.0;
        if (s2 > 0.0) {
          const double nrm = sqrt(alpha * alpha + s2);
          beta = alpha >= 0.0 ? -nrm : nrm;
          tau = (beta - alpha) / beta;
          scal = 1.0 / (alpha - beta);
        }
        if (t > c) {
          const double vt = a[cc0] * scal;
#pragma unroll
          for (int j = 0; j < kW; ++j)
            if (j > c) a[j] -= tau * vt * (rowc[j] + scal * gsum[j]);
          a[cc0] = vt;
        } else if (t == c) {
#pragma unroll
          for (int j = 0; j < kW; ++j)
            if (j > c) a[j] -= tau * (rowc[j] + scal * gsum[j]);
          a[cc0] = beta;
        }
        if (t == 0) taus[cc0] = tau;
      }
      // the T update above reads taus[c-1] written in the previous step and
      // gsum of this step; the next step rewrites gsum only after its first
      // barrier, which every thread reaches after finishing this step.
    }
  }
  __syncthreads();

  // reflectors (unit lower trapezoid), T, and the triangle in the head rows
  double* Y = Yws + q * (kL * kW);
#pragma unroll
  for (int j = 0; j < kW; ++j) {
    double y = 0.0;
    if (j < nsteps && t < cnt) y = t > j ? a[j] : (t == j ? 1.0 : 0.0);
    Y[t * kW + j] = y;
  }
  double* Tg = Tws + q * (kW * kW);
  for (int e = t; e < kW * kW; e += kL) {
    const int i = e / kW, j = e % kW;
    Tg[e] = (i < nsteps && j < nsteps) ? T[i][j] : 0.0;
  }
  if (row >= 0) {
#pragma unroll
    for (int j = 0; j < kW; ++j)
      if (j < g.w) A[row * lda + g.j0 + j] = (t < nsteps && j >= t) ? a[j] : 0.0;
  }
}

// C <- (I - Y T^T Y^T) C on the node's rows, 64 trailing columns per block.
constexpr int kUC = 64;

__global__ void __launch_bounds__(kL)
    qr_update_kernel(double* __restrict__ A, int64_t lda, NodeGeom g,
                     const double* __restrict__ Yws,
                     const double* __restrict__ Tws, int64_t col0,
                     int64_t ncols) {
  __shared__ int64_t rows[kL];
  __shared__ double Ys[kL][kW];
  __shared__ double Wp[4][kW][kUC];
  __shared__ double Ts[kW][kW];

  const int t = threadIdx.x;
  const int lc = t & 63;
  const int grp = t >> 6;
  const int64_t q = blockIdx.x;
  const int cnt = node_rows(g, q, rows);
  const double* Y = Yws + q * (kL * kW);
  for (int e = t; e < kL * kW; e += kL) (&Ys[0][0])[e] = Y[e];
  const double* Tg = Tws + q * (kW * kW);
  for (int e = t; e < kW * kW; e += kL) (&Ts[0][0])[e] = Tg[e];
  __syncthreads();

  const int64_t col = col0 + static_cast<int64_t>(blockIdx.y) * kUC + lc;
  const bool cok = col < col0 + ncols;

  double w1[kW];
#pragma unroll
  for (int i = 0; i < kW; ++i) w1[i] = 0.0;
  const int rlo = grp * 64;
  const int rhi = cnt < rlo + 64 ? cnt : rlo + 64;
  if (cok) {
#pragma unroll 2
    for (int tt = rlo; tt < rhi; ++tt) {
      const double cv = A[rows[tt] * lda + col];
#pragma unroll
      for (int i = 0; i < kW; ++i) w1[i] += Ys[tt][i] * cv;
    }
  }
#pragma unroll
  for (int i = 0; i < kW; ++i) Wp[grp][i][lc] = w1[i];
  __syncthreads();
  // W1 = sum over the four row groups (kept in Wp[0])
#pragma unroll
  for (int ii = 0; ii < kW / 4; ++ii) {
    const int i = grp * (kW / 4) + ii;
    Wp[0][i][lc] = Wp[0][i][lc] + Wp[1][i][lc] + Wp[2][i][lc] + Wp[3][i][lc];
  }
  __syncthreads();
  // W2 = T^T W1 -> Wp[1]
#pragma unroll
  for (int ii = 0; ii < kW / 4; ++ii) {
    const int i = grp * (kW / 4) + ii;
    double s = 0.0;
    for (int l = 0; l <= i; ++l) s += Ts[l][i] * Wp[0][l][lc];
    Wp[1][i][lc] = s;
  }
  __syncthreads();
  double w2[kW];
#pragma unroll
  for (int i = 0; i < kW; ++i) w2[i] = Wp[1][i][lc];
  if (cok) {
#pragma unroll 2
    for (int tt = rlo; tt < rhi; ++tt) {
      double u = 0.0;
#pragma unroll
      for (int i = 0; i < kW; ++i) u += Ys[tt][i] * w2[i];
      double* p = A + rows[tt] * lda + col;
      *p = *p - u;
    }
  }
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

size_t qr_scratch_bytes(int64_t m, int64_t d) {
  (void)d;
  const int64_t leaves = (m + kL - 1) / kL;
  return static_cast<size_t>(leaves) * (kL * kW + kW * kW) * sizeof(double);
}

void qr_factor(double* a, int64_t m, int64_t d, double* r_out, void* scratch,
               hipStream_t s) {
  const int64_t leaves_max = (m + kL - 1) / kL;
  double* Yws = static_cast<double*>(scratch);
  double* Tws = Yws + leaves_max * (kL * kW);
  for (int64_t j0 = 0; j0 < d; j0 += kW) {
    NodeGeom g;
    g.m = m;
    g.j0 = j0;
    g.w = static_cast<int>(d - j0 < kW ? d - j0 : kW);
    g.nleaves = (m - j0 + kL - 1) / kL;
    g.level = 0;
    g.child_span = 0;
    g.child_leaves = 0;
    g.nchild = 0;
    int64_t nodes = g.nleaves;
    int64_t span = kL;       // rows spanned by a node of the current level
    int64_t leaves_per = 1;  // leaves per node of the current level
    const int64_t tc0 = j0 + g.w;
    const int64_t tcols = d - tc0;
    for (;;) {
      prof_begin(kKQrNode, s);
      qr_node_kernel<<<static_cast<unsigned>(nodes), kL, 0, s>>>(a, d, g, Yws,
                                                                 Tws);
      prof_end(kKQrNode, s);
      if (tcols > 0) {
        dim3 grid(static_cast<unsigned>(nodes),
                  static_cast<unsigned>((tcols + kUC - 1) / kUC));
        prof_begin(kKQrUpdate, s);
        qr_update_kernel<<<grid, kL, 0, s>>>(a, d, g, Yws, Tws, tc0, tcols);
        prof_end(kKQrUpdate, s);
      }
      if (nodes == 1) break;
      g.level += 1;
      g.child_span = span;
      g.child_leaves = leaves_per;
      g.nchild = nodes;
      span *= kF;
      leaves_per *= kF;
      nodes = (nodes + kF - 1) / kF;
    }
  }
  const int64_t dd = d * d;
  prof_begin(kKQrExtract, s);
  extract_r_kernel<<<static_cast<unsigned>((dd + 255) / 256), 256, 0, s>>>(
      a, d, d, r_out);
  prof_end(kKQrExtract, s);
}

void launch_diag_stats(const double* r, int64_t d, double* out,
                       hipStream_t s) {
  diag_stats_kernel<<<1, 256, 0, s>>>(r, d, out);
}

}  // namespace slso
