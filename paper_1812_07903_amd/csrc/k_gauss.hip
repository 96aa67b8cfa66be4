// Gaussian sketch S X of FP32 input (Sec. 2.1; Algorithm 2 step 1, the plain
// FP32 path) and the Gram matrix X^T X of the refinement pass; the BF16 and
// FP8 paths of both live in k_gauss_q.hip, whose partial sums the reduction
// kernels here also finish.
//
// Entries of S = G / sqrt(r): G[j][i] is produced on the fly from the seed
// (one Philox4x32-10 block per four consecutive data rows i of one sketch
// row j, FP32 Box-Muller with polynomial logarithm, Newton square root and
// Taylor sine/cosine, every operation separately rounded so the value is
// reproducible exactly), multiplied on v_mfma_f32_32x32x2_f32. Sums are FP32
// within one workgroup's slice of rows (split-K) and FP64 across slices, in a
// fixed order, so the result is deterministic.
//
// Tiling: a workgroup of eight waves owns 256 sketch rows x 256 columns;
// wave w owns rows 32 w .. 32 w + 31 (8 accumulator tiles of 32 x 32). Per
// step of 16 data rows, the X tile (16 x 256) is staged in LDS and each lane
// generates its own 8 entries of G (two Philox blocks). The MFMA K-slots are
// permuted (slot 2s + h <-> data row 8h + s) so that each lane's 8 entries of
// G are 8 consecutive data rows.
#include "internal.h"

namespace slso {
namespace {

typedef float f16v __attribute__((ext_vector_type(16)));

// ---- the FP32 Gaussian generator -------------------------------------------
#pragma clang fp contract(off)
__device__ __forceinline__ void box_muller_f32(uint32_t wa, uint32_t wb,
                                               float& z0, float& z1) {
  const float u1 = static_cast<float>((wa >> 8) + 1u) * 0x1p-24f;
  const float u2 = static_cast<float>(wb >> 8) * 0x1p-24f;
  const uint32_t bits = __float_as_uint(u1);
  int e = static_cast<int>(bits >> 23) - 127;
  float m = __uint_as_float((bits & 0x7FFFFFu) | 0x3F800000u);
  if (m > 1.4142135381698608f) {
    m = m * 0.5f;
    e += 1;
  }
  const float t = m - 1.0f;
  float q = -0.10134056955575943f;
  q = q * t;
  q = q + 0.1623418927192688f;
  q = q * t;
  q = q + -0.17247013747692108f;
  q = q * t;
  q = q + 0.19898565113544464f;
  q = q * t;
  q = q + -0.24970071017742157f;
  q = q * t;
  q = q + 0.33335113525390625f;
  q = q * t;
  q = q + -0.5000036358833313f;
  q = q * t;
  q = q + 0.9999999403953552f;
  const float lnm = t * q;
  float ln_u = static_cast<float>(e) * 0.6931471824645996f;
  ln_u = ln_u + lnm;
  const float L = -2.0f * ln_u;
  float y = __uint_as_float(0x5F3759DFu - (__float_as_uint(L) >> 1));
  const float hl = 0.5f * L;
  for (int it = 0; it < 3; ++it) {
    const float y2 = y * y;
    const float t2 = hl * y2;
    const float t3 = 1.5f - t2;
    y = y * t3;
  }
  const float rad = (L == 0.0f) ? 0.0f : L * y;
  const float q4 = u2 * 4.0f;
  const int k = static_cast<int>(q4);
  const float f = q4 - static_cast<float>(k);
  const float x = (f - 0.5f) * 1.5707963705062866f;
  const float x2 = x * x;
  float c = 1.0f / 40320.0f;
  c = c * x2;
  c = c + -1.0f / 720.0f;
  c = c * x2;
  c = c + 1.0f / 24.0f;
  c = c * x2;
  c = c + -0.5f;
  float cosx = c * x2;
  cosx = cosx + 1.0f;
  float s = 1.0f / 362880.0f;
  s = s * x2;
  s = s + -1.0f / 5040.0f;
  s = s * x2;
  s = s + 1.0f / 120.0f;
  s = s * x2;
  s = s + -1.0f / 6.0f;
  float sinx = s * x2;
  sinx = sinx * x;
  sinx = sinx + x;
  const float h = 0.7071067690849304f;
  const float ca = (k == 0 || k == 3) ? h : -h;
  const float sa = (k < 2) ? h : -h;
  const float p1 = ca * cosx;
  const float p2 = sa * sinx;
  const float cos_t = p1 - p2;
  const float p3 = sa * cosx;
  const float p4 = ca * sinx;
  const float sin_t = p3 + p4;
  z0 = rad * cos_t;
  z1 = rad * sin_t;
}

// G[j][4 g .. 4 g + 3] for sketch row j and data-row group g.
__device__ __forceinline__ void gauss4(uint64_t seed, uint64_t g, uint32_t j,
                                       float (&z)[4]) {
  U4 c{static_cast<uint32_t>(g), static_cast<uint32_t>(g >> 32), j,
       static_cast<uint32_t>(kStreamGaussS)};
  const U4 o = philox10(c, static_cast<uint32_t>(seed),
                        static_cast<uint32_t>(seed >> 32));
  box_muller_f32(o.x, o.y, z[0], z[1]);
  box_muller_f32(o.z, o.w, z[2], z[3]);
}
#pragma clang fp contract(on)

constexpr int kTR = 256;  // sketch rows per workgroup
constexpr int kTD = 256;  // columns per workgroup
constexpr int kKS = 16;   // data rows per step

__global__ void __launch_bounds__(512)
    gauss_sketch_kernel(const float* __restrict__ x, int64_t n, int64_t d,
                        int64_t ld, uint64_t seed, int64_t r,
                        int64_t rows_per_split, float* __restrict__ partial) {
  // XS[row][col]
  __shared__ float XS[kKS * kTD];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int l32 = lane & 31;
  const int h = lane >> 5;
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * kTR;  // sketch rows
  const int64_t col0 = static_cast<int64_t>(blockIdx.y) * kTD;
  const int64_t i_begin = static_cast<int64_t>(blockIdx.z) * rows_per_split;
  int64_t i_end = i_begin + rows_per_split;
  if (i_end > n) i_end = n;
  const int64_t jrow = row0 + wave * 32 + l32;  // this lane's sketch row
  const uint32_t jg = static_cast<uint32_t>(jrow < r ? jrow : 0);

  f16v acc[8];
#pragma unroll
  for (int ct = 0; ct < 8; ++ct)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[ct][e] = 0.0f;

  // staging assignment: thread t loads 8 consecutive columns of one row
  const int srow = t >> 5;            // 0..15
  const int scol = (t & 31) * 8;      // 0..248

  for (int64_t k0 = i_begin; k0 < i_end; k0 += kKS) {
    __syncthreads();
    {
      const int64_t gi = k0 + srow;
      const int64_t gc = col0 + scol;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool ok = gi < i_end && gc + u < d;
        XS[srow * kTD + scol + u] = ok ? x[gi * ld + gc + u] : 0.0f;
      }
    }
    __syncthreads();
    // this lane's 8 entries of G: sketch row jrow, data rows k0 + 8h + s
    float gz[8];
    {
      const uint64_t g0 = static_cast<uint64_t>(k0 + 8 * h) >> 2;
      float z4[4];
      gauss4(seed, g0, jg, z4);
#pragma unroll
      for (int s = 0; s < 4; ++s) gz[s] = z4[s];
      gauss4(seed, g0 + 1, jg, z4);
#pragma unroll
      for (int s = 0; s < 4; ++s) gz[4 + s] = z4[s];
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
#pragma unroll
      for (int ct = 0; ct < 8; ++ct) {
        const float b = XS[(8 * h + s) * kTD + ct * 32 + l32];
        acc[ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(gz[s], b, acc[ct], 0, 0, 0);
      }
    }
  }
  // partial[split][j][c]; accumulator register e of lane l holds
  // D[(e % 4) + 8 (e / 4) + 4 (l / 32)][l % 32]
  float* P = partial + static_cast<int64_t>(blockIdx.z) * r * d;
#pragma unroll
  for (int ct = 0; ct < 8; ++ct) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int64_t j = row0 + wave * 32 + (e % 4) + 8 * (e / 4) + 4 * h;
      const int64_t c = col0 + ct * 32 + l32;
      if (j < r && c < d) P[j * d + c] = acc[ct][e];
    }
  }
}

// sx[j][c] = (sum_s partial[s][j][c]) * colscale[c] * dscale[c] / sqrt(r)
__global__ void gauss_reduce_kernel(const float* __restrict__ partial,
                                    int64_t splits, int64_t r, int64_t d,
                                    const float* __restrict__ col_scale,
                                    const double* __restrict__ dscale,
                                    double inv_sqrt_r, double* __restrict__ sx) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= r * d) return;
  const int64_t c = e % d;
  double s = 0.0;
  for (int64_t p = 0; p < splits; ++p) s += static_cast<double>(partial[p * r * d + e]);
  double f = inv_sqrt_r;
  if (col_scale) f *= static_cast<double>(col_scale[c]);
  s = s * f;
  if (dscale) s *= dscale[c];
  sx[e] = s;
}

// G[i][j] = D_i D_j cs_i cs_j sum_s partial[s][min][max] (symmetric fill)
__global__ void gram_reduce_kernel(const float* __restrict__ partial,
                                   int64_t splits, int64_t d,
                                   const float* __restrict__ col_scale,
                                   const double* __restrict__ dscale,
                                   double* __restrict__ g) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= d * d) return;
  int64_t i = e / d, j = e % d;
  // the tile that holds (i, j) has block(i) <= block(j); swap otherwise
  if (i / kTD > j / kTD) {
    const int64_t tmp = i;
    i = j;
    j = tmp;
  }
  double s = 0.0;
  for (int64_t p = 0; p < splits; ++p)
    s += static_cast<double>(partial[p * d * d + i * d + j]);
  if (col_scale)
    s *= static_cast<double>(col_scale[i]) * static_cast<double>(col_scale[j]);
  if (dscale) s *= dscale[i] * dscale[j];
  g[e] = s;
}

// ---- Gram matrix of FP32 input on the FP64 MFMA ------------------------------
// Products of FP32 values are exact in FP64 and the sums are FP64, so G is
// accurate to FP64 rounding whatever the conditioning of X (the FP32-
// accumulated form loses about kappa(X)^2 * 1e-7 in the refined R).
// Output tile 64 x 64 of column blocks (a, b), a <= b; four waves, wave w
// owns the 32 x 32 quarter (w / 2, w % 2) as 2 x 2 blocks of
// v_mfma_f64_16x16x4f64 (A lane l = A[l % 16][l / 16], B lane l =
// B[l / 16][l % 16], accumulator v of lane l = D[4 v + l / 16][l % 16]).
constexpr int kGT = 64;   // tile edge
constexpr int kGK = 16;   // data rows per step
constexpr int kGP = 80;   // padded LDS row (doubles)

__global__ void __launch_bounds__(256)
    gram_f64_kernel(const float* __restrict__ x, int64_t n, int64_t d,
                    int64_t ld, int nb, int64_t rows_per_split,
                    double* __restrict__ partial) {
  typedef double f64x4 __attribute__((ext_vector_type(4)));
  __shared__ double XA[kGK][kGP];
  __shared__ double XB[kGK][kGP];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  int ta = 0, rem = static_cast<int>(blockIdx.x);
  while (rem >= nb - ta) {
    rem -= nb - ta;
    ++ta;
  }
  const int tb = ta + rem;
  const bool diag = ta == tb;
  const int64_t a0 = static_cast<int64_t>(ta) * kGT;
  const int64_t b0 = static_cast<int64_t>(tb) * kGT;
  const int64_t i_begin = static_cast<int64_t>(blockIdx.z) * rows_per_split;
  int64_t i_end = i_begin + rows_per_split;
  if (i_end > n) i_end = n;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;

  f64x4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[bi][bj][v] = 0.0;

  // staging: thread t loads 4 consecutive columns of row t / 16
  const int srow = t >> 4;
  const int scol = (t & 15) * 4;
  for (int64_t k0 = i_begin; k0 < i_end; k0 += kGK) {
    __syncthreads();
    const int64_t gi = k0 + srow;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t ca = a0 + scol + u, cb = b0 + scol + u;
      XA[srow][scol + u] =
          (gi < i_end && ca < d) ? static_cast<double>(x[gi * ld + ca]) : 0.0;
      if (!diag)
        XB[srow][scol + u] =
            (gi < i_end && cb < d) ? static_cast<double>(x[gi * ld + cb]) : 0.0;
    }
    __syncthreads();
    const double (*B)[kGP] = diag ? XA : XB;
#pragma unroll
    for (int kk = 0; kk < kGK; kk += 4) {
      double av[2], bv[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        av[q] = XA[kk + lk][wr + 16 * q + lr];
        bv[q] = B[kk + lk][wc + 16 * q + lr];
      }
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
          acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bi], bv[bj],
                                                            acc[bi][bj], 0, 0, 0);
    }
  }
  double* P = partial + static_cast<int64_t>(blockIdx.z) * d * d;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = a0 + wr + 16 * bi + 4 * v + lk;
        const int64_t j = b0 + wc + 16 * bj + lr;
        if (i < d && j < d) P[i * d + j] = acc[bi][bj][v];
      }
}

// G[i][j] = D_i D_j sum_s partial[s][i'][j'] with (i', j') the entry of the
// computed tile (block(i') <= block(j'))
__global__ void gram_reduce_f64_kernel(const double* __restrict__ partial,
                                       int64_t splits, int64_t d,
                                       const double* __restrict__ dscale,
                                       double* __restrict__ g) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= d * d) return;
  int64_t i = e / d, j = e % d;
  if (i / kGT > j / kGT) {
    const int64_t tmp = i;
    i = j;
    j = tmp;
  }
  double s = 0.0;
  for (int64_t p = 0; p < splits; ++p) s += partial[p * d * d + i * d + j];
  if (dscale) s *= dscale[i] * dscale[j];
  g[e] = s;
}

__global__ void gauss_entries_kernel(uint64_t seed, int64_t r, int64_t n,
                                     int64_t row0, float* __restrict__ out) {
  // out[j * n + i] = G[j][row0 + i]
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= r * n) return;
  const int64_t j = e / n, i = row0 + (e % n);
  float z[4];
  gauss4(seed, static_cast<uint64_t>(i) >> 2, static_cast<uint32_t>(j), z);
  out[e] = z[i & 3];
}

inline int64_t split_rows(int64_t n, int64_t max_rows, int64_t* splits) {
  int64_t s = (n + max_rows - 1) / max_rows;
  if (s < 1) s = 1;
  int64_t per = (n + s - 1) / s;
  per = (per + kKS - 1) / kKS * kKS;
  *splits = (n + per - 1) / per;
  return per;
}

constexpr int64_t kMaxRowsPerSplit = 65536;

}  // namespace

size_t gauss_partial_bytes(int64_t n, int64_t r, int64_t d, int dtype) {
  if (gauss_q_dtype(dtype)) return gauss_q_partial_bytes(n, r, d);
  int64_t splits;
  split_rows(n, kMaxRowsPerSplit, &splits);
  return static_cast<size_t>(splits * r * d) * sizeof(float);
}

void launch_gauss_sketch(const void* x, int dtype, int64_t n, int64_t d,
                         int64_t ld, const float* col_scale, uint64_t seed,
                         int64_t r, const double* dscale, float* partial,
                         double* sx, hipStream_t s) {
  int64_t splits;
  if (gauss_q_dtype(dtype)) {
    launch_gauss_q_sketch(x, dtype, n, d, ld, seed, r, partial, &splits,
                          col_scale, nullptr, nullptr, s);
  } else {
    const int64_t per = split_rows(n, kMaxRowsPerSplit, &splits);
    dim3 grid(static_cast<unsigned>((r + kTR - 1) / kTR),
              static_cast<unsigned>((d + kTD - 1) / kTD),
              static_cast<unsigned>(splits));
    prof_begin(kKGaussSketch, s);
    gauss_sketch_kernel<<<grid, 512, 0, s>>>(static_cast<const float*>(x), n, d,
                                             ld, seed, r, per, partial);
    prof_end(kKGaussSketch, s);
  }
  const int64_t tot = r * d;
  gauss_reduce_kernel<<<static_cast<unsigned>((tot + 255) / 256), 256, 0, s>>>(
      partial, splits, r, d, dtype == 3 ? col_scale : nullptr, dscale,
      1.0 / sqrt(static_cast<double>(r)), sx);
}

void launch_gauss_sketch_eq(const void* x, int dtype, int64_t n, int64_t d,
                            int64_t ld, const float* col_scale, uint64_t seed,
                            int64_t r, uint64_t* colmax_bits, int* nonfinite,
                            double* dscale_out, float* partial, double* sx,
                            hipStream_t s) {
  launch_fill_u64(colmax_bits, d, 0, s);
  int64_t splits;
  launch_gauss_q_sketch(x, dtype, n, d, ld, seed, r, partial, &splits,
                        col_scale, colmax_bits, nonfinite, s);
  launch_colscale(colmax_bits, d, dscale_out, s);
  const int64_t tot = r * d;
  gauss_reduce_kernel<<<static_cast<unsigned>((tot + 255) / 256), 256, 0, s>>>(
      partial, splits, r, d, dtype == 3 ? col_scale : nullptr, dscale_out,
      1.0 / sqrt(static_cast<double>(r)), sx);
}

// FP64 Gram of FP32 input: enough row splits for about 2048 workgroups,
// each of at least 1024 rows
inline int64_t gram_f64_split(int64_t n, int64_t d, int64_t* splits) {
  const int64_t nb = (d + kGT - 1) / kGT;
  const int64_t tiles = nb * (nb + 1) / 2;
  int64_t want = (2048 + tiles - 1) / tiles;
  const int64_t cap = (n + 1023) / 1024;
  if (want > cap) want = cap;
  if (want < 1) want = 1;
  int64_t per = (n + want - 1) / want;
  per = (per + kGK - 1) / kGK * kGK;
  *splits = (n + per - 1) / per;
  return per;
}

size_t gram_partial_bytes(int64_t n, int64_t d, int dtype) {
  if (gauss_q_dtype(dtype)) return gram_q_partial_bytes(n, d);
  int64_t splits;
  if (dtype == 1) {
    gram_f64_split(n, d, &splits);
    return static_cast<size_t>(splits * d * d) * sizeof(double);
  }
  split_rows(n, kMaxRowsPerSplit, &splits);
  return static_cast<size_t>(splits * d * d) * sizeof(float);
}

void launch_gram(const void* x, int dtype, int64_t n, int64_t d, int64_t ld,
                 const float* col_scale, const double* dscale, void* scratch,
                 double* g, hipStream_t s) {
  int64_t splits;
  if (dtype == 1) {
    const int64_t per = gram_f64_split(n, d, &splits);
    const int nb = static_cast<int>((d + kGT - 1) / kGT);
    dim3 grid(static_cast<unsigned>(nb * (nb + 1) / 2), 1,
              static_cast<unsigned>(splits));
    double* partial = static_cast<double*>(scratch);
    prof_begin(kKGram, s);
    gram_f64_kernel<<<grid, 256, 0, s>>>(static_cast<const float*>(x), n, d, ld,
                                         nb, per, partial);
    prof_end(kKGram, s);
    gram_reduce_f64_kernel<<<static_cast<unsigned>((d * d + 255) / 256), 256, 0,
                             s>>>(partial, splits, d, dscale, g);
    return;
  }
  float* partial = static_cast<float*>(scratch);
  launch_gram_q(x, dtype, n, d, ld, partial, &splits, s);
  gram_reduce_kernel<<<static_cast<unsigned>((d * d + 255) / 256), 256, 0, s>>>(
      partial, splits, d, dtype == 3 ? col_scale : nullptr, dscale, g);
}

void launch_gauss_entries(uint64_t seed, int64_t r, int64_t n, int64_t row0,
                          float* out, hipStream_t s) {
  const int64_t tot = r * n;
  if (tot <= 0) return;
  gauss_entries_kernel<<<static_cast<unsigned>((tot + 255) / 256), 256, 0, s>>>(
      seed, r, n, row0, out);
}

}  // namespace slso
