// Row scores l_i = ||x_i M||^2 (Algorithm 2 step 4 / Algorithm 3 step 5),
// with the product x_i M never written out: each workgroup keeps a 64-row x
// 64-column tile of X M in registers and reduces its squares.
//
// Precision: FP32 input is multiplied with the FP32 copy of M in FP32, the
// contraction over d is accumulated in FP32 within 32-wide chunks and in FP64
// across chunks (plain FP32 accumulation over d = 784 loses ~8e-6 relative
// on cancellation-prone rows; chunking keeps it ~3e-6). FP64 input uses FP64
// throughout. CSR rows gather the FP32 rows of M and accumulate in FP64.
#include "internal.h"

namespace slso {
namespace {

constexpr int kRows = 64;   // rows per workgroup
constexpr int kCols = 64;   // columns of M per workgroup
constexpr int kChunk = 32;  // contraction chunk

template <typename T>
struct Ld;
template <>
struct Ld<float> {
  using acc = float;
  __device__ static float get(const float* p, int64_t i) { return p[i]; }
};
template <>
struct Ld<uint16_t> {
  using acc = float;
  __device__ static float get(const uint16_t* p, int64_t i) {
    return bf16_to_f32(p[i]);
  }
};
template <>
struct Ld<uint8_t> {  // FP8-e4m3 code; the column scale is folded into M
  using acc = float;
  __device__ static float get(const uint8_t* p, int64_t i) {
    return e4m3_to_f32(p[i]);
  }
};
template <>
struct Ld<double> {
  using acc = double;
  __device__ static double get(const double* p, int64_t i) { return p[i]; }
};

template <typename T, typename MT>
__global__ void __launch_bounds__(256)
    score_dense_kernel(const T* __restrict__ x, int64_t n, int64_t d,
                       int64_t ld, const MT* __restrict__ m, int64_t k,
                       double* __restrict__ partial, float* __restrict__ out) {
  using A = typename Ld<T>::acc;
  __shared__ A Xs[kRows][kChunk + 1];
  __shared__ A Ms[kChunk][kCols];
  const int t = threadIdx.x;
  const int tr = t >> 4;   // rows 4*tr .. 4*tr+3
  const int tc = t & 15;   // cols 4*tc .. 4*tc+3
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * kRows;
  const int64_t col0 = static_cast<int64_t>(blockIdx.y) * kCols;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;

  for (int64_t c0 = 0; c0 < d; c0 += kChunk) {
    // stage X (64 x 32) and M (32 x 64)
    for (int e = t; e < kRows * kChunk; e += 256) {
      const int i = e / kChunk, l = e % kChunk;
      const int64_t row = row0 + i, col = c0 + l;
      Xs[i][l] = (row < n && col < d) ? Ld<T>::get(x, row * ld + col) : A(0);
    }
    for (int e = t; e < kChunk * kCols; e += 256) {
      const int l = e / kCols, j = e % kCols;
      const int64_t dr = c0 + l, mc = col0 + j;
      Ms[l][j] = (dr < d && mc < k) ? static_cast<A>(m[dr * k + mc]) : A(0);
    }
    __syncthreads();
    A part[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) part[i][j] = A(0);
#pragma unroll 8
    for (int l = 0; l < kChunk; ++l) {
      A xv[4], mv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) xv[i] = Xs[4 * tr + i][l];
#pragma unroll
      for (int j = 0; j < 4; ++j) mv[j] = Ms[l][4 * tc + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) part[i][j] += xv[i] * mv[j];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] += static_cast<double>(part[i][j]);
    __syncthreads();
  }
  // sum of squares over this tile's columns; the 16 threads sharing rows are
  // 16 consecutive lanes
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) s += acc[i][j] * acc[i][j];
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    const int64_t row = row0 + 4 * tr + i;
    if (tc == 0 && row < n) {
      if (partial)
        partial[static_cast<int64_t>(blockIdx.y) * n + row] = s;
      else
        out[row] = static_cast<float>(s);
    }
  }
}

__global__ void sum_partials_kernel(const double* __restrict__ partial,
                                    int64_t n, int64_t tiles,
                                    float* __restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t t = 0; t < tiles; ++t) s += partial[t * n + i];
  out[i] = static_cast<float>(s);
}

// One wave per CSR row; lanes own columns of M (64 at a time).
__global__ void __launch_bounds__(256)
    score_csr_kernel(const int64_t* __restrict__ row_ptr,
                     const int32_t* __restrict__ col_idx,
                     const float* __restrict__ val, int64_t n,
                     const float* __restrict__ m, int64_t k,
                     float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t row = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const int64_t e0 = row_ptr[row], e1 = row_ptr[row + 1];
  double tot = 0.0;
  for (int64_t c0 = 0; c0 < k; c0 += 64) {
    const int64_t c = c0 + lane;
    double y = 0.0;
    if (c < k) {
      for (int64_t e = e0; e < e1; ++e) {
        const int64_t j = col_idx[e];
        y += static_cast<double>(val[e]) * static_cast<double>(m[j * k + c]);
      }
    }
    tot += y * y;
  }
  tot = wave_sum_d(tot);
  if (lane == 0) out[row] = static_cast<float>(tot);
}

}  // namespace

size_t scores_partial_bytes(int64_t n, int64_t k, int format) {
  const int64_t tiles = (k + kCols - 1) / kCols;
  if (format == 1 || tiles <= 1) return 0;
  return static_cast<size_t>(tiles * n) * sizeof(double);
}

void launch_scores(const void* x, int dtype, int format, int64_t n, int64_t d,
                   int64_t ld, const int64_t* row_ptr, const int32_t* col_idx,
                   const float* col_scale, const float* row_scale,
                   const double* m64, const float* m32, int64_t k,
                   float* scores, hipStream_t s, double* partial) {
  (void)m64;
  (void)col_scale;
  (void)row_scale;
  if (n <= 0) return;
  if (format == 1) {
    prof_begin(kKScore, s);
    score_csr_kernel<<<static_cast<unsigned>((n + 3) / 4), 256, 0, s>>>(
        row_ptr, col_idx, static_cast<const float*>(x), n, m32, k, scores);
    prof_end(kKScore, s);
    return;
  }
  const int64_t tiles = (k + kCols - 1) / kCols;
  dim3 grid(static_cast<unsigned>((n + kRows - 1) / kRows),
            static_cast<unsigned>(tiles));
  double* part = tiles > 1 ? partial : nullptr;
  switch (dtype) {
    case 0:
      prof_begin(kKScore, s);
      score_dense_kernel<double, double><<<grid, 256, 0, s>>>(
          static_cast<const double*>(x), n, d, ld, m64, k, part, scores);
      prof_end(kKScore, s);
      break;
    case 1:
      prof_begin(kKScore, s);
      score_dense_kernel<float, float><<<grid, 256, 0, s>>>(
          static_cast<const float*>(x), n, d, ld, m32, k, part, scores);
      prof_end(kKScore, s);
      break;
    case 3:
      prof_begin(kKScore, s);
      score_dense_kernel<uint8_t, float><<<grid, 256, 0, s>>>(
          static_cast<const uint8_t*>(x), n, d, ld, m32, k, part, scores);
      prof_end(kKScore, s);
      break;
    case 2:
      prof_begin(kKScore, s);
      score_dense_kernel<uint16_t, float><<<grid, 256, 0, s>>>(
          static_cast<const uint16_t*>(x), n, d, ld, m32, k, part, scores);
      prof_end(kKScore, s);
      break;
    default:
      break;
  }
  if (part)
    sum_partials_kernel<<<static_cast<unsigned>((n + 255) / 256), 256, 0, s>>>(
        part, n, tiles, scores);
}

}  // namespace slso
