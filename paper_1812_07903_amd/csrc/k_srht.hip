// SRHT sketch S X = (1/sqrt(r)) P H D X (the randomized Hadamard transform of
// Sec. 2.1 and Table 1): D the row signs (parity of the polynomial hash of
// stream 7), X padded with zero rows to n' = 2^ceil(log2 n), H the
// unnormalised Walsh-Hadamard transform in Sylvester order, P the r Hadamard
// rows with the smallest stream-8 words (ties by ascending row), in that
// order; the 1/sqrt(r) (and the column factors) are applied once at the end.
//
// The transform runs in passes of up to 8 stages. A workgroup owns the 2^k
// rows that differ only in the pass's bits (row base + m 2^s, m < 2^k) and 32
// columns, keeps them in LDS and applies the stages in increasing order,
// each butterfly forming (y_a + y_b, y_a - y_b) for rows a < b = a + 2^t, so
// every value is the one of the stage-by-stage definition. The first pass
// reads X (with the signs, zero past row n), the last one writes only the
// sampled rows, straight into the sketch.
#include <cmath>

#include "internal.h"

namespace slso {
namespace {

constexpr int kHB = 8;   // stages per pass
constexpr int kHC = 32;  // columns per workgroup

template <typename T>
struct SrhtIn;
template <>
struct SrhtIn<double> {
  __device__ static double get(const double* p, int64_t i) { return p[i]; }
};
template <>
struct SrhtIn<float> {
  __device__ static double get(const float* p, int64_t i) {
    return static_cast<double>(p[i]);
  }
};
template <>
struct SrhtIn<uint16_t> {
  __device__ static double get(const uint16_t* p, int64_t i) {
    return static_cast<double>(bf16_to_f32(p[i]));
  }
};
template <>
struct SrhtIn<uint8_t> {  // FP8-e4m3 code (the column scale is applied apart)
  __device__ static double get(const uint8_t* p, int64_t i) {
    return static_cast<double>(e4m3_to_f32(p[i]));
  }
};

__global__ void srht_keys_kernel(uint64_t seed, int64_t n2, uint32_t* keys) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n2) return;
  U4 c;
  c.x = static_cast<uint32_t>(i);
  c.y = static_cast<uint32_t>(static_cast<uint64_t>(i) >> 32);
  c.z = 0u;
  c.w = kStreamSrhtRows;
  keys[i] = philox10(c, static_cast<uint32_t>(seed),
                     static_cast<uint32_t>(seed >> 32)).x;
}

__global__ void srht_tmap_kernel(const uint32_t* __restrict__ order, int64_t r,
                                 int32_t* __restrict__ tmap) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < r) tmap[order[t]] = static_cast<int32_t>(t);
}

// One pass over the stages s .. s + k - 1 (k <= 8) for row set blockIdx.x and
// columns 32 blockIdx.y ..
template <typename T, bool kFirst, bool kLast>
__global__ void __launch_bounds__(256)
    fwht_pass_kernel(const T* __restrict__ x, int64_t n, int64_t ld,
                     HashCoeffs hs, const double* __restrict__ yin,
                     double* __restrict__ yout, int64_t n2, int64_t d, int s,
                     int k, const int32_t* __restrict__ tmap, double cscale,
                     const double* __restrict__ colfac, double* __restrict__ sx) {
  __shared__ double Y[1 << kHB][kHC + 1];
  __shared__ double sgn[1 << kHB];
  const int t = threadIdx.x, c = t % kHC, g = t / kHC;  // 8 row groups
  const int rows = 1 << k;
  const int64_t q = blockIdx.x;
  const int64_t lo = q & ((int64_t{1} << s) - 1), hi = q >> s;
  const int64_t base = (hi << (s + k)) | lo;
  const int64_t col = static_cast<int64_t>(blockIdx.y) * kHC + c;
  const bool okc = col < d;
  if (kFirst) {
    // the rows' signs, once per row (zero past n)
    for (int m = t; m < rows; m += 256) {
      const int64_t row = base + (static_cast<int64_t>(m) << s);
      sgn[m] = row >= n ? 0.0
               : ((poly61(hs, static_cast<uint64_t>(row)) & 1u) ? -1.0 : 1.0);
    }
    __syncthreads();
  }
  // load without branches (a row past the set, past n or a column past d
  // reads a clamped address and becomes zero), every load issued before any
  // is stored, so they are in flight together
  constexpr int kPer = (1 << kHB) / (256 / kHC);  // rows per thread
  double v[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int m = g + (256 / kHC) * u;
    const int mm = m < rows ? m : rows - 1;
    const int64_t row = base + (static_cast<int64_t>(mm) << s);
    if (kFirst) {
      const bool ok = okc && row < n;
      v[u] = SrhtIn<T>::get(x, ok ? row * ld + col : 0);
    } else {
      v[u] = yin[okc ? row * d + col : 0];
    }
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int m = g + (256 / kHC) * u;
    if (m < rows) {
      const int64_t row = base + (static_cast<int64_t>(m) << s);
      if (kFirst)
        Y[m][c] = (okc && row < n) ? sgn[m] * v[u] : 0.0;
      else
        Y[m][c] = okc ? v[u] : 0.0;
    }
  }
  __syncthreads();
  for (int b = 0; b < k; ++b) {
    const int h = 1 << b;
    for (int p = g; p < rows / 2; p += 256 / kHC) {
      const int m = ((p >> b) << (b + 1)) | (p & (h - 1));
      const double a = Y[m][c], e = Y[m + h][c];
      Y[m][c] = a + e;
      Y[m + h][c] = a - e;
    }
    __syncthreads();
  }
  if (!okc) return;
  const double cf = kLast && colfac ? colfac[col] : 1.0;
  for (int m = g; m < rows; m += 256 / kHC) {
    const int64_t row = base + (static_cast<int64_t>(m) << s);
    if (kLast) {
      const int32_t tt = tmap[row];
      if (tt >= 0) sx[static_cast<int64_t>(tt) * d + col] = Y[m][c] * cscale * cf;
    } else {
      yout[row * d + col] = Y[m][c];
    }
  }
}

// A full pass of 8 stages with few LDS trips: thread (g, c) first holds the
// 32 consecutive rows 32 g .. 32 g + 31 of column c and applies stages 0-4 in
// registers; through LDS, thread (l, cc) then holds rows l + 32 v (v < 8) of
// columns cc + 8 w (w < 4) and applies stages 5-7; back through LDS for
// coalesced stores. The stages still run in increasing order, on the same
// pairs, so the values are those of fwht_pass_kernel.
template <typename T, bool kFirst, bool kLast>
__global__ void __launch_bounds__(256)
    fwht8_kernel(const T* __restrict__ x, int64_t n, int64_t ld,
                 HashCoeffs hs, const double* __restrict__ yin,
                 double* __restrict__ yout, int64_t d, int s,
                 const int32_t* __restrict__ tmap, double cscale,
                 const double* __restrict__ colfac, double* __restrict__ sx) {
  __shared__ double Y[256][kHC + 1];
  __shared__ double sgn[256];
  const int t = threadIdx.x;
  const int g = t / kHC, c = t % kHC;      // layout A
  const int l = t % 32, cc = t / 32;       // layout B
  const int64_t q = blockIdx.x;
  const int64_t lo = q & ((int64_t{1} << s) - 1), hi = q >> s;
  const int64_t base = (hi << (s + 8)) | lo;
  const int64_t col0 = static_cast<int64_t>(blockIdx.y) * kHC;
  const int64_t col = col0 + c;
  const bool okc = col < d;
  if (kFirst) {
    const int64_t row = base + (static_cast<int64_t>(t) << s);
    sgn[t] = row >= n ? 0.0
             : ((poly61(hs, static_cast<uint64_t>(row)) & 1u) ? -1.0 : 1.0);
  }
  double v[32];
#pragma unroll
  for (int u = 0; u < 32; ++u) {
    const int64_t row = base + (static_cast<int64_t>(32 * g + u) << s);
    if (kFirst) {
      const bool ok = okc && row < n;
      v[u] = SrhtIn<T>::get(x, ok ? row * ld + col : 0);
    } else {
      v[u] = yin[okc ? row * d + col : 0];
    }
  }
  if (kFirst) __syncthreads();  // sgn
#pragma unroll
  for (int u = 0; u < 32; ++u) {
    if (kFirst) {
      const int64_t row = base + (static_cast<int64_t>(32 * g + u) << s);
      v[u] = (okc && row < n) ? sgn[32 * g + u] * v[u] : 0.0;
    } else {
      v[u] = okc ? v[u] : 0.0;
    }
  }
  // stages 0-4 (row bits 0-4: inside the thread)
#pragma unroll
  for (int b = 0; b < 5; ++b) {
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      if (u & (1 << b)) continue;
      const double a = v[u], e = v[u + (1 << b)];
      v[u] = a + e;
      v[u + (1 << b)] = a - e;
    }
  }
#pragma unroll
  for (int u = 0; u < 32; ++u) Y[32 * g + u][c] = v[u];
  __syncthreads();
  // stages 5-7 (row bits 5-7) in layout B
  double z[8][4];
#pragma unroll
  for (int vv = 0; vv < 8; ++vv)
#pragma unroll
    for (int w = 0; w < 4; ++w) z[vv][w] = Y[l + 32 * vv][cc + 8 * w];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
#pragma unroll
    for (int vv = 0; vv < 8; ++vv) {
      if (vv & (1 << b)) continue;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const double a = z[vv][w], e = z[vv + (1 << b)][w];
        z[vv][w] = a + e;
        z[vv + (1 << b)][w] = a - e;
      }
    }
  }
#pragma unroll
  for (int vv = 0; vv < 8; ++vv)
#pragma unroll
    for (int w = 0; w < 4; ++w) Y[l + 32 * vv][cc + 8 * w] = z[vv][w];
  __syncthreads();
  if (!okc) return;
  const double cf = kLast && colfac ? colfac[col] : 1.0;
#pragma unroll
  for (int u = 0; u < 32; ++u) {
    const int64_t row = base + (static_cast<int64_t>(32 * g + u) << s);
    const double y = Y[32 * g + u][c];
    if (kLast) {
      const int32_t tt = tmap[row];
      if (tt >= 0) sx[static_cast<int64_t>(tt) * d + col] = y * cscale * cf;
    } else {
      yout[row * d + col] = y;
    }
  }
}

inline unsigned grid1(int64_t n, int t) {
  return static_cast<unsigned>((n + t - 1) / t);
}

template <typename T>
void run_passes(const T* x, int64_t n, int64_t d, int64_t ld,
                const HashCoeffs& hs, double* y, int64_t n2, int L,
                const int32_t* tmap, double cscale, const double* colfac,
                double* sx, hipStream_t s) {
  const unsigned gy = static_cast<unsigned>((d + kHC - 1) / kHC);
  const int passes = L == 0 ? 1 : (L + kHB - 1) / kHB;
  for (int p = 0; p < passes; ++p) {
    const int s0 = p * kHB;
    const int k = L - s0 < kHB ? L - s0 : kHB;
    const dim3 grid(static_cast<unsigned>(n2 >> k), gy);
    const bool first = p == 0, last = p == passes - 1;
    if (k == kHB) {
      if (first && last)
        fwht8_kernel<T, true, true><<<grid, 256, 0, s>>>(
            x, n, ld, hs, nullptr, nullptr, d, s0, tmap, cscale, colfac, sx);
      else if (first)
        fwht8_kernel<T, true, false><<<grid, 256, 0, s>>>(
            x, n, ld, hs, nullptr, y, d, s0, nullptr, 1.0, nullptr, nullptr);
      else if (last)
        fwht8_kernel<double, false, true><<<grid, 256, 0, s>>>(
            nullptr, n, ld, hs, y, nullptr, d, s0, tmap, cscale, colfac, sx);
      else
        fwht8_kernel<double, false, false><<<grid, 256, 0, s>>>(
            nullptr, n, ld, hs, y, y, d, s0, nullptr, 1.0, nullptr, nullptr);
      continue;
    }
    if (first && last)
      fwht_pass_kernel<T, true, true><<<grid, 256, 0, s>>>(
          x, n, ld, hs, nullptr, nullptr, n2, d, s0, k, tmap, cscale, colfac, sx);
    else if (first)
      fwht_pass_kernel<T, true, false><<<grid, 256, 0, s>>>(
          x, n, ld, hs, nullptr, y, n2, d, s0, k, nullptr, 1.0, nullptr, nullptr);
    else if (last)
      fwht_pass_kernel<double, false, true><<<grid, 256, 0, s>>>(
          nullptr, n, ld, hs, y, nullptr, n2, d, s0, k, tmap, cscale, colfac, sx);
    else
      fwht_pass_kernel<double, false, false><<<grid, 256, 0, s>>>(
          nullptr, n, ld, hs, y, y, n2, d, s0, k, nullptr, 1.0, nullptr, nullptr);
  }
}

}  // namespace

int64_t srht_rows_padded(int64_t n) {
  int64_t n2 = 1;
  while (n2 < n) n2 <<= 1;
  return n2;
}

size_t srht_scratch_bytes(int64_t n, int64_t d) {
  const int64_t n2 = srht_rows_padded(n);
  return static_cast<size_t>(n2 * d) * sizeof(double) +
         static_cast<size_t>(6 * n2 + 64) * sizeof(uint32_t) +
         radix_sort_scratch_bytes(n2) + 1024;
}

int launch_srht(const void* x, int dtype, int64_t n, int64_t d, int64_t ld,
                uint64_t seed, int64_t r, const double* colfac, void* scratch,
                double* sx, hipStream_t s) {
  const int64_t n2 = srht_rows_padded(n);
  if (r > n2 || d <= 0) return -1;
  int L = 0;
  while ((int64_t{1} << L) < n2) ++L;
  char* p = static_cast<char*>(scratch);
  auto take = [&](size_t bytes) {
    char* q = p;
    p += (bytes + 255) / 256 * 256;
    return q;
  };
  double* y = reinterpret_cast<double*>(take(static_cast<size_t>(n2 * d) * 8));
  uint32_t* keys = reinterpret_cast<uint32_t*>(take(n2 * 4));
  uint32_t* keys_o = reinterpret_cast<uint32_t*>(take(n2 * 4));
  uint32_t* order = reinterpret_cast<uint32_t*>(take(n2 * 4));
  uint32_t* keys_t = reinterpret_cast<uint32_t*>(take(n2 * 4));
  uint32_t* vals_t = reinterpret_cast<uint32_t*>(take(n2 * 4));
  int32_t* tmap = reinterpret_cast<int32_t*>(take(n2 * 4));
  void* sws = take(radix_sort_scratch_bytes(n2));
  // the row choice (its sort is profiled as the sort's own groups)
  srht_keys_kernel<<<grid1(n2, 256), 256, 0, s>>>(seed, n2, keys);
  radix_sort_pairs(keys, nullptr, keys_o, order, keys_t, vals_t, n2, 32, sws, s);
  launch_fill_i32(tmap, n2, -1, s);
  srht_tmap_kernel<<<grid1(r, 256), 256, 0, s>>>(order, r, tmap);
  prof_begin(kKSketch, s);
  const HashCoeffs hs = make_hash_coeffs(seed, kStreamSrhtSign);
  const double cscale = 1.0 / std::sqrt(static_cast<double>(r));
  switch (dtype) {
    case 0:
      run_passes(static_cast<const double*>(x), n, d, ld, hs, y, n2, L, tmap,
                 cscale, colfac, sx, s);
      break;
    case 1:
      run_passes(static_cast<const float*>(x), n, d, ld, hs, y, n2, L, tmap,
                 cscale, colfac, sx, s);
      break;
    case 2:
      run_passes(static_cast<const uint16_t*>(x), n, d, ld, hs, y, n2, L, tmap,
                 cscale, colfac, sx, s);
      break;
    default:
      run_passes(static_cast<const uint8_t*>(x), n, d, ld, hs, y, n2, L, tmap,
                 cscale, colfac, sx, s);
      break;
  }
  prof_end(kKSketch, s);
  return 0;
}

}  // namespace slso
