// The sampling policies "dec, swr" and "dec, swor" of Algorithm 4 step 4
// (Sec. 5.2), drawn from P_i = L_i / sum_j L_j (step 3) with a seeded stream
// per epoch. A score that is not a positive finite number has probability 0.
//
// Draw stream: for item t and epoch, one Philox4x32-10 block with counter
// (lo32(t), hi32(t), epoch, stream) and key (lo32(seed), hi32(seed)).
//
// dec-swr (stream 5): n draws with replacement, in draw order. P is held
// exactly as integer weights w_i = floor(L_i 2^(30 - e)), 2^(e-1) <= max L <
// 2^e, so the cumulative weights C_i are exact int64 (W = C_{n-1} < n 2^30);
// draw t takes m_t = ((w0 << 32) | w1) >> 11 (53 bits) and the smallest i with
// C_i > floor(m_t W / 2^53). Kernels: the maximum (bit patterns of
// non-negative floats order like their values), the weights with a
// workgroup-local inclusive scan, the scan of the workgroup totals, the
// offsets added, then one thread per draw with a binary search.
//
// dec-swor (stream 6): the permutation of weighted sampling without
// replacement, in draw order, by the exponential keys of Efraimidis and
// Spirakis: key_i = E_i / L_i, E_i = 0 - ln u_i with u_i = ((w0 >> 8) + 1)
// 2^-24 and the FP32 logarithm of the Gaussian generator (separately rounded
// operations); rows sorted by ascending key (non-negative floats: their bit
// patterns order like the values), ties by ascending row, probability-0 rows
// (key +inf) last.
#include "internal.h"

namespace slso {
namespace {

constexpr int kSwrItems = 8;             // weights per thread of a scan block
constexpr int kSwrBlock = 256 * kSwrItems;

__device__ __forceinline__ U4 sample_block(uint64_t seed, uint32_t stream,
                                           uint32_t epoch, uint64_t t) {
  U4 c;
  c.x = static_cast<uint32_t>(t);
  c.y = static_cast<uint32_t>(t >> 32);
  c.z = epoch;
  c.w = stream;
  return philox10(c, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
}

__device__ __forceinline__ bool positive(float v) {
  return v > 0.0f && v <= 3.402823466e38f;
}

// ln u for u = ((w >> 8) + 1) 2^-24, every operation rounded separately (the
// logarithm of the FP32 Gaussian generator)
#pragma clang fp contract(off)
__device__ __forceinline__ float ln_unit_f32(uint32_t w) {
  const float u1 = static_cast<float>((w >> 8) + 1u) * 0x1p-24f;
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
  const float ln_u = static_cast<float>(e) * 0.6931471824645996f;
  return ln_u + lnm;
}

__global__ void swor_keys_kernel(const float* __restrict__ scores, int64_t n,
                                 uint64_t seed, uint32_t epoch,
                                 uint32_t* __restrict__ keys) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float l = scores[t];
  const U4 w = sample_block(seed, kStreamSwor, epoch, static_cast<uint64_t>(t));
  const float e = 0.0f - ln_unit_f32(w.x);
  const float k = positive(l) ? e / l : __builtin_inff();
  keys[t] = __float_as_uint(k);
}
#pragma clang fp contract(on)

__global__ void swr_max_kernel(const float* __restrict__ scores, int64_t n,
                               unsigned int* __restrict__ mbits) {
  __shared__ unsigned int red[4];
  unsigned int m = 0u;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
       i < n; i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const float v = scores[i];
    const unsigned int b = positive(v) ? __float_as_uint(v) : 0u;
    m = b > m ? b : m;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned int x = __shfl_xor(m, o, 64);
    m = x > m ? x : m;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned int b = red[0];
    for (int k = 1; k < 4; ++k) b = red[k] > b ? red[k] : b;
    if (b) atomicMax(mbits, b);
  }
}

// weights of block blockIdx.x, inclusive prefix inside the block into cum,
// the block's total into tot[blockIdx.x]
__global__ void __launch_bounds__(256)
    swr_weights_kernel(const float* __restrict__ scores, int64_t n,
                       const unsigned int* __restrict__ mbits,
                       int64_t* __restrict__ cum, int64_t* __restrict__ tot) {
  __shared__ int64_t wsum[4];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  int e;
  frexp(static_cast<double>(__uint_as_float(*mbits)), &e);
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kSwrBlock + t * kSwrItems;
  int64_t w[kSwrItems];
  int64_t run = 0;
#pragma unroll
  for (int u = 0; u < kSwrItems; ++u) {
    const int64_t i = base + u;
    const float v = i < n ? scores[i] : 0.0f;
    w[u] = positive(v) ? static_cast<int64_t>(floor(ldexp(static_cast<double>(v), 30 - e)))
                       : 0;
    run += w[u];
  }
  // exclusive scan of the thread totals over the workgroup
  int64_t inc = run;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  int64_t off = inc - run;
#pragma unroll
  for (int k = 0; k < 4; ++k) off += k < wv ? wsum[k] : 0;
#pragma unroll
  for (int u = 0; u < kSwrItems; ++u) {
    off += w[u];
    if (base + u < n) cum[base + u] = off;
  }
  if (t == 255) tot[blockIdx.x] = off;
}

// exclusive prefix of the block totals in place; one workgroup
__global__ void __launch_bounds__(1024)
    swr_scan_totals_kernel(int64_t* __restrict__ tot, int64_t nblk) {
  __shared__ int64_t wsum[16];
  __shared__ int64_t carry;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  if (t == 0) carry = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < nblk; b0 += 1024) {
    const int64_t i = b0 + t;
    const int64_t v = i < nblk ? tot[i] : 0;
    int64_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t y = __shfl_up(inc, o, 64);
      if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    int64_t off = carry + inc - v;
    for (int k = 0; k < wv; ++k) off += wsum[k];
    if (i < nblk) tot[i] = off;
    __syncthreads();
    if (t == 1023) carry = off + v;
    __syncthreads();
  }
}

__global__ void swr_add_kernel(int64_t* __restrict__ cum, int64_t n,
                               const int64_t* __restrict__ tot) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) cum[i] += tot[i / kSwrBlock];
}

__global__ void swr_draw_kernel(const int64_t* __restrict__ cum, int64_t n,
                                uint64_t seed, uint32_t epoch,
                                int32_t* __restrict__ out) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const uint64_t total = static_cast<uint64_t>(cum[n - 1]);
  const U4 w = sample_block(seed, kStreamSwr, epoch, static_cast<uint64_t>(t));
  const uint64_t m = ((static_cast<uint64_t>(w.x) << 32) | w.y) >> 11;
  // floor(m W / 2^53) from the 128-bit product
  const uint64_t lo = m * total, hi = __umul64hi(m, total);
  const int64_t target = static_cast<int64_t>((hi << 11) | (lo >> 53));
  int64_t a = 0, b = n - 1;
  while (a < b) {
    const int64_t mid = a + (b - a) / 2;
    if (cum[mid] > target)
      b = mid;
    else
      a = mid + 1;
  }
  out[t] = static_cast<int32_t>(a);
}

inline unsigned grid1(int64_t n, int t) {
  return static_cast<unsigned>((n + t - 1) / t);
}

}  // namespace

size_t swr_scratch_bytes(int64_t n) {
  const int64_t nblk = (n + kSwrBlock - 1) / kSwrBlock;
  return static_cast<size_t>(n + nblk + 8) * sizeof(int64_t);
}

void launch_swor_keys(const float* scores, int64_t n, uint64_t seed,
                      uint32_t epoch, uint32_t* keys, hipStream_t s) {
  if (n <= 0) return;
  swor_keys_kernel<<<grid1(n, 256), 256, 0, s>>>(scores, n, seed, epoch, keys);
}

void launch_swr_prefix(const float* scores, int64_t n, void* scratch,
                       hipStream_t s) {
  if (n <= 0) return;
  int64_t* cum = static_cast<int64_t*>(scratch);
  const int64_t nblk = (n + kSwrBlock - 1) / kSwrBlock;
  int64_t* tot = cum + n;
  unsigned int* mbits = reinterpret_cast<unsigned int*>(tot + nblk);
  launch_fill_i32(reinterpret_cast<int32_t*>(mbits), 1, 0, s);
  const int64_t gmax = grid1(n, 256) < 1024 ? grid1(n, 256) : 1024;
  swr_max_kernel<<<static_cast<unsigned>(gmax), 256, 0, s>>>(scores, n, mbits);
  swr_weights_kernel<<<static_cast<unsigned>(nblk), 256, 0, s>>>(scores, n, mbits,
                                                                  cum, tot);
  swr_scan_totals_kernel<<<1, 1024, 0, s>>>(tot, nblk);
  swr_add_kernel<<<grid1(n, 256), 256, 0, s>>>(cum, n, tot);
}

void launch_swr_draws(const void* scratch, int64_t n, uint64_t seed,
                      uint32_t epoch, int32_t* out, hipStream_t s) {
  if (n <= 0) return;
  swr_draw_kernel<<<grid1(n, 256), 256, 0, s>>>(
      static_cast<const int64_t*>(scratch), n, seed, epoch, out);
}

}  // namespace slso
