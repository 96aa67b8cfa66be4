// Random streams on the device and the stable LSD radix sort that serves
// both the CountSketch bucket partition (rows grouped by bucket, ascending
// row within a bucket: the streaming order of Sec. 3.1.2) and the "dec"
// ordering of Sec. 5.2 (scores decreasing, ties by ascending row).
//
// Radix sort: 8-bit digits, tiles of 256 kItems keys per 256-thread
// workgroup. Per pass: (1) per-tile digit histogram in LDS, (2) one exclusive
// scan of the digit-major histogram table, (3) a stable scatter in which each
// wave ranks equal digits with eight ballots and the waves of a tile are
// ordered through LDS prefix counts, so equal keys keep their input order.
// Up to kFusedTiles tiles, step (2) is folded into (3): the histogram is
// stored tile-major and each scatter workgroup sums the few columns it needs
// (its tile's predecessors and the digit totals), which saves a launch and a
// single-workgroup pass per digit.
#include "internal.h"

namespace slso {
namespace {

constexpr int kThreads = 256;
// keys per thread of the histogram and scatter passes: 16 for large inputs,
// 4 below kSmallSort keys (more workgroups: the passes are latency bound there)
constexpr int kItemsLarge = 16;
constexpr int kItemsSmall = 4;
constexpr int64_t kSmallSort = int64_t{1} << 20;
constexpr int kFusedTiles = 128;

__global__ void hash_pack_kernel(HashCoeffs hb, HashCoeffs hs, uint64_t r,
                                 int64_t row0, int64_t n, uint32_t* keys,
                                 uint32_t* vals) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t g = static_cast<uint64_t>(row0 + i);
  keys[i] = static_cast<uint32_t>(poly61(hb, g) % r);
  const uint32_t neg = static_cast<uint32_t>(poly61(hs, g) & 1u);
  vals[i] = static_cast<uint32_t>(i) | (neg << 31);
}

__global__ void hash_pack_osnap_kernel(OsnapCoeffs h, int nnz, uint64_t b,
                                       int64_t n, uint32_t* keys,
                                       uint32_t* vals) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n * nnz) return;
  const int j = static_cast<int>(e / n);
  const uint64_t i = static_cast<uint64_t>(e - static_cast<int64_t>(j) * n);
  keys[e] = static_cast<uint32_t>(static_cast<uint64_t>(j) * b + poly61(h.hb[j], i) % b);
  const uint32_t neg = static_cast<uint32_t>(poly61(h.hs[j], i) & 1u);
  vals[e] = static_cast<uint32_t>(i) | (neg << 31);
}

__global__ void hash_out_kernel(HashCoeffs hb, HashCoeffs hs, uint64_t r,
                                int64_t row0, int64_t n, int32_t* bucket,
                                int8_t* sign) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t g = static_cast<uint64_t>(row0 + i);
  bucket[i] = static_cast<int32_t>(poly61(hb, g) % r);
  sign[i] = (poly61(hs, g) & 1u) ? int8_t(-1) : int8_t(1);
}

__global__ void gaussian_kernel(uint64_t seed, uint32_t stream_id, int64_t rows,
                                int64_t cols, double divisor, double* out) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= rows * cols) return;
  const int64_t a = t / cols, b = t - a * cols;
  out[t] = gauss64(seed, stream_id, static_cast<uint64_t>(a),
                   static_cast<uint64_t>(b)) / divisor;
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void score_keys_kernel(const float* s, int64_t n, uint32_t* keys) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t u = __float_as_uint(s[i]);
  const uint32_t asc = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  keys[i] = ~asc;  // ascending key order = descending score order
}

// tile-major (hist[tile][digit]) when kFused, else digit-major
template <int kItems, bool kFused>
__global__ void __launch_bounds__(kThreads)
    rs_hist_kernel(const uint32_t* __restrict__ keys, int64_t n, int shift,
                   uint32_t* __restrict__ hist, int nblocks) {
  constexpr int kTile = kThreads * kItems;
  __shared__ uint32_t h[256];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kTile;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const int64_t p = base + j * kThreads + tid;
    if (p < n) atomicAdd(&h[(keys[p] >> shift) & 255u], 1u);
  }
  __syncthreads();
  if (kFused)
    hist[static_cast<int64_t>(blockIdx.x) * 256 + tid] = h[tid];
  else
    hist[static_cast<int64_t>(tid) * nblocks + blockIdx.x] = h[tid];
}

// Exclusive scan of len entries in place, one workgroup of 1024 threads:
// thread t owns one contiguous segment; its entries are read 16 at a time
// with all loads in flight together.
__global__ void __launch_bounds__(1024)
    rs_scan_kernel(uint32_t* __restrict__ hist, int64_t len) {
  __shared__ uint32_t s[1024];
  const int tid = threadIdx.x;
  const int64_t seg = (len + 1023) / 1024;
  const int64_t lo = tid * seg;
  const int64_t hi = lo + seg < len ? lo + seg : len;
  uint32_t sum = 0;
  for (int64_t c = lo; c < hi; c += 16) {
    uint32_t v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = c + u < hi ? hist[c + u] : 0u;
#pragma unroll
    for (int u = 0; u < 16; ++u) sum += v[u];
  }
  s[tid] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const uint32_t v = tid >= o ? s[tid - o] : 0u;
    __syncthreads();
    s[tid] += v;
    __syncthreads();
  }
  uint32_t run = s[tid] - sum;
  for (int64_t c = lo; c < hi; c += 16) {
    uint32_t v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = c + u < hi ? hist[c + u] : 0u;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      if (c + u < hi) hist[c + u] = run;
      run += v[u];
    }
  }
}

// Exclusive scan of len entries in place by chunks of kScanChunk: the
// chunk sums (one workgroup per chunk), their exclusive scan (one
// workgroup, up to 1024 chunks), and each chunk's scan from its offset.
constexpr int kScanChunk = 2048;

__global__ void __launch_bounds__(256)
    rs_chunk_sum_kernel(const uint32_t* __restrict__ hist, int64_t len,
                        uint32_t* __restrict__ sums) {
  __shared__ uint32_t ws[4];
  const int tid = threadIdx.x;
  const int64_t c0 = static_cast<int64_t>(blockIdx.x) * kScanChunk;
  uint32_t v = 0;
#pragma unroll
  for (int u = 0; u < kScanChunk / 256; ++u) {
    const int64_t i = c0 + u * 256 + tid;
    v += i < len ? hist[i] : 0u;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((tid & 63) == 0) ws[tid >> 6] = v;
  __syncthreads();
  if (tid == 0) sums[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

__global__ void __launch_bounds__(1024)
    rs_sums_scan_kernel(uint32_t* __restrict__ sums, int nchunks) {
  __shared__ uint32_t s[1024];
  const int tid = threadIdx.x;
  const uint32_t v = tid < nchunks ? sums[tid] : 0u;
  s[tid] = v;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const uint32_t y = tid >= o ? s[tid - o] : 0u;
    __syncthreads();
    s[tid] += y;
    __syncthreads();
  }
  if (tid < nchunks) sums[tid] = s[tid] - v;
}

__global__ void __launch_bounds__(256)
    rs_chunk_scan_kernel(uint32_t* __restrict__ hist, int64_t len,
                         const uint32_t* __restrict__ sums) {
  // thread tid scans entries c0 + 8 tid .. + 7, then the 256 thread sums
  __shared__ uint32_t ws[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t c0 = static_cast<int64_t>(blockIdx.x) * kScanChunk + 8 * tid;
  uint32_t v[8], tot = 0;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    v[u] = c0 + u < len ? hist[c0 + u] : 0u;
    tot += v[u];
  }
  uint32_t inc = tot;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) ws[wave] = inc;
  __syncthreads();
  uint32_t run = sums[blockIdx.x] + inc - tot;
#pragma unroll
  for (int w = 0; w < 4; ++w) run += w < wave ? ws[w] : 0u;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    if (c0 + u < len) hist[c0 + u] = run;
    run += v[u];
  }
}

template <int kItems, bool kFused>
__global__ void __launch_bounds__(kThreads)
    rs_scatter_kernel(const uint32_t* __restrict__ keys_in,
                      const uint32_t* __restrict__ vals_in,
                      uint32_t* __restrict__ keys_out,
                      uint32_t* __restrict__ vals_out, int64_t n, int shift,
                      const uint32_t* __restrict__ hist, int nblocks) {
  constexpr int kTile = kThreads * kItems;
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcount[4][256];
  __shared__ uint32_t wpref[4][256];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  if (kFused) {
    // start of digit tid in this tile's output: keys of smaller digits in
    // all tiles, plus keys of digit tid in the tiles before this one
    __shared__ uint32_t wsum[4];
    // 32 entries per round trip (clamped addresses, masked after the load)
    uint32_t tot = 0, before = 0;
    for (int b0 = 0; b0 < nblocks; b0 += 32) {
      uint32_t v[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) {
        const int b = b0 + u < nblocks ? b0 + u : nblocks - 1;
        v[u] = hist[static_cast<int64_t>(b) * 256 + tid];
      }
#pragma unroll
      for (int u = 0; u < 32; ++u) {
        const uint32_t x = b0 + u < nblocks ? v[u] : 0u;
        tot += x;
        before += b0 + u < static_cast<int>(blockIdx.x) ? x : 0u;
      }
    }
    uint32_t inc = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(inc, o, 64);
      if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t off = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) off += w < wave ? wsum[w] : 0u;
    run[tid] = off + inc - tot + before;
  } else {
    run[tid] = hist[static_cast<int64_t>(tid) * nblocks + blockIdx.x];
  }
#pragma unroll
  for (int w = 0; w < 4; ++w) wcount[w][tid] = 0;
  __syncthreads();
  const uint64_t lt_mask = (1ull << lane) - 1ull;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kTile;
  for (int j = 0; j < kItems; ++j) {
    const int64_t p = base + j * kThreads + tid;
    const bool valid = p < n;
    const uint32_t k = valid ? keys_in[p] : 0u;
    const uint32_t v =
        valid ? (vals_in ? vals_in[p] : static_cast<uint32_t>(p)) : 0u;
    const uint32_t dig = (k >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (dig >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = __popcll(peers & lt_mask);
    if (valid && rank == 0) wcount[wave][dig] = __popcll(peers);
    __syncthreads();
    {
      uint32_t r = run[tid];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const uint32_t c = wcount[w][tid];
        wcount[w][tid] = 0;
        wpref[w][tid] = r;
        r += c;
      }
      run[tid] = r;
    }
    __syncthreads();
    if (valid) {
      const uint32_t pos = wpref[wave][dig] + rank;
      keys_out[pos] = k;
      vals_out[pos] = v;
    }
  }
}

__global__ void bucket_offsets_kernel(const uint32_t* __restrict__ keys,
                                      int64_t n, int64_t r,
                                      int32_t* __restrict__ off) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p > n) return;
  const int64_t prev = p == 0 ? -1 : static_cast<int64_t>(keys[p - 1]);
  const int64_t cur = p == n ? r : static_cast<int64_t>(keys[p]);
  for (int64_t b = prev + 1; b <= cur; ++b) off[b] = static_cast<int32_t>(p);
}

inline unsigned grid1(int64_t n, int t) {
  return static_cast<unsigned>((n + t - 1) / t);
}

}  // namespace

void launch_hash_pack(const HashCoeffs& hb, const HashCoeffs& hs, int64_t r,
                      int64_t row0, int64_t n, uint32_t* keys, uint32_t* vals,
                      hipStream_t s) {
  if (n <= 0) return;
  prof_begin(kKHash, s);
  hash_pack_kernel<<<grid1(n, 256), 256, 0, s>>>(hb, hs, static_cast<uint64_t>(r),
                                                  row0, n, keys, vals);
  prof_end(kKHash, s);
}

void launch_hash_pack_osnap(const OsnapCoeffs& h, int nnz, int64_t r,
                            int64_t n, uint32_t* keys, uint32_t* vals,
                            hipStream_t s) {
  if (n <= 0 || nnz <= 0) return;
  prof_begin(kKHash, s);
  hash_pack_osnap_kernel<<<grid1(n * nnz, 256), 256, 0, s>>>(
      h, nnz, static_cast<uint64_t>(r / nnz), n, keys, vals);
  prof_end(kKHash, s);
}

void launch_hash_out(const HashCoeffs& hb, const HashCoeffs& hs, int64_t r,
                     int64_t row0, int64_t n, int32_t* bucket, int8_t* sign,
                     hipStream_t s) {
  if (n <= 0) return;
  hash_out_kernel<<<grid1(n, 256), 256, 0, s>>>(hb, hs, static_cast<uint64_t>(r),
                                                 row0, n, bucket, sign);
}

void launch_gaussian(uint64_t seed, uint32_t stream_id, int64_t rows,
                     int64_t cols, double divisor, double* out, hipStream_t s) {
  if (rows * cols <= 0) return;
  prof_begin(kKGauss, s);
  gaussian_kernel<<<grid1(rows * cols, 256), 256, 0, s>>>(seed, stream_id, rows,
                                                          cols, divisor, out);
  prof_end(kKGauss, s);
}

void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return;
  fill_i32_kernel<<<grid1(n, 256), 256, 0, s>>>(p, n, v);
}

void launch_score_keys(const float* scores, int64_t n, uint32_t* keys,
                       hipStream_t s) {
  if (n <= 0) return;
  score_keys_kernel<<<grid1(n, 256), 256, 0, s>>>(scores, n, keys);
}

namespace {
int sort_items(int64_t n) { return n < kSmallSort ? kItemsSmall : kItemsLarge; }
}  // namespace

size_t radix_sort_scratch_bytes(int64_t n) {
  const int64_t tile = static_cast<int64_t>(kThreads) * sort_items(n);
  const int64_t nblocks = (n + tile - 1) / tile;
  const int64_t len = 256 * nblocks;
  const int64_t nchunks = (len + kScanChunk - 1) / kScanChunk;
  return static_cast<size_t>(len + nchunks) * sizeof(uint32_t);
}

void radix_sort_pairs(const uint32_t* keys_in, const uint32_t* vals_in,
                      uint32_t* keys_out, uint32_t* vals_out,
                      uint32_t* keys_tmp, uint32_t* vals_tmp, int64_t n,
                      int nbits, void* scratch, hipStream_t s) {
  if (n <= 0) return;
  const int items = sort_items(n);
  const int64_t tile = static_cast<int64_t>(kThreads) * items;
  const int nblocks = static_cast<int>((n + tile - 1) / tile);
  uint32_t* hist = static_cast<uint32_t*>(scratch);
  const int passes = nbits <= 0 ? 1 : (nbits + 7) / 8;
  const uint32_t* ksrc = keys_in;
  const uint32_t* vsrc = vals_in;
  for (int p = 0; p < passes; ++p) {
    const bool to_out = ((passes - 1 - p) % 2) == 0;
    uint32_t* kdst = to_out ? keys_out : keys_tmp;
    uint32_t* vdst = to_out ? vals_out : vals_tmp;
    const int shift = 8 * p;
    if (nblocks <= kFusedTiles && items == kItemsSmall) {
      prof_begin(kKSortHist, s);
      rs_hist_kernel<kItemsSmall, true><<<nblocks, kThreads, 0, s>>>(
          ksrc, n, shift, hist, nblocks);
      prof_end(kKSortHist, s);
      prof_begin(kKSortScatter, s);
      rs_scatter_kernel<kItemsSmall, true><<<nblocks, kThreads, 0, s>>>(
          ksrc, vsrc, kdst, vdst, n, shift, hist, nblocks);
      prof_end(kKSortScatter, s);
    } else {
      prof_begin(kKSortHist, s);
      if (items == kItemsSmall)
        rs_hist_kernel<kItemsSmall, false><<<nblocks, kThreads, 0, s>>>(
            ksrc, n, shift, hist, nblocks);
      else
        rs_hist_kernel<kItemsLarge, false><<<nblocks, kThreads, 0, s>>>(
            ksrc, n, shift, hist, nblocks);
      prof_end(kKSortHist, s);
      prof_begin(kKSortScan, s);
      const int64_t len = static_cast<int64_t>(256) * nblocks;
      const int64_t nchunks = (len + kScanChunk - 1) / kScanChunk;
      if (nchunks <= 1024) {
        uint32_t* sums = hist + len;
        rs_chunk_sum_kernel<<<static_cast<unsigned>(nchunks), 256, 0, s>>>(
            hist, len, sums);
        rs_sums_scan_kernel<<<1, 1024, 0, s>>>(sums, static_cast<int>(nchunks));
        rs_chunk_scan_kernel<<<static_cast<unsigned>(nchunks), 256, 0, s>>>(
            hist, len, sums);
      } else {
        rs_scan_kernel<<<1, 1024, 0, s>>>(hist, len);
      }
      prof_end(kKSortScan, s);
      prof_begin(kKSortScatter, s);
      if (items == kItemsSmall)
        rs_scatter_kernel<kItemsSmall, false><<<nblocks, kThreads, 0, s>>>(
            ksrc, vsrc, kdst, vdst, n, shift, hist, nblocks);
      else
        rs_scatter_kernel<kItemsLarge, false><<<nblocks, kThreads, 0, s>>>(
            ksrc, vsrc, kdst, vdst, n, shift, hist, nblocks);
      prof_end(kKSortScatter, s);
    }
    ksrc = kdst;
    vsrc = vdst;
  }
}

void launch_bucket_offsets(const uint32_t* sorted_keys, int64_t n, int64_t r,
                           int32_t* offsets, hipStream_t s) {
  prof_begin(kKOffsets, s);
  bucket_offsets_kernel<<<grid1(n + 1, 256), 256, 0, s>>>(sorted_keys, n, r,
                                                          offsets);
  prof_end(kKOffsets, s);
}

}  // namespace slso
