// Gaussian sketch S X (Sec. 2.1; Algorithm 2 step 1) for BF16 and FP8 input,
// with the quantile form of the sketch entries: G[j][i] is a signed midpoint
// quantile of |Z| (Z standard normal) on 2^15 equiprobable cells,
//   t_m = sqrt(2) erfinv((2 m + 1) / 65536),
// rounded to BF16 for BF16 input and to e4m3 for FP8 input, chosen by a
// 16-bit half of a Philox4x32-10 block (one block per eight consecutive
// data rows of one sketch row: counter (lo32(i >> 3), hi32(i >> 3), j, 9),
// half (i & 1) of word (i >> 1) & 3; top bit the sign, low 15 bits the
// cell). The sketch products run on the BF16 MFMA (e4m3 values are exact in
// BF16; products are exact in FP32); sums are FP32 within one workgroup's
// slice of rows and FP64 across slices, in a fixed order.
//
// The tables are computed on the host at context creation (FP64 erfinv by
// Newton steps on erf / erfc, rounded to nearest even) and copied into a
// device array; every t_m lies more than 1e-9 of itself from a rounding
// boundary of either format, so this evaluation gives the exact tables.
//
// Tiling: one workgroup of eight waves owns 128 sketch rows x 512 columns of
// one slice of data rows, so each entry of G is generated once per column
// chunk of 512 (once in all for d <= 512) and feeds 2 x 512 flops. A step
// takes 32 data rows: each thread draws one Philox block (8 entries of one
// sketch row) and stages a 4-row x 8-column block of X, transposed in
// registers so that each column's 4 rows are one 8-byte LDS write. Wave w
// owns sketch rows 64 (w & 1) .. + 63 and columns 128 (w >> 1) .. + 127 as
// 2 x 4 MFMA blocks of 32 x 32 (v_mfma_f32_32x32x16_bf16). The next step's
// entries are drawn while the current step's products run, so the
// generator's VALU work overlaps the matrix unit, and rows are loaded two
// steps ahead.
#include <cmath>
#include <cstring>
#include <mutex>

#include "internal.h"

namespace slso {

constexpr int kQCells = 1 << 15;

// BF16 bit patterns of the entry magnitudes: [0] t_m rounded to BF16,
// [1] t_m rounded to e4m3 (held as the BF16 pattern of the same value)
__device__ __attribute__((aligned(16))) uint16_t g_qtab[2][kQCells];

namespace {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kQR = 128;        // sketch rows per workgroup
constexpr int kQD = 512;        // columns per workgroup
constexpr int kQK = 32;         // data rows per step
constexpr int kQP = 40;         // LDS pitch (elements) along the data rows
constexpr int kQThreads = 512;  // eight waves

// ---- host: the quantile tables ---------------------------------------------
// erfinv(p) for 0 < p < 1: the Winitzki estimate refined by Newton steps on
// erf (on erfc above one half, where 1 - p is exact and erf would cancel)
double erfinv_host(double p) {
  const double a = 0.147;
  const double ln1 = std::log((1.0 - p) * (1.0 + p));
  const double t = 2.0 / (M_PI * a) + 0.5 * ln1;
  double x = std::sqrt(std::sqrt(t * t - ln1 / a) - t);
  const double q = 1.0 - p;  // exact for p = (2m + 1) / 65536
  for (int it = 0; it < 8; ++it) {
    const double f = p <= 0.5 ? std::erf(x) - p : q - std::erfc(x);
    x -= f / (1.1283791670955126 * std::exp(-x * x));
  }
  return x;
}

// value of t rounded to nearest even with `sig` significant bits and
// exponent at least emin (subnormal spacing below it)
double round_sig(double t, int sig, int emin) {
  int ex = 0;
  (void)std::frexp(t, &ex);
  int e = ex - 1;
  if (e < emin) e = emin;
  const double sp = std::ldexp(1.0, e - (sig - 1));
  return std::nearbyint(t / sp) * sp;
}

uint16_t bf16_pattern(double v) {
  const float f = static_cast<float>(v);  // exact: v has at most 8 bits
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return static_cast<uint16_t>(u >> 16);
}

struct QTables {
  uint16_t t[2][kQCells];
  QTables() {
    for (int m = 0; m < kQCells; ++m) {
      const double p = (2.0 * m + 1.0) / 65536.0;
      const double tm = M_SQRT2 * erfinv_host(p);
      t[0][m] = bf16_pattern(round_sig(tm, 8, -126));
      double v8 = round_sig(tm, 4, -6);
      if (v8 > 448.0) v8 = 448.0;
      t[1][m] = bf16_pattern(v8);
    }
  }
};

const QTables& host_tables() {
  static const QTables tabs;
  return tabs;
}

// ---- device -------------------------------------------------------------------
template <int IT>
struct QIn;
template <>
struct QIn<1> {  // BF16
  using T = uint16_t;
};
template <>
struct QIn<2> {  // FP8-e4m3 codes
  using T = uint8_t;
};

// 8 entries of sketch row j for data rows 8 q .. 8 q + 7, as 4 words of
// BF16 pairs (lower data row in the low half)
__device__ __forceinline__ void draw8(uint64_t q, uint32_t j, uint32_t k0,
                                      uint32_t k1, const uint16_t* tab,
                                      uint32_t (&gw)[4]) {
  U4 c{static_cast<uint32_t>(q), static_cast<uint32_t>(q >> 32), j,
       static_cast<uint32_t>(kStreamGaussQ)};
  const U4 o = philox10(c, k0, k1);
  const uint32_t w4[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const uint32_t v = w4[u];
    const uint32_t lo = tab[v & 0x7FFFu];
    const uint32_t hi = tab[(v >> 16) & 0x7FFFu];
    gw[u] = (lo | (hi << 16)) | (v & 0x80008000u);
  }
}

// e4m3 code -> BF16 bits of its value (exact; NaN codes give a NaN)
__device__ __forceinline__ uint32_t e4m3_bf16_bits(uint32_t q) {
  return __float_as_uint(e4m3_to_f32(static_cast<uint8_t>(q))) >> 16;
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// ---- staging of X blocks (shared by the sketch and the Gram pass) ------------
// A thread stages rows row .. row + 3 and columns gcol .. gcol + 7 of X. The
// loads are issued unconditionally (rows past i_end read row i_end - 1) into
// raw registers and only used a step or two later, so nothing waits for
// them at the issue point; rows at or past i_end are zeroed when the block
// is unpacked (stage_unpack) into BF16 pairs xr[u][v] = row + u, columns
// 2 v (low half) and 2 v + 1. FP8 codes are decoded through the 256-entry
// table dec8 (exact in BF16).
template <int IT>
struct RawBlock;
template <>
struct RawBlock<1> {  // BF16: 8 elements per row, 16 bytes
  uint4 q[4];
};
template <>
struct RawBlock<2> {  // FP8 codes: 8 per row, 8 bytes
  uint2 q[4];
};

template <int IT, bool VEC>
__device__ __forceinline__ void stage_issue(
    const typename QIn<IT>::T* __restrict__ x, int64_t ld, int64_t d,
    int64_t gcol, int64_t row, int64_t i_end, RawBlock<IT>& raw) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t gi = row + u < i_end ? row + u : i_end - 1;
    const typename QIn<IT>::T* p = x + gi * ld + gcol;
    if constexpr (VEC) {
      if constexpr (IT == 1)
        raw.q[u] = *reinterpret_cast<const uint4*>(p);
      else
        raw.q[u] = *reinterpret_cast<const uint2*>(p);
    } else {
      uint32_t e8[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t c = gcol + e < d ? e : 0;
        e8[e] = p[c];
      }
      if constexpr (IT == 1) {
        raw.q[u] = make_uint4(e8[0] | (e8[1] << 16), e8[2] | (e8[3] << 16),
                              e8[4] | (e8[5] << 16), e8[6] | (e8[7] << 16));
      } else {
        raw.q[u] = make_uint2(e8[0] | (e8[1] << 8) | (e8[2] << 16) | (e8[3] << 24),
                              e8[4] | (e8[5] << 8) | (e8[6] << 16) | (e8[7] << 24));
      }
    }
  }
}

// nvalid = rows of the block inside the slice (i_end - row, clamped to 0..4)
template <int IT>
__device__ __forceinline__ void stage_unpack(const RawBlock<IT>& raw,
                                             int64_t nvalid,
                                             const uint16_t* dec8,
                                             uint32_t (&xr)[4][4]) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    uint32_t v4[4];
    if constexpr (IT == 1) {
      v4[0] = raw.q[u].x;
      v4[1] = raw.q[u].y;
      v4[2] = raw.q[u].z;
      v4[3] = raw.q[u].w;
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const uint32_t w = v < 2 ? raw.q[u].x : raw.q[u].y;
        const int sh = 16 * (v & 1);
        v4[v] = static_cast<uint32_t>(dec8[(w >> sh) & 0xFFu]) |
                (static_cast<uint32_t>(dec8[(w >> (sh + 8)) & 0xFFu]) << 16);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) xr[u][v] = u < nvalid ? v4[v] : 0u;
  }
}

// The staged block into a K-contiguous LDS tile (pitch kQP): column col + e
// gets its four rows at k .. k + 3 as one 8-byte write.
__device__ __forceinline__ void stage_store(uint16_t* T, int col, int k,
                                            const uint32_t (&xr)[4][4]) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const uint32_t sel = (e & 1) ? 0x07060302u : 0x05040100u;
    uint2 v;
    v.x = __builtin_amdgcn_perm(xr[1][e >> 1], xr[0][e >> 1], sel);
    v.y = __builtin_amdgcn_perm(xr[3][e >> 1], xr[2][e >> 1], sel);
    *reinterpret_cast<uint2*>(&T[(col + e) * kQP + k]) = v;
  }
}

// |x| of the block folded into per-column maxima of BF16 bit patterns
// (packed pairs like xr): for non-negative values the pattern order is the
// numeric order, and Inf / NaN patterns (>= 0x7F80) exceed every finite one
__device__ __forceinline__ void stage_max(const uint32_t (&xr)[4][4],
                                          uint32_t (&mx)[4]) {
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const u16x2 a = __builtin_bit_cast(u16x2, mx[v]);
      const u16x2 b = __builtin_bit_cast(u16x2, xr[u][v] & 0x7FFF7FFFu);
      mx[v] = __builtin_bit_cast(uint32_t, __builtin_elementwise_max(a, b));
    }
}

// Column maxima of the eight row groups of a column chunk (lanes 8 c ..
// 8 c + 7 of a wave) into colmax (FP64 bit patterns, times |cs| for FP8
// codes); a non-finite value sets *nonfinite
__device__ __forceinline__ void flush_max(uint32_t (&mx)[4], int rg,
                                          int64_t col, int64_t d,
                                          const float* __restrict__ cs,
                                          unsigned long long* colmax,
                                          int* nonfinite) {
#pragma unroll
  for (int off = 1; off < 8; off <<= 1)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const uint32_t o = __shfl_xor(mx[v], off, 64);
      mx[v] = __builtin_bit_cast(
          uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, mx[v]),
                                              __builtin_bit_cast(u16x2, o)));
    }
  if (rg != 0) return;
  bool bad = false;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int64_t c = col + e;
    const uint32_t b = (mx[e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
    if (c >= d) continue;
    if (b >= 0x7F80u) {
      bad = true;
      continue;
    }
    double v = static_cast<double>(__uint_as_float(b << 16));
    if (cs) v *= fabs(static_cast<double>(cs[c]));
    if (v > 0.0)
      atomicMax(&colmax[c],
                static_cast<unsigned long long>(__double_as_longlong(v)));
  }
  if (bad) atomicExch(nonfinite, 1);
}

// logical workgroup id: with a grid that is a multiple of 8 each XCD
// (blockIdx mod 8) gets a contiguous range of ids, so workgroups that share
// a slice of rows of X share that XCD's L2
__device__ __forceinline__ unsigned xcd_logical() {
  const unsigned nb = gridDim.x;
  if ((nb & 7u) != 0u) return blockIdx.x;
  return (blockIdx.x & 7u) * (nb >> 3) + (blockIdx.x >> 3);
}

template <int IT>
__device__ __forceinline__ void load_dec8(uint16_t* dec8, int t) {
  if (IT == 2 && t < 256) dec8[t] = static_cast<uint16_t>(e4m3_bf16_bits(t));
}

template <int IT, bool VEC>
__global__ void __launch_bounds__(kQThreads)
    gauss_q_kernel(const typename QIn<IT>::T* __restrict__ x, int64_t n,
                   int64_t d, int64_t ld, uint64_t seed, int64_t r,
                   int64_t rows_per_split, int nrt, int nct,
                   float* __restrict__ partial, const float* __restrict__ cs,
                   unsigned long long* __restrict__ colmax,
                   int* __restrict__ nonfinite) {
  __shared__ __attribute__((aligned(16))) uint16_t tab[kQCells];
  __shared__ __attribute__((aligned(16))) uint16_t XT[kQD * kQP];
  __shared__ __attribute__((aligned(16))) uint16_t GT[kQR * kQP];
  __shared__ uint16_t dec8[256];
  const int t = threadIdx.x;
  // consecutive logical ids share a slice of rows
  const unsigned L = xcd_logical();
  const int rt = static_cast<int>(L % static_cast<unsigned>(nrt));
  const int ct = static_cast<int>((L / static_cast<unsigned>(nrt)) %
                                  static_cast<unsigned>(nct));
  const int64_t sp = static_cast<int64_t>(L / static_cast<unsigned>(nrt * nct));
  const int64_t row0 = static_cast<int64_t>(rt) * kQR;
  const int64_t col0 = static_cast<int64_t>(ct) * kQD;
  const int64_t i_begin = sp * rows_per_split;
  int64_t i_end = i_begin + rows_per_split;
  if (i_end > n) i_end = n;

  {
    const uint4* src = reinterpret_cast<const uint4*>(g_qtab[IT == 2 ? 1 : 0]);
    uint4* dst = reinterpret_cast<uint4*>(tab);
    for (int e = t; e < kQCells / 8; e += kQThreads) dst[e] = src[e];
    load_dec8<IT>(dec8, t);
  }

  // staging role: rows 4 rg .. 4 rg + 3 of a step, columns col0 + 8 cc ..;
  // columns past d read column 0 (their products land in output columns
  // that are never stored)
  const int rg = t & 7, cc = t >> 3;
  const int64_t gcol = col0 + 8 * cc < d ? col0 + 8 * cc : 0;
  // generation role: sketch row row0 + jr, data rows 8 gq .. 8 gq + 7
  const int jr = t >> 2, gq = t & 3;
  const uint32_t jctr = static_cast<uint32_t>(row0 + jr);
  const uint32_t sk0 = static_cast<uint32_t>(seed);
  const uint32_t sk1 = static_cast<uint32_t>(seed >> 32);
  // product role
  const int lane = t & 63, w = t >> 6, l32 = lane & 31, h = lane >> 5;
  const int wr = w & 1, wc = w >> 1;

  f16v acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[a][b][e] = 0.0f;

  // column maxima (when colmax is given): the nrt row-tile workgroups of a
  // slice take turns, step s by the workgroup with s mod nrt = rt
  uint32_t mx[4] = {0u, 0u, 0u, 0u};
  // rows are loaded two steps ahead (two raw buffers, steps taken in pairs
  // so that each buffer keeps its registers)
  RawBlock<IT> ra, rb;
  uint32_t gw[4];
  __syncthreads();  // tables in LDS
  stage_issue<IT, VEC>(x, ld, d, gcol, i_begin + 4 * rg, i_end, ra);
  stage_issue<IT, VEC>(x, ld, d, gcol, i_begin + kQK + 4 * rg, i_end, rb);
  draw8(static_cast<uint64_t>(i_begin >> 3) + gq, jctr, sk0, sk1, tab, gw);

  auto step = [&](int64_t k0, int st, RawBlock<IT>& raw) {
    uint32_t xr[4][4];
    stage_unpack<IT>(raw, i_end - (k0 + 4 * rg), dec8, xr);
    if (colmax && st % nrt == rt) stage_max(xr, mx);
    __syncthreads();  // the previous step's operands have been read
    stage_store(XT, 8 * cc, 4 * rg, xr);
    *reinterpret_cast<uint4*>(&GT[jr * kQP + 8 * gq]) =
        make_uint4(gw[0], gw[1], gw[2], gw[3]);
    __syncthreads();
    // two steps ahead (past the slice: rows clamped, never used)
    stage_issue<IT, VEC>(x, ld, d, gcol, k0 + 2 * kQK + 4 * rg, i_end, raw);
#pragma unroll
    for (int kh = 0; kh < 2; ++kh) {
      bf16x8 av[2], bv[4];
#pragma unroll
      for (int a = 0; a < 2; ++a)
        av[a] = *reinterpret_cast<const bf16x8*>(
            &GT[(64 * wr + 32 * a + l32) * kQP + 16 * kh + 8 * h]);
#pragma unroll
      for (int b = 0; b < 4; ++b)
        bv[b] = *reinterpret_cast<const bf16x8*>(
            &XT[(128 * wc + 32 * b + l32) * kQP + 16 * kh + 8 * h]);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[a], bv[b],
                                                              acc[a][b], 0, 0, 0);
    }
    draw8(static_cast<uint64_t>((k0 + kQK) >> 3) + gq, jctr, sk0, sk1, tab,
          gw);
  };
  int st = 0;
  for (int64_t k0 = i_begin; k0 < i_end; k0 += 2 * kQK, st += 2) {
    step(k0, st, ra);
    if (k0 + kQK < i_end) step(k0 + kQK, st + 1, rb);
  }
  if (colmax) flush_max(mx, rg, col0 + 8 * cc, d, cs, colmax, nonfinite);

  // partial[slice][j][c]; accumulator register e of lane l holds
  // D[(e % 4) + 8 (e / 4) + 4 (l / 32)][l % 32]
  float* P = partial + sp * r * d;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t j = row0 + 64 * wr + 32 * a + (e % 4) + 8 * (e / 4) + 4 * h;
        const int64_t c = col0 + 128 * wc + 32 * b + l32;
        if (j < r && c < d) P[j * d + c] = acc[a][b][e];
      }
}

// ---- Gram matrix X^T X of BF16 / FP8 input (the refinement pass) -------------
// Output tile 256 x 256 of column blocks (A, B), A <= B, over one slice of
// rows; eight waves, wave w owns rows 64 (w & 3) .. + 63 and columns
// 128 (w >> 2) .. + 127 of the tile as 2 x 4 MFMA blocks. Threads 0-255
// stage block A and 256-511 block B (the diagonal tiles stage A only) into
// K-contiguous tiles, which serve both as the A^T and the B operand.
constexpr int kGB = 256;

template <int IT, bool VEC>
__global__ void __launch_bounds__(kQThreads)
    gram_q_kernel(const typename QIn<IT>::T* __restrict__ x, int64_t n,
                  int64_t d, int64_t ld, int nb, int ntiles,
                  int64_t rows_per_split, float* __restrict__ partial) {
  __shared__ __attribute__((aligned(16))) uint16_t TA[kGB * kQP];
  __shared__ __attribute__((aligned(16))) uint16_t TB[kGB * kQP];
  __shared__ uint16_t dec8[256];
  const int t = threadIdx.x;
  const unsigned L = xcd_logical();
  int rem = static_cast<int>(L % static_cast<unsigned>(ntiles));
  const int64_t sp = static_cast<int64_t>(L / static_cast<unsigned>(ntiles));
  int ta = 0;
  while (rem >= nb - ta) {
    rem -= nb - ta;
    ++ta;
  }
  const int tb = ta + rem;
  const bool diag = ta == tb;
  const int64_t i_begin = sp * rows_per_split;
  int64_t i_end = i_begin + rows_per_split;
  if (i_end > n) i_end = n;
  load_dec8<IT>(dec8, t);

  const int side = t >> 8, ts = t & 255;
  const int rg = ts & 7, cc = ts >> 3;  // 32 chunks of 8 columns
  const int64_t c0 = static_cast<int64_t>(side ? tb : ta) * kGB + 8 * cc;
  const int64_t gcol = c0 < d ? c0 : 0;
  const bool stager = side == 0 || !diag;
  uint16_t* T = side ? TB : TA;
  const uint16_t* TBr = diag ? TA : TB;
  const int lane = t & 63, w = t >> 6, l32 = lane & 31, h = lane >> 5;
  const int wr = w & 3, wc = w >> 2;

  f16v acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[a][b][e] = 0.0f;

  RawBlock<IT> ra, rb;
  __syncthreads();  // dec8
  if (stager) {
    stage_issue<IT, VEC>(x, ld, d, gcol, i_begin + 4 * rg, i_end, ra);
    stage_issue<IT, VEC>(x, ld, d, gcol, i_begin + kQK + 4 * rg, i_end, rb);
  }
  auto step = [&](int64_t k0, RawBlock<IT>& raw) {
    uint32_t xr[4][4];
    if (stager) stage_unpack<IT>(raw, i_end - (k0 + 4 * rg), dec8, xr);
    __syncthreads();
    if (stager) stage_store(T, 8 * cc, 4 * rg, xr);
    __syncthreads();
    if (stager)
      stage_issue<IT, VEC>(x, ld, d, gcol, k0 + 2 * kQK + 4 * rg, i_end, raw);
#pragma unroll
    for (int kh = 0; kh < 2; ++kh) {
      bf16x8 av[2], bv[4];
#pragma unroll
      for (int a = 0; a < 2; ++a)
        av[a] = *reinterpret_cast<const bf16x8*>(
            &TA[(64 * wr + 32 * a + l32) * kQP + 16 * kh + 8 * h]);
#pragma unroll
      for (int b = 0; b < 4; ++b)
        bv[b] = *reinterpret_cast<const bf16x8*>(
            &TBr[(128 * wc + 32 * b + l32) * kQP + 16 * kh + 8 * h]);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[a], bv[b],
                                                              acc[a][b], 0, 0, 0);
    }
  };
  for (int64_t k0 = i_begin; k0 < i_end; k0 += 2 * kQK) {
    step(k0, ra);
    if (k0 + kQK < i_end) step(k0 + kQK, rb);
  }
  float* P = partial + sp * d * d;
  const int64_t a0 = static_cast<int64_t>(ta) * kGB, b0 = static_cast<int64_t>(tb) * kGB;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t i = a0 + 64 * wr + 32 * a + (e % 4) + 8 * (e / 4) + 4 * h;
        const int64_t j = b0 + 128 * wc + 32 * b + l32;
        if (i < d && j < d) P[i * d + j] = acc[a][b][e];
      }
}

__global__ void gauss_q_entries_kernel(uint64_t seed, int64_t r, int64_t n,
                                       int64_t row0, int fmt,
                                       float* __restrict__ out) {
  // out[j * n + i] = G[j][row0 + i] (quantile form, fmt 0 BF16, 1 e4m3)
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= r * n) return;
  const int64_t j = e / n, i = row0 + (e % n);
  U4 c{static_cast<uint32_t>(static_cast<uint64_t>(i) >> 3),
       static_cast<uint32_t>(static_cast<uint64_t>(i) >> 35),
       static_cast<uint32_t>(j), static_cast<uint32_t>(kStreamGaussQ)};
  const U4 o = philox10(c, static_cast<uint32_t>(seed),
                        static_cast<uint32_t>(seed >> 32));
  const uint32_t w4[4] = {o.x, o.y, o.z, o.w};
  const uint32_t v = (w4[(i >> 1) & 3] >> (16 * (i & 1))) & 0xFFFFu;
  const uint32_t b = g_qtab[fmt][v & 0x7FFFu] | (v & 0x8000u);
  out[e] = __uint_as_float(b << 16);
}

// Slices of rows for a grid of `tiles` workgroups per slice: slices of at
// most 2^18 rows (multiples of kQK), as many as fit the 256 CUs in one round
// of one workgroup each (at least one slice, at least one step per slice)
int64_t q_split(int64_t n, int64_t tiles, int64_t* splits) {
  const int64_t steps = (n + kQK - 1) / kQK;
  int64_t s = 256 / tiles;
  const int64_t need = (n + (int64_t{1} << 18) - 1) >> 18;
  if (s < need) s = need;
  if (s > steps) s = steps;
  if (s < 1) s = 1;
  int64_t per = (steps + s - 1) / s * kQK;
  *splits = (n + per - 1) / per;
  return per;
}

std::mutex g_qtab_mu;
bool g_qtab_ready[64] = {};

inline bool vec_ok(int dtype, int64_t d, int64_t ld, const void* x) {
  const uintptr_t addr = reinterpret_cast<uintptr_t>(x);
  return d % 8 == 0 && ld % 8 == 0 && addr % (dtype == 2 ? 16 : 8) == 0;
}

}  // namespace

int init_quantile_tables(int device) {
  std::lock_guard<std::mutex> g(g_qtab_mu);
  if (device >= 0 && device < 64 && g_qtab_ready[device]) return 0;
  const QTables& tabs = host_tables();
  if (hipMemcpyToSymbol(HIP_SYMBOL(g_qtab), tabs.t, sizeof(tabs.t), 0,
                        hipMemcpyHostToDevice) != hipSuccess)
    return -1;
  if (device >= 0 && device < 64) g_qtab_ready[device] = true;
  return 0;
}

size_t gauss_q_partial_bytes(int64_t n, int64_t r, int64_t d) {
  const int64_t tiles = ((r + kQR - 1) / kQR) * ((d + kQD - 1) / kQD);
  int64_t splits;
  q_split(n, tiles, &splits);
  return static_cast<size_t>(splits * r * d) * sizeof(float);
}

// the quantile form applies to BF16 (dtype 2) and FP8 (dtype 3) input
bool gauss_q_dtype(int dtype) { return dtype == 2 || dtype == 3; }

void launch_gauss_q_sketch(const void* x, int dtype, int64_t n, int64_t d,
                           int64_t ld, uint64_t seed, int64_t r,
                           float* partial, int64_t* splits_out,
                           const float* col_scale, uint64_t* colmax,
                           int* nonfinite, hipStream_t s) {
  const int nrt = static_cast<int>((r + kQR - 1) / kQR);
  const int nct = static_cast<int>((d + kQD - 1) / kQD);
  int64_t splits;
  const int64_t per = q_split(n, static_cast<int64_t>(nrt) * nct, &splits);
  *splits_out = splits;
  const unsigned grid = static_cast<unsigned>(splits * nrt * nct);
  const bool vec = vec_ok(dtype, d, ld, x);
  unsigned long long* cm = reinterpret_cast<unsigned long long*>(colmax);
  const float* cs = dtype == 3 ? col_scale : nullptr;
  prof_begin(kKGaussSketch, s);
  if (dtype == 2) {
    const uint16_t* xp = static_cast<const uint16_t*>(x);
    if (vec)
      gauss_q_kernel<1, true><<<grid, kQThreads, 0, s>>>(
          xp, n, d, ld, seed, r, per, nrt, nct, partial, cs, cm, nonfinite);
    else
      gauss_q_kernel<1, false><<<grid, kQThreads, 0, s>>>(
          xp, n, d, ld, seed, r, per, nrt, nct, partial, cs, cm, nonfinite);
  } else {
    const uint8_t* xp = static_cast<const uint8_t*>(x);
    if (vec)
      gauss_q_kernel<2, true><<<grid, kQThreads, 0, s>>>(
          xp, n, d, ld, seed, r, per, nrt, nct, partial, cs, cm, nonfinite);
    else
      gauss_q_kernel<2, false><<<grid, kQThreads, 0, s>>>(
          xp, n, d, ld, seed, r, per, nrt, nct, partial, cs, cm, nonfinite);
  }
  prof_end(kKGaussSketch, s);
}

size_t gram_q_partial_bytes(int64_t n, int64_t d) {
  const int64_t nb = (d + kGB - 1) / kGB;
  int64_t splits;
  q_split(n, nb * (nb + 1) / 2, &splits);
  return static_cast<size_t>(splits * d * d) * sizeof(float);
}

void launch_gram_q(const void* x, int dtype, int64_t n, int64_t d, int64_t ld,
                   float* partial, int64_t* splits_out, hipStream_t s) {
  const int nb = static_cast<int>((d + kGB - 1) / kGB);
  const int ntiles = nb * (nb + 1) / 2;
  int64_t splits;
  const int64_t per = q_split(n, ntiles, &splits);
  *splits_out = splits;
  const unsigned grid = static_cast<unsigned>(splits * ntiles);
  const bool vec = vec_ok(dtype, d, ld, x);
  prof_begin(kKGram, s);
  if (dtype == 2) {
    const uint16_t* xp = static_cast<const uint16_t*>(x);
    if (vec)
      gram_q_kernel<1, true><<<grid, kQThreads, 0, s>>>(xp, n, d, ld, nb, ntiles,
                                                       per, partial);
    else
      gram_q_kernel<1, false><<<grid, kQThreads, 0, s>>>(xp, n, d, ld, nb,
                                                        ntiles, per, partial);
  } else {
    const uint8_t* xp = static_cast<const uint8_t*>(x);
    if (vec)
      gram_q_kernel<2, true><<<grid, kQThreads, 0, s>>>(xp, n, d, ld, nb, ntiles,
                                                       per, partial);
    else
      gram_q_kernel<2, false><<<grid, kQThreads, 0, s>>>(xp, n, d, ld, nb,
                                                        ntiles, per, partial);
  }
  prof_end(kKGram, s);
}

void launch_gauss_q_entries(uint64_t seed, int64_t r, int64_t n, int64_t row0,
                            int fmt, float* out, hipStream_t s) {
  const int64_t tot = r * n;
  if (tot <= 0) return;
  gauss_q_entries_kernel<<<static_cast<unsigned>((tot + 255) / 256), 256, 0,
                           s>>>(seed, r, n, row0, fmt, out);
}

}  // namespace slso
