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
// takes 16 data rows through one of two LDS buffers: every thread stages a
// 2-row x 8-column block of X (one 4-byte LDS write per column), half the
// threads draw one Philox block each (8 entries of one sketch row), and wave
// w multiplies sketch rows 64 (w & 1) .. + 63 by columns 128 (w >> 1) ..
// + 127 as 2 x 4 MFMA blocks of 32 x 32 (v_mfma_f32_32x32x16_bf16). While a
// step's products run, the next step is written into the other buffer, rows
// three steps ahead are loaded and the entries two steps ahead drawn, so the
// generator's VALU work, the loads and the matrix unit overlap, with one
// barrier per step.
#include <cmath>
#include <cstring>
#include <mutex>
#include <type_traits>

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
constexpr int kQK = 16;         // data rows per step of the Gram pass
constexpr int kQP = 24;         // LDS pitch (elements) of its 16-row tiles
constexpr int kQThreads = 512;  // eight waves
constexpr int kSK = 32;         // data rows per step of the sketch

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

// a ^ b ^ k in one instruction (k uniform): gfx950's three-input logic op
// with the truth table of a three-way xor (0x96); the compiler forms two
// two-input xors here, and the generator's VALU work bounds the sketch
__device__ __forceinline__ uint32_t xor3k(uint32_t a, uint32_t b, uint32_t k) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "s"(k), "v"(a), "v"(b));
  return r;
}

// The Philox4x32-10 block of sketch row j for data rows 8 q .. 8 q + 7 (the
// same rounds as philox10, with the key folded in by xor3k)
__device__ __forceinline__ void draw_raw(uint64_t q, uint32_t j, uint32_t k0,
                                         uint32_t k1, uint32_t (&o4)[4]) {
  uint32_t c0 = static_cast<uint32_t>(q), c1 = static_cast<uint32_t>(q >> 32);
  uint32_t c2 = j, c3 = static_cast<uint32_t>(kStreamGaussQ);
#pragma unroll
  for (int rd = 0; rd < 10; ++rd) {
    if (rd > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = static_cast<uint64_t>(c0) * 0xD2511F53u;
    const uint64_t p1 = static_cast<uint64_t>(c2) * 0xCD9E8D57u;
    const uint32_t n0 = xor3k(static_cast<uint32_t>(p1 >> 32), c1, k0);
    const uint32_t n2 = xor3k(static_cast<uint32_t>(p0 >> 32), c3, k1);
    c1 = static_cast<uint32_t>(p1);
    c3 = static_cast<uint32_t>(p0);
    c0 = n0;
    c2 = n2;
  }
  o4[0] = c0;
  o4[1] = c1;
  o4[2] = c2;
  o4[3] = c3;
}

// its 8 entries as 4 words of BF16 pairs (lower data row in the low half)
__device__ __forceinline__ void entries8(const uint32_t (&o4)[4],
                                         const uint16_t* tab,
                                         uint32_t (&gw)[4]) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const uint32_t v = o4[u];
    const uint32_t lo = tab[v & 0x7FFFu];
    const uint32_t hi = tab[(v >> 16) & 0x7FFFu];
    gw[u] = (lo | (hi << 16)) | (v & 0x80008000u);
  }
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

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

// logical workgroup id: workgroups are dealt to the eight XCDs in turn
// (XCD = blockIdx mod 8), so numbering each XCD's workgroups consecutively
// (the XCDs before it hold q + 1 or q of the nb = 8 q + rem workgroups)
// gives workgroups that share a slice of rows of X the same XCD and L2
__device__ __forceinline__ unsigned xcd_logical() {
  const unsigned nb = gridDim.x, b = blockIdx.x;
  const unsigned xcd = b & 7u, q = nb >> 3, rem = nb & 7u;
  return xcd * q + (xcd < rem ? xcd : rem) + (b >> 3);
}

// ---- staging of X (shared by the sketch and the Gram pass) ------------------
// A step takes 16 data rows; a thread stages rows row, row + 1 and columns
// gcol .. gcol + 7 of X. The loads are issued unconditionally (rows past
// i_end read row i_end - 1, in bounds) into raw registers and only used a
// step or two later, so nothing waits for them at the issue point; rows at or
// past i_end are zeroed when the block is unpacked (pair_unpack) into BF16
// pairs xr[u][v] = row + u, columns 2 v (low half) and 2 v + 1. FP8 codes
// are decoded by the hardware conversion (e4m3x2_to_bf16x2, exact in BF16).
template <int IT>
struct RawPair;
template <>
struct RawPair<1> {
  uint4 q[2];
};
template <>
struct RawPair<2> {
  uint2 q[2];
};

template <int IT, bool VEC>
__device__ __forceinline__ void pair_issue(
    const typename QIn<IT>::T* __restrict__ x, int64_t ld, int64_t d,
    int64_t gcol, int64_t row, int64_t i_end, RawPair<IT>& raw) {
#pragma unroll
  for (int u = 0; u < 2; ++u) {
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

template <int IT>
__device__ __forceinline__ void pair_unpack(const RawPair<IT>& raw,
                                            int64_t nvalid,
                                            uint32_t (&xr)[2][4]) {
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    uint32_t v4[4];
    if constexpr (IT == 1) {
      v4[0] = raw.q[u].x;
      v4[1] = raw.q[u].y;
      v4[2] = raw.q[u].z;
      v4[3] = raw.q[u].w;
    } else {
      v4[0] = e4m3x2_to_bf16x2<false>(raw.q[u].x);
      v4[1] = e4m3x2_to_bf16x2<true>(raw.q[u].x);
      v4[2] = e4m3x2_to_bf16x2<false>(raw.q[u].y);
      v4[3] = e4m3x2_to_bf16x2<true>(raw.q[u].y);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) xr[u][v] = u < nvalid ? v4[v] : 0u;
  }
}

// |x| of the block folded into per-column maxima of BF16 bit patterns
// (packed pairs like xr): for non-negative values the pattern order is the
// numeric order, and Inf / NaN patterns (>= 0x7F80) exceed every finite one
__device__ __forceinline__ void pair_max(const uint32_t (&xr)[2][4],
                                         uint32_t (&mx)[4]) {
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const u16x2 a = __builtin_bit_cast(u16x2, mx[v]);
      const u16x2 b = __builtin_bit_cast(u16x2, xr[u][v] & 0x7FFF7FFFu);
      mx[v] = __builtin_bit_cast(uint32_t, __builtin_elementwise_max(a, b));
    }
}

// Rows k, k + 1 of a tile's columns 8 cc + e (e = 0..7, cc < NC) into a
// K-contiguous tile of 8 NC slots (pitch kQP): column 8 cc + e goes to
// slot NC e + cc, so that the 64 lanes of one store (eight chunks cc, eight
// row pairs) fall on the banks two lanes per bank, where a slot per column
// in order would put the eight chunks of a wave on the same banks
template <int NC>
__device__ __forceinline__ int q_slot_col(int slot) {
  return 8 * (slot % NC) + slot / NC;
}

template <int NC>
__device__ __forceinline__ void pair_store(uint16_t* T, int cc, int k,
                                           const uint32_t (&xr)[2][4]) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const uint32_t sel = (e & 1) ? 0x07060302u : 0x05040100u;
    *reinterpret_cast<uint32_t*>(&T[(NC * e + cc) * kQP + k]) =
        __builtin_amdgcn_perm(xr[1][e >> 1], xr[0][e >> 1], sel);
  }
}

// ---- the sketch's 32-row tiles ------------------------------------------------
// A slot (an X column or a sketch row) holds its 32 data rows contiguously as
// four 8-element groups, group q stored at position q ^ ((slot >> 1) & 3):
// the MFMA operand reads (16 bytes per lane, 32 consecutive slots, one group)
// and the staging writes below then spread over all banks, without padding.
__device__ __forceinline__ int qsw(int slot, int grp) {
  return slot * kSK + 8 * (grp ^ ((slot >> 1) & 3));
}

// Four-row blocks: a thread stages rows row .. row + 3 and columns gcol ..
// gcol + 7, loaded and masked as the two-row blocks above.
template <int IT>
struct RawQuad;
template <>
struct RawQuad<1> {
  uint4 q[4];
};
template <>
struct RawQuad<2> {
  uint2 q[4];
};

template <int IT, bool VEC>
__device__ __forceinline__ void quad_issue(
    const typename QIn<IT>::T* __restrict__ x, int64_t ld, int64_t d,
    int64_t gcol, int64_t row, int64_t i_end, RawQuad<IT>& raw) {
  RawPair<IT> lo, hi;
  pair_issue<IT, VEC>(x, ld, d, gcol, row, i_end, lo);
  pair_issue<IT, VEC>(x, ld, d, gcol, row + 2, i_end, hi);
  raw.q[0] = lo.q[0];
  raw.q[1] = lo.q[1];
  raw.q[2] = hi.q[0];
  raw.q[3] = hi.q[1];
}

template <int IT>
__device__ __forceinline__ void quad_unpack(const RawQuad<IT>& raw,
                                            int64_t nvalid,
                                            uint32_t (&xr)[4][4]) {
  RawPair<IT> lo, hi;
  lo.q[0] = raw.q[0];
  lo.q[1] = raw.q[1];
  hi.q[0] = raw.q[2];
  hi.q[1] = raw.q[3];
  uint32_t a[2][4], b[2][4];
  pair_unpack<IT>(lo, nvalid, a);
  pair_unpack<IT>(hi, nvalid - 2, b);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    xr[0][v] = a[0][v];
    xr[1][v] = a[1][v];
    xr[2][v] = b[0][v];
    xr[3][v] = b[1][v];
  }
}

// The same four rows where every row read is inside X and inside the slice:
// p points at row `row`, column gcol; no clamping and no masking.
template <int IT, bool VEC>
__device__ __forceinline__ void quad_issue_fast(
    const typename QIn<IT>::T* __restrict__ p, int64_t ld, int64_t d,
    int64_t gcol, RawQuad<IT>& raw) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const typename QIn<IT>::T* q = p + u * ld;
    if constexpr (VEC) {
      if constexpr (IT == 1)
        raw.q[u] = *reinterpret_cast<const uint4*>(q);
      else
        raw.q[u] = *reinterpret_cast<const uint2*>(q);
    } else {
      uint32_t e8[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) e8[e] = q[gcol + e < d ? e : 0];
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

template <int IT>
__device__ __forceinline__ void quad_unpack_fast(const RawQuad<IT>& raw,
                                                 uint32_t (&xr)[4][4]) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    if constexpr (IT == 1) {
      xr[u][0] = raw.q[u].x;
      xr[u][1] = raw.q[u].y;
      xr[u][2] = raw.q[u].z;
      xr[u][3] = raw.q[u].w;
    } else {
      xr[u][0] = e4m3x2_to_bf16x2<false>(raw.q[u].x);
      xr[u][1] = e4m3x2_to_bf16x2<true>(raw.q[u].x);
      xr[u][2] = e4m3x2_to_bf16x2<false>(raw.q[u].y);
      xr[u][3] = e4m3x2_to_bf16x2<true>(raw.q[u].y);
    }
  }
}

// rows 4 rg .. 4 rg + 3 of columns 8 cc + e into slot NC e + cc of a 32-row
// tile (one 8-byte write per column)
template <int NC>
__device__ __forceinline__ void quad_store(uint16_t* T, int cc, int rg,
                                           const uint32_t (&xr)[4][4]) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const uint32_t sel = (e & 1) ? 0x07060302u : 0x05040100u;
    uint2 v;
    v.x = __builtin_amdgcn_perm(xr[1][e >> 1], xr[0][e >> 1], sel);
    v.y = __builtin_amdgcn_perm(xr[3][e >> 1], xr[2][e >> 1], sel);
    *reinterpret_cast<uint2*>(&T[qsw(NC * e + cc, rg >> 1) + 4 * (rg & 1)]) = v;
  }
}

// Steps of 32 data rows through two LDS buffers, every thread doing the same
// work in every step: it writes the next step's block of X (four rows x
// eight columns, transposed) and its Philox block of the next step's entries
// (sketch row jr, data rows 8 g .. 8 g + 7) into the other buffer, issues the
// loads for three steps ahead, draws its block for two steps ahead and
// multiplies the current buffer; one barrier per step. With no branch in the
// step, the generator's VALU work can issue between the MFMAs.
template <int IT, bool VEC>
__global__ void __launch_bounds__(kQThreads)
    gauss_q_kernel(const typename QIn<IT>::T* __restrict__ x, int64_t n,
                   int64_t d, int64_t ld, uint64_t seed, int64_t r,
                   int64_t rows_per_split, int nrt, int nct,
                   float* __restrict__ partial, const float* __restrict__ cs,
                   unsigned long long* __restrict__ colmax,
                   int* __restrict__ nonfinite) {
  __shared__ __attribute__((aligned(16))) uint16_t tab[kQCells];
  __shared__ __attribute__((aligned(16))) uint16_t XT[2][kQD * kSK];
  __shared__ __attribute__((aligned(16))) uint16_t GT[2][kQR * kSK];
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
  const int nsteps = static_cast<int>((i_end - i_begin + kSK - 1) / kSK);

  {
    const uint4* src = reinterpret_cast<const uint4*>(g_qtab[IT == 2 ? 1 : 0]);
    uint4* dst = reinterpret_cast<uint4*>(tab);
    for (int e = t; e < kQCells / 8; e += kQThreads) dst[e] = src[e];
  }

  // staging role: rows 4 rg .. 4 rg + 3 of a step, columns col0 + 8 cc ..;
  // columns past d read column 0 (their products land in output columns
  // that are never stored)
  const int rg = t & 7, cc = t >> 3;
  const int64_t gcol = col0 + 8 * cc < d ? col0 + 8 * cc : 0;
  // generation role: sketch row row0 + jr, data rows 8 g .. 8 g + 7
  const int jr = t >> 2, g = t & 3;
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
  auto krow = [&](int st) { return i_begin + static_cast<int64_t>(st) * kSK; };
  auto draw_step = [&](int st, uint32_t (&o4)[4]) {
    draw_raw(static_cast<uint64_t>(krow(st) >> 3) + g, jctr, sk0, sk1, o4);
  };
  auto mma = [&](int st) {
    const int b = st & 1;
#pragma unroll
    for (int kh = 0; kh < 2; ++kh) {
      bf16x8 av[2], bv[4];
#pragma unroll
      for (int a = 0; a < 2; ++a)
        av[a] = *reinterpret_cast<const bf16x8*>(
            &GT[b][qsw(64 * wr + 32 * a + l32, 2 * kh + h)]);
#pragma unroll
      for (int c4 = 0; c4 < 4; ++c4)
        bv[c4] = *reinterpret_cast<const bf16x8*>(
            &XT[b][qsw(128 * wc + 32 * c4 + l32, 2 * kh + h)]);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c4 = 0; c4 < 4; ++c4)
          acc[a][c4] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              av[a], bv[c4], acc[a][c4], 0, 0, 0);
    }
  };

  // SAFE: rows are clamped into the slice and masked past its end (the last
  // slices). Otherwise every step lies inside the slice, whose row count is
  // even in steps, and the three steps of look-ahead past its end are still
  // rows of X, so rows are read and staged as they are.
  auto run = [&](auto safe_tag) {
    constexpr bool SAFE = decltype(safe_tag)::value;
    const int64_t stride = kSK * ld;
    const typename QIn<IT>::T* pnext = x + (i_begin + 4 * rg) * ld + gcol;
    auto issue = [&](int st, RawQuad<IT>& raw) {
      if constexpr (SAFE) {
        quad_issue<IT, VEC>(x, ld, d, gcol, krow(st) + 4 * rg, i_end, raw);
      } else {
        quad_issue_fast<IT, VEC>(pnext, ld, d, gcol, raw);
        pnext += stride;
      }
    };
    auto write_step = [&](int st, const RawQuad<IT>& raw,
                          const uint32_t (&o4)[4]) {
      const int b = st & 1;
      uint32_t gw[4];
      entries8(o4, tab, gw);
      uint32_t xr[4][4];
      if constexpr (SAFE)
        quad_unpack<IT>(raw, i_end - (krow(st) + 4 * rg), xr);
      else
        quad_unpack_fast<IT>(raw, xr);
      if (colmax && st % nrt == rt) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const u16x2 a = __builtin_bit_cast(u16x2, mx[v]);
            const u16x2 c = __builtin_bit_cast(u16x2, xr[u][v] & 0x7FFF7FFFu);
            mx[v] = __builtin_bit_cast(uint32_t, __builtin_elementwise_max(a, c));
          }
      }
      quad_store<kQD / 8>(XT[b], cc, rg, xr);
      *reinterpret_cast<uint4*>(&GT[b][qsw(jr, g)]) =
          make_uint4(gw[0], gw[1], gw[2], gw[3]);
    };

    RawQuad<IT> ra, rb;  // steps of even / odd index
    uint32_t o4[4];       // Philox words of the next step's block
    issue(0, ra);
    issue(1, rb);
    draw_step(0, o4);
    write_step(0, ra, o4);
    issue(2, ra);
    draw_step(1, o4);
    __syncthreads();
    // iteration st: buffer st & 1 holds step st. Steps past the slice's end
    // (SAFE) read its last row and stage zeros, so the loop body has no
    // conditional memory operations and runs in pairs (an odd count gets
    // one all-zero step).
    auto iter = [&](int st, RawQuad<IT>& rnext) {
      write_step(st + 1, rnext, o4);
      issue(st + 3, rnext);
      draw_step(st + 2, o4);
      mma(st);
      __syncthreads();
      // keeps the next step's unpacking (and its wait for the loads) after
      // the barrier
      __builtin_amdgcn_sched_barrier(0);
    };
    for (int st = 0; st < nsteps; st += 2) {
      iter(st, rb);
      iter(st + 1, ra);
    }
  };
  __syncthreads();  // tables in LDS
  // (element-wise loads of unaligned input always take the SAFE form)
  if constexpr (VEC) {
    if ((i_end - i_begin) % (2 * kSK) == 0 && i_end + 3 * kSK <= n) {
      run(std::false_type{});
    } else {
      run(std::true_type{});
    }
  } else {
    run(std::true_type{});
  }
  if (colmax) flush_max(mx, rg, col0 + 8 * cc, d, cs, colmax, nonfinite);

  // partial[slice][j][c]; accumulator register e of lane l holds
  // D[(e % 4) + 8 (e / 4) + 4 (l / 32)][l % 32], the column of slot l % 32
  // of the block
  float* P = partial + sp * r * d;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t c = col0 + q_slot_col<kQD / 8>(128 * wc + 32 * b + l32);
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t j = row0 + 64 * wr + 32 * a + (e % 4) + 8 * (e / 4) + 4 * h;
        if (j < r && c < d) P[j * d + c] = acc[a][b][e];
      }
    }
}

// ---- Gram matrix X^T X of BF16 / FP8 input (the refinement pass) -------------
// Output tile 256 x 256 of column blocks (A, B), A <= B, over one slice of
// rows; eight waves, wave w owns rows 64 (w & 3) .. + 63 and columns
// 128 (w >> 2) .. + 127 of the tile as 2 x 4 MFMA blocks. Threads 0-255
// stage block A and 256-511 block B (on the diagonal both stage the same
// block) into K-contiguous tiles, which serve both as the A^T and the B
// operand. Steps of 16 rows through two buffers with one barrier per step,
// loads three steps ahead, as in the sketch.
constexpr int kGB = 256;

template <int IT, bool VEC>
__global__ void __launch_bounds__(kQThreads)
    gram_q_kernel(const typename QIn<IT>::T* __restrict__ x, int64_t n,
                  int64_t d, int64_t ld, int nb, int ntiles,
                  int64_t rows_per_split, float* __restrict__ partial) {
  __shared__ __attribute__((aligned(16))) uint16_t TA[2][kGB * kQP];
  __shared__ __attribute__((aligned(16))) uint16_t TB[2][kGB * kQP];
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
  const int64_t i_begin = sp * rows_per_split;
  int64_t i_end = i_begin + rows_per_split;
  if (i_end > n) i_end = n;
  const int nsteps = static_cast<int>((i_end - i_begin + kQK - 1) / kQK);

  constexpr int kNC = kGB / 8;  // 32 chunks of 8 columns
  const int side = t >> 8, ts = t & 255;
  const int rp = ts & 7, cc = ts >> 3;
  const int64_t c0 = static_cast<int64_t>(side ? tb : ta) * kGB + 8 * cc;
  const int64_t gcol = c0 < d ? c0 : 0;
  const int lane = t & 63, w = t >> 6, l32 = lane & 31, h = lane >> 5;
  const int wr = w & 3, wc = w >> 2;

  f16v acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[a][b][e] = 0.0f;

  auto krow = [&](int st) { return i_begin + static_cast<int64_t>(st) * kQK; };
  auto write_step = [&](int st, const RawPair<IT>& raw) {
    uint32_t xr[2][4];
    pair_unpack<IT>(raw, i_end - (krow(st) + 2 * rp), xr);
    pair_store<kNC>(side ? TB[st & 1] : TA[st & 1], cc, 2 * rp, xr);
  };
  auto mma = [&](int st) {
    const uint16_t* A = TA[st & 1];
    const uint16_t* B = TB[st & 1];
    bf16x8 av[2], bv[4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
      av[a] = *reinterpret_cast<const bf16x8*>(
          &A[(64 * wr + 32 * a + l32) * kQP + 8 * h]);
#pragma unroll
    for (int b = 0; b < 4; ++b)
      bv[b] = *reinterpret_cast<const bf16x8*>(
          &B[(128 * wc + 32 * b + l32) * kQP + 8 * h]);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[a], bv[b],
                                                            acc[a][b], 0, 0, 0);
  };

  RawPair<IT> ra, rb, rc, rd;
  // four register buffers: step s is loaded into buffer s mod 4, five steps
  // (80 rows) ahead of its products
  pair_issue<IT, VEC>(x, ld, d, gcol, krow(0) + 2 * rp, i_end, ra);
  pair_issue<IT, VEC>(x, ld, d, gcol, krow(1) + 2 * rp, i_end, rb);
  pair_issue<IT, VEC>(x, ld, d, gcol, krow(2) + 2 * rp, i_end, rc);
  pair_issue<IT, VEC>(x, ld, d, gcol, krow(3) + 2 * rp, i_end, rd);
  write_step(0, ra);
  pair_issue<IT, VEC>(x, ld, d, gcol, krow(4) + 2 * rp, i_end, ra);
  __syncthreads();
  auto iter = [&](int st, RawPair<IT>& rnext) {
    write_step(st + 1, rnext);
    pair_issue<IT, VEC>(x, ld, d, gcol, krow(st + 5) + 2 * rp, i_end, rnext);
    mma(st);
    __syncthreads();
    __builtin_amdgcn_sched_barrier(0);
  };
  // steps past the slice's end read its last row and stage zeros (slices
  // hold whole groups of four steps except the last)
  for (int st = 0; st < nsteps; st += 4) {
    iter(st, rb);
    iter(st + 1, rc);
    iter(st + 2, rd);
    iter(st + 3, ra);
  }

  float* P = partial + sp * d * d;
  const int64_t a0 = static_cast<int64_t>(ta) * kGB, b0 = static_cast<int64_t>(tb) * kGB;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t j = b0 + q_slot_col<kNC>(128 * wc + 32 * b + l32);
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t i =
            a0 + q_slot_col<kNC>(64 * wr + 32 * a + (e % 4) + 8 * (e / 4) + 4 * h);
        if (i < d && j < d) P[i * d + j] = acc[a][b][e];
      }
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
// most 2^18 rows (multiples of 64, pairs of steps of both kernels), as many as
// fit the 256 CUs in one round of one workgroup each (at least one slice, at
// least one step per slice)
int64_t q_split(int64_t n, int64_t tiles, int64_t* splits) {
  const int64_t steps = (n + 2 * kSK - 1) / (2 * kSK);
  int64_t s = 256 / tiles;
  const int64_t need = (n + (int64_t{1} << 18) - 1) >> 18;
  if (s < need) s = need;
  if (s > steps) s = steps;
  if (s < 1) s = 1;
  int64_t per = (steps + s - 1) / s * (2 * kSK);
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
