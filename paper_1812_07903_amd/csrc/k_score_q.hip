// Scores l_i = ||x_i M||^2 (Algorithm 2 step 4) for BF16 and FP8 input with
// d a multiple of 16 up to 512 and k <= 64: the pass that reads X once per
// job, so it is priced against HBM.
//
// M (d x 64, zero past k) enters the BF16 MFMA as BF16 parts held in LDS
// for the whole kernel, so a workgroup reads M once: three parts
// Mh = bf16(M), Mm = bf16(M - Mh), Ml = bf16(M - Mh - Mm) (M to FP32
// precision) while they fit, d <= 352 (at most 151 KB); two, Mh and
// bf16(M - Mh) (M to 2^-17 of each entry), for 352 < d <= 512 (133 KB at
// d = 512). X goes from HBM straight into MFMA operand registers: for
// v_mfma_f32_16x16x32_bf16 lane l takes row l % 16 and 8 K-values, here 16
// contiguous bytes of a row-major row (8 BF16, or 16 FP8 codes for two
// K-steps, decoded by the packed FP8 conversion). A wave owns blocks of 32
// rows (persistent: blocks wave, wave + W, ...), each taken in units of load
// steps through a ring of register buffers, each unit's loads issued one
// ring ahead. Sums are FP32 (products exact); the epilogue squares and adds
// the 64 columns in FP32.
#include "internal.h"

namespace slso {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kSQThreads = 512;  // eight waves
constexpr int kSQMaxD = 512;     // largest d
constexpr int kSQMaxD3 = 352;    // largest d with three parts of M
// M's depth in LDS is d rounded up to a load step (64 columns for FP8)
constexpr int kSQLds = 3 * 64 * (384 + 8) > 2 * 64 * (kSQMaxD + 8)
                           ? 3 * 64 * (384 + 8)
                           : 2 * 64 * (kSQMaxD + 8);

__device__ __forceinline__ uint16_t bf16_bits_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
  return static_cast<uint16_t>(u);
}

// Mh, Ml by column (k contiguous, ldm = d), 64 columns, zero past k
__global__ void split_m2_kernel(const double* __restrict__ m64, int64_t d,
                                int64_t k, uint16_t* __restrict__ mh,
                                uint16_t* __restrict__ ml) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= 64 * d) return;
  const int64_t c = e / d, j = e % d;
  const double v = c < k ? m64[j * k + c] : 0.0;
  const uint16_t hb = bf16_bits_rne(static_cast<float>(v));
  const double rest = v - static_cast<double>(__uint_as_float(
                              static_cast<uint32_t>(hb) << 16));
  mh[c * d + j] = hb;
  ml[c * d + j] = bf16_bits_rne(static_cast<float>(rest));
}

// Mh, Mm, Ml by column: Mh = bf16(M), Mm = bf16(M - Mh), Ml = bf16(M - Mh - Mm)
__global__ void split_m3_kernel(const double* __restrict__ m64, int64_t d,
                                int64_t k, uint16_t* __restrict__ mh,
                                uint16_t* __restrict__ mm,
                                uint16_t* __restrict__ ml) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= 64 * d) return;
  const int64_t c = e / d, j = e % d;
  double v = c < k ? m64[j * k + c] : 0.0;
  const uint16_t hb = bf16_bits_rne(static_cast<float>(v));
  v -= static_cast<double>(__uint_as_float(static_cast<uint32_t>(hb) << 16));
  const uint16_t mb = bf16_bits_rne(static_cast<float>(v));
  v -= static_cast<double>(__uint_as_float(static_cast<uint32_t>(mb) << 16));
  mh[c * d + j] = hb;
  mm[c * d + j] = mb;
  ml[c * d + j] = bf16_bits_rne(static_cast<float>(v));
}

template <int IT>
struct SQIn;
template <>
struct SQIn<1> {
  using T = uint16_t;
};
template <>
struct SQIn<2> {
  using T = uint8_t;
};

// MFMA operand (8 BF16) from a lane's 16 loaded bytes: BF16 as is; FP8
// codes 8 e .. 8 e + 7 decoded by the packed conversion
template <int IT>
__device__ __forceinline__ bf16x8 operand(const uint4& r, int e) {
  if constexpr (IT == 1) {
    (void)e;
    return __builtin_bit_cast(bf16x8, r);
  } else {
    const uint32_t w0 = e == 0 ? r.x : r.z, w1 = e == 0 ? r.y : r.w;
    uint4 o;
    o.x = e4m3x2_to_bf16x2<false>(w0);
    o.y = e4m3x2_to_bf16x2<true>(w0);
    o.z = e4m3x2_to_bf16x2<false>(w1);
    o.w = e4m3x2_to_bf16x2<true>(w1);
    return __builtin_bit_cast(bf16x8, o);
  }
}

__device__ __forceinline__ f4v mfma16(bf16x8 a, bf16x8 b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// NP parts of M: mp[0] = Mh, mp[NP - 1] = the smallest part; d <= MAXD
// (sizes the register ring); KU register buffers (units of load steps) per
// 32-row block
template <int IT, int NP, int MAXD, int KU>
__global__ void __launch_bounds__(kSQThreads)
    score_q_kernel(const typename SQIn<IT>::T* __restrict__ x, int64_t n,
                   int64_t d, int64_t ld, const uint16_t* __restrict__ mh,
                   const uint16_t* __restrict__ mm,
                   const uint16_t* __restrict__ ml, float* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) uint16_t sm[kSQLds];
  using T = typename SQIn<IT>::T;
  constexpr int kLW = IT == 1 ? 32 : 64;  // columns of X per load step
  constexpr int kCW = kLW / 4;            // of them per lane (16 bytes)
  const int nls = static_cast<int>((d + kLW - 1) / kLW);
  const int dp = nls * kLW;               // depth of M in LDS, zero past d
  const int pm = dp + 8;                  // LDS pitch of M (elements)
  uint16_t* Mh = sm;
  uint16_t* Mm = sm + 64 * pm;            // NP == 3 only
  uint16_t* Ml = sm + (NP - 1) * 64 * pm;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  // M into LDS, 8 elements per access (d is a multiple of 16)
  for (int e = t; e < 8 * dp; e += kSQThreads) {
    const int c = e / (dp / 8), j = 8 * (e % (dp / 8));
    uint4 vh = {0u, 0u, 0u, 0u}, vm = vh, vl = vh;
    if (j < d) {
      vh = *reinterpret_cast<const uint4*>(&mh[c * d + j]);
      vl = *reinterpret_cast<const uint4*>(&ml[c * d + j]);
      if (NP == 3) vm = *reinterpret_cast<const uint4*>(&mm[c * d + j]);
    }
    *reinterpret_cast<uint4*>(&Mh[c * pm + j]) = vh;
    *reinterpret_cast<uint4*>(&Ml[c * pm + j]) = vl;
    if (NP == 3) *reinterpret_cast<uint4*>(&Mm[c * pm + j]) = vm;
  }
  __syncthreads();

  // A wave owns blocks of 32 rows as two 16-row MFMA tiles. Load step s
  // gives lane (row r16, group g) 16 contiguous bytes of its row, columns
  // kLW s + kCW g .. + kCW - 1, so one load instruction reads 64 contiguous
  // bytes of each of 16 rows (a read pattern that streams about a tenth
  // faster than 32 bytes of each of 32 rows). The MFMA pairs element i of
  // lane group g in A with the same element of the same group in B, so any
  // assignment of columns to (step, group, element) gives x_i M as long as M
  // is read with it: BF16 step s is one K-step (columns 32 s + 8 g + i), an
  // FP8 step two (columns 64 s + 16 g + 8 e + i, e = 0, 1).
  const int64_t nblk = (n + 31) / 32;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 8;
  int64_t blk = static_cast<int64_t>(blockIdx.x) * 8 + w;
  const int clast = static_cast<int>(d) - kCW;
  auto rowptr = [&](int64_t b, int rb) -> const T* {
    int64_t row = b * 32 + 16 * rb + r16;
    if (row >= n) row = n - 1;  // in bounds; the score is not written
    return x + row * ld;
  };
  // units of kUS load steps through a ring of KU register buffers: a unit's
  // loads are issued KU - 1 units ahead of its products. Loads are
  // unconditional (a block past the last reads the last block, a step past
  // d the last columns of the row), so no wait is placed at a branch; a
  // lane's columns past d enter the MFMA as zeros. slso_tune chooses KU per
  // (d, dtype); every choice gives the same bits (the K-steps are summed in
  // one order).
  constexpr int kMaxLS = (MAXD + kLW - 1) / kLW;  // load steps at d = MAXD
  constexpr int kUS = (kMaxLS + KU - 1) / KU;      // load steps per unit
  const int64_t blk0 = blk;
  uint4 Q[KU][kUS][2];
  auto issue = [&](uint4 (&buf)[kUS][2], int64_t u, int q) {
    int64_t b = blk0 + (u / KU) * stride;
    if (b >= nblk) b = nblk - 1;
    const T* p0 = rowptr(b, 0);
    const T* p1 = rowptr(b, 1);
#pragma unroll
    for (int s = 0; s < kUS; ++s) {
      int c = kLW * (kUS * q + s) + kCW * g;
      c = c < clast ? c : clast;
      buf[s][0] = *reinterpret_cast<const uint4*>(p0 + c);
      buf[s][1] = *reinterpret_cast<const uint4*>(p1 + c);
    }
  };
  f4v acc[2][4];
  // the products of a unit as a sequence of (step, half, column tile)
  // items; each item's NP LDS reads of M are issued one item ahead, so their
  // latency runs under the previous item's MFMAs. Per accumulator the parts
  // are added smallest first.
  constexpr int kE = IT == 1 ? 1 : 2;  // K-steps per load step
  constexpr int kJ = kUS * kE * 4;
  struct BOp {
    bf16x8 p[NP];
  };
  auto read_b = [&](int j, int q, BOp& b) {
    const int s = j / (4 * kE), e = (j / 4) % kE, ct = j % 4;
    const int o = (16 * ct + r16) * pm + kLW * (kUS * q + s) + kCW * g + 8 * e;
    b.p[0] = *reinterpret_cast<const bf16x8*>(&Ml[o]);
    if constexpr (NP == 3) b.p[1] = *reinterpret_cast<const bf16x8*>(&Mm[o]);
    b.p[NP - 1] = *reinterpret_cast<const bf16x8*>(&Mh[o]);
  };
  auto compute = [&](const uint4 (&buf)[kUS][2], int q) {
    BOp bb[2];
    read_b(0, q, bb[0]);
    bf16x8 a0 = bf16x8{}, a1 = bf16x8{};
#pragma unroll
    for (int j = 0; j < kJ; ++j) {
      const int s = j / (4 * kE), e = (j / 4) % kE, ct = j % 4;
      const int ls = kUS * q + s;
      // (nothing moves across: the scheduler would otherwise hoist every
      // item's reads and run out of registers)
      __builtin_amdgcn_sched_barrier(0);
      if (j + 1 < kJ) read_b(j + 1, q, bb[(j + 1) & 1]);
      if (ct == 0) {
        a0 = operand<IT>(buf[s][0], e);
        a1 = operand<IT>(buf[s][1], e);
        if (kLW * ls + kCW * g + kCW > d) {
          a0 = bf16x8{};
          a1 = bf16x8{};
        }
      }
      if (ls < nls) {
#pragma unroll
        for (int pp = 0; pp < NP; ++pp) {
          acc[0][ct] = mfma16(a0, bb[j & 1].p[pp], acc[0][ct]);
          acc[1][ct] = mfma16(a1, bb[j & 1].p[pp], acc[1][ct]);
        }
      }
    }
  };
  if (blk0 < nblk) {
#pragma unroll
    for (int j = 0; j + 1 < KU; ++j) issue(Q[j], j, j);
  }
  int64_t u0 = 0;
  for (; blk < nblk; blk += stride, u0 += KU) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) acc[rb][ct] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int q = 0; q < KU; ++q) {
      // the buffer the previous unit used takes the unit KU - 1 ahead
      constexpr int kLast = KU - 1;
      const int nb = (q + kLast) % KU;
      issue(Q[nb], u0 + q + kLast, nb);
      compute(Q[q], q);
    }
    // l_i = sum over the 64 columns of the squares: register v of lane l
    // of tile (rb, ct) holds row 16 rb + 4 (l / 16) + v, column 16 ct + l % 16
    float v[8];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        float sq = acc[rb][0][e] * acc[rb][0][e];
#pragma unroll
        for (int ct = 1; ct < 4; ++ct) sq += acc[rb][ct][e] * acc[rb][ct][e];
        v[4 * rb + e] = sq;
      }
#pragma unroll
    for (int o = 1; o < 16; o <<= 1)
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] += __shfl_xor(v[e], o, 64);
    if (r16 < 8) {
      const int e = r16;
      const int64_t row = blk * 32 + 16 * (e >> 2) + 4 * g + (e & 3);
      float val = v[0];
#pragma unroll
      for (int q = 1; q < 8; ++q) val = e == q ? v[q] : val;
      if (row < n) out[row] = val;
    }
  }
}

}  // namespace

bool score_q_ok(const void* x, int dtype, int format, int64_t d, int64_t ld,
                int64_t k) {
  if (format != 0 || (dtype != 2 && dtype != 3) || k > 64 || k < 1) return false;
  // 16-byte loads: 8 BF16 or 16 FP8 codes at a multiple of as many columns
  if (d % 16 != 0 || d > kSQMaxD || ld % (dtype == 2 ? 8 : 16) != 0) return false;
  return reinterpret_cast<uintptr_t>(x) % 16 == 0;
}

size_t score_q_scratch_bytes(int64_t d) {
  return static_cast<size_t>(3 * 64 * d) * sizeof(uint16_t);
}

void launch_score_q(const void* x, int dtype, int64_t n, int64_t d, int64_t ld,
                    const double* m64, int64_t k, void* scratch, float* scores,
                    hipStream_t s, int choice) {
  uint16_t* mh = static_cast<uint16_t*>(scratch);
  uint16_t* mm = mh + 64 * d;
  uint16_t* ml = mm + 64 * d;
  const bool three = d <= kSQMaxD3;
  const unsigned gs = static_cast<unsigned>((64 * d + 255) / 256);
  if (three)
    split_m3_kernel<<<gs, 256, 0, s>>>(m64, d, k, mh, mm, ml);
  else
    split_m2_kernel<<<gs, 256, 0, s>>>(m64, d, k, mh, ml);
  const int64_t nblk = (n + 31) / 32;
  int64_t grid = (nblk + 7) / 8;
  if (grid > 256) grid = 256;
  const unsigned g = static_cast<unsigned>(grid);
  // register ring: choice 0, 1, 2 = 2, 4, 8 units per block; untuned, two
  // (the fastest for BF16 and FP8 at the precision shape: 0.75 / 0.50 ms
  // against 0.80-0.84 / 0.56 ms)
  if (choice < 0 || choice >= kScoreRingChoices) choice = tune_choice(kTuneScore, d, dtype);
  if (choice < 0) choice = 0;
  prof_begin(kKScore, s);
#define SLSO_SQ(IT_, T_, NP_, MAXD_)                                             \
  do {                                                                           \
    const T_* xp = static_cast<const T_*>(x);                                    \
    if (choice == 0)                                                             \
      score_q_kernel<IT_, NP_, MAXD_, 2><<<g, kSQThreads, 0, s>>>(               \
          xp, n, d, ld, mh, mm, ml, scores);                                     \
    else if (choice == 1)                                                        \
      score_q_kernel<IT_, NP_, MAXD_, 4><<<g, kSQThreads, 0, s>>>(               \
          xp, n, d, ld, mh, mm, ml, scores);                                     \
    else                                                                         \
      score_q_kernel<IT_, NP_, MAXD_, 8><<<g, kSQThreads, 0, s>>>(               \
          xp, n, d, ld, mh, mm, ml, scores);                                     \
  } while (0)
  // the ring holds a block's loads at the class's largest d: d <= 128 and
  // d <= 352 (three parts of M), d <= 512 (two)
  if (dtype == 2) {
    if (d <= 128)
      SLSO_SQ(1, uint16_t, 3, 128);
    else if (three)
      SLSO_SQ(1, uint16_t, 3, kSQMaxD3);
    else
      SLSO_SQ(1, uint16_t, 2, kSQMaxD);
  } else {
    if (d <= 128)
      SLSO_SQ(2, uint8_t, 3, 128);
    else if (three)
      SLSO_SQ(2, uint8_t, 3, kSQMaxD3);
    else
      SLSO_SQ(2, uint8_t, 2, kSQMaxD);
  }
#undef SLSO_SQ
  prof_end(kKScore, s);
}

}  // namespace slso
