// Scores l_i = ||x_i M||^2 (Algorithm 2 step 4) for BF16 and FP8 input with
// d a multiple of 16 up to 512 and k <= 64: the pass that reads X once per
// job, so it is priced against HBM.
//
// M (d x 64, zero past k) enters the BF16 MFMA as BF16 parts held in LDS
// for the whole kernel, so a workgroup reads M once: three parts
// Mh = bf16(M), Mm = bf16(M - Mh), Ml = bf16(M - Mh - Mm) (M to FP32
// precision) while they fit, d <= 352 (138 KB); two, Mh and bf16(M - Mh)
// (M to 2^-17 of each entry), for 352 < d <= 512 (133 KB at d = 512). X goes from HBM straight into MFMA operand
// registers: for v_mfma_f32_32x32x16_bf16 lane l takes row l % 32 and 8
// consecutive columns, which are 16 contiguous bytes of a row-major BF16 row
// (8 bytes of FP8 codes, decoded by the packed FP8 conversion). A wave
// owns blocks of 32 rows (persistent: blocks wave, wave + W, ...), each
// taken in units of K-steps through a ring of register buffers (two halves
// for BF16, four quarters for FP8), each unit's loads issued one ring ahead. Sums are FP32 (products exact); the epilogue squares and adds the
// 64 columns in FP32.
#include "internal.h"

namespace slso {
namespace {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kSQThreads = 512;  // eight waves
constexpr int kSQHalf = 16;      // K-steps per half block
constexpr int kSQMaxD = 512;     // largest d (two halves of 16 K-steps)
constexpr int kSQMaxD3 = 352;    // largest d with three parts of M
constexpr int kSQLds = 3 * 64 * (kSQMaxD3 + 8) > 2 * 64 * (kSQMaxD + 8)
                           ? 3 * 64 * (kSQMaxD3 + 8)
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

// A operand (8 BF16) of K-step s for this lane: row `row`, columns
// 16 s + 8 h .. + 7 (raw: 16 bytes of BF16, or 8 bytes of FP8 codes)
template <int IT>
struct Raw;
template <>
struct Raw<1> {
  uint4 v;
};
template <>
struct Raw<2> {
  uint2 v;
};

template <int IT>
__device__ __forceinline__ Raw<IT> load_raw(const typename SQIn<IT>::T* p) {
  Raw<IT> r;
  if constexpr (IT == 1)
    r.v = *reinterpret_cast<const uint4*>(p);
  else
    r.v = *reinterpret_cast<const uint2*>(p);
  return r;
}

template <int IT>
__device__ __forceinline__ bf16x8 operand(const Raw<IT>& r) {
  if constexpr (IT == 1) {
    return __builtin_bit_cast(bf16x8, r.v);
  } else {
    uint4 o;
    o.x = e4m3x2_to_bf16x2<false>(r.v.x);
    o.y = e4m3x2_to_bf16x2<true>(r.v.x);
    o.z = e4m3x2_to_bf16x2<false>(r.v.y);
    o.w = e4m3x2_to_bf16x2<true>(r.v.y);
    return __builtin_bit_cast(bf16x8, o);
  }
}

// NP parts of M: mp[0] = Mh, mp[NP - 1] = the smallest part; KU register
// buffers (units of 32 / KU K-steps) per 32-row block
template <int IT, int NP, int KU>
__global__ void __launch_bounds__(kSQThreads)
    score_q_kernel(const typename SQIn<IT>::T* __restrict__ x, int64_t n,
                   int64_t d, int64_t ld, const uint16_t* __restrict__ mh,
                   const uint16_t* __restrict__ mm,
                   const uint16_t* __restrict__ ml, float* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) uint16_t sm[kSQLds];
  const int pm = static_cast<int>(d) + 8;  // LDS pitch of M (elements)
  uint16_t* Mh = sm;
  uint16_t* Mm = sm + 64 * pm;             // NP == 3 only
  uint16_t* Ml = sm + (NP - 1) * 64 * pm;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int l32 = lane & 31, h = lane >> 5;
  const int steps = static_cast<int>(d / 16);
  // M into LDS, 8 elements per access (d is a multiple of 16)
  for (int64_t e = t; e < 8 * d; e += kSQThreads) {
    const int64_t c = e / (d / 8), j = 8 * (e % (d / 8));
    *reinterpret_cast<uint4*>(&Mh[c * pm + j]) =
        *reinterpret_cast<const uint4*>(&mh[c * d + j]);
    *reinterpret_cast<uint4*>(&Ml[c * pm + j]) =
        *reinterpret_cast<const uint4*>(&ml[c * d + j]);
    if (NP == 3)
      *reinterpret_cast<uint4*>(&Mm[c * pm + j]) =
          *reinterpret_cast<const uint4*>(&mm[c * d + j]);
  }
  __syncthreads();

  const int64_t nblk = (n + 31) / 32;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 8;
  int64_t blk = static_cast<int64_t>(blockIdx.x) * 8 + w;
  using T = typename SQIn<IT>::T;
  auto rowptr = [&](int64_t b) -> const T* {
    int64_t row = b * 32 + l32;
    if (row >= n) row = n - 1;  // in bounds; the score is not written
    return x + row * ld + 8 * h;
  };
  // units of kUS K-steps (a block of at most 32 K-steps has kU of them)
  // through a ring of kU register buffers: a unit's loads are issued kU - 1
  // units ahead of its products. Loads are unconditional (a block past the
  // last reads the last block, a K-step past d reads the last K-step), so no
  // wait is placed at a branch. Measured at the precision shape: BF16 halves
  // (0.72 ms; quarters 0.73, eighths 0.77), FP8 quarters (0.55 ms; halves
  // 0.63, eighths 0.58): the defaults; slso_tune chooses per (d, dtype).
  // Every choice gives the same bits (the K-steps are summed in one order).
  constexpr int kU = KU;
  constexpr int kUS = 2 * kSQHalf / kU;  // K-steps per unit
  const int64_t blk0 = blk;
  Raw<IT> Q[kU][kUS];
  auto issue = [&](Raw<IT> (&buf)[kUS], int64_t u, int q) {
    int64_t b = blk0 + (u / kU) * stride;
    if (b >= nblk) b = nblk - 1;
    const T* p = rowptr(b);
#pragma unroll
    for (int s = 0; s < kUS; ++s) {
      const int ks = kUS * q + s < steps ? kUS * q + s : steps - 1;
      buf[s] = load_raw<IT>(p + 16 * ks);
    }
  };
  f16v acc[2];
  auto compute = [&](const Raw<IT> (&buf)[kUS], int q) {
#pragma unroll
    for (int s = 0; s < kUS; ++s) {
      const int ks = kUS * q + s;
      if (ks < steps) {
        const bf16x8 a = operand<IT>(buf[s]);
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          const int o = (32 * ct + l32) * pm + 16 * ks + 8 * h;
          const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&Ml[o]);
          acc[ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bl, acc[ct], 0, 0, 0);
          if constexpr (NP == 3) {
            const bf16x8 bm = *reinterpret_cast<const bf16x8*>(&Mm[o]);
            acc[ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bm, acc[ct], 0, 0, 0);
          }
          const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&Mh[o]);
          acc[ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bh, acc[ct], 0, 0, 0);
        }
      }
    }
  };
  if (blk0 < nblk) {
#pragma unroll
    for (int j = 0; j + 1 < kU; ++j) issue(Q[j], j, j);
  }
  int64_t u0 = 0;
  for (; blk < nblk; blk += stride, u0 += kU) {
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[ct][e] = 0.0f;
#pragma unroll
    for (int q = 0; q < kU; ++q) {
      // the buffer the previous unit used takes the unit kU - 1 ahead
      constexpr int kLast = kU - 1;
      const int nb = (q + kLast) % kU;
      issue(Q[nb], u0 + q + kLast, nb);
      compute(Q[q], q);
    }
    // l_i = sum over the 64 columns of the squares: register e of lane l
    // holds row (e % 4) + 8 (e / 4) + 4 h, column l % 32 (+ 32 ct)
    float v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e)
      v[e] = acc[0][e] * acc[0][e] + acc[1][e] * acc[1][e];
#pragma unroll
    for (int o = 1; o < 32; o <<= 1)
#pragma unroll
      for (int e = 0; e < 16; ++e) v[e] += __shfl_xor(v[e], o, 64);
    if (l32 < 16) {
      const int e = l32;
      const int64_t row = blk * 32 + (e % 4) + 8 * (e / 4) + 4 * h;
      float val = v[0];
#pragma unroll
      for (int q = 1; q < 16; ++q) val = e == q ? v[q] : val;
      if (row < n) out[row] = val;
    }
  }
}

}  // namespace

bool score_q_ok(const void* x, int dtype, int format, int64_t d, int64_t ld,
                int64_t k) {
  if (format != 0 || (dtype != 2 && dtype != 3) || k > 64 || k < 1) return false;
  if (d % 16 != 0 || d > kSQMaxD || ld % 8 != 0) return false;
  const uintptr_t a = reinterpret_cast<uintptr_t>(x);
  return a % (dtype == 2 ? 16 : 8) == 0;
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
  // register ring: choice 0, 1, 2 = 2, 4, 8 units per block
  if (choice < 0 || choice >= kScoreRingChoices) choice = tune_choice(kTuneScore, d, dtype);
  if (choice < 0) choice = dtype == 2 ? 0 : 1;
  prof_begin(kKScore, s);
#define SLSO_SQ(IT_, T_, NP_)                                                    \
  do {                                                                           \
    const T_* xp = static_cast<const T_*>(x);                                    \
    if (choice == 0)                                                             \
      score_q_kernel<IT_, NP_, 2><<<g, kSQThreads, 0, s>>>(xp, n, d, ld, mh, mm, \
                                                           ml, scores);          \
    else if (choice == 1)                                                        \
      score_q_kernel<IT_, NP_, 4><<<g, kSQThreads, 0, s>>>(xp, n, d, ld, mh, mm, \
                                                           ml, scores);          \
    else                                                                         \
      score_q_kernel<IT_, NP_, 8><<<g, kSQThreads, 0, s>>>(xp, n, d, ld, mh, mm, \
                                                           ml, scores);          \
  } while (0)
  if (dtype == 2) {
    if (three)
      SLSO_SQ(1, uint16_t, 3);
    else
      SLSO_SQ(1, uint16_t, 2);
  } else {
    if (three)
      SLSO_SQ(2, uint8_t, 3);
    else
      SLSO_SQ(2, uint8_t, 2);
  }
#undef SLSO_SQ
  prof_end(kKScore, s);
}

}  // namespace slso
