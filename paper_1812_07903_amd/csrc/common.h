// Shared device/host helpers of the slso library (gfx950, HIP).
//
// Random streams (the paper names no hash family or generator; these are the
// library's readings, implemented here from the published definitions):
//   * SplitMix64 finaliser (Steele, Lea & Flood 2014) derives the hash
//     coefficients from the seed on the host;
//   * CountSketch bucket/sign: degree-3 Carter-Wegman polynomial over the
//     Mersenne prime 2^61-1 (4-wise independent), Horner evaluation, bucket =
//     P1(i) mod r, sign = +1 when P2(i) is even;
//   * Gaussian entries: Philox4x32-10 (Salmon et al., SC'11) keyed by the seed
//     with counter (b>>1, lo32(a), hi32(a), stream), two 53-bit uniforms and
//     the Box-Muller transform in FP64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace slso {

constexpr uint64_t kP61 = (1ull << 61) - 1;

enum StreamId : uint32_t {
  kStreamBucket = 1,
  kStreamSign = 2,
  kStreamGaussS = 3,
  kStreamPi2 = 4,
  kStreamSwr = 5,
  kStreamSwor = 6,
  kStreamSrhtSign = 7,
  kStreamSrhtRows = 8,
  kStreamGaussQ = 9
};

struct HashCoeffs {
  uint64_t a[4];  // a0 + a1 i + a2 i^2 + a3 i^3 mod 2^61-1
};

// OSNAP hash j (block construction, at most kMaxOsnapNnz nonzeros per column
// of S): hash 0 takes the CountSketch streams, hash j >= 1 streams 16 + 2j
// (bucket) and 17 + 2j (sign).
constexpr int kMaxOsnapNnz = 16;
inline uint32_t osnap_bucket_stream(int j) {
  return j == 0 ? kStreamBucket : static_cast<uint32_t>(16 + 2 * j);
}
inline uint32_t osnap_sign_stream(int j) {
  return j == 0 ? kStreamSign : static_cast<uint32_t>(17 + 2 * j);
}
struct OsnapCoeffs {
  HashCoeffs hb[kMaxOsnapNnz], hs[kMaxOsnapNnz];
};

// ---- host: coefficient derivation ----------------------------------------
inline uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

inline HashCoeffs make_hash_coeffs(uint64_t seed, uint32_t stream) {
  HashCoeffs h;
  uint64_t state = seed ^ (static_cast<uint64_t>(stream) * 0xD1B54A32D192ED03ull);
  for (int m = 0; m < 4; ++m) {
    state += 0x9E3779B97F4A7C15ull;
    h.a[m] = sm64_mix(state) % kP61;
  }
  return h;
}

// ---- device: arithmetic mod 2^61-1 ---------------------------------------
__device__ __forceinline__ uint64_t fold61(uint64_t x) {
  // x < 2^63: one fold gives <= 2^61, a conditional subtraction finishes
  x = (x & kP61) + (x >> 61);
  return x >= kP61 ? x - kP61 : x;
}

__device__ __forceinline__ uint64_t mulmod61(uint64_t a, uint64_t b) {
  // a, b < 2^61: a*b = hi*2^64 + lo with hi < 2^58, and 2^64 = 8 (mod p)
  const uint64_t lo = a * b;
  const uint64_t hi = __umul64hi(a, b);
  return fold61((lo & kP61) + (lo >> 61) + (hi << 3));
}

__device__ __forceinline__ uint64_t poly61(const HashCoeffs& h, uint64_t i) {
  uint64_t acc = fold61(mulmod61(h.a[3], i) + h.a[2]);
  acc = fold61(mulmod61(acc, i) + h.a[1]);
  acc = fold61(mulmod61(acc, i) + h.a[0]);
  return acc;
}

// ---- device: Philox4x32-10 and Box-Muller ----------------------------------
struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    // one 32 x 32 -> 64-bit product per multiplier (v_mad_u64_u32): faster
    // here than separate low and high halves
    const uint64_t p0 = static_cast<uint64_t>(c.x) * 0xD2511F53u;
    const uint64_t p1 = static_cast<uint64_t>(c.z) * 0xCD9E8D57u;
    U4 n;
    n.x = static_cast<uint32_t>(p1 >> 32) ^ c.y ^ k0;
    n.y = static_cast<uint32_t>(p1);
    n.z = static_cast<uint32_t>(p0 >> 32) ^ c.w ^ k1;
    n.w = static_cast<uint32_t>(p0);
    c = n;
  }
  return c;
}

// Standard normal entry (a, b) of a stream, FP64.
__device__ __forceinline__ double gauss64(uint64_t seed, uint32_t stream,
                                          uint64_t a, uint64_t b) {
  U4 c{static_cast<uint32_t>(b >> 1), static_cast<uint32_t>(a),
       static_cast<uint32_t>(a >> 32), stream};
  const U4 o = philox10(c, static_cast<uint32_t>(seed),
                        static_cast<uint32_t>(seed >> 32));
  const uint64_t m1 =
      ((static_cast<uint64_t>(o.x) << 21) | (o.y >> 11)) & ((1ull << 53) - 1);
  const uint64_t m2 =
      ((static_cast<uint64_t>(o.z) << 21) | (o.w >> 11)) & ((1ull << 53) - 1);
  const double u1 = (static_cast<double>(m1) + 1.0) * 0x1p-53;
  const double u2 = static_cast<double>(m2) * 0x1p-53;
  const double rad = sqrt(-2.0 * log(u1));
  const double ang = 6.283185307179586 * u2;  // (2 * pi in FP64) * u2
  return (b & 1) ? rad * sin(ang) : rad * cos(ang);
}

// ---- device: input element decoding ---------------------------------------
__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
  return __uint_as_float(static_cast<uint32_t>(b) << 16);
}

// Two OCP e4m3fn codes, bytes 0 and 1 of the low (HI false) or high 16-bit
// half of w, as two BF16 values packed low / high. gfx950's packed FP8 ->
// FP32 conversion decodes e4m3fn exactly (all 256 codes checked against the
// decoding below, subnormals and NaN included); an e4m3 value has at most
// four significant bits, so the FP32 result's low 16 bits are zero and its
// high half is the BF16 value.
template <bool HI>
__device__ __forceinline__ uint32_t e4m3x2_to_bf16x2(uint32_t w) {
  const auto f = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(w), HI);
  return __builtin_amdgcn_perm(__float_as_uint(f[1]), __float_as_uint(f[0]),
                               0x07060302u);
}

// OCP fp8 e4m3fn: sign, 4 exponent bits (bias 7), 3 mantissa bits; the
// all-ones exponent with all-ones mantissa is NaN, there is no infinity.
__device__ __forceinline__ float e4m3_to_f32(uint8_t q) {
  const uint32_t s = (q >> 7) & 1u, e = (q >> 3) & 15u, m = q & 7u;
  float v;
  if (e == 0)
    v = static_cast<float>(m) * 0x1p-9f;
  else if (e == 15 && m == 7)
    v = __uint_as_float(0x7fc00000u);
  else
    v = __uint_as_float(((e + 120u) << 23) | (m << 20));
  return s ? -v : v;
}

// ---- wave helpers (wave64) -------------------------------------------------
__device__ __forceinline__ double shfl_xor_d(double v, int mask) {
  return __shfl_xor(v, mask, 64);
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace slso
