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

#include <type_traits>

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

// One wave per CSR row; lanes own columns of M (64 at a time). The row's
// entries are read by one lane each (64 at a time) and taken in order from
// there, so the loads of M's rows do not wait on the index loads one by one:
// eight of them are issued before their products are added (FP64, in entry
// order).
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
    const int64_t cc = c < k ? c : k - 1;  // in bounds; its sum is dropped
    double y = 0.0;
    for (int64_t eb = e0; eb < e1; eb += 64) {
      const int ne = static_cast<int>(e1 - eb < 64 ? e1 - eb : 64);
      int32_t jl = 0;
      float vl = 0.0f;
      if (lane < ne) {
        jl = col_idx[eb + lane];
        vl = val[eb + lane];
      }
      constexpr int kU = 8;  // (16 measured slower)
      for (int q0 = 0; q0 < ne; q0 += kU) {
        float mv[kU], vv[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int q = q0 + u < ne ? q0 + u : ne - 1;
          const int64_t j = __builtin_amdgcn_readlane(jl, q);
          vv[u] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vl), q));
          mv[u] = m[j * k + cc];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u)
          if (q0 + u < ne)
            y += static_cast<double>(vv[u]) * static_cast<double>(mv[u]);
      }
    }
    if (c >= k) y = 0.0;
    tot += y * y;
  }
  tot = wave_sum_d(tot);
  if (lane == 0) out[row] = static_cast<float>(tot);
}

// ---- MFMA scoring for k <= 64 ------------------------------------------------
// A workgroup of four waves scores 128 rows; wave w owns rows 32w .. 32w + 31
// and all 64 columns of M (two 32 x 32 accumulator tiles). The contraction
// over d runs in chunks of 32: X (128 x 32) and M (32 x 64) are staged in
// LDS, double-buffered (the next chunk is loaded into registers while this
// one multiplies), the chunk's products summed on MFMA in FP32 and added
// to FP64 accumulators, so the error is that of 32-term FP32 sums.
//   FP32 input: v_mfma_f32_32x32x2f32 on FP32 X and FP32 M.
//   BF16 / FP8 input: v_mfma_f32_32x32x16_bf16 on X (exact in BF16) and three
//   BF16 parts of M (M = Mh + Mm + Ml, |M - Mh - Mm - Ml| <= 2^-24 |M|).
//   FP32 input, split form (IT 3): split-BF16 emulation of the FP32 product
//   (Henry, Tang and Heinecke 2019). Each X operand is cut, as it leaves LDS,
//   into X1 = bf16(X), X2 = bf16(X - X1), X3 = bf16(X - X1 - X2), which sum to
//   X exactly for normal FP32 values; with M's three parts, the six products
//   Xi Mj with i + j <= 4 are taken (smallest first) on the BF16 MFMA, each
//   exact in the FP32 accumulation; the three dropped ones are below 2^-23
//   |X| |M| together. It needs a sixth of the FP32 MFMA's cycles per flop
//   times six products: the pass is then bound by reading X.
// Epilogue: l_i = sum over the 64 columns of the squared FP64 accumulators.
// Accumulator register e of lane l holds row (e % 4) + 8 (e / 4) + 4 (l / 32)
// and column l % 32 of its tile.
constexpr int kMR = 128;     // rows per workgroup
constexpr int kMC = 32;      // contraction chunk
constexpr int kXS32 = 33;    // LDS row stride (floats) of the FP32 X tile
constexpr int kXS36 = 36;    // the same for the split form (16-byte rows)
constexpr int kXS16 = 40;    // LDS row stride (bf16) of the BF16 tiles

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
  return static_cast<uint16_t>(u);
}

template <int IT>
struct XIn;
template <>
struct XIn<0> {
  using T = float;
};
template <>
struct XIn<1> {
  using T = uint16_t;
};
template <>
struct XIn<2> {
  using T = uint8_t;
};
// FP32 input multiplied as three BF16 parts (see the kernel header)
template <>
struct XIn<3> {
  using T = float;
};

// BF16 bits of input element v (FP8 e4m3 values are exact in BF16)
__device__ __forceinline__ uint16_t in_bf16(uint16_t v) { return v; }
__device__ __forceinline__ uint16_t in_bf16(uint8_t q) {
  return f32_to_bf16_bits(e4m3_to_f32(q));
}

// 32-lane butterfly sum (lanes l and l ^ 32 are kept apart)
__device__ __forceinline__ double sum32(double v) {
#pragma unroll
  for (int o = 1; o < 32; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// kVec (the split form, IT 3: ld a multiple of 4, d of 8, 16-byte aligned X
// and parts of M): the staging loads are 4-float vectors of X and 8-element
// vectors of M's parts, a fraction of the load instructions and cache-line
// lookups of the element-wise form
template <int IT, bool kVec = false>
__global__ void __launch_bounds__(256)
    score_mfma_kernel(const typename XIn<IT>::T* __restrict__ x, int64_t n,
                      int64_t d, int64_t ld, const float* __restrict__ m32,
                      int64_t k, const uint16_t* __restrict__ mh,
                      const uint16_t* __restrict__ mm,
                      const uint16_t* __restrict__ ml, int64_t ldm,
                      float* __restrict__ out) {
  // FP32: X[2][128][33] f32 + M[2][32][64] f32; BF16: X[2][128][40] bf16 +
  // Mh, Mm, Ml[2][64][40] bf16 (M stored by column, k contiguous)
  static_assert(!kVec || IT == 3, "vector staging is the split form's");
  constexpr int kXBytes = IT == 0   ? kMR * kXS32 * 4
                          : IT == 3 ? kMR * kXS36 * 4
                                    : kMR * kXS16 * 2;
  constexpr int kMBytes = IT == 0 ? kMC * 64 * 4 : 3 * 64 * kXS16 * 2;
  __shared__ __attribute__((aligned(16))) unsigned char lds[2 * (kXBytes + kMBytes)];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int l32 = lane & 31, h = lane >> 5;
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * kMR;
  const int nch = static_cast<int>((d + kMC - 1) / kMC);

  f16v acc[2];
  double a64[2][16];
#pragma unroll
  for (int tt = 0; tt < 2; ++tt)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      acc[tt][e] = 0.0f;
      a64[tt][e] = 0.0;
    }

  // staging registers: X 16 elements per thread (row t/8 + 32 p, columns
  // 4 (t%8) .. +3), M 8 elements per thread
  using XT = typename XIn<IT>::T;
  // raw loaded values and which of them lie inside the matrix: the zeros
  // are put in when the stage goes to LDS, so no load is waited for early
  struct SStage {
    XT xr[16];
    float mr[8];
    uint16_t mhr[8], mmr[8], mlr[8];
    uint4 mq[3];  // split form: 8 k of one column of Mh, Mm, Ml
    uint32_t okx, okm;
  };
  auto load_chunk = [&](int ch, SStage& st) {
    const int64_t c0 = static_cast<int64_t>(ch) * kMC;
    st.okx = 0u;
    st.okm = 0u;
    if constexpr (kVec) {
      // X: row t/8 + 32 pp, columns 4 (t%8) .. +3 as one vector
#pragma unroll
      for (int pp = 0; pp < 4; ++pp) {
        const int64_t gr = row0 + t / 8 + 32 * pp;
        const int64_t gc = c0 + 4 * (t % 8);
        const bool ok = gr < n && gc < d;
        const float4 q = *reinterpret_cast<const float4*>(x + (ok ? gr * ld + gc : 0));
        st.xr[4 * pp] = q.x;
        st.xr[4 * pp + 1] = q.y;
        st.xr[4 * pp + 2] = q.z;
        st.xr[4 * pp + 3] = q.w;
        st.okx |= ok ? (0xfu << (4 * pp)) : 0u;
      }
      // M: column t / 4 of each part, k = c0 + 8 (t % 4) .. + 7 (d is a
      // multiple of 8, so the eight are all inside or all outside)
      const int64_t gk = c0 + 8 * (t % 4);
      const bool ok = gk < d;
      const int64_t i = ok ? (t / 4) * ldm + gk : 0;
      st.mq[0] = *reinterpret_cast<const uint4*>(mh + i);
      st.mq[1] = *reinterpret_cast<const uint4*>(mm + i);
      st.mq[2] = *reinterpret_cast<const uint4*>(ml + i);
      st.okm = ok ? 1u : 0u;
      return;
    }
    if constexpr (!kVec) {
#pragma unroll
    for (int pp = 0; pp < 4; ++pp) {
      const int r = t / 8 + 32 * pp;
      const int64_t gr = row0 + r;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        // an entry outside reads x[0] (zeroed at the store)
        const int64_t gc = c0 + 4 * (t % 8) + u;
        const bool ok = gr < n && gc < d;
        st.xr[4 * pp + u] = x[ok ? gr * ld + gc : 0];
        st.okx |= ok ? (1u << (4 * pp + u)) : 0u;
      }
    }
    }
    if constexpr (IT == 0) {
      // M rows c0 .. c0 + 31, 64 columns: element e = t + 256 v
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int e = t + 256 * v;
        const int kr = e / 64, cc = e % 64;
        const int64_t gk = c0 + kr;
        const bool ok = gk < d && cc < k;
        st.mr[v] = m32[ok ? gk * k + cc : 0];
        st.okm |= ok ? (1u << v) : 0u;
      }
    } else {
      // Mh / Ml by column: 64 columns x 32 k, element e = t + 256 v
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int e = t + 256 * v;
        const int cc = e / 32, kr = e % 32;
        const int64_t gk = c0 + kr;
        const bool ok = gk < d;
        const int64_t i = ok ? cc * ldm + gk : 0;
        st.mhr[v] = mh[i];
        st.mmr[v] = mm[i];
        st.mlr[v] = ml[i];
        st.okm |= ok ? (1u << v) : 0u;
      }
    }
  };
  auto store_chunk = [&](int buf, const SStage& st) {
    unsigned char* xb = lds + buf * kXBytes;
    unsigned char* mb = lds + 2 * kXBytes + buf * kMBytes;
    if constexpr (IT == 3) {
      float* X = reinterpret_cast<float*>(xb);
#pragma unroll
      for (int pp = 0; pp < 4; ++pp) {
        float4 q;
        q.x = ((st.okx >> (4 * pp)) & 1u) ? st.xr[4 * pp] : 0.0f;
        q.y = ((st.okx >> (4 * pp + 1)) & 1u) ? st.xr[4 * pp + 1] : 0.0f;
        q.z = ((st.okx >> (4 * pp + 2)) & 1u) ? st.xr[4 * pp + 2] : 0.0f;
        q.w = ((st.okx >> (4 * pp + 3)) & 1u) ? st.xr[4 * pp + 3] : 0.0f;
        *reinterpret_cast<float4*>(&X[(t / 8 + 32 * pp) * kXS36 + 4 * (t % 8)]) = q;
      }
    }
    if constexpr (IT == 0) {
      float* X = reinterpret_cast<float*>(xb);
#pragma unroll
      for (int pp = 0; pp < 4; ++pp)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          X[(t / 8 + 32 * pp) * kXS32 + 4 * (t % 8) + u] =
              ((st.okx >> (4 * pp + u)) & 1u) ? st.xr[4 * pp + u] : 0.0f;
      float* M = reinterpret_cast<float*>(mb);
#pragma unroll
      for (int v = 0; v < 8; ++v)
        M[t + 256 * v] = ((st.okm >> v) & 1u) ? st.mr[v] : 0.0f;
    } else {
      if constexpr (IT != 3) {
        uint16_t* X = reinterpret_cast<uint16_t*>(xb);
#pragma unroll
        for (int pp = 0; pp < 4; ++pp)
#pragma unroll
          for (int u = 0; u < 4; ++u)
            X[(t / 8 + 32 * pp) * kXS16 + 4 * (t % 8) + u] =
                ((st.okx >> (4 * pp + u)) & 1u) ? in_bf16(st.xr[4 * pp + u]) : uint16_t(0);
      }
      uint16_t* Mh = reinterpret_cast<uint16_t*>(mb);
      uint16_t* Mm = Mh + 64 * kXS16;
      uint16_t* Ml = Mm + 64 * kXS16;
      if constexpr (IT == 3 && kVec) {
        const uint32_t mk = st.okm ? 0xffffffffu : 0u;
        const int o = (t / 4) * kXS16 + 8 * (t % 4);
        uint4* dst[3] = {reinterpret_cast<uint4*>(Mh + o), reinterpret_cast<uint4*>(Mm + o),
                         reinterpret_cast<uint4*>(Ml + o)};
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          uint4 v;
          v.x = st.mq[j].x & mk;
          v.y = st.mq[j].y & mk;
          v.z = st.mq[j].z & mk;
          v.w = st.mq[j].w & mk;
          *dst[j] = v;
        }
        return;
      }
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int e = t + 256 * v;
        const bool ok = (st.okm >> v) & 1u;
        Mh[(e / 32) * kXS16 + e % 32] = ok ? st.mhr[v] : uint16_t(0);
        Mm[(e / 32) * kXS16 + e % 32] = ok ? st.mmr[v] : uint16_t(0);
        Ml[(e / 32) * kXS16 + e % 32] = ok ? st.mlr[v] : uint16_t(0);
      }
    }
  };
  // products of the chunk in buffer buf, added to the FP64 accumulators
  auto compute = [&](int buf) {
    const unsigned char* xb = lds + buf * kXBytes;
    const unsigned char* mb = lds + 2 * kXBytes + buf * kMBytes;
    if constexpr (IT == 0) {
      const float* X = reinterpret_cast<const float*>(xb);
      const float* M = reinterpret_cast<const float*>(mb);
      // operands of eight steps read before their products, so one LDS
      // round trip serves sixteen MFMAs
#pragma unroll
      for (int k0 = 0; k0 < kMC / 2; k0 += 8) {
        float av[8], bv[8][2];
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
          av[kk] = X[(32 * w + l32) * kXS32 + 2 * (k0 + kk) + h];
#pragma unroll
          for (int tt = 0; tt < 2; ++tt)
            bv[kk][tt] = M[(2 * (k0 + kk) + h) * 64 + 32 * tt + l32];
        }
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
#pragma unroll
          for (int tt = 0; tt < 2; ++tt)
            acc[tt] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[kk], bv[kk][tt],
                                                            acc[tt], 0, 0, 0);
      }
    } else if constexpr (IT == 3) {
      const float* X = reinterpret_cast<const float*>(xb);
      const __bf16* Mh = reinterpret_cast<const __bf16*>(mb);
      const __bf16* Mm = Mh + 64 * kXS16;
      const __bf16* Ml = Mm + 64 * kXS16;
#pragma unroll
      for (int kk = 0; kk < kMC / 16; ++kk) {
        const float* xp = &X[(32 * w + l32) * kXS36 + 16 * kk + 8 * h];
        const float4 q0 = *reinterpret_cast<const float4*>(xp);
        const float4 q1 = *reinterpret_cast<const float4*>(xp + 4);
        const float xv[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
        bf16x8 a1, a2, a3;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const __bf16 p1 = static_cast<__bf16>(xv[j]);
          const float r1 = xv[j] - static_cast<float>(p1);  // exact
          const __bf16 p2 = static_cast<__bf16>(r1);
          const float r2 = r1 - static_cast<float>(p2);     // exact
          a1[j] = p1;
          a2[j] = p2;
          a3[j] = static_cast<__bf16>(r2);
        }
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
          const int col = 32 * tt + l32;
          const bf16x8 bh = *reinterpret_cast<const bf16x8*>(
              &Mh[col * kXS16 + 16 * kk + 8 * h]);
          const bf16x8 bm = *reinterpret_cast<const bf16x8*>(
              &Mm[col * kXS16 + 16 * kk + 8 * h]);
          const bf16x8 bl = *reinterpret_cast<const bf16x8*>(
              &Ml[col * kXS16 + 16 * kk + 8 * h]);
          // i + j = 4, then 3, then 2
          acc[tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a3, bh, acc[tt], 0, 0, 0);
          acc[tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2, bm, acc[tt], 0, 0, 0);
          acc[tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, bl, acc[tt], 0, 0, 0);
          acc[tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2, bh, acc[tt], 0, 0, 0);
          acc[tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, bm, acc[tt], 0, 0, 0);
          acc[tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, bh, acc[tt], 0, 0, 0);
        }
      }
    } else {
      const __bf16* X = reinterpret_cast<const __bf16*>(xb);
      const __bf16* Mh = reinterpret_cast<const __bf16*>(mb);
      const __bf16* Mm = Mh + 64 * kXS16;
      const __bf16* Ml = Mm + 64 * kXS16;
#pragma unroll
      for (int kk = 0; kk < kMC / 16; ++kk) {
        const bf16x8 av = *reinterpret_cast<const bf16x8*>(
            &X[(32 * w + l32) * kXS16 + 16 * kk + 8 * h]);
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
          const int col = 32 * tt + l32;
          const bf16x8 bh = *reinterpret_cast<const bf16x8*>(
              &Mh[col * kXS16 + 16 * kk + 8 * h]);
          const bf16x8 bm = *reinterpret_cast<const bf16x8*>(
              &Mm[col * kXS16 + 16 * kk + 8 * h]);
          const bf16x8 bl = *reinterpret_cast<const bf16x8*>(
              &Ml[col * kXS16 + 16 * kk + 8 * h]);
          // smallest part first
          acc[tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bl, acc[tt], 0, 0, 0);
          acc[tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bm, acc[tt], 0, 0, 0);
          acc[tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bh, acc[tt], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        a64[tt][e] += static_cast<double>(acc[tt][e]);
        acc[tt][e] = 0.0f;
      }
  };

  // Chunk ch is read from buffer ch % 2 after the barrier that follows its
  // store; the store of chunk ch + 1 goes to the other buffer, whose last
  // reader (chunk ch - 1) finished before that same barrier, so one barrier
  // per chunk suffices. kVec: two register stages, and chunk ch + 2 is
  // loaded into the stage chunk ch has left (already in LDS) before chunk ch
  // multiplies, so two chunks of X are in flight while one multiplies; the
  // other forms load chunk ch + 1 there (one stage, fewer registers).
  SStage st[kVec ? 2 : 1];
  load_chunk(0, st[0]);
  store_chunk(0, st[0]);
  if (kVec && nch > 1) load_chunk(1, st[kVec ? 1 : 0]);
  __syncthreads();
  auto step = [&](int ch, auto stage) {
    constexpr int S = decltype(stage)::value;
    constexpr int kIn = kVec ? S : 0, kNext = kVec ? 1 - S : 0;
    if (kVec) {
      if (ch + 2 < nch) load_chunk(ch + 2, st[kIn]);
    } else {
      if (ch + 1 < nch) load_chunk(ch + 1, st[0]);
    }
    compute(ch & 1);
    if (ch + 1 < nch) {
      store_chunk((ch + 1) & 1, st[kNext]);
      __syncthreads();
    }
  };
  for (int ch = 0; ch < nch; ch += 2) {
    step(ch, std::integral_constant<int, 0>{});
    if (ch + 1 < nch) step(ch + 1, std::integral_constant<int, 1>{});
  }
  // l_i = sum_c y_ic^2: square and add the two tiles, then 32 lanes
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    double sq = a64[0][e] * a64[0][e] + a64[1][e] * a64[1][e];
    sq = sum32(sq);
    const int64_t row = row0 + 32 * w + (e % 4) + 8 * (e / 4) + 4 * h;
    if (l32 == 0 && row < n) out[row] = static_cast<float>(sq);
  }
}

__device__ __forceinline__ double bf16_bits_to_double(uint16_t b) {
  return static_cast<double>(__uint_as_float(static_cast<uint32_t>(b) << 16));
}

// Mh, Mm, Ml (64 x ldm bf16, column c of M stored contiguously): the BF16
// rounding of M, of the remainder, and of the remainder after that
__global__ void split_m_kernel(const double* __restrict__ m64, int64_t d,
                               int64_t k, int64_t ldm, uint16_t* __restrict__ mh,
                               uint16_t* __restrict__ mm,
                               uint16_t* __restrict__ ml) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= 64 * d) return;
  const int64_t c = e / d, j = e % d;
  double v = c < k ? m64[j * k + c] : 0.0;
  const uint16_t hb = f32_to_bf16_bits(static_cast<float>(v));
  v -= bf16_bits_to_double(hb);
  const uint16_t mb = f32_to_bf16_bits(static_cast<float>(v));
  v -= bf16_bits_to_double(mb);
  mh[c * ldm + j] = hb;
  mm[c * ldm + j] = mb;
  ml[c * ldm + j] = f32_to_bf16_bits(static_cast<float>(v));
}

}  // namespace

size_t scores_partial_bytes(int64_t n, int64_t d, int64_t k, int format,
                            int dtype) {
  if (format == 0 && dtype != 0 && k <= 64) {
    // the three BF16 parts of M (reduced-precision input, and FP32 input in
    // the split form)
    return static_cast<size_t>(3 * 64 * d) * sizeof(uint16_t);
  }
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
  if (score_q_ok(x, dtype, format, d, ld, k) &&
      reinterpret_cast<uintptr_t>(partial) % 16 == 0) {
    launch_score_q(x, dtype, n, d, ld, m64, k, partial, scores, s);
    return;
  }
  if (dtype != 0 && k <= 64) {
    const unsigned g = static_cast<unsigned>((n + kMR - 1) / kMR);
    if (dtype == 1) {
      // the split form: 4-float X loads and 8-element loads of M's parts
      // (the parts hold 64 columns, zero past k, so any k <= 64)
      const bool vec = ld % 4 == 0 && d % 8 == 0 &&
                       reinterpret_cast<uintptr_t>(x) % 16 == 0 &&
                       reinterpret_cast<uintptr_t>(partial) % 16 == 0;
      if (vec) {
        uint16_t* mh = reinterpret_cast<uint16_t*>(partial);
        uint16_t* mm = mh + 64 * d;
        uint16_t* ml = mm + 64 * d;
        split_m_kernel<<<static_cast<unsigned>((64 * d + 255) / 256), 256, 0, s>>>(
            m64, d, k, d, mh, mm, ml);
        prof_begin(kKScore, s);
        score_mfma_kernel<3, true><<<g, 256, 0, s>>>(
            static_cast<const float*>(x), n, d, ld, nullptr, k, mh, mm, ml, d,
            scores);
        prof_end(kKScore, s);
        return;
      }
      prof_begin(kKScore, s);
      score_mfma_kernel<0><<<g, 256, 0, s>>>(static_cast<const float*>(x), n, d,
                                             ld, m32, k, nullptr, nullptr,
                                             nullptr, 0, scores);
      prof_end(kKScore, s);
    } else {
      uint16_t* mh = reinterpret_cast<uint16_t*>(partial);
      uint16_t* mm = mh + 64 * d;
      uint16_t* ml = mm + 64 * d;
      split_m_kernel<<<static_cast<unsigned>((64 * d + 255) / 256), 256, 0, s>>>(
          m64, d, k, d, mh, mm, ml);
      prof_begin(kKScore, s);
      if (dtype == 2)
        score_mfma_kernel<1><<<g, 256, 0, s>>>(static_cast<const uint16_t*>(x), n,
                                               d, ld, nullptr, k, mh, mm, ml, d,
                                               scores);
      else
        score_mfma_kernel<2><<<g, 256, 0, s>>>(static_cast<const uint8_t*>(x), n,
                                               d, ld, nullptr, k, mh, mm, ml, d,
                                               scores);
      prof_end(kKScore, s);
    }
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
