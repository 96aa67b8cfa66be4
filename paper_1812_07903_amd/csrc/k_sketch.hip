// CountSketch S*X (Algorithm 2 step 1; Sec. 2.1) and the power-of-two column
// equilibration applied before sketching.
//
// Design: rows are first grouped by bucket with the stable radix sort
// (k_sort.hip), so every sketch row is owned by exactly one wave, which
// streams the rows of its bucket in ascending order and accumulates the
// signed sums privately (registers for dense input, an LDS row segment for
// CSR input), then writes its sketch row once. No atomics touch S*X: the FP64
// sums are deterministic and taken in the same order as the streaming model
// of Sec. 3.1.2. Dense rows are read contiguously (64 lanes x 4 columns per
// pass); CSR rows are read as contiguous (col_idx, value) runs.
#include "internal.h"

namespace slso {
namespace {

template <typename T>
struct Elem;
template <>
struct Elem<double> {
  __device__ static double get(const double* p, int64_t i) { return p[i]; }
};
template <>
struct Elem<float> {
  __device__ static double get(const float* p, int64_t i) {
    return static_cast<double>(p[i]);
  }
};
template <>
struct Elem<uint16_t> {
  __device__ static double get(const uint16_t* p, int64_t i) {
    return static_cast<double>(bf16_to_f32(p[i]));
  }
};
template <>
struct Elem<uint8_t> {  // FP8-e4m3 code (the column scale is applied apart)
  __device__ static double get(const uint8_t* p, int64_t i) {
    return static_cast<double>(e4m3_to_f32(p[i]));
  }
};

__global__ void fill_u64_kernel(uint64_t* p, int64_t n, uint64_t v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename T>
__global__ void __launch_bounds__(256)
    colmax_dense_kernel(const T* __restrict__ x, int64_t n, int64_t d,
                        int64_t ld, int64_t rows_per_block,
                        unsigned long long* __restrict__ colmax, int* nonfinite,
                        const float* __restrict__ col_scale) {
  const int64_t col = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (col >= d) return;
  const double cs = col_scale ? fabs(static_cast<double>(col_scale[col])) : 1.0;
  const int64_t r0 = static_cast<int64_t>(blockIdx.y) * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < n ? r0 + rows_per_block : n;
  double m = 0.0;
  bool bad = false;
  for (int64_t row = r0; row < r1; ++row) {
    const double v = fabs(Elem<T>::get(x, row * ld + col)) * cs;
    bad |= !isfinite(v);
    m = fmax(m, v);
  }
  if (bad) atomicExch(nonfinite, 1);
  if (m > 0.0) atomicMax(&colmax[col], static_cast<unsigned long long>(__double_as_longlong(m)));
}

// CSR column max: LDS-privatised per workgroup when d fits (d <= 8192).
__global__ void __launch_bounds__(256)
    colmax_csr_kernel(const int32_t* __restrict__ col_idx,
                      const float* __restrict__ val, int64_t nnz, int64_t d,
                      int64_t per_block, unsigned long long* __restrict__ colmax,
                      int* nonfinite) {
  extern __shared__ unsigned long long lmax[];
  const bool priv = d <= 8192;
  if (priv)
    for (int64_t c = threadIdx.x; c < d; c += 256) lmax[c] = 0ull;
  __syncthreads();
  const int64_t p0 = static_cast<int64_t>(blockIdx.x) * per_block;
  const int64_t p1 = p0 + per_block < nnz ? p0 + per_block : nnz;
  bool bad = false;
  for (int64_t p = p0 + threadIdx.x; p < p1; p += 256) {
    const double v = fabs(static_cast<double>(val[p]));
    bad |= !isfinite(v);
    const unsigned long long b =
        static_cast<unsigned long long>(__double_as_longlong(v));
    if (priv)
      atomicMax(&lmax[col_idx[p]], b);
    else
      atomicMax(&colmax[col_idx[p]], b);
  }
  if (bad) atomicExch(nonfinite, 1);
  __syncthreads();
  if (priv)
    for (int64_t c = threadIdx.x; c < d; c += 256)
      if (lmax[c]) atomicMax(&colmax[c], lmax[c]);
}

__global__ void colscale_kernel(const unsigned long long* __restrict__ colmax,
                                int64_t d, double* __restrict__ dscale) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= d) return;
  const double m = __longlong_as_double(static_cast<long long>(colmax[j]));
  double s = 1.0;
  if (m > 0.0 && isfinite(m)) {
    int e;
    frexp(m, &e);           // m = f 2^e, f in [0.5, 1)
    s = ldexp(1.0, -(e - 1));  // m * s in [1, 2)
  }
  dscale[j] = s;
}

// One wave per bucket; 4 columns per lane per pass (256 columns).
template <typename T>
__global__ void __launch_bounds__(256)
    countsketch_dense_kernel(const T* __restrict__ x, int64_t d, int64_t ld,
                             const uint32_t* __restrict__ sorted_vals,
                             const int32_t* __restrict__ off, int64_t r,
                             const double* __restrict__ dscale,
                             double* __restrict__ sx, double sscale) {
  const int lane = threadIdx.x & 63;
  const int64_t b = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (b >= r) return;
  const int p0 = off[b], p1 = off[b + 1];
  for (int64_t c0 = 0; c0 < d; c0 += 256) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int p = p0; p < p1; ++p) {
      const uint32_t v = sorted_vals[p];
      const int64_t row = static_cast<int64_t>(v & 0x7fffffffu);
      const bool neg = (v >> 31) != 0;
      const int64_t rb = row * ld;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t c = c0 + lane + 64 * u;
        if (c < d) {
          const double xv = Elem<T>::get(x, rb + c);
          acc[u] += neg ? -xv : xv;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t c = c0 + lane + 64 * u;
      if (c < d) sx[b * d + c] = acc[u] * sscale * (dscale ? dscale[c] : 1.0);
    }
  }
}

// One wave per bucket, a workgroup of one wave with an LDS accumulator of
// kCsrChunk FP64 columns (8 KB, so up to twenty workgroups per CU); wider
// matrices take the columns in chunks, each reading the bucket's rows again
// (from L2; at d = 4096, 1024 columns measured faster than 512, 2048 or all
// 4096 at once). Lane q first reads the extent and sign of the
// bucket's row p0 + q (the rows in groups of 64), so the rows' CSR offsets
// arrive in one round trip; the first 64 entries of eight rows (one per
// lane) are loaded together, then added row by row, so every column
// receives its rows' values in bucket order (the columns of one row are
// distinct, and the wave's LDS updates take effect in program order).
constexpr int kCsrChunk = 1024;

__device__ __forceinline__ int64_t readlane_i64(int64_t v, int l) {
  const uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(v), l);
  const uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(v >> 32), l);
  return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}

__global__ void __launch_bounds__(64)
    countsketch_csr_kernel(const int64_t* __restrict__ row_ptr,
                           const int32_t* __restrict__ col_idx,
                           const float* __restrict__ val, int64_t n,
                           int64_t d, const uint32_t* __restrict__ sorted_vals,
                           const int32_t* __restrict__ off, int64_t r,
                           const double* __restrict__ dscale,
                           double* __restrict__ sx, double sscale) {
  __shared__ double acc[kCsrChunk];
  const int lane = threadIdx.x;
  const int64_t b = blockIdx.x;
  if (b >= r) return;
  const int p0 = off[b], p1 = off[b + 1];
  // with no entries at all there is no index to clamp the loads to
  const bool any = row_ptr[n] > 0;
  for (int64_t c0 = 0; c0 < d; c0 += kCsrChunk) {
    const int nc = static_cast<int>(d - c0 < kCsrChunk ? d - c0 : kCsrChunk);
    for (int c = lane; c < nc; c += 64) acc[c] = 0.0;
    for (int pg = p0; any && pg < p1; pg += 64) {
      const int np = p1 - pg < 64 ? p1 - pg : 64;
      int64_t e0 = 0, e1 = 0;
      uint32_t sg = 0;
      if (lane < np) {
        const uint32_t v = sorted_vals[pg + lane];
        const int64_t row = static_cast<int64_t>(v & 0x7fffffffu);
        sg = v >> 31;
        e0 = row_ptr[row];
        e1 = row_ptr[row + 1];
      }
      // entry e0_q + lane of row q (clamped into the row, or to entry 0 for
      // an empty row; lanes past its length add nothing); rows in batches of
      // eight, the batch's loads issued together, then its rows added in order
      constexpr int kB = 8;
      for (int qb = 0; qb < np; qb += kB) {
        int32_t cb[kB];
        float xb[kB];
        bool ib[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          const int q = qb + u < np ? qb + u : np - 1;
          const int64_t qe0 = readlane_i64(e0, q), qe1 = readlane_i64(e1, q);
          const int64_t e = qe0 + lane;
          ib[u] = qb + u < np && e < qe1;
          const int64_t ec = e < qe1 ? e : (qe1 > qe0 ? qe1 - 1 : 0);
          cb[u] = col_idx[ec];
          xb[u] = val[ec];
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          const int q = qb + u;
          if (q >= np) break;
          const bool neg = __builtin_amdgcn_readlane(sg, q) != 0u;
          if (ib[u] && cb[u] >= c0 && cb[u] < c0 + nc) {
            const double xv = static_cast<double>(xb[u]);
            acc[cb[u] - c0] += neg ? -xv : xv;
          }
          // a row longer than 64 entries: the rest in order
          const int64_t qe0 = readlane_i64(e0, q), qe1 = readlane_i64(e1, q);
          for (int64_t e = qe0 + 64 + lane; e < qe1; e += 64) {
            const int64_t c = col_idx[e];
            if (c >= c0 && c < c0 + nc) {
              const double xv = static_cast<double>(val[e]);
              acc[c - c0] += neg ? -xv : xv;
            }
          }
        }
      }
    }
    for (int c = lane; c < nc; c += 64)
      sx[b * d + c0 + c] = acc[c] * sscale * (dscale ? dscale[c0 + c] : 1.0);
  }
}

__global__ void mul_scale_kernel(const double* __restrict__ a,
                                 const float* __restrict__ b, int64_t d,
                                 double* __restrict__ out) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j < d) out[j] = (a ? a[j] : 1.0) * static_cast<double>(b[j]);
}

// ---- CountSketch with the column maxima in the same pass ----------------------
// Dense F32 / BF16 / FP8 input whose rows start on 4-element boundaries. One
// wave per bucket (waves stride over the buckets); lane l owns columns
// 4 (l + 64 u) .. + 3, u < U, of each 256 U-column chunk (U = 1, 2 or 4, the
// fewest that cover d up to 1024) and reads them as one 4-element vector per
// row, so a row is one pass of coalesced loads. NR rows of the bucket are
// loaded at a time (16, 8 or 4: narrower rows leave registers for more
// loads in flight), and the next NR row-list entries are read while they
// are summed. The signed FP64 sums are those of countsketch_dense_kernel,
// in the same order, times the FP8 column scale; the power-of-two
// equilibration D is left to the consumer (scaling by a power of two is
// exact, so the consumer sees the same numbers); OSNAP sums are multiplied
// once by 1/sqrt(nnz). Every row is read (nnz times for OSNAP), so the
// column max-abs values come from the same loads: per workgroup into
// parts[blockIdx][col], reduced by colmax_parts_kernel.
constexpr int kSkMaxGroups = 1024;

__device__ __forceinline__ void load4(const float* p, float (&v)[4]) {
  const float4 q = *reinterpret_cast<const float4*>(p);
  v[0] = q.x;
  v[1] = q.y;
  v[2] = q.z;
  v[3] = q.w;
}
__device__ __forceinline__ void load4(const uint16_t* p, float (&v)[4]) {
  const uint2 q = *reinterpret_cast<const uint2*>(p);
  v[0] = bf16_to_f32(static_cast<uint16_t>(q.x & 0xffffu));
  v[1] = bf16_to_f32(static_cast<uint16_t>(q.x >> 16));
  v[2] = bf16_to_f32(static_cast<uint16_t>(q.y & 0xffffu));
  v[3] = bf16_to_f32(static_cast<uint16_t>(q.y >> 16));
}
// four e4m3fn codes by gfx950's packed FP8 -> FP32 conversion (exact for
// every code, as e4m3_to_f32)
__device__ __forceinline__ void load4(const uint8_t* p, float (&v)[4]) {
  const int q = *reinterpret_cast<const int*>(p);
  const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8(q, false);
  const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8(q, true);
  v[0] = lo[0];
  v[1] = lo[1];
  v[2] = hi[0];
  v[3] = hi[1];
}
__device__ __forceinline__ float elem_f(const float* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float elem_f(const uint16_t* p, int64_t i) {
  return bf16_to_f32(p[i]);
}
__device__ __forceinline__ float elem_f(const uint8_t* p, int64_t i) {
  return e4m3_to_f32(p[i]);
}

// kTail: d % 4 != 0 (rows end in a partial vector)
template <typename T, bool kTail, int U, int NR>
__global__ void __launch_bounds__(256)
    countsketch_colmax_kernel(const T* __restrict__ x, int64_t d, int64_t ld,
                              const float* __restrict__ col_scale,
                              const uint32_t* __restrict__ sorted_vals,
                              const int32_t* __restrict__ off, int64_t r,
                              float* __restrict__ parts, int* nonfinite,
                              double* __restrict__ sx, double sscale) {
  constexpr bool kFp8 = sizeof(T) == 1;  // codes times the column scale
  constexpr int kW = 256 * U;            // columns per chunk
  constexpr int kE = 4 * U;              // columns per lane
  __shared__ float wmax[4][kW];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * 4;
  bool bad = false;
  for (int64_t c0 = 0; c0 < d; c0 += kW) {
    float cm[kE];
    double cs[kE];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t c = c0 + 4 * (lane + 64 * u) + e;
        cm[4 * u + e] = 0.0f;
        cs[4 * u + e] = (kFp8 && c < d) ? static_cast<double>(col_scale[c]) : 1.0;
      }
    for (int64_t b = static_cast<int64_t>(blockIdx.x) * 4 + wv; b < r; b += nwaves) {
      const int p0 = off[b], p1 = off[b + 1];
      double acc[kE];
#pragma unroll
      for (int e = 0; e < kE; ++e) acc[e] = 0.0;
      // the row-list entries of the first NR rows (a row past the bucket
      // repeats its last row and is masked below)
      uint32_t vn[NR];
#pragma unroll
      for (int j = 0; j < NR; ++j)
        vn[j] = p0 < p1 ? sorted_vals[p0 + j < p1 ? p0 + j : p1 - 1] : 0u;
      for (int p = p0; p < p1; p += NR) {
        bool neg[NR];
        const T* xr[NR];
#pragma unroll
        for (int j = 0; j < NR; ++j) {
          neg[j] = (vn[j] >> 31) != 0;
          xr[j] = x + static_cast<int64_t>(vn[j] & 0x7fffffffu) * ld;
        }
        // branch-free loads (a vector past the end reads the row start and
        // is masked), all in flight together, then the next entries
        float xv[NR][kE];
#pragma unroll
        for (int j = 0; j < NR; ++j)
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int64_t c = c0 + 4 * (lane + 64 * u);
            const bool full = c + 4 <= d;
            float q[4];
            load4(xr[j] + (full ? c : 0), q);
#pragma unroll
            for (int e = 0; e < 4; ++e) xv[j][4 * u + e] = full ? q[e] : 0.0f;
          }
        const int pn = p + NR;
#pragma unroll
        for (int j = 0; j < NR; ++j)
          vn[j] = sorted_vals[pn + j < p1 ? pn + j : p1 - 1];
        if (kTail) {
          // the partial last vector of each row, element by element
#pragma unroll
          for (int j = 0; j < NR; ++j)
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const int64_t c = c0 + 4 * (lane + 64 * u);
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const bool ok = c + 4 > d && c + e < d;
                const float sv = elem_f(xr[j], ok ? c + e : 0);
                xv[j][4 * u + e] = ok ? sv : xv[j][4 * u + e];
              }
            }
        }
        // sums in row order; a repeated row (past the bucket) is added with
        // weight zero and changes no maximum
#pragma unroll
        for (int j = 0; j < NR; ++j) {
          const double sg = p + j < p1 ? (neg[j] ? -1.0 : 1.0) : 0.0;
#pragma unroll
          for (int e = 0; e < kE; ++e) {
            const float a = fabsf(xv[j][e]);
            bad |= !(a <= 3.402823466e38f);
            cm[e] = fmaxf(cm[e], a);
            acc[e] = fma(sg, static_cast<double>(xv[j][e]), acc[e]);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t c = c0 + 4 * (lane + 64 * u) + e;
          if (c < d)
            sx[b * d + c] = kFp8 ? acc[4 * u + e] * sscale * cs[4 * u + e]
                                 : acc[4 * u + e] * sscale;
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) wmax[wv][4 * (lane + 64 * u) + e] = cm[4 * u + e];
    __syncthreads();
    for (int j = threadIdx.x; j < kW; j += 256) {
      const float m = fmaxf(fmaxf(wmax[0][j], wmax[1][j]), fmaxf(wmax[2][j], wmax[3][j]));
      if (c0 + j < d) parts[static_cast<int64_t>(blockIdx.x) * d + c0 + j] = m;
    }
    __syncthreads();
  }
  if (bad) atomicExch(nonfinite, 1);
}

// dscale[col] = D_col from the largest of the groups' maxima (times |cs|, the
// FP8 column scale), as colscale_kernel. Four columns per workgroup, 64
// threads per column.
__global__ void __launch_bounds__(256)
    colmax_parts_kernel(const float* __restrict__ parts, int64_t groups,
                        int64_t d, const float* __restrict__ col_scale,
                        int* nonfinite, double* __restrict__ dscale) {
  __shared__ float red[4][4];
  const int t = threadIdx.x, cl = t & 3, g = t >> 2, lane = t & 63, wv = t >> 6;
  const int64_t col = static_cast<int64_t>(blockIdx.x) * 4 + cl;
  float m = 0.0f;
  if (col < d) {
    for (int64_t j0 = 0; j0 < groups; j0 += 64 * 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t j = j0 + g + 64 * u;
        v[u] = j < groups ? parts[j * d + col] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) m = fmaxf(m, v[u]);
    }
  }
#pragma unroll
  for (int o = 4; o < 64; o <<= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if (lane < 4) red[wv][lane] = m;
  __syncthreads();
  if (t < 4) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 4 + t;
    if (c < d) {
      const float mx = fmaxf(fmaxf(red[0][t], red[1][t]), fmaxf(red[2][t], red[3][t]));
      const double mm = static_cast<double>(mx) *
                        (col_scale ? fabs(static_cast<double>(col_scale[c])) : 1.0);
      if (!isfinite(mm)) atomicExch(nonfinite, 1);
      double sc = 1.0;
      if (mm > 0.0 && isfinite(mm)) {
        int e;
        frexp(mm, &e);
        sc = ldexp(1.0, -(e - 1));
      }
      dscale[c] = sc;
    }
  }
}

inline unsigned grid1(int64_t n, int t) {
  return static_cast<unsigned>((n + t - 1) / t);
}

}  // namespace

void launch_mul_scale(const double* a, const float* b, int64_t d, double* out,
                      hipStream_t s) {
  if (d <= 0) return;
  mul_scale_kernel<<<grid1(d, 256), 256, 0, s>>>(a, b, d, out);
}

void launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s) {
  if (n <= 0) return;
  fill_u64_kernel<<<grid1(n, 256), 256, 0, s>>>(p, n, v);
}

void launch_colmax(const void* x, int dtype, int format, int64_t n, int64_t d,
                   int64_t ld, const int64_t* row_ptr, const int32_t* col_idx,
                   int64_t nnz, const float* col_scale, const float* row_scale,
                   uint64_t* colmax_bits, int* nonfinite, hipStream_t s) {
  (void)row_ptr;
  (void)row_scale;
  auto* cm = reinterpret_cast<unsigned long long*>(colmax_bits);
  if (format == 1) {  // CSR, FP32 values
    if (nnz <= 0) return;
    const int64_t per_block = 16384;
    const size_t shm = d <= 8192 ? static_cast<size_t>(d) * 8 : 0;
    prof_begin(kKColmax, s);
    colmax_csr_kernel<<<grid1(nnz, static_cast<int>(per_block)), 256, shm, s>>>(
        col_idx, static_cast<const float*>(x), nnz, d, per_block, cm, nonfinite);
    prof_end(kKColmax, s);
    return;
  }
  const int64_t cb = (d + 255) / 256;
  int64_t rpb = 64;
  while ((n + rpb - 1) / rpb * cb > 4096) rpb *= 2;
  dim3 grid(static_cast<unsigned>(cb), static_cast<unsigned>((n + rpb - 1) / rpb));
  switch (dtype) {
    case 0:
      prof_begin(kKColmax, s);
      colmax_dense_kernel<double><<<grid, 256, 0, s>>>(
          static_cast<const double*>(x), n, d, ld, rpb, cm, nonfinite, nullptr);
      prof_end(kKColmax, s);
      break;
    case 1:
      prof_begin(kKColmax, s);
      colmax_dense_kernel<float><<<grid, 256, 0, s>>>(
          static_cast<const float*>(x), n, d, ld, rpb, cm, nonfinite, nullptr);
      prof_end(kKColmax, s);
      break;
    case 3:
      prof_begin(kKColmax, s);
      colmax_dense_kernel<uint8_t><<<grid, 256, 0, s>>>(
          static_cast<const uint8_t*>(x), n, d, ld, rpb, cm, nonfinite,
          col_scale);
      prof_end(kKColmax, s);
      break;
    case 2:
      prof_begin(kKColmax, s);
      colmax_dense_kernel<uint16_t><<<grid, 256, 0, s>>>(
          static_cast<const uint16_t*>(x), n, d, ld, rpb, cm, nonfinite, nullptr);
      prof_end(kKColmax, s);
      break;
    default:
      break;
  }
}

void launch_colscale(const uint64_t* colmax_bits, int64_t d, double* dscale,
                     hipStream_t s) {
  colscale_kernel<<<grid1(d, 256), 256, 0, s>>>(
      reinterpret_cast<const unsigned long long*>(colmax_bits), d, dscale);
}

void launch_countsketch(const void* x, int dtype, int format, int64_t n,
                        int64_t d, int64_t ld, const int64_t* row_ptr,
                        const int32_t* col_idx, const float* col_scale,
                        const float* row_scale, const uint32_t* sorted_vals,
                        const int32_t* offsets, int64_t r,
                        const double* dscale, double* sx, hipStream_t s,
                        double sscale) {
  (void)col_scale;
  (void)row_scale;
  const unsigned grid = grid1(r, 4);
  if (format == 1) {
    prof_begin(kKSketch, s);
    countsketch_csr_kernel<<<static_cast<unsigned>(r), 64, 0, s>>>(
        row_ptr, col_idx, static_cast<const float*>(x), n, d, sorted_vals,
        offsets, r, dscale, sx, sscale);
    prof_end(kKSketch, s);
    return;
  }
  switch (dtype) {
    case 0:
      prof_begin(kKSketch, s);
      countsketch_dense_kernel<double><<<grid, 256, 0, s>>>(
          static_cast<const double*>(x), d, ld, sorted_vals, offsets, r, dscale,
          sx, sscale);
      prof_end(kKSketch, s);
      break;
    case 1:
      prof_begin(kKSketch, s);
      countsketch_dense_kernel<float><<<grid, 256, 0, s>>>(
          static_cast<const float*>(x), d, ld, sorted_vals, offsets, r, dscale,
          sx, sscale);
      prof_end(kKSketch, s);
      break;
    case 2:
      prof_begin(kKSketch, s);
      countsketch_dense_kernel<uint16_t><<<grid, 256, 0, s>>>(
          static_cast<const uint16_t*>(x), d, ld, sorted_vals, offsets, r,
          dscale, sx, sscale);
      prof_end(kKSketch, s);
      break;
    case 3:
      prof_begin(kKSketch, s);
      countsketch_dense_kernel<uint8_t><<<grid, 256, 0, s>>>(
          static_cast<const uint8_t*>(x), d, ld, sorted_vals, offsets, r,
          dscale, sx, sscale);
      prof_end(kKSketch, s);
      break;
    default:
      break;
  }
}

int64_t countsketch_colmax_groups(int64_t r) {
  const int64_t g = (r + 3) / 4;
  return g < 1 ? 1 : (g < kSkMaxGroups ? g : kSkMaxGroups);
}

bool countsketch_colmax_ok(const void* x, int dtype, int format, int64_t ld) {
  const int esz = dtype == 1 ? 4 : (dtype == 2 ? 2 : (dtype == 3 ? 1 : 0));
  return format == 0 && esz != 0 && ld % 4 == 0 &&
         reinterpret_cast<uintptr_t>(x) % (4 * esz) == 0;
}

bool launch_countsketch_colmax(const void* x, int dtype, int64_t d, int64_t ld,
                               const float* col_scale,
                               const uint32_t* sorted_vals,
                               const int32_t* offsets, int64_t r, float* parts,
                               int* nonfinite, double* dscale, double* sx,
                               hipStream_t s, double sscale, int choice) {
  if (!countsketch_colmax_ok(x, dtype, 0, ld) || d <= 0 || r <= 0) return false;
  const int64_t groups = countsketch_colmax_groups(r);
  const unsigned g = static_cast<unsigned>(groups);
  prof_begin(kKSketch, s);
  const bool tail = d % 4 != 0;
  // chunk width 256 U: one chunk for d up to 1024. Rows in flight per
  // bucket wave: choice 0 or 1 (default 1) = 8 or 16 (U = 1), 4 or 8
  // (U = 2), 2 or 4 (U = 4); every choice sums the same rows in the same
  // order, so the bits do not depend on it
  const int U = d <= 256 ? 1 : (d <= 512 ? 2 : 4);
  if (choice < 0 || choice >= kCsChoices) choice = tune_choice(kTuneCountSketch, d, dtype);
  if (choice < 0) choice = 1;
  const bool big = choice == 1;
#define SLSO_CS_GO(T, CS, TL, UU, NR)                                           \
  countsketch_colmax_kernel<T, TL, UU, NR><<<g, 256, 0, s>>>(                   \
      static_cast<const T*>(x), d, ld, CS, sorted_vals, offsets, r, parts,     \
      nonfinite, sx, sscale)
#define SLSO_CS_TL(T, CS, TL)                                                   \
  do {                                                                          \
    if (U == 1) {                                                               \
      if (big) SLSO_CS_GO(T, CS, TL, 1, 16); else SLSO_CS_GO(T, CS, TL, 1, 8);  \
    } else if (U == 2) {                                                        \
      if (big) SLSO_CS_GO(T, CS, TL, 2, 8); else SLSO_CS_GO(T, CS, TL, 2, 4);   \
    } else {                                                                    \
      if (big) SLSO_CS_GO(T, CS, TL, 4, 4); else SLSO_CS_GO(T, CS, TL, 4, 2);   \
    }                                                                           \
  } while (0)
#define SLSO_CS_LAUNCH(T, CS)                                                   \
  do {                                                                          \
    if (tail)                                                                   \
      SLSO_CS_TL(T, CS, true);                                                  \
    else                                                                        \
      SLSO_CS_TL(T, CS, false);                                                 \
  } while (0)
  if (dtype == 1)
    SLSO_CS_LAUNCH(float, nullptr);
  else if (dtype == 2)
    SLSO_CS_LAUNCH(uint16_t, nullptr);
  else
    SLSO_CS_LAUNCH(uint8_t, col_scale);
#undef SLSO_CS_LAUNCH
#undef SLSO_CS_TL
#undef SLSO_CS_GO
  prof_end(kKSketch, s);
  colmax_parts_kernel<<<grid1(d, 4), 256, 0, s>>>(
      parts, groups, d, dtype == 3 ? col_scale : nullptr, nonfinite, dscale);
  return true;
}

}  // namespace slso
