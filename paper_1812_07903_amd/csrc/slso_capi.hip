// C ABI of the slso library: argument validation, the context's device
// workspace, and the order of stages of the sketched leverage path
// (Algorithms 2 and 3 in QR form with the second projection Pi_2, and the
// "dec" ordering of Sec. 5.2).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <optional>
#include <string>
#include <vector>

#include "internal.h"
#include "slso.h"

struct slso_ctx {
  // the arguments of a no-sync slso_leverage call awaiting
  // slso_leverage_finish
  struct Pending {
    bool valid = false;   // the arguments of the last no-sync call
    bool active = false;  // its work may still be in flight
    slso_matrix X{};
    uint64_t seed = 0;
    int64_t r = 0, k = 0;
    slso_options o{};
    float* scores = nullptr;
    hipStream_t s = nullptr;
    size_t ds_off = 0;
  } pend;
  int device = 0;
  void* scratch = nullptr;  // this device's address of the scoring scratch
  void* ws = nullptr;       // device workspace
  size_t ws_bytes = 0;
  bool ws_fixed = false;    // allocated once by slso_create, never grown
  hipEvent_t ws_done = nullptr;  // recorded after the last work using ws
  hipEvent_t side_done = nullptr;  // joins the side stream into a call's stream
  slso::QrStreams qs;            // QR look-ahead stream and events
  void* host_buf = nullptr; // pinned host staging for small read-backs
  std::string err;
};


// ---- launch profiler -------------------------------------------------------
namespace slso {
namespace {
struct ProfEntry {
  int kid;
  hipEvent_t a, b;
};
struct Profiler {
  bool on = false;
  int only = -1;  // record only this kernel id (-1: all)
  std::mutex mu;
  std::vector<hipEvent_t> pool;
  std::vector<ProfEntry> pending;
  double ms[kKCount] = {};
  int64_t count[kKCount] = {};
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
Profiler& prof() {
  static Profiler p;
  return p;
}
// the launch being timed by this host thread (threads may share a process)
thread_local int open_kid = -1;
thread_local hipEvent_t open_ev = nullptr;
}  // namespace

void prof_begin(int kid, hipStream_t s) {
  Profiler& p = prof();
  if (!p.on || (p.only >= 0 && p.only != kid)) return;
  std::lock_guard<std::mutex> g(p.mu);
  hipEvent_t e = p.get();
  if (!e) return;
  if (hipEventRecord(e, s) != hipSuccess) {
    p.pool.push_back(e);
    return;
  }
  open_kid = kid;
  open_ev = e;
}

void prof_end(int kid, hipStream_t s) {
  Profiler& p = prof();
  if (!p.on) return;
  std::lock_guard<std::mutex> g(p.mu);
  if (open_kid != kid || !open_ev) return;
  hipEvent_t e = p.get();
  if (!e) return;
  if (hipEventRecord(e, s) != hipSuccess) {
    p.pool.push_back(e);
    return;
  }
  p.pending.push_back({kid, open_ev, e});
  open_kid = -1;
  open_ev = nullptr;
}
int ctx_reserve_workspace(slso_ctx* c, size_t bytes);
int ctx_release_workspace(slso_ctx* c) {
  if (!c) return SLSO_EINVAL;
  if (!c->ws) return SLSO_OK;
  if (hipSetDevice(c->device) != hipSuccess ||
      hipEventSynchronize(c->ws_done) != hipSuccess ||
      hipFree(c->ws) != hipSuccess)
    return SLSO_EDEVICE;
  c->ws = nullptr;
  c->ws_bytes = 0;
  return SLSO_OK;
}
}  // namespace slso

// ---- the scratch of the allocation-free scoring call ------------------------
// One array per device, alive until the process ends, shared by every
// slso_scores_noalloc call on that device. Host code never uses the array's
// name as an address: slso_create looks up this device's address once
// (hipGetSymbolAddress, with the device current) and every launch takes that
// pointer.
constexpr size_t kNoAllocScratchBytes = SLSO_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

using namespace slso;

constexpr size_t kAlign = 256;

struct Arena {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    T* p = reinterpret_cast<T*>(base + off);
    off += count * sizeof(T);
    return p;
  }
};

// Bytes an arena layout needs: replay the same sequence of take() calls.
struct Sizer {
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    off += count * sizeof(T);
    return nullptr;
  }
};

int set_err(slso_ctx* c, int st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

#define SLSO_HIP(ctx, call)                                                  \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess)                                                    \
      return set_err(ctx, SLSO_EDEVICE,                                      \
                     std::string(#call) + ": " + hipGetErrorString(e_));     \
  } while (0)

// Bytes a context allocates for a workspace request (rounded to 2 MiB).
size_t ws_alloc_bytes(size_t need) {
  const size_t g = size_t{1} << 21;
  return (need + g - 1) / g * g;
}

// Orders a call's use of the context's workspace after every earlier call's,
// whatever streams the two were made on: the call's stream first waits for
// ws_done (recorded by the previous call), and when the call returns, after
// all of its work has been enqueued, whatever it left on the side stream is
// joined into its stream and ws_done is recorded there.
struct WsMark {
  slso_ctx* c;
  hipStream_t s;
  WsMark(slso_ctx* ctx, hipStream_t stream) : c(ctx), s(stream) {
    (void)hipStreamWaitEvent(s, c->ws_done, 0);
  }
  ~WsMark() {
    if (c->qs.side && hipEventRecord(c->side_done, c->qs.side) == hipSuccess)
      (void)hipStreamWaitEvent(s, c->side_done, 0);
    (void)hipEventRecord(c->ws_done, s);
  }
  WsMark(const WsMark&) = delete;
  WsMark& operator=(const WsMark&) = delete;
};

int ensure_ws(slso_ctx* c, size_t bytes) {
  if (bytes <= c->ws_bytes) return SLSO_OK;
  if (c->ws_fixed)
    return set_err(c, SLSO_ENOMEM,
                   "the call needs " + std::to_string(bytes) +
                       " bytes of workspace; the context was created with a "
                       "fixed workspace of " +
                       std::to_string(c->ws_bytes) + " bytes");
  SLSO_HIP(c, hipSetDevice(c->device));
  if (c->ws) {
    // only this context's own earlier work can still be using the buffer
    // (a pending no-sync call recorded no event: its stream is waited for)
    SLSO_HIP(c, hipEventSynchronize(c->ws_done));
    if (c->pend.active) SLSO_HIP(c, hipStreamSynchronize(c->pend.s));
    SLSO_HIP(c, hipFree(c->ws));
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  const size_t want = ws_alloc_bytes(bytes);
  if (hipMalloc(&c->ws, want) != hipSuccess) {
    c->ws = nullptr;
    (void)hipGetLastError();
    return set_err(c, SLSO_ENOMEM,
                   "workspace allocation of " + std::to_string(want) +
                       " bytes failed");
  }
  c->ws_bytes = want;
  return SLSO_OK;
}

// this device's address of the scratch array (see its definition)
std::mutex g_scratch_mu;
void* g_scratch_addr[64] = {};

// the array's address on `device` (current); nullptr when it cannot be had
void* scratch_address(int device) {
  if (device < 0 || device >= 64) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_addr[device] = p;
  }
  return g_scratch_addr[device];
}

int check_launch(slso_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return set_err(c, SLSO_EDEVICE,
                   std::string(what) + ": " + hipGetErrorString(e));
  return SLSO_OK;
}

int bits_for(int64_t r) {
  int b = 0;
  while ((static_cast<int64_t>(1) << b) < r) ++b;
  return b;
}

int validate_matrix(slso_ctx* c, const slso_matrix* X) {
  if (!X) return set_err(c, SLSO_EINVAL, "X is NULL");
  if (X->n < 1 || X->d < 1) return set_err(c, SLSO_EINVAL, "n and d must be >= 1");
  if (X->n >= (static_cast<int64_t>(1) << 31))
    return set_err(c, SLSO_EINVAL, "n must be < 2^31");
  if (!X->values) return set_err(c, SLSO_EINVAL, "X->values is NULL");
  if (X->row_scale)
    return set_err(c, SLSO_EUNSUPPORTED, "row_scale is not provided");
  if (X->dtype == SLSO_FP8_E4M3) {
    if (!X->col_scale)
      return set_err(c, SLSO_EUNSUPPORTED, "FP8 input needs col_scale");
  } else if (X->col_scale) {
    return set_err(c, SLSO_EINVAL, "col_scale is only read for FP8 input");
  }
  if (X->format == SLSO_DENSE) {
    if (X->ld < X->d) return set_err(c, SLSO_EINVAL, "ld must be >= d");
    if (X->dtype != SLSO_F64 && X->dtype != SLSO_F32 &&
        X->dtype != SLSO_BF16 && X->dtype != SLSO_FP8_E4M3)
      return set_err(c, SLSO_EINVAL, "unknown dtype");
  } else if (X->format == SLSO_CSR) {
    if (!X->row_ptr || !X->col_idx)
      return set_err(c, SLSO_EINVAL, "CSR needs row_ptr and col_idx");
    if (X->nnz < 0) return set_err(c, SLSO_EINVAL, "nnz must be >= 0");
    if (X->dtype != SLSO_F32)
      return set_err(c, SLSO_EUNSUPPORTED, "CSR values must be F32");
  } else {
    return set_err(c, SLSO_EINVAL, "unknown format");
  }
  return SLSO_OK;
}

// The Gaussian sketch and the Gram pass of the refinement run on MFMA for
// dense F32, BF16 and FP8 input.
bool mfma_input(const slso_matrix* X) {
  return X->format == SLSO_DENSE &&
         (X->dtype == SLSO_F32 || X->dtype == SLSO_BF16 ||
          X->dtype == SLSO_FP8_E4M3);
}

struct SketchBufs {
  uint32_t *keys, *vals, *keys_s, *vals_s, *keys_t, *vals_t;
  int32_t* off;
  void* sort_ws;
};

template <typename A>
SketchBufs take_sketch_bufs(A& a, int64_t n, int64_t r) {
  SketchBufs b{};
  b.keys = a.template take<uint32_t>(n);
  b.vals = a.template take<uint32_t>(n);
  b.keys_s = a.template take<uint32_t>(n);
  b.vals_s = a.template take<uint32_t>(n);
  b.keys_t = a.template take<uint32_t>(n);
  b.vals_t = a.template take<uint32_t>(n);
  b.off = a.template take<int32_t>(r + 1);
  b.sort_ws = a.template take<char>(radix_sort_scratch_bytes(n));
  return b;
}

void size_sketch_bufs(Sizer& z, int64_t n, int64_t r) {
  for (int i = 0; i < 6; ++i) z.take<uint32_t>(n);
  z.take<int32_t>(r + 1);
  z.take<char>(radix_sort_scratch_bytes(n));
}

// Nonzeros per column of S for the hashed sketches: 1 for CountSketch, the
// option (default 2) for OSNAP, 0 for the Gaussian sketch.
int sketch_nnz(const slso_options& o) {
  if (o.sketch == SLSO_COUNTSKETCH) return 1;
  if (o.sketch == SLSO_OSNAP) return o.nnz_per_col == 0 ? 2 : o.nnz_per_col;
  return 0;
}
// 1 / sqrt(nnz), applied once to every FP64 sum of a hashed sketch
double sketch_scale(int nnz) {
  return nnz <= 1 ? 1.0 : 1.0 / std::sqrt(static_cast<double>(nnz));
}
int check_sketch_kind(slso_ctx* c, const slso_options& o, int64_t r,
                      const slso_matrix* X) {
  if (o.sketch != SLSO_COUNTSKETCH && o.sketch != SLSO_GAUSSIAN &&
      o.sketch != SLSO_OSNAP && o.sketch != SLSO_SRHT)
    return set_err(c, SLSO_EINVAL, "unknown sketch kind");
  if (o.sketch == SLSO_SRHT) {
    if (X->format != SLSO_DENSE)
      return set_err(c, SLSO_EUNSUPPORTED, "the SRHT takes dense input");
    if (r > srht_rows_padded(X->n))
      return set_err(c, SLSO_EINVAL, "SRHT needs r <= n rounded up to a power of two");
  }
  if ((o.flags & ~(SLSO_OPT_SVD_RANK | SLSO_OPT_EPS_HAT | SLSO_OPT_NO_SYNC)) != 0)
    return set_err(c, SLSO_EINVAL, "unknown option flags");
  if (o.sketch == SLSO_OSNAP) {
    const int s = sketch_nnz(o);
    if (s < 1 || s > kMaxOsnapNnz || r % s != 0)
      return set_err(c, SLSO_EINVAL,
                     "OSNAP needs 1 <= nnz_per_col <= 16 dividing r");
  }
  return SLSO_OK;
}

// Bucket partition of the rows (hash, stable sort by bucket, offsets) for
// nnz entries per row (entry j n + i: hash j of row i): it reads no input
// values. Entries of one bucket come from one hash, in ascending row order.
void enqueue_partition(int64_t n, int nnz, uint64_t seed, int64_t r,
                       const SketchBufs& b, hipStream_t s) {
  if (nnz == 1) {
    const HashCoeffs hb = make_hash_coeffs(seed, kStreamBucket);
    const HashCoeffs hs = make_hash_coeffs(seed, kStreamSign);
    launch_hash_pack(hb, hs, r, 0, n, b.keys, b.vals, s);
  } else {
    OsnapCoeffs h{};
    for (int j = 0; j < nnz; ++j) {
      h.hb[j] = make_hash_coeffs(seed, osnap_bucket_stream(j));
      h.hs[j] = make_hash_coeffs(seed, osnap_sign_stream(j));
    }
    launch_hash_pack_osnap(h, nnz, r, n, b.keys, b.vals, s);
  }
  const int64_t ne = n * nnz;
  radix_sort_pairs(b.keys, b.vals, b.keys_s, b.vals_s, b.keys_t, b.vals_t, ne,
                   bits_for(r), b.sort_ws, s);
  launch_bucket_offsets(b.keys_s, ne, r, b.off, s);
}
void enqueue_gather(const slso_matrix* X, int nnz, int64_t r,
                    const SketchBufs& b, const double* dscale, double* sx,
                    hipStream_t s) {
  launch_countsketch(X->values, X->dtype, X->format, X->n, X->d, X->ld,
                     X->row_ptr, X->col_idx, X->col_scale, X->row_scale,
                     b.vals_s, b.off, r, dscale, sx, s, sketch_scale(nnz));
}
// Bucket partition + hashed sketch into sx (r x d), optionally column-scaled.
void enqueue_countsketch(const slso_matrix* X, int nnz, uint64_t seed,
                         int64_t r, const SketchBufs& b, const double* dscale,
                         double* sx, hipStream_t s) {
  enqueue_partition(X->n, nnz, seed, r, b, s);
  enqueue_gather(X, nnz, r, b, dscale, sx, s);
}

size_t gemm_partial_bytes(const slso_matrix* X, int64_t r, bool gauss,
                          bool refine) {
  const int64_t n = X->n, d = X->d;
  const size_t g = gauss ? gauss_partial_bytes(n, r, d, X->dtype) : size_t{0};
  const size_t m = refine ? gram_partial_bytes(n, d, X->dtype) : size_t{0};
  return std::max(g, m);
}

// Workspace of slso_leverage; the arena in slso_leverage takes the same
// buffers in the same order.
size_t leverage_ws_bytes(const slso_matrix* X, int64_t r, int64_t k,
                         const slso_options& o) {
  const int64_t n = X->n, d = X->d;
  const int64_t kk = k == 0 ? d : k;
  const int nnz = sketch_nnz(o);
  const bool gauss = o.sketch == SLSO_GAUSSIAN;
  const bool refine = o.refine == 1;
  // the refinement's Gram and Cholesky also run for the distortion report
  const bool gram = refine || (o.flags & SLSO_OPT_EPS_HAT) != 0;
  Sizer z;
  if (nnz > 0) {
    size_sketch_bufs(z, n * nnz, r);
    z.take<float>(countsketch_colmax_groups(r) * d);  // column maxima parts
  }
  if (o.sketch == SLSO_SRHT) z.take<char>(srht_scratch_bytes(n, d));
  z.take<uint64_t>(d);             // colmax bits
  z.take<double>(d);               // dscale D
  z.take<double>(d);               // D * col_scale (FP8)
  z.take<int>(64);                 // flags
  z.take<double>(8);               // diag stats
  z.take<double>(r * d);           // sketch
  z.take<char>(gemm_partial_bytes(X, r, gauss, gram));
  z.take<char>(qr_scratch_bytes(r, d));
  z.take<double>(d * d);           // R_D of the sketch
  if (gram) {
    for (int i = 0; i < 3; ++i) z.take<double>(d * d);  // G, R1, refined R
    z.take<char>(chol_tiled_scratch_bytes(d));            // its Cholesky
  }
  z.take<double>(d * kk);          // Pi_2 -> M'
  z.take<double>(d * kk);          // M (FP64)
  z.take<float>(d * kk);           // M (FP32)
  z.take<char>(scores_partial_bytes(n, d, kk, X->format, X->dtype));
  z.take<char>(trsm_blocked_scratch(d, gram ? d : kk));
  if (o.flags & SLSO_OPT_EPS_HAT) {  // Jacobi SVD of R1
    z.take<char>(jacobi_svd_scratch_bytes(d));
    z.take<double>(d * d);
    z.take<double>(d);
  }
  return z.off;
}

size_t order_ws_bytes(int64_t n) {
  Sizer z;
  for (int i = 0; i < 4; ++i) z.take<uint32_t>(n);
  z.take<char>(radix_sort_scratch_bytes(n));
  return z.off;
}

int check_leverage(slso_ctx* c, const slso_matrix* X, int64_t r, int64_t k,
                   const slso_options* opt, slso_options* o) {
  int st = validate_matrix(c, X);
  if (st) return st;
  if (r < X->d || r >= (static_cast<int64_t>(1) << 31))
    return set_err(c, SLSO_EINVAL, "need d <= r < 2^31");
  if (k < 0) return set_err(c, SLSO_EINVAL, "k must be >= 0");
  *o = slso_options{};
  if (opt) *o = *opt;
  if ((st = check_sketch_kind(c, *o, r, X))) return st;
  if (o->refine != 0 && o->refine != 1)
    return set_err(c, SLSO_EINVAL, "refine must be 0 or 1");
  if ((o->flags & SLSO_OPT_NO_SYNC) != 0 &&
      (o->refine != 0 || (o->flags & (SLSO_OPT_EPS_HAT | SLSO_OPT_SVD_RANK)) != 0))
    return set_err(c, SLSO_EUNSUPPORTED,
                   "SLSO_OPT_NO_SYNC takes neither the refinement, the "
                   "distortion report nor the SVD rank mode");
  if ((o->sketch == SLSO_GAUSSIAN || o->refine == 1 ||
       (o->flags & SLSO_OPT_EPS_HAT) != 0) &&
      !mfma_input(X))
    return set_err(c, SLSO_EUNSUPPORTED,
                   "the Gaussian sketch, the refinement and the distortion "
                   "report take dense F32, BF16 or FP8 input");
  return SLSO_OK;
}

}  // namespace

extern "C" {

const char* slso_status_string(int status) {
  switch (status) {
    case SLSO_OK: return "ok";
    case SLSO_RANK_DEFICIENT: return "rank deficient (truncated)";
    case SLSO_EINVAL: return "invalid argument";
    case SLSO_ENOMEM: return "out of device memory";
    case SLSO_ENONFINITE: return "input holds Inf or NaN";
    case SLSO_EDEVICE: return "HIP runtime error";
    case SLSO_EUNSUPPORTED: return "unsupported combination";
    default: return "unknown status";
  }
}

const char* slso_last_error(const slso_ctx* ctx) {
  return ctx ? ctx->err.c_str() : "";
}

int slso_create(slso_ctx** out, int device, size_t workspace_bytes) {
  if (!out) return SLSO_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return SLSO_EINVAL;
  slso_ctx* c = new slso_ctx();
  c->device = device;
  if (hipSetDevice(device) != hipSuccess ||
      init_quantile_tables(device) != 0 ||
      hipHostMalloc(&c->host_buf, 4096, hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&c->ws_done, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->side_done, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&c->qs.side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->qs.factored, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->qs.bulk_done, hipEventDisableTiming) != hipSuccess ||
      (c->scratch = scratch_address(device)) == nullptr) {
    if (c->qs.bulk_done) (void)hipEventDestroy(c->qs.bulk_done);
    if (c->qs.factored) (void)hipEventDestroy(c->qs.factored);
    if (c->qs.side) (void)hipStreamDestroy(c->qs.side);
    if (c->side_done) (void)hipEventDestroy(c->side_done);
    if (c->ws_done) (void)hipEventDestroy(c->ws_done);
    if (c->host_buf) (void)hipHostFree(c->host_buf);
    delete c;
    return SLSO_EDEVICE;
  }
  if (workspace_bytes > 0) {
    if (ensure_ws(c, workspace_bytes) != SLSO_OK) {
      (void)slso_destroy(c);
      return SLSO_ENOMEM;
    }
    c->ws_fixed = true;
  }
  *out = c;
  return SLSO_OK;
}

int slso_destroy(slso_ctx* c) {
  if (!c) return SLSO_EINVAL;
  (void)hipSetDevice(c->device);
  (void)hipEventSynchronize(c->ws_done);
  if (c->pend.active) (void)hipStreamSynchronize(c->pend.s);
  if (c->ws) (void)hipFree(c->ws);
  (void)hipEventDestroy(c->ws_done);
  (void)hipEventDestroy(c->side_done);
  (void)hipStreamSynchronize(c->qs.side);
  (void)hipEventDestroy(c->qs.factored);
  (void)hipEventDestroy(c->qs.bulk_done);
  (void)hipStreamDestroy(c->qs.side);
  if (c->host_buf) (void)hipHostFree(c->host_buf);
  delete c;
  return SLSO_OK;
}

int slso_hash(uint64_t seed, int64_t r, int64_t row0, int64_t n,
              int32_t* bucket, int8_t* sign, void* stream) {
  if (r < 1 || r >= (static_cast<int64_t>(1) << 31) || n < 0 || row0 < 0 ||
      (n > 0 && (!bucket || !sign)))
    return SLSO_EINVAL;
  launch_hash_out(make_hash_coeffs(seed, kStreamBucket),
                  make_hash_coeffs(seed, kStreamSign), r, row0, n, bucket, sign,
                  static_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? SLSO_OK : SLSO_EDEVICE;
}

int slso_gaussian(uint64_t seed, int32_t stream_id, int64_t rows, int64_t cols,
                  double* out, void* stream) {
  if (rows < 0 || cols < 0 || (rows * cols > 0 && !out)) return SLSO_EINVAL;
  launch_gaussian(seed, static_cast<uint32_t>(stream_id), rows, cols, 1.0, out,
                  static_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? SLSO_OK : SLSO_EDEVICE;
}

int slso_gaussian_sketch_entries(uint64_t seed, int64_t r, int64_t row0,
                                 int64_t n, float* out, void* stream) {
  if (r < 0 || n < 0 || row0 < 0 || (r * n > 0 && !out)) return SLSO_EINVAL;
  launch_gauss_entries(seed, r, n, row0, out, static_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? SLSO_OK : SLSO_EDEVICE;
}

int slso_gaussian_sketch_entries_q(uint64_t seed, int32_t dtype, int64_t r,
                                   int64_t row0, int64_t n, float* out,
                                   void* stream) {
  if (r < 0 || n < 0 || row0 < 0 || (r * n > 0 && !out)) return SLSO_EINVAL;
  if (dtype != SLSO_BF16 && dtype != SLSO_FP8_E4M3) return SLSO_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || init_quantile_tables(dev) != 0)
    return SLSO_EDEVICE;
  launch_gauss_q_entries(seed, r, n, row0, dtype == SLSO_BF16 ? 0 : 1, out,
                         static_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? SLSO_OK : SLSO_EDEVICE;
}

int slso_sketch(slso_ctx* c, const slso_matrix* X, uint64_t seed, int64_t r,
                const slso_options* opt, double* sx, void* stream) {
  if (!c) return SLSO_EINVAL;
  int st = validate_matrix(c, X);
  if (st) return st;
  if (r < X->d || r >= (static_cast<int64_t>(1) << 31))
    return set_err(c, SLSO_EINVAL, "need d <= r < 2^31");
  if (!sx) return set_err(c, SLSO_EINVAL, "sx is NULL");
  slso_options o{};
  if (opt) o = *opt;
  if ((st = check_sketch_kind(c, o, r, X))) return st;
  const int kind = o.sketch;
  const int nnz = sketch_nnz(o);
  if (kind == SLSO_GAUSSIAN && !mfma_input(X))
    return set_err(c, SLSO_EUNSUPPORTED,
                   "the Gaussian sketch takes dense F32, BF16 or FP8 input");
  SLSO_HIP(c, hipSetDevice(c->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Sizer z;
  if (kind == SLSO_SRHT) {
    z.take<char>(srht_scratch_bytes(X->n, X->d));
    z.take<double>(X->d);
  } else if (nnz > 0) {
    size_sketch_bufs(z, X->n * nnz, r);
    z.take<double>(X->d);
  } else {
    z.take<char>(gauss_partial_bytes(X->n, r, X->d, X->dtype));
  }
  if ((st = ensure_ws(c, z.off))) return st;
  WsMark mark_{c, s};
  Arena a{static_cast<char*>(c->ws)};
  if (kind == SLSO_SRHT) {
    void* ws = a.take<char>(srht_scratch_bytes(X->n, X->d));
    double* cs = a.take<double>(X->d);
    if (X->dtype == SLSO_FP8_E4M3)
      launch_mul_scale(nullptr, X->col_scale, X->d, cs, s);
    if (launch_srht(X->values, X->dtype, X->n, X->d, X->ld, seed, r,
                    X->dtype == SLSO_FP8_E4M3 ? cs : nullptr, ws, sx, s) != 0)
      return set_err(c, SLSO_EINVAL, "SRHT needs r <= n'");
  } else if (nnz > 0) {
    SketchBufs b = take_sketch_bufs(a, X->n * nnz, r);
    double* cs = a.take<double>(X->d);
    if (X->dtype == SLSO_FP8_E4M3)
      launch_mul_scale(nullptr, X->col_scale, X->d, cs, s);
    enqueue_countsketch(X, nnz, seed, r, b,
                        X->dtype == SLSO_FP8_E4M3 ? cs : nullptr, sx, s);
  } else {
    float* part = a.take<float>(gauss_partial_bytes(X->n, r, X->d, X->dtype) / 4);
    launch_gauss_sketch(X->values, X->dtype, X->n, X->d, X->ld, X->col_scale,
                        seed, r, nullptr, part, sx, s);
  }
  return check_launch(c, "slso_sketch");
}

int slso_sketch_svd(slso_ctx* c, const slso_matrix* X, uint64_t seed,
                    int64_t r, const slso_options* opt, double* sx,
                    double* sigma, double* v, void* stream) {
  if (!c) return SLSO_EINVAL;
  if (!sx || !sigma || !v) return set_err(c, SLSO_EINVAL, "sx, sigma or v is NULL");
  int st = slso_sketch(c, X, seed, r, opt, sx, stream);
  if (st) return st;
  const int64_t d = X->d;
  // R of S X into v, then its SVD (A and V of the sweeps in the workspace)
  if ((st = slso_qr_r(c, sx, r, d, v, stream))) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = ensure_ws(c, jacobi_svd_scratch_bytes(d)))) return st;
  WsMark mark_{c, s};
  if (jacobi_svd(v, d, sigma, v, c->ws, s) != 0)
    return set_err(c, SLSO_EDEVICE, "Jacobi SVD failed");
  return check_launch(c, "slso_sketch_svd");
}

int slso_qr_r_path(slso_ctx* c, double* a, int64_t m, int64_t d,
                   double* r_out, int path, int32_t* path_used, void* stream) {
  if (!c) return SLSO_EINVAL;
  if (!a || !r_out || d < 1 || m < d)
    return set_err(c, SLSO_EINVAL, "need a, r_out and m >= d >= 1");
  if (path < SLSO_QR_AUTO || path > SLSO_QR_TREE)
    return set_err(c, SLSO_EINVAL, "unknown QR path");
  SLSO_HIP(c, hipSetDevice(c->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Sizer z;
  z.take<char>(qr_scratch_bytes(m, d));
  z.take<double>(m * d);  // copy of a for the fallbacks
  z.take<int>(64);
  int st = ensure_ws(c, z.off);
  if (st) return st;
  WsMark mark_{c, s};
  Arena ar{static_cast<char*>(c->ws)};
  void* qws = ar.take<char>(qr_scratch_bytes(m, d));
  double* copy = ar.take<double>(m * d);
  int* status = ar.take<int>(64);
  const size_t bytes = static_cast<size_t>(m * d) * sizeof(double);
  int* hf = static_cast<int*>(c->host_buf);
  auto read_status = [&]() -> int {
    SLSO_HIP(c, hipMemcpyAsync(hf, status, sizeof(int), hipMemcpyDeviceToHost, s));
    SLSO_HIP(c, hipStreamSynchronize(s));
    return SLSO_OK;
  };
  if (path != SLSO_QR_TREE)
    SLSO_HIP(c, hipMemcpyAsync(copy, a, bytes, hipMemcpyDeviceToDevice, s));
  int used = path;
  bool done = false;
  if (path == SLSO_QR_AUTO) {
    qr_factor(a, m, d, r_out, qws, status, c->qs, s);
    if ((st = check_launch(c, "slso_qr_r"))) return st;
    if ((st = read_status())) return st;
    if (*hf == 2) {
      qr_factor_finish(m, d, r_out, qws, status, s);
      if ((st = check_launch(c, "slso_qr_r"))) return st;
      if ((st = read_status())) return st;
      used = SLSO_QR_CHOLQR2_FULL;
    } else {
      used = SLSO_QR_CHOLQR2;
    }
    done = *hf == 0;
  }
  if (!done && path != SLSO_QR_TREE) {
    if (path == SLSO_QR_AUTO)
      SLSO_HIP(c, hipMemcpyAsync(a, copy, bytes, hipMemcpyDeviceToDevice, s));
    qr_factor_panel(a, m, d, r_out, qws, status, c->qs, s);
    if ((st = check_launch(c, "slso_qr_r"))) return st;
    if ((st = read_status())) return st;
    used = SLSO_QR_PANEL;
    done = *hf == 0;
    if (!done) SLSO_HIP(c, hipMemcpyAsync(a, copy, bytes, hipMemcpyDeviceToDevice, s));
  }
  if (!done) {
    qr_factor_robust(a, m, d, r_out, qws, s);
    used = SLSO_QR_TREE;
  }
  if (path_used) *path_used = used;
  return check_launch(c, "slso_qr_r");
}

int slso_qr_r(slso_ctx* c, double* a, int64_t m, int64_t d, double* r_out,
              void* stream) {
  return slso_qr_r_path(c, a, m, d, r_out, SLSO_QR_AUTO, nullptr, stream);
}

int slso_solve_upper(slso_ctx* c, const double* r, int64_t d, double* b,
                     int64_t k, void* stream) {
  if (!c) return SLSO_EINVAL;
  if (!r || !b || d < 1 || k < 1)
    return set_err(c, SLSO_EINVAL, "need r, b, d >= 1, k >= 1");
  SLSO_HIP(c, hipSetDevice(c->device));
  int st = ensure_ws(c, trsm_blocked_scratch(d, k));
  if (st) return st;
  WsMark mark_{c, static_cast<hipStream_t>(stream)};
  solve_upper(r, d, b, k, static_cast<hipStream_t>(stream),
              static_cast<double*>(c->ws));
  return check_launch(c, "slso_solve_upper");
}

}  // extern "C"

namespace {
// Layout of the scoring call's buffers, from `base` (workspace or scratch)
template <typename A>
void score_layout(A& a, const slso_matrix* X, int64_t k, double** cs,
                  double** m64, float** m32, double** part) {
  *cs = a.template take<double>(X->d);
  *m64 = a.template take<double>(X->d * k);
  *m32 = a.template take<float>(X->d * k);
  *part = a.template take<double>(
      scores_partial_bytes(X->n, X->d, k, X->format, X->dtype) / 8);
}

size_t score_bytes(const slso_matrix* X, int64_t k) {
  Sizer z;
  double *cs, *m64, *part;
  float* m32;
  score_layout(z, X, k, &cs, &m64, &m32, &part);
  return z.off;
}

void score_enqueue(const slso_matrix* X, const double* m, int64_t k,
                   float* scores, char* base, hipStream_t s) {
  Arena a{base};
  double *cs, *m64, *part;
  float* m32;
  score_layout(a, X, k, &cs, &m64, &m32, &part);
  // FP8 codes: the column scales are folded into the rows of M
  const bool fp8 = X->dtype == SLSO_FP8_E4M3;
  if (fp8) launch_mul_scale(nullptr, X->col_scale, X->d, cs, s);
  launch_scale_rows(m, fp8 ? cs : nullptr, X->d, k, m64, m32, s);
  launch_scores(X->values, X->dtype, X->format, X->n, X->d, X->ld, X->row_ptr,
                X->col_idx, X->col_scale, X->row_scale, m64, m32, k, scores, s,
                part);
}
}  // namespace

extern "C" {

int slso_scores(slso_ctx* c, const slso_matrix* X, const double* m, int64_t k,
                float* scores, void* stream) {
  if (!c) return SLSO_EINVAL;
  int st = validate_matrix(c, X);
  if (st) return st;
  if (!m || !scores || k < 1)
    return set_err(c, SLSO_EINVAL, "need m, scores and k >= 1");
  SLSO_HIP(c, hipSetDevice(c->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = ensure_ws(c, score_bytes(X, k)))) return st;
  WsMark mark_{c, s};
  score_enqueue(X, m, k, scores, static_cast<char*>(c->ws), s);
  return check_launch(c, "slso_scores");
}

int slso_scores_noalloc(slso_ctx* c, const slso_matrix* X, const double* m,
                        int64_t k, float* scores, void* stream) {
  if (!c) return SLSO_EINVAL;
  int st = validate_matrix(c, X);
  if (st) return st;
  if (!m || !scores || k < 1)
    return set_err(c, SLSO_EINVAL, "need m, scores and k >= 1");
  const size_t need = score_bytes(X, k);
  if (need > kNoAllocScratchBytes)
    return set_err(c, SLSO_EINVAL,
                   "slso_scores_noalloc needs " + std::to_string(need) +
                       " bytes of scratch; the limit is " +
                       std::to_string(kNoAllocScratchBytes));
  if (!c->scratch)
    return set_err(c, SLSO_EDEVICE, "no scratch address on this device");
  SLSO_HIP(c, hipSetDevice(c->device));
  score_enqueue(X, m, k, scores, static_cast<char*>(c->scratch),
                static_cast<hipStream_t>(stream));
  return check_launch(c, "slso_scores_noalloc");
}

int slso_leverage(slso_ctx* c, const slso_matrix* X, uint64_t seed, int64_t r,
                  int64_t k, const slso_options* opt, float* scores,
                  slso_info* info, void* stream) {
  if (!c) return SLSO_EINVAL;
  if (!scores) return set_err(c, SLSO_EINVAL, "scores is NULL");
  slso_options o{};
  int st = check_leverage(c, X, r, k, opt, &o);
  if (st) return st;
  const bool gauss = o.sketch == SLSO_GAUSSIAN;
  const int nnz = sketch_nnz(o);
  const bool refine = o.refine == 1;
  const bool want_eps = (o.flags & SLSO_OPT_EPS_HAT) != 0;
  // the refinement's Gram and Cholesky run for the refinement and for the
  // distortion report
  const bool gram = refine || want_eps;
  const bool fp8 = X->dtype == SLSO_FP8_E4M3;
  const double tol = o.rank_tol == 0.0 ? 1e-10 : o.rank_tol;
  const int64_t n = X->n, d = X->d;
  const int64_t kk = k == 0 ? d : k;
  SLSO_HIP(c, hipSetDevice(c->device));
  hipStream_t s = static_cast<hipStream_t>(stream);

  // no-sync: every decision on the device, nothing waited for on the host
  // and no other stream involved (the call can be captured in a graph); the
  // caller orders calls that share the context and calls
  // slso_leverage_finish
  const bool nosync = (o.flags & SLSO_OPT_NO_SYNC) != 0;
  const size_t gemm_part = gemm_partial_bytes(X, r, gauss, gram);
  Sizer z;
  z.off = leverage_ws_bytes(X, r, k, o);
  if ((st = ensure_ws(c, z.off))) return st;
  std::optional<WsMark> mark_;
  if (!nosync) mark_.emplace(c, s);
  Arena a{static_cast<char*>(c->ws)};
  SketchBufs sb{};
  float* cparts = nullptr;
  if (nnz > 0) {
    sb = take_sketch_bufs(a, n * nnz, r);
    cparts = a.take<float>(countsketch_colmax_groups(r) * d);
  }
  const bool srht = o.sketch == SLSO_SRHT;
  void* srht_ws = srht ? a.take<char>(srht_scratch_bytes(n, d)) : nullptr;
  uint64_t* colmax = a.take<uint64_t>(d);
  double* dscale = a.take<double>(d);
  double* eff = a.take<double>(d);
  int* flags = a.take<int>(64);
  double* dstat = a.take<double>(8);
  double* sx = a.take<double>(r * d);
  void* gpart = a.take<char>(gemm_part);
  void* qws = a.take<char>(qr_scratch_bytes(r, d));
  double* RS = a.take<double>(d * d);
  double *G = nullptr, *R1 = nullptr, *RR = nullptr;
  void* ctws = nullptr;
  if (gram) {
    G = a.take<double>(d * d);
    R1 = a.take<double>(d * d);
    RR = a.take<double>(d * d);
    ctws = a.take<char>(chol_tiled_scratch_bytes(d));
  }
  double* pi = a.take<double>(d * kk);
  double* m64 = a.take<double>(d * kk);
  float* m32 = a.take<float>(d * kk);
  double* part = a.take<double>(scores_partial_bytes(n, d, kk, X->format, X->dtype) / 8);
  double* tws = a.take<double>(trsm_blocked_scratch(d, gram ? d : kk) / 8);
  void* jws = nullptr;
  double *jv = nullptr, *jsig = nullptr;
  if (want_eps) {
    jws = a.take<char>(jacobi_svd_scratch_bytes(d));
    jv = a.take<double>(d * d);
    jsig = a.take<double>(d);
  }

  // Dense F32 / BF16 / FP8 input: the column maxima are taken in the
  // CountSketch's own pass over X, and D is applied by the QR as it reads the
  // sketch (exact: powers of two). Otherwise a pass of its own comes first.
  const bool fuse = nnz > 0 && countsketch_colmax_ok(X->values, X->dtype,
                                                     X->format, X->ld);
  // BF16 / FP8 input to the Gaussian sketch: the column maxima are taken in
  // the sketch's own pass, and D is applied when its slices are summed
  const bool gauss_eq = gauss && gauss_q_dtype(X->dtype);
  // 0. the bucket partition needs no input values: without the fused pass it
  // runs on the context's second stream while the column maxima are taken
  const bool side_partition = nnz > 0 && !fuse && c->qs.side && !nosync;
  if (side_partition) {
    SLSO_HIP(c, hipEventRecord(c->qs.factored, s));
    SLSO_HIP(c, hipStreamWaitEvent(c->qs.side, c->qs.factored, 0));
    enqueue_partition(n, nnz, seed, r, sb, c->qs.side);
    SLSO_HIP(c, hipEventRecord(c->qs.bulk_done, c->qs.side));
  }
  // 1. column equilibration D (power of two) from column max-abs of X
  launch_fill_i32(flags, 64, 0, s);
  // Pi_2 depends only on the seed, d and k: it is formed here, ahead of the
  // sketch, rather than after the rank-screen read-back, where the GPU would
  // wait for its launch
  if (k == 0)
    launch_eye(pi, d, s);
  else
    launch_gaussian(seed, kStreamPi2, d, k, std::sqrt(static_cast<double>(k)),
                    pi, s);
  if (!fuse && !gauss_eq) {
    launch_fill_u64(colmax, d, 0, s);
    launch_colmax(X->values, X->dtype, X->format, n, d, X->ld, X->row_ptr,
                  X->col_idx, X->nnz, X->col_scale, X->row_scale, colmax, flags,
                  s);
    launch_colscale(colmax, d, dscale, s);
    if (fp8) launch_mul_scale(dscale, X->col_scale, d, eff, s);
  }
  // per-column factor applied to stored values: D, times the FP8 scales
  const double* rowfac = fp8 ? eff : dscale;
  // 2. sketch of X D (Algorithm 2 step 1), 3. Householder QR of the sketch
  // (Algorithm 2 step 2, QR form), 3b. refinement: G = (X D)^T (X D);
  // G' = R_S^-T G R_S^-1 = R1^T R1; R = R1 R_S is the R factor of X D.
  // The QR's 64-column panels use Cholesky-QR2; when one is too ill-
  // conditioned for it (flags[2]), the sketch is formed again and factored
  // column by column. unscaled: sx holds S X without D (the fused pass).
  bool partitioned = false, fused_done = false, unscaled = false;
  auto sketch = [&]() {
    unscaled = false;
    if (gauss_eq) {
      launch_gauss_sketch_eq(X->values, X->dtype, n, d, X->ld, X->col_scale,
                             seed, r, colmax, flags, dscale,
                             static_cast<float*>(gpart), sx, s);
      if (fp8) launch_mul_scale(dscale, X->col_scale, d, eff, s);
      return;
    }
    if (gauss) {
      launch_gauss_sketch(X->values, X->dtype, n, d, X->ld, X->col_scale, seed,
                          r, dscale, static_cast<float*>(gpart), sx, s);
      return;
    }
    if (srht) {
      (void)launch_srht(X->values, X->dtype, n, d, X->ld, seed, r, rowfac,
                        srht_ws, sx, s);
      return;
    }
    if (!partitioned) {
      if (side_partition)
        (void)hipStreamWaitEvent(s, c->qs.bulk_done, 0);
      else
        enqueue_partition(n, nnz, seed, r, sb, s);
      partitioned = true;
    }
    if (fuse && !fused_done) {
      (void)launch_countsketch_colmax(X->values, X->dtype, d, X->ld,
                                      X->col_scale, sb.vals_s, sb.off, r,
                                      cparts, flags, dscale, sx, s,
                                      sketch_scale(nnz));
      if (fp8) launch_mul_scale(dscale, X->col_scale, d, eff, s);
      fused_done = true;
      unscaled = true;
    } else {
      enqueue_gather(X, nnz, r, sb, rowfac, sx, s);
    }
  };
  // post(r_formed): rank-screen statistics of the R just formed (when
  // Cholesky-QR2 ran without forming R it wrote them itself), then the
  // refinement, which needs R_S
  auto post = [&](bool r_formed) {
    if (r_formed) launch_diag_stats(RS, d, dstat, s);
    if (gram) {
      launch_fill_i32(flags + 1, 1, 0, s);
      launch_gram(X->values, X->dtype, n, d, X->ld, X->col_scale, dscale, gpart,
                  G, s);
      solve_upper_trans(RS, d, G, d, s, tws);     // W = R_S^-T G
      launch_transpose(G, d, R1, s);         // W^T
      solve_upper_trans(RS, d, R1, d, s, tws);    // R_S^-T W^T = G'
      chol_tiled(R1, d, G, ctws, flags + 1, s);  // G (reused) = R1
      launch_trmm_upper(G, RS, d, RR, s);    // R = R1 R_S
      launch_diag_stats(RR, d, dstat + 2, s);
    }
  };
  // 4. rank screen read-back
  char* hb = static_cast<char*>(c->host_buf);
  double ds[4];
  int fl[3];
  // flags and dstat are consecutive arena blocks: one copy brings both (the
  // GPU idles while it runs, so a second copy would add its whole latency)
  const size_t ds_off = static_cast<size_t>(reinterpret_cast<char*>(dstat) -
                                            reinterpret_cast<char*>(flags));
  auto readback = [&]() -> int {
    SLSO_HIP(c, hipMemcpyAsync(hb, flags, ds_off + 4 * sizeof(double),
                               hipMemcpyDeviceToHost, s));
    SLSO_HIP(c, hipStreamSynchronize(s));
    std::memcpy(fl, hb, sizeof(fl));
    std::memcpy(ds, hb + ds_off, sizeof(ds));
    return check_launch(c, "slso_leverage: sketch/QR");
  };
  // The sketch's R by Cholesky-QR2 (which overwrites the sketch); when that
  // does not apply (flags[2] = 1: the sketch is too ill-conditioned), the
  // sketch is formed again and factored by the Householder panel path, and
  // should that fail too, column by column.
  // Without the refinement R itself is only needed if the rank screen trips:
  // Cholesky-QR2 then keeps R^{-1} in factored form and applies it to Pi_2.
  // One pass of Cholesky-QR is taken (flags[2] = 3) when R1's condition
  // estimate bounds the scores' error far below the gate, or, with the
  // refinement (R only preconditions it), R^T R close enough to X's Gram.
  const bool want_r = gram;
  bool cholqr2 = true, second = false, one = false, r_formed = want_r;
  int32_t info_flags = 0;
  if (nosync) {
    // the common path with its branches taken on the device: the second
    // pass runs only after status 2, the factored R^{-1} applies the form
    // the passes left; a Householder fallback, a failed second pass, a
    // truncation or non-finite input leave flags[15] set, and
    // slso_leverage_finish then reruns the job on the synchronous path
    sketch();
    qr_factor(sx, r, d, RS, qws, flags + 2, c->qs, s, false, dstat,
              unscaled ? dscale : nullptr, 2);
    qr_finish_dev(r, d, qws, flags + 2, flags + 8, dstat, s);
    cholqr2_decide_dev(flags + 2, flags + 8, dstat, tol, flags, flags + 12, s);
    qr_apply_rinv_dev(r, d, qws, flags + 12, pi, kk, s);
    launch_scale_rows(pi, rowfac, d, kk, m64, m32, s);
    launch_scores(X->values, X->dtype, X->format, n, d, X->ld, X->row_ptr,
                  X->col_idx, X->col_scale, X->row_scale, m64, m32, kk, scores,
                  s, part);
    SLSO_HIP(c, hipMemcpyAsync(c->host_buf, flags, ds_off + 4 * sizeof(double),
                               hipMemcpyDeviceToHost, s));
    if ((st = check_launch(c, "slso_leverage (no-sync)"))) return st;
    c->pend.valid = true;
    c->pend.active = true;
    c->pend.X = *X;
    c->pend.seed = seed;
    c->pend.r = r;
    c->pend.k = k;
    c->pend.o = o;
    c->pend.scores = scores;
    c->pend.s = s;
    c->pend.ds_off = ds_off;
    if (info) *info = slso_info{};
    return SLSO_OK;
  }
  sketch();
  qr_factor(sx, r, d, RS, qws, flags + 2, c->qs, s, want_r, dstat,
            unscaled ? dscale : nullptr, refine ? 1 : (want_r ? 0 : 2));
  post(want_r);
  if ((st = readback())) return st;
  if (fl[0]) return set_err(c, SLSO_ENONFINITE, "X holds Inf or NaN");
  if (fl[2] == 3) {
    info_flags |= SLSO_INFO_QR_ONE_PASS;
    one = true;
    fl[2] = 0;
  }
  if (fl[2] == 2) {
    info_flags |= SLSO_INFO_QR_SECOND_CHOLESKY;
    second = true;
    qr_factor_finish(r, d, RS, qws, flags + 2, s, want_r, dstat);
    post(want_r);
    if ((st = readback())) return st;
  }
  if (fl[2] != 0) {
    info_flags |= SLSO_INFO_QR_HOUSEHOLDER;
    cholqr2 = false;
    r_formed = true;
    sketch();
    qr_factor_panel(sx, r, d, RS, qws, flags + 2, c->qs, s);
    post(true);
    if ((st = readback())) return st;
    if (fl[2] != 0) {
      info_flags |= SLSO_INFO_QR_TREE;
      sketch();
      qr_factor_robust(sx, r, d, RS, qws, s);
      post(true);
      if ((st = readback())) return st;
    }
  }
  const double* R = RS;
  double dmin = ds[0], dmax = ds[1];
  if (refine) {
    const bool ok = fl[1] == 0 && std::isfinite(ds[2]) && std::isfinite(ds[3]);
    if (ok) {
      R = RR;
      dmin = ds[2];
      dmax = ds[3];
      info_flags |= SLSO_INFO_REFINED;
    } else {
      info_flags |= SLSO_INFO_REFINE_FAILED;
    }
  }
  bool full = true;
  if (tol >= 0.0)
    full = (o.flags & SLSO_OPT_SVD_RANK) == 0 && dmax > 0.0 &&
           dmin > std::sqrt(tol) * dmax;
  // 5. M = D pinv(R_D) Pi_2 (Algorithm 2 step 3 / Algorithm 3 step 4)
  int64_t rank = d;
  if (full) {
    if (cholqr2 && !want_r)
      qr_apply_rinv(r, d, qws, one ? 2 : (second ? 1 : 0), pi, kk, s);
    else
      solve_upper(R, d, pi, kk, s, tws);
    launch_scale_rows(pi, rowfac, d, kk, m64, m32, s);
  } else {
    if (!r_formed) qr_write_r(r, d, RS, qws, one ? 2 : (second ? 1 : 0), s);
    Sizer jz;
    jz.take<char>(jacobi_scratch_bytes(d, kk));
    // the Jacobi scratch reuses the sketch area, which is no longer needed
    if (static_cast<size_t>(r * d) * sizeof(double) < jz.off) {
      return set_err(c, SLSO_EUNSUPPORTED,
                     "truncation scratch exceeds the sketch area");
    }
    if (jacobi_truncated_apply(R, d, pi, kk, tol, m64, &rank, sx, s) != 0)
      return set_err(c, SLSO_EDEVICE, "Jacobi SVD failed");
    launch_scale_rows(m64, rowfac, d, kk, pi, m32, s);
    m64 = pi;
  }
  // 6. scores l_i = ||x_i M||^2 (Algorithm 2 step 4)
  launch_scores(X->values, X->dtype, X->format, n, d, X->ld, X->row_ptr,
                X->col_idx, X->col_scale, X->row_scale, m64, m32, kk, scores, s,
                part);
  if ((st = check_launch(c, "slso_leverage: scores"))) return st;
  // 7. realised distortion (Def. 1 / Thm. 1): R = R1 R_S is the R of X D, so
  // S U = Q_S R_S R^-1 = Q_S R1^-1 and sigma(S U) = 1 / sigma(R1)
  double eps_hat = std::nan("");
  if (want_eps && fl[1] == 0) {
    if (jacobi_svd(G, d, jsig, jv, jws, s) != 0)
      return set_err(c, SLSO_EDEVICE, "Jacobi SVD of R1 failed");
    double* hs = reinterpret_cast<double*>(hb + 2048);
    SLSO_HIP(c, hipMemcpyAsync(hs, jsig, sizeof(double), hipMemcpyDeviceToHost, s));
    SLSO_HIP(c, hipMemcpyAsync(hs + 1, jsig + d - 1, sizeof(double),
                               hipMemcpyDeviceToHost, s));
    SLSO_HIP(c, hipStreamSynchronize(s));
    if (hs[1] > 0.0) {
      const double su_max = 1.0 / hs[1], su_min = 1.0 / hs[0];
      eps_hat = std::max(su_max * su_max - 1.0, 1.0 - su_min * su_min);
    }
  }
  if (info) {
    info->rank = rank;
    info->screen_full = full ? 1 : 0;
    info->flags = info_flags;
    info->diag_min = dmin;
    info->diag_max = dmax;
    info->eps_hat = eps_hat;
  }
  return rank < d ? SLSO_RANK_DEFICIENT : SLSO_OK;
}

int slso_leverage_finish(slso_ctx* c, slso_info* info) {
  if (!c) return SLSO_EINVAL;
  if (!c->pend.valid)
    return set_err(c, SLSO_EINVAL, "no no-sync slso_leverage call was made");
  const slso_ctx::Pending p = c->pend;
  SLSO_HIP(c, hipSetDevice(c->device));
  SLSO_HIP(c, hipStreamSynchronize(p.s));
  c->pend.active = false;
  int fl[16];
  double ds[4];
  const char* hb = static_cast<const char*>(c->host_buf);
  std::memcpy(fl, hb, sizeof(fl));
  std::memcpy(ds, hb + p.ds_off, sizeof(ds));
  if (fl[0]) return set_err(c, SLSO_ENONFINITE, "X holds Inf or NaN");
  if (fl[15]) {
    slso_options o = p.o;
    o.flags &= ~SLSO_OPT_NO_SYNC;
    const int st = slso_leverage(c, &p.X, p.seed, p.r, p.k, &o, p.scores, info,
                                 p.s);
    if (st >= 0 && info) info->flags |= SLSO_INFO_RERUN;
    return st;
  }
  if (info) {
    info->rank = p.X.d;
    info->screen_full = 1;
    info->flags = (fl[2] == 3 ? SLSO_INFO_QR_ONE_PASS : 0) |
                  (fl[2] == 2 ? SLSO_INFO_QR_SECOND_CHOLESKY : 0);
    info->diag_min = ds[0];
    info->diag_max = ds[1];
    info->eps_hat = std::nan("");
  }
  return SLSO_OK;
}

}  // extern "C"

// ---- tuned launch shapes ---------------------------------------------------
namespace {
std::mutex g_tune_mu;
std::unordered_map<uint64_t, int> g_tune;  // (pass, dtype, d) -> choice

uint64_t tune_key(int pass, int64_t d, int dtype) {
  return (static_cast<uint64_t>(pass) << 56) |
         (static_cast<uint64_t>(dtype & 0xff) << 48) |
         (static_cast<uint64_t>(d) & ((uint64_t{1} << 48) - 1));
}
int tune_choices(int pass) {
  return pass == kTuneScore ? kScoreRingChoices
                            : (pass == kTuneCountSketch ? kCsChoices : 0);
}

// the tuner's buffers (also sized by a Sizer)
struct TuneBufs {
  double* m64 = nullptr;
  void* sq = nullptr;
  float* out = nullptr;
  SketchBufs sb{};
  float* parts = nullptr;
  int* flags = nullptr;
  double* dscale = nullptr;
  double* sx = nullptr;
};
template <typename A>
TuneBufs tune_layout(A& a, const slso_matrix* X, int64_t r, bool score,
                     int nnz) {
  TuneBufs b;
  if (score) {
    b.m64 = a.template take<double>(X->d * 64);
    b.sq = a.template take<char>(score_q_scratch_bytes(X->d));
    b.out = a.template take<float>(X->n);
  }
  if (nnz > 0) {
    b.sb = take_sketch_bufs(a, X->n * nnz, r);
    b.parts = a.template take<float>(countsketch_colmax_groups(r) * X->d);
    b.flags = a.template take<int>(64);
    b.dscale = a.template take<double>(X->d);
    b.sx = a.template take<double>(r * X->d);
  }
  return b;
}
}  // namespace

namespace slso {
int tune_choice(int pass, int64_t d, int dtype) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  const auto it = g_tune.find(tune_key(pass, d, dtype));
  return it == g_tune.end() ? -1 : it->second;
}
}  // namespace slso

extern "C" {

int slso_tune_get(int pass, int64_t d, int dtype, int* choice) {
  if (!choice || tune_choices(pass) == 0 || d < 1) return SLSO_EINVAL;
  *choice = tune_choice(pass, d, dtype);
  return SLSO_OK;
}

int slso_tune_set(int pass, int64_t d, int dtype, int choice) {
  const int nc = tune_choices(pass);
  if (nc == 0 || d < 1 || choice < -1 || choice >= nc) return SLSO_EINVAL;
  std::lock_guard<std::mutex> g(g_tune_mu);
  if (choice < 0)
    g_tune.erase(tune_key(pass, d, dtype));
  else
    g_tune[tune_key(pass, d, dtype)] = choice;
  return SLSO_OK;
}

int slso_tune(slso_ctx* c, const slso_matrix* X, int64_t r, int64_t k,
              const slso_options* opt, void* stream) {
  if (!c) return SLSO_EINVAL;
  slso_options o{};
  int st = check_leverage(c, X, r, k, opt, &o);
  if (st) return st;
  const int nnz = sketch_nnz(o);
  const int64_t kk = k == 0 ? X->d : k;
  const bool score =
      score_q_ok(X->values, X->dtype, X->format, X->d, X->ld, kk);
  const bool cs = nnz > 0 && countsketch_colmax_ok(X->values, X->dtype,
                                                   X->format, X->ld);
  if (!score && !cs) return SLSO_OK;
  Sizer z;
  tune_layout(z, X, r, score, cs ? nnz : 0);
  SLSO_HIP(c, hipSetDevice(c->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = ensure_ws(c, z.off))) return st;
  WsMark mark_{c, s};
  Arena a{static_cast<char*>(c->ws)};
  const TuneBufs b = tune_layout(a, X, r, score, cs ? nnz : 0);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  SLSO_HIP(c, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return set_err(c, SLSO_EDEVICE, "hipEventCreate failed");
  }
  // mean of three runs after one untimed run
  auto timed = [&](const auto& launch) -> float {
    launch();
    float ms = 1e30f;
    if (hipEventRecord(e0, s) != hipSuccess) return ms;
    for (int i = 0; i < 3; ++i) launch();
    if (hipEventRecord(e1, s) != hipSuccess ||
        hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      return 1e30f;
    return ms / 3.0f;
  };
  if (score) {
    // M's values do not change the time: zeros
    launch_fill_u64(reinterpret_cast<uint64_t*>(b.m64), X->d * 64, 0, s);
    int best = -1;
    float bt = 1e30f;
    for (int ch = 0; ch < kScoreRingChoices; ++ch) {
      const float t = timed([&]() {
        launch_score_q(X->values, X->dtype, X->n, X->d, X->ld, b.m64, kk, b.sq,
                       b.out, s, ch);
      });
      if (t < bt) {
        bt = t;
        best = ch;
      }
    }
    if (best >= 0) (void)slso_tune_set(kTuneScore, X->d, X->dtype, best);
  }
  if (cs) {
    enqueue_partition(X->n, nnz, 1, r, b.sb, s);
    launch_fill_i32(b.flags, 64, 0, s);
    int best = -1;
    float bt = 1e30f;
    for (int ch = 0; ch < kCsChoices; ++ch) {
      const float t = timed([&]() {
        (void)launch_countsketch_colmax(X->values, X->dtype, X->d, X->ld,
                                        X->col_scale, b.sb.vals_s, b.sb.off, r,
                                        b.parts, b.flags, b.dscale, b.sx, s,
                                        sketch_scale(nnz), ch);
      });
      if (t < bt) {
        bt = t;
        best = ch;
      }
    }
    if (best >= 0) (void)slso_tune_set(kTuneCountSketch, X->d, X->dtype, best);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return check_launch(c, "slso_tune");
}

int slso_workspace_size(const slso_matrix* X, int64_t r, int64_t k,
                        const slso_options* opt, size_t* bytes) {
  if (!bytes) return SLSO_EINVAL;
  slso_options o{};
  const int st = check_leverage(nullptr, X, r, k, opt, &o);
  if (st) return st;
  *bytes = ws_alloc_bytes(std::max(
      leverage_ws_bytes(X, r, k, o),
      order_ws_bytes(X->n)));
  return SLSO_OK;
}

int slso_order(slso_ctx* c, const float* scores, int64_t n, int32_t* perm,
               void* stream) {
  if (!c) return SLSO_EINVAL;
  if (!scores || !perm || n < 1 || n >= (static_cast<int64_t>(1) << 31))
    return set_err(c, SLSO_EINVAL, "need scores, perm and 1 <= n < 2^31");
  SLSO_HIP(c, hipSetDevice(c->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  int st = ensure_ws(c, order_ws_bytes(n));
  if (st) return st;
  WsMark mark_{c, s};
  Arena a{static_cast<char*>(c->ws)};
  uint32_t* keys = a.take<uint32_t>(n);
  uint32_t* keys_o = a.take<uint32_t>(n);
  uint32_t* keys_t = a.take<uint32_t>(n);
  uint32_t* vals_t = a.take<uint32_t>(n);
  void* sws = a.take<char>(radix_sort_scratch_bytes(n));
  launch_score_keys(scores, n, keys, s);
  radix_sort_pairs(keys, nullptr, keys_o, reinterpret_cast<uint32_t*>(perm),
                   keys_t, vals_t, n, 32, sws, s);
  return check_launch(c, "slso_order");
}

int slso_order_sample(slso_ctx* c, const float* scores, int64_t n,
                      int32_t policy, uint64_t seed, uint32_t epoch,
                      int32_t* out, void* stream) {
  if (!c) return SLSO_EINVAL;
  if (policy == SLSO_ORDER_DEC) return slso_order(c, scores, n, out, stream);
  if (!scores || !out || n < 1 || n >= (static_cast<int64_t>(1) << 31))
    return set_err(c, SLSO_EINVAL, "need scores, out and 1 <= n < 2^31");
  if (policy != SLSO_ORDER_SWR && policy != SLSO_ORDER_SWOR)
    return set_err(c, SLSO_EINVAL, "unknown ordering policy");
  SLSO_HIP(c, hipSetDevice(c->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t need = policy == SLSO_ORDER_SWR ? swr_scratch_bytes(n)
                                               : order_ws_bytes(n);
  int st = ensure_ws(c, need);
  if (st) return st;
  WsMark mark_{c, s};
  Arena a{static_cast<char*>(c->ws)};
  if (policy == SLSO_ORDER_SWOR) {
    uint32_t* keys = a.take<uint32_t>(n);
    uint32_t* keys_o = a.take<uint32_t>(n);
    uint32_t* keys_t = a.take<uint32_t>(n);
    uint32_t* vals_t = a.take<uint32_t>(n);
    void* sws = a.take<char>(radix_sort_scratch_bytes(n));
    launch_swor_keys(scores, n, seed, epoch, keys, s);
    radix_sort_pairs(keys, nullptr, keys_o, reinterpret_cast<uint32_t*>(out),
                     keys_t, vals_t, n, 32, sws, s);
    return check_launch(c, "slso_order_sample");
  }
  void* scratch = a.take<char>(swr_scratch_bytes(n));
  launch_swr_prefix(scores, n, scratch, s);
  // W = 0 (no positive score) has no distribution to draw from
  int64_t w = 0;
  SLSO_HIP(c, hipMemcpyAsync(c->host_buf, static_cast<int64_t*>(scratch) + (n - 1),
                             sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SLSO_HIP(c, hipStreamSynchronize(s));
  std::memcpy(&w, c->host_buf, sizeof(w));
  if (w <= 0) return set_err(c, SLSO_EINVAL, "dec-swr needs a positive score");
  launch_swr_draws(scratch, n, seed, epoch, out, s);
  return check_launch(c, "slso_order_sample");
}

int slso_profile_enable(int on) {
  slso::Profiler& p = slso::prof();
  std::lock_guard<std::mutex> g(p.mu);
  p.on = on != 0;
  return SLSO_OK;
}

int slso_profile_only(int id) {
  if (id < -1 || id >= slso::kKCount) return SLSO_EINVAL;
  slso::Profiler& p = slso::prof();
  std::lock_guard<std::mutex> g(p.mu);
  p.only = id;
  return SLSO_OK;
}

int slso_profile_read(double* ms, int64_t* launches, int n) {
  slso::Profiler& p = slso::prof();
  if (hipDeviceSynchronize() != hipSuccess) return SLSO_EDEVICE;
  std::lock_guard<std::mutex> g(p.mu);
  for (const auto& e : p.pending) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, e.a, e.b) == hipSuccess) {
      p.ms[e.kid] += t;
      p.count[e.kid] += 1;
    }
    p.pool.push_back(e.a);
    p.pool.push_back(e.b);
  }
  p.pending.clear();
  for (int i = 0; i < n && i < slso::kKCount; ++i) {
    if (ms) ms[i] = p.ms[i];
    if (launches) launches[i] = p.count[i];
    p.ms[i] = 0.0;
    p.count[i] = 0;
  }
  return slso::kKCount;
}

const char* slso_profile_name(int id) {
  static const char* names[] = {
      "hash_pack", "sort_hist", "sort_scan", "sort_scatter", "bucket_offsets",
      "colmax", "countsketch", "qr_node", "qr_update", "qr_extract", "trsm",
      "score", "gaussian", "gauss_sketch", "gram", "cholesky", "cq_gram",
      "cq_sum", "cq_chol", "cq_q1", "cq_z", "cq_recon", "cq_w", "cq_update", "cq2_gram",
      "cq2_gram_edge", "cq2_gram_sum", "cq2_chol", "cq2_solve", "cq2_r"};
  if (id < 0 || id >= slso::kKCount) return "";
  return names[id];
}

}  // extern "C"

namespace slso {
// grow the context's workspace to at least `bytes` now (the serving loop's
// headroom); nothing happens when it is that large already
int ctx_reserve_workspace(slso_ctx* c, size_t bytes) {
  if (!c) return SLSO_EINVAL;
  if (hipSetDevice(c->device) != hipSuccess) return SLSO_EDEVICE;
  return ensure_ws(c, bytes);
}
}  // namespace slso
