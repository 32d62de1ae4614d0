// C ABI of the emulation library: argument validation, workspace layout and
// dispatch to the kernels.  Nothing here allocates device memory per call or
// synchronises a stream.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "ozk.h"
#include "ozk_internal.hpp"

// Size class of a GEMM configuration: the operation, scheme and slice or
// modulus count, and ceil(log2) of M, N and K.
struct ozk_cfg_key {
  int op, scheme, p_or_s, mb, nb, kb;
  bool operator<(const ozk_cfg_key& o) const {
    return std::tie(op, scheme, p_or_s, mb, nb, kb) < std::tie(o.op, o.scheme, o.p_or_s, o.mb, o.nb, o.kb);
  }
};

struct ozk_cfg_entry {
  ozk_gemm_config cfg;
  float ms;  // tuned time of the GEMM kernel(s), 0 if set by hand
};

// The workspace of ozk_dgemm_noalloc: a fixed buffer in device memory, one
// copy per device, held by every device the library runs on until the
// process ends.  In host code `scratch` only names the symbol; its device
// address comes from hipGetSymbolAddress (scratch_of) and is the only form
// that reaches a kernel or a copy.
static __device__ __align__(256) unsigned char scratch[OZK_NOALLOC_SCRATCH_BYTES];

struct ozk_ctx {
  int device = 0;
  int last_arg = 0;
  void* scratch = nullptr;       // device address of `scratch` on this device
  uint32_t* dflags = nullptr;    // device: [0] condition flags, [1] the last value taken
  int64_t k_split_override = 0;  // > 0: shorter K runs (testing the fold path)
  float* sel_w = nullptr;        // selector parameters on the device (or null)
  float sel_thr[OZK_SELECTOR_HEADS];  // per-head decision thresholds
  int sel_margin = 0;
  std::map<ozk_cfg_key, ozk_cfg_entry> configs;  // tuned or set GEMM configurations
};

using ozk::round_up;

namespace {

ozk_status fail(ozk_ctx* c, ozk_status s, int arg) {
  if (c) c->last_arg = arg;
  return s;
}

// Device address of `scratch` on the current device `device`, looked up once
// per device (each device holds its own copy at its own address).
hipError_t scratch_of(int device, void** out) {
  static std::mutex mu;
  static std::map<int, void*> addr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(device);
  if (it == addr.end()) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return e != hipSuccess ? e : hipErrorInvalidSymbol;
    it = addr.emplace(device, p).first;
  }
  *out = it->second;
  return hipSuccess;
}

ozk_status hip_status(ozk_ctx* c, hipError_t e) {
  if (e == hipSuccess) return OZK_OK;
  if (c) c->last_arg = 0;
  return OZK_ERR_HIP;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

int64_t k_split_of(const ozk_ctx* c, int p) {
  const int64_t per_k = p == 1 ? (1 << 12) : (int64_t)(p - 1) << 14;
  int64_t k = ((int64_t)0x7fffffff / per_k) / OZK_K_CHUNK * OZK_K_CHUNK;
  if (c && c->k_split_override > 0 && c->k_split_override < k) k = c->k_split_override;
  return k;
}

struct S1Plan {
  size_t off_e, off_f, off_a, off_b, off_z, total;
  int64_t nsplit, steps_per_split, nchunk;
};

// Workspace layout of Scheme I.  `split` asks for at least that many K runs
// (a configuration's choice); INT32 exactness may need more.
S1Plan s1_plan(const ozk_ctx* c, int p, int64_t M, int64_t N, int64_t K, int split = 1) {
  S1Plan pl;
  const int64_t kp = round_up(K, OZK_K_CHUNK);
  pl.nchunk = kp / OZK_K_CHUNK;
  const int64_t ks = k_split_of(c, p);
  pl.steps_per_split = ks / OZK_K_CHUNK;
  if (split > 1 && pl.nchunk > 1) {
    const int64_t want = (pl.nchunk + split - 1) / split;
    if (want < pl.steps_per_split) pl.steps_per_split = want;
  }
  pl.nsplit = pl.nchunk <= pl.steps_per_split ? 1 : (pl.nchunk + pl.steps_per_split - 1) / pl.steps_per_split;
  if (pl.nchunk == 0) pl.nsplit = 1;
  size_t o = 0;
  pl.off_e = o; o = align256(o + 4 * (size_t)(M > 0 ? M : 1));
  pl.off_f = o; o = align256(o + 4 * (size_t)(N > 0 ? N : 1));
  pl.off_a = o; o = align256(o + ozk_s1_packed_bytes(M, K, p));
  pl.off_b = o; o = align256(o + ozk_s1_packed_bytes(N, K, p));
  pl.off_z = o;
  if (pl.nsplit > 1) o = align256(o + 16 * (size_t)pl.nsplit * M * N);
  pl.total = o;
  return pl;
}

struct S2Plan {
  size_t off_sig, off_tau, off_a, off_b, off_res, total;
};

S2Plan s2_plan(int s, bool cplx, int64_t M, int64_t N, int64_t K) {
  S2Plan pl;
  size_t o = 0;
  pl.off_sig = o; o = align256(o + 4 * (size_t)(M > 0 ? M : 1));
  pl.off_tau = o; o = align256(o + 4 * (size_t)(N > 0 ? N : 1));
  pl.off_a = o; o = align256(o + ozk_s2_packed_bytes(M, K, s, cplx));
  pl.off_b = o; o = align256(o + ozk_s2_packed_bytes(N, K, s, cplx));
  pl.off_res = o; o = align256(o + (size_t)s * (cplx ? 2 : 1) * M * N);
  pl.total = o;
  return pl;
}

// Workspace of the 4M Scheme I complex product: the Scheme I plan of the
// real embedding (M x 2K times 2K x 2N), then the M x 2N real parts of the
// product before the complex alpha/beta update (16 MN bytes).
struct S1ZPlan {
  S1Plan s1;
  ozk_gemm_config cfg;
  size_t off_h, total;
};

S1ZPlan s1z_plan(const ozk_ctx* c, int p, int64_t M, int64_t N, int64_t K);

// Median time (ms) of `reps` runs of fn on the stream, after one untimed run.
template <class F>
static hipError_t time_median(hipStream_t st, int reps, F&& fn, float* ms) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return hipErrorUnknown;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return hipErrorUnknown;
  }
  hipError_t err = fn();
  std::vector<float> t;
  for (int r = 0; r < reps && err == hipSuccess; ++r) {
    err = hipEventRecord(a, st);
    if (err == hipSuccess) err = fn();
    if (err == hipSuccess) err = hipEventRecord(b, st);
    if (err == hipSuccess) err = hipEventSynchronize(b);
    float x = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&x, a, b);
    t.push_back(x);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (err != hipSuccess) return err;
  std::sort(t.begin(), t.end());
  *ms = t[t.size() / 2];
  return hipSuccess;
}

// Workspace of the auto path: room for Scheme I at p = 8 or Scheme II at
// s = 20 (only the chosen scheme's buffers are used), then 256 bytes of
// selector counters and 256 bytes of decision (info).
struct AutoPlan {
  S1Plan s1;
  S2Plan s2;
  size_t off_cnt, off_info, total;
};

AutoPlan auto_plan(const ozk_ctx* c, int64_t M, int64_t N, int64_t K) {
  AutoPlan ap;
  ap.s1 = s1_plan(c, OZK_MAX_P, M, N, K);
  ap.s2 = s2_plan(OZK_MAX_S, false, M, N, K);
  const size_t base = std::max(ap.s1.total, ap.s2.total);
  ap.off_cnt = base;
  ap.off_info = base + 256;
  ap.total = base + 512;
  return ap;
}

bool bad_rows(int64_t r) { return r < 0 || r > OZK_MAX_ROWS; }

bool bad_dims(int64_t M, int64_t N, int64_t K) {
  return bad_rows(M) || bad_rows(N) || K < 0 || K > ((int64_t)1 << 40);
}

// Scheme II scales need K <= OZK_S2_MAX_K (exact 64-bit norm-bound sums).
bool s2_long_k(int64_t K) { return K > OZK_S2_MAX_K; }

int log2_class(int64_t x) {
  int b = 0;
  while (b < 62 && ((int64_t)1 << b) < x) ++b;
  return b;
}

ozk_cfg_key cfg_key(int op, int scheme, int p_or_s, int64_t M, int64_t N, int64_t K) {
  return ozk_cfg_key{op, scheme, p_or_s, log2_class(M), log2_class(N), log2_class(K)};
}

ozk_gemm_config default_config() { return ozk_gemm_config{0, 0, 4, 1}; }

// The configuration for this size class: the tuned or set one, else the default.
ozk_gemm_config config_for(const ozk_ctx* c, int op, int scheme, int p_or_s, int64_t M, int64_t N, int64_t K) {
  if (c) {
    auto it = c->configs.find(cfg_key(op, scheme, p_or_s, M, N, K));
    if (it != c->configs.end()) return it->second.cfg;
  }
  return default_config();
}

S1ZPlan s1z_plan(const ozk_ctx* c, int p, int64_t M, int64_t N, int64_t K) {
  S1ZPlan z;
  z.cfg = config_for(c, OZK_OP_DGEMM, OZK_SCHEME1, p, M, 2 * N, 2 * K);  // the embedded real product's class
  z.s1 = s1_plan(c, p, M, 2 * N, 2 * K, z.cfg.split);
  z.off_h = z.s1.total;
  z.total = align256(z.off_h + 16 * (size_t)(M > 0 ? M : 1) * (size_t)(N > 0 ? N : 1));
  return z;
}

bool valid_config(int scheme, const ozk_gemm_config& g) {
  const int nv = scheme == OZK_SCHEME1 ? OZK_S1_VARIANTS : OZK_S2_VARIANTS;
  return g.variant >= 0 && g.variant < nv && (g.raster == 0 || g.raster == 1) && g.group >= 1 && g.group <= 64 &&
         g.split >= 1 && g.split <= 64;
}

}  // namespace

extern "C" {

const char* ozk_version(void) { return "0.1.0"; }

const char* ozk_status_string(ozk_status s) {
  switch (s) {
    case OZK_OK: return "ok";
    case OZK_ERR_INVALID_ARG: return "invalid argument";
    case OZK_ERR_UNSUPPORTED: return "unsupported slice or modulus count";
    case OZK_ERR_WORKSPACE: return "workspace missing or too small";
    case OZK_ERR_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

ozk_status ozk_create(ozk_ctx** ctx, int device) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  *ctx = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) return OZK_ERR_HIP;
  if (device < 0 || device >= n) return OZK_ERR_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return OZK_ERR_HIP;
  ozk_ctx* c = new (std::nothrow) ozk_ctx();
  if (!c) return OZK_ERR_HIP;
  c->device = device;
  if (ozk::s2_upload_crt_tables() != hipSuccess) {  // CRT constants of every s for the auto path
    delete c;
    return OZK_ERR_HIP;
  }
  if (scratch_of(device, &c->scratch) != hipSuccess) {  // the buffer of ozk_dgemm_noalloc
    delete c;
    return OZK_ERR_HIP;
  }
  if (hipMalloc(&c->dflags, 256) != hipSuccess) {
    c->dflags = nullptr;
    delete c;
    return OZK_ERR_HIP;
  }
  if (hipMemset(c->dflags, 0, 256) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(c->dflags);
    delete c;
    return OZK_ERR_HIP;
  }
  *ctx = c;
  return OZK_OK;
}

ozk_status ozk_destroy(ozk_ctx* ctx) {
  if (ctx && ctx->sel_w) (void)hipFree(ctx->sel_w);
  if (ctx && ctx->dflags) (void)hipFree(ctx->dflags);
  delete ctx;
  return OZK_OK;
}

int ozk_last_arg(const ozk_ctx* ctx) { return ctx ? ctx->last_arg : 0; }

ozk_status ozk_get_flags(ozk_ctx* ctx, hipStream_t stream, uint32_t* flags) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (!flags) return fail(ctx, OZK_ERR_INVALID_ARG, 3);
  hipError_t err = hipSetDevice(ctx->device);
  if (err == hipSuccess) err = ozk::flag_take(ctx->dflags, ctx->dflags + 1, stream);
  if (err == hipSuccess) err = hipStreamSynchronize(stream);
  uint32_t v = 0;
  if (err == hipSuccess) err = hipMemcpy(&v, ctx->dflags + 1, sizeof(v), hipMemcpyDeviceToHost);
  if (err != hipSuccess) return hip_status(ctx, err);
  *flags = v;
  return OZK_OK;
}

ozk_status ozk_set_k_split(ozk_ctx* ctx, int64_t k) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (k < 0 || k % OZK_K_CHUNK != 0) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  ctx->k_split_override = k;
  return OZK_OK;
}

size_t ozk_s1_packed_bytes(int64_t rows, int64_t K, int p) {
  if (rows < 0 || K < 0 || p < 1) return 0;
  return (size_t)round_up(rows, OZK_ROW_ALIGN) * (size_t)round_up(K, OZK_K_CHUNK) * (size_t)p;
}

size_t ozk_s2_packed_bytes(int64_t rows, int64_t K, int s, int complex_planes) {
  if (rows < 0 || K < 0 || s < 1) return 0;
  return (size_t)round_up(rows, OZK_ROW_ALIGN) * (size_t)round_up(K, OZK_K_CHUNK) * (size_t)s *
         (complex_planes ? 3 : 1);
}

int64_t ozk_s1_k_split(int p) {
  if (p < 1 || p > OZK_MAX_P) return 0;
  return k_split_of(nullptr, p);
}

ozk_status ozk_workspace_size(ozk_ctx* ctx, ozk_op op, ozk_scheme scheme, int64_t M, int64_t N, int64_t K,
                              int p_or_s, size_t* bytes) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (!bytes) return fail(ctx, OZK_ERR_INVALID_ARG, 8);
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, 4);
  if (op == OZK_OP_DGEMM && scheme == OZK_SCHEME1) {
    if (p_or_s == 0) {  // the auto path (either scheme)
      *bytes = auto_plan(ctx, M, N, K).total;
      return OZK_OK;
    }
    if (p_or_s < 1 || p_or_s > OZK_MAX_P) return fail(ctx, OZK_ERR_UNSUPPORTED, 7);
    *bytes = s1_plan(ctx, p_or_s, M, N, K, config_for(ctx, op, scheme, p_or_s, M, N, K).split).total;
    return OZK_OK;
  }
  if (op == OZK_OP_ZGEMM && scheme == OZK_SCHEME1) {  // 4M on the real embedding
    if (p_or_s < 1 || p_or_s > OZK_MAX_P) return fail(ctx, OZK_ERR_UNSUPPORTED, 7);
    if (2 * N > OZK_MAX_ROWS || 2 * K > ((int64_t)1 << 40)) return fail(ctx, OZK_ERR_INVALID_ARG, 5);
    *bytes = s1z_plan(ctx, p_or_s, M, N, K).total;
    return OZK_OK;
  }
  if (op == OZK_OP_ZGEMM && scheme == OZK_SCHEME2 && p_or_s == 0) {  // the automatic ZGEMM
    *bytes = align256(s2_plan(OZK_MAX_S, true, M, N, K).total) + 512;
    return OZK_OK;
  }
  if (scheme == OZK_SCHEME2 && (op == OZK_OP_DGEMM || op == OZK_OP_ZGEMM)) {
    if (p_or_s < 1 || p_or_s > OZK_MAX_S) return fail(ctx, OZK_ERR_UNSUPPORTED, 7);
    *bytes = s2_plan(p_or_s, op == OZK_OP_ZGEMM, M, N, K).total;
    return OZK_OK;
  }
  if (op != OZK_OP_DGEMM && op != OZK_OP_ZGEMM) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  return fail(ctx, OZK_ERR_UNSUPPORTED, 3);
}

ozk_status ozk_s1_split_rows(ozk_ctx* ctx, int p, int64_t rows, int64_t K, const double* X, int64_t ldx,
                             int32_t* e, int8_t* packed, hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (p < 1 || p > OZK_MAX_P) return fail(ctx, OZK_ERR_UNSUPPORTED, 2);
  if (bad_rows(rows)) return fail(ctx, OZK_ERR_INVALID_ARG, 3);
  if (K < 0 || K > ((int64_t)1 << 40)) return fail(ctx, OZK_ERR_INVALID_ARG, 4);
  if (!X && rows > 0 && K > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 5);
  if (ldx < (K > 0 ? K : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 6);
  if (!e && rows > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 7);
  if (!packed && rows > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 8);
  return hip_status(ctx, ozk::s1_split_rows(p, X, ldx, rows, K, e, packed, stream));
}

ozk_status ozk_s1_split_cols(ozk_ctx* ctx, int p, int64_t K, int64_t cols, const double* X, int64_t ldx,
                             int32_t* f, int8_t* packed, hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (p < 1 || p > OZK_MAX_P) return fail(ctx, OZK_ERR_UNSUPPORTED, 2);
  if (K < 0 || K > ((int64_t)1 << 40)) return fail(ctx, OZK_ERR_INVALID_ARG, 3);
  if (bad_rows(cols)) return fail(ctx, OZK_ERR_INVALID_ARG, 4);
  if (!X && cols > 0 && K > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 5);
  if (ldx < (cols > 0 ? cols : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 6);
  if (!f && cols > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 7);
  if (!packed && cols > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 8);
  return hip_status(ctx, ozk::s1_split_cols(p, X, ldx, K, cols, f, packed, stream));
}

// The Scheme I GEMM of packed operands with configuration cfg (the check
// entry point writing diagonals always uses the default).
static ozk_status s1_gemm_common(ozk_ctx* ctx, int p, int64_t M, int64_t N, int64_t K, const int8_t* Ap,
                                 const int32_t* e, const int8_t* Bp, const int32_t* f, double alpha,
                                 double beta, double* C, int64_t ldc, void* ws, size_t ws_bytes,
                                 int32_t* diag, hipStream_t stream, ozk_gemm_config cfg, float* C32 = nullptr) {
  if (diag) cfg = default_config();
  const S1Plan pl = s1_plan(ctx, p, M, N, K, cfg.split);
  ozk::S1GemmArgs g;
  g.variant = cfg.variant;
  g.raster = cfg.raster;
  g.group = cfg.group;
  g.M = M;
  g.N = N;
  g.Ap = Ap;
  g.Bp = Bp;
  g.nchunk = pl.nchunk;
  g.steps_per_split = pl.nsplit > 1 ? pl.steps_per_split : (pl.nchunk > 0 ? pl.nchunk : 1);
  g.nsplit = pl.nsplit;
  g.e = e;
  g.f = f;
  g.alpha = alpha;
  g.beta = beta;
  g.C = C;
  g.ldc = ldc;
  g.zpart = nullptr;
  g.diag = diag;
  g.C32 = C32;
  if (!diag && pl.nsplit > 1) {
    const size_t need = 16 * (size_t)pl.nsplit * M * N;
    if (!ws || ws_bytes < need) return fail(ctx, OZK_ERR_WORKSPACE, 15);
    g.zpart = (int64_t*)ws;
  }
  return hip_status(ctx, ozk::s1_gemm(p, g, stream));
}

ozk_status ozk_s1_gemm(ozk_ctx* ctx, int p, int64_t M, int64_t N, int64_t K, const int8_t* packedA,
                       const int32_t* e, const int8_t* packedB, const int32_t* f, double alpha, double beta,
                       double* C, int64_t ldc, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (p < 1 || p > OZK_MAX_P) return fail(ctx, OZK_ERR_UNSUPPORTED, 2);
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, 3);
  if (M > 0 && N > 0) {
    if (!packedA) return fail(ctx, OZK_ERR_INVALID_ARG, 6);
    if (!e) return fail(ctx, OZK_ERR_INVALID_ARG, 7);
    if (!packedB) return fail(ctx, OZK_ERR_INVALID_ARG, 8);
    if (!f) return fail(ctx, OZK_ERR_INVALID_ARG, 9);
    if (!C) return fail(ctx, OZK_ERR_INVALID_ARG, 12);
  }
  if (ldc < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 13);
  return s1_gemm_common(ctx, p, M, N, K, packedA, e, packedB, f, alpha, beta, C, ldc, ws, ws_bytes, nullptr,
                        stream, config_for(ctx, OZK_OP_DGEMM, OZK_SCHEME1, p, M, N, K));
}

ozk_status ozk_s1_diagonals(ozk_ctx* ctx, int p, int64_t M, int64_t N, int64_t K, const int8_t* packedA,
                            const int8_t* packedB, int32_t* Cd, hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (p < 1 || p > OZK_MAX_P) return fail(ctx, OZK_ERR_UNSUPPORTED, 2);
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, 3);
  if (K > k_split_of(ctx, p)) return fail(ctx, OZK_ERR_UNSUPPORTED, 5);
  if (M > 0 && N > 0 && (!packedA || !packedB || !Cd)) return fail(ctx, OZK_ERR_INVALID_ARG, 6);
  return s1_gemm_common(ctx, p, M, N, K, packedA, nullptr, packedB, nullptr, 1.0, 0.0, nullptr, N > 0 ? N : 1,
                        nullptr, 0, Cd, stream, default_config());
}

// The DGEMM pipeline after argument checks; trans_a / trans_b: the operand
// is stored transposed (A as K x M, B as N x K, row-major).
// swap_budgets: the row operand takes Scheme II's column budget T_B and the
// column operand T_A (a column-major problem run as its row-major transpose
// keeps each operand's own budget; T_A and T_B differ by one bit when
// ceil(log2 P) is odd).
static ozk_status dgemm_run(ozk_ctx* ctx, ozk_scheme scheme, int p_or_s, bool trans_a, bool trans_b, int64_t M,
                            int64_t N, int64_t K, double alpha, const double* A, int64_t lda, const double* B,
                            int64_t ldb, double beta, double* C, int64_t ldc, void* ws, size_t ws_bytes,
                            hipStream_t stream, int ws_arg, bool swap_budgets = false) {
  if (scheme == OZK_SCHEME2) {
    const int s = p_or_s;
    if (s < 1 || s > OZK_MAX_S) return fail(ctx, OZK_ERR_UNSUPPORTED, 3);
    // K is argument 6 of ozk_dgemm (workspace 15) and 8 of ozk_dgemm_t (workspace 19)
    if (s2_long_k(K)) return fail(ctx, OZK_ERR_UNSUPPORTED, ws_arg == 15 ? 6 : 8);
    const S2Plan pl = s2_plan(s, false, M, N, K);
    if (!ws || ws_bytes < pl.total) return fail(ctx, OZK_ERR_WORKSPACE, ws_arg);
    if (M == 0 || N == 0) return OZK_OK;
    char* w = (char*)ws;
    int32_t* sig = (int32_t*)(w + pl.off_sig);
    int32_t* tau = (int32_t*)(w + pl.off_tau);
    int8_t* Ap = (int8_t*)(w + pl.off_a);
    int8_t* Bp = (int8_t*)(w + pl.off_b);
    int8_t* res = (int8_t*)(w + pl.off_res);
    int ta_bits, tb_bits;
    ozk::s2_targets(s, ta_bits, tb_bits);
    if (swap_budgets) std::swap(ta_bits, tb_bits);
    // a transposed operand is read by the other pass, with its own bit budget
    hipError_t err = trans_a ? ozk::s2_split_cols(s, false, A, lda, K, M, sig, Ap, stream, ta_bits)
                             : ozk::s2_split_rows(s, false, A, lda, M, K, sig, Ap, stream, ta_bits);
    if (err == hipSuccess)
      err = trans_b ? ozk::s2_split_rows(s, false, B, ldb, N, K, tau, Bp, stream, tb_bits)
                    : ozk::s2_split_cols(s, false, B, ldb, K, N, tau, Bp, stream, tb_bits);
    if (err == hipSuccess) err = ozk::flag_nonfinite(sig, M, tau, N, ctx->dflags, stream);
    const ozk_gemm_config cfg = config_for(ctx, OZK_OP_DGEMM, OZK_SCHEME2, s, M, N, K);
    if (cfg.variant == OZK_S2_FUSED_CRT) {
      if (err == hipSuccess)
        err = ozk::s2_gemm_crt(s, M, N, K, Ap, Bp, sig, tau, alpha, beta, C, ldc, cfg.raster, cfg.group, stream);
      return hip_status(ctx, err);
    }
    if (err == hipSuccess)
      err = ozk::s2_gemm_mod(s, false, M, N, K, Ap, Bp, res, stream, cfg.variant, cfg.raster, cfg.group);
    const double al[2] = {alpha, 0.0}, be[2] = {beta, 0.0};
    if (err == hipSuccess) err = ozk::s2_crt(s, false, M, N, res, sig, tau, al, be, C, ldc, stream);
    return hip_status(ctx, err);
  }
  const int p = p_or_s;
  if (p < 1 || p > OZK_MAX_P) return fail(ctx, OZK_ERR_UNSUPPORTED, 3);
  const ozk_gemm_config cfg = config_for(ctx, OZK_OP_DGEMM, OZK_SCHEME1, p, M, N, K);
  const S1Plan pl = s1_plan(ctx, p, M, N, K, cfg.split);
  if (!ws || ws_bytes < pl.total) return fail(ctx, OZK_ERR_WORKSPACE, ws_arg);
  if (M == 0 || N == 0) return OZK_OK;
  char* w = (char*)ws;
  int32_t* e = (int32_t*)(w + pl.off_e);
  int32_t* f = (int32_t*)(w + pl.off_f);
  int8_t* Ap = (int8_t*)(w + pl.off_a);
  int8_t* Bp = (int8_t*)(w + pl.off_b);
  // a transposed operand is read by the other pass (same packed layout)
  hipError_t err = trans_a ? ozk::s1_split_cols(p, A, lda, K, M, e, Ap, stream)
                           : ozk::s1_split_rows(p, A, lda, M, K, e, Ap, stream);
  if (err == hipSuccess)
    err = trans_b ? ozk::s1_split_rows(p, B, ldb, N, K, f, Bp, stream) : ozk::s1_split_cols(p, B, ldb, K, N, f, Bp, stream);
  if (err == hipSuccess) err = ozk::flag_nonfinite(e, M, f, N, ctx->dflags, stream);
  if (err != hipSuccess) return hip_status(ctx, err);
  return s1_gemm_common(ctx, p, M, N, K, Ap, e, Bp, f, alpha, beta, C, ldc, w + pl.off_z,
                        pl.total - pl.off_z, nullptr, stream, cfg);
}

ozk_status ozk_dgemm(ozk_ctx* ctx, ozk_scheme scheme, int p_or_s, int64_t M, int64_t N, int64_t K,
                     double alpha, const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                     double* C, int64_t ldc, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (scheme != OZK_SCHEME1 && scheme != OZK_SCHEME2) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, M < 0 ? 4 : (N < 0 ? 5 : 6));
  if (!A && M > 0 && K > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 8);
  if (lda < (K > 0 ? K : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 9);
  if (!B && K > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 10);
  if (ldb < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 11);
  if (!C && M > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 13);
  if (ldc < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 14);
  return dgemm_run(ctx, scheme, p_or_s, false, false, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, ws_bytes,
                   stream, 15);
}

ozk_status ozk_dgemm_noalloc(ozk_ctx* ctx, ozk_scheme scheme, int p_or_s, int64_t M, int64_t N, int64_t K,
                             double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                             double beta, double* C, int64_t ldc, hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (scheme != OZK_SCHEME1 && scheme != OZK_SCHEME2) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, M < 0 ? 4 : (N < 0 ? 5 : 6));
  if (!A && M > 0 && K > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 8);
  if (lda < (K > 0 ? K : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 9);
  if (!B && K > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 10);
  if (ldb < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 11);
  if (!C && M > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 13);
  if (ldc < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 14);
  if (scheme == OZK_SCHEME2 && (p_or_s < 1 || p_or_s > OZK_MAX_S)) return fail(ctx, OZK_ERR_UNSUPPORTED, 3);
  if (scheme == OZK_SCHEME1 && (p_or_s < 1 || p_or_s > OZK_MAX_P)) return fail(ctx, OZK_ERR_UNSUPPORTED, 3);
  if (scheme == OZK_SCHEME2 && s2_long_k(K)) return fail(ctx, OZK_ERR_UNSUPPORTED, 6);
  if (!ctx->scratch) return fail(ctx, OZK_ERR_HIP, 0);
  // the workspace ozk_dgemm would take must fit the fixed buffer
  size_t need = 0;
  const ozk_status st = ozk_workspace_size(ctx, OZK_OP_DGEMM, scheme, M, N, K, p_or_s, &need);
  if (st != OZK_OK) return fail(ctx, st, 4);
  if (need > (size_t)OZK_NOALLOC_SCRATCH_BYTES) return fail(ctx, OZK_ERR_WORKSPACE, 4);
  return dgemm_run(ctx, scheme, p_or_s, false, false, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ctx->scratch,
                   OZK_NOALLOC_SCRATCH_BYTES, stream, 15);
}

ozk_status ozk_dgemm_t(ozk_ctx* ctx, ozk_scheme scheme, int p_or_s, int trans_a, int trans_b, int64_t M, int64_t N,
                       int64_t K, double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                       double beta, double* C, int64_t ldc, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (scheme != OZK_SCHEME1 && scheme != OZK_SCHEME2) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  if (trans_a != 0 && trans_a != 1) return fail(ctx, OZK_ERR_INVALID_ARG, 4);
  if (trans_b != 0 && trans_b != 1) return fail(ctx, OZK_ERR_INVALID_ARG, 5);
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, M < 0 ? 6 : (N < 0 ? 7 : 8));
  const int64_t acols = trans_a ? M : K, bcols = trans_b ? K : N;  // row lengths as stored
  const bool a_empty = M == 0 || K == 0, b_empty = K == 0 || N == 0;
  if (!A && !a_empty) return fail(ctx, OZK_ERR_INVALID_ARG, 10);
  if (lda < (acols > 0 ? acols : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 11);
  if (!B && !b_empty) return fail(ctx, OZK_ERR_INVALID_ARG, 12);
  if (ldb < (bcols > 0 ? bcols : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 13);
  if (!C && M > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 15);
  if (ldc < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 16);
  if (scheme == OZK_SCHEME2 && (p_or_s < 1 || p_or_s > OZK_MAX_S)) return fail(ctx, OZK_ERR_UNSUPPORTED, 3);
  if (scheme == OZK_SCHEME1 && (p_or_s < 1 || p_or_s > OZK_MAX_P)) return fail(ctx, OZK_ERR_UNSUPPORTED, 3);
  return dgemm_run(ctx, scheme, p_or_s, trans_a != 0, trans_b != 0, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws,
                   ws_bytes, stream, 19);
}

// The unfused baseline: the DGEMM pre-pass, then one INT8 GEMM per slice
// pair writing INT32 planes, then the reconstruction.
static size_t s1_unfused_ws(const ozk_ctx* ctx, int p, int64_t M, int64_t N, int64_t K, S1Plan& pl) {
  pl = s1_plan(ctx, p, M, N, K, 1);
  return align256(pl.off_z) + (size_t)ozk::s1_unfused_planes_bytes(p, M, N);
}

ozk_status ozk_s1_unfused_workspace_size(ozk_ctx* ctx, int p, int64_t M, int64_t N, int64_t K, size_t* bytes) {
  if (!ctx || !bytes) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (p < 1 || p > OZK_MAX_P) return fail(ctx, OZK_ERR_UNSUPPORTED, 2);
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, 3);
  S1Plan pl;
  *bytes = s1_unfused_ws(ctx, p, M, N, K, pl);
  return OZK_OK;
}

ozk_status ozk_s1_dgemm_unfused(ozk_ctx* ctx, int p, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                                int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                                void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (p < 1 || p > OZK_MAX_P) return fail(ctx, OZK_ERR_UNSUPPORTED, 2);
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, M < 0 ? 3 : (N < 0 ? 4 : 5));
  if (K > 131071) return fail(ctx, OZK_ERR_UNSUPPORTED, 5);  // |sum| <= K 2^14 < 2^31
  if (!A && M > 0 && K > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 7);
  if (lda < (K > 0 ? K : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 8);
  if (!B && K > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 9);
  if (ldb < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 10);
  if (!C && M > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 12);
  if (ldc < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 13);
  S1Plan pl;
  const size_t need = s1_unfused_ws(ctx, p, M, N, K, pl);
  if (!ws || ws_bytes < need) return fail(ctx, OZK_ERR_WORKSPACE, 15);
  if (M == 0 || N == 0) return OZK_OK;
  char* w = (char*)ws;
  int32_t* e = (int32_t*)(w + pl.off_e);
  int32_t* f = (int32_t*)(w + pl.off_f);
  int8_t* Ap = (int8_t*)(w + pl.off_a);
  int8_t* Bp = (int8_t*)(w + pl.off_b);
  int32_t* planes = (int32_t*)(w + align256(pl.off_z));
  hipError_t err = ozk::s1_split_rows(p, A, lda, M, K, e, Ap, stream);
  if (err == hipSuccess) err = ozk::s1_split_cols(p, B, ldb, K, N, f, Bp, stream);
  if (err == hipSuccess) err = ozk::flag_nonfinite(e, M, f, N, ctx->dflags, stream);
  if (err == hipSuccess)
    err = ozk::s1_gemm_unfused(p, M, N, K, Ap, e, Bp, f, alpha, beta, C, ldc, planes, stream);
  return hip_status(ctx, err);
}

ozk_status ozk_sgemm(ozk_ctx* ctx, ozk_scheme scheme, int p_or_s, int64_t M, int64_t N, int64_t K, float alpha,
                     const float* A, int64_t lda, const float* B, int64_t ldb, float beta, float* C, int64_t ldc,
                     void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (scheme != OZK_SCHEME1 && scheme != OZK_SCHEME2) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, M < 0 ? 4 : (N < 0 ? 5 : 6));
  if (!A && M > 0 && K > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 8);
  if (lda < (K > 0 ? K : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 9);
  if (!B && K > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 10);
  if (ldb < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 11);
  if (!C && M > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 13);
  if (ldc < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 14);
  // the GEMM steps are the DGEMM ones (same packed operands), so they share their configurations
  if (scheme == OZK_SCHEME2) {
    const int s = p_or_s;
    if (s < 1 || s > OZK_MAX_S) return fail(ctx, OZK_ERR_UNSUPPORTED, 3);
    if (s2_long_k(K)) return fail(ctx, OZK_ERR_UNSUPPORTED, 6);
    const S2Plan pl = s2_plan(s, false, M, N, K);
    if (!ws || ws_bytes < pl.total) return fail(ctx, OZK_ERR_WORKSPACE, 15);
    if (M == 0 || N == 0) return OZK_OK;
    char* w = (char*)ws;
    int32_t* sig = (int32_t*)(w + pl.off_sig);
    int32_t* tau = (int32_t*)(w + pl.off_tau);
    int8_t* Ap = (int8_t*)(w + pl.off_a);
    int8_t* Bp = (int8_t*)(w + pl.off_b);
    int8_t* res = (int8_t*)(w + pl.off_res);
    hipError_t err = ozk::s2_split_rows(s, false, A, lda, M, K, sig, Ap, stream);
    if (err == hipSuccess) err = ozk::s2_split_cols(s, false, B, ldb, K, N, tau, Bp, stream);
    if (err == hipSuccess) err = ozk::flag_nonfinite(sig, M, tau, N, ctx->dflags, stream);
    const ozk_gemm_config cfg = config_for(ctx, OZK_OP_DGEMM, OZK_SCHEME2, s, M, N, K);
    if (err == hipSuccess)  // the fused-CRT variant writes binary64: the separate kernels here
      err = ozk::s2_gemm_mod(s, false, M, N, K, Ap, Bp, res, stream, cfg.variant, cfg.raster, cfg.group);
    const float al[2] = {alpha, 0.0f}, be[2] = {beta, 0.0f};
    if (err == hipSuccess) err = ozk::s2_crt(s, false, M, N, res, sig, tau, al, be, C, ldc, stream);
    return hip_status(ctx, err);
  }
  const int p = p_or_s;
  if (p < 1 || p > OZK_MAX_P) return fail(ctx, OZK_ERR_UNSUPPORTED, 3);
  const ozk_gemm_config cfg = config_for(ctx, OZK_OP_DGEMM, OZK_SCHEME1, p, M, N, K);
  const S1Plan pl = s1_plan(ctx, p, M, N, K, cfg.split);
  if (!ws || ws_bytes < pl.total) return fail(ctx, OZK_ERR_WORKSPACE, 15);
  if (M == 0 || N == 0) return OZK_OK;
  char* w = (char*)ws;
  int32_t* e = (int32_t*)(w + pl.off_e);
  int32_t* f = (int32_t*)(w + pl.off_f);
  int8_t* Ap = (int8_t*)(w + pl.off_a);
  int8_t* Bp = (int8_t*)(w + pl.off_b);
  hipError_t err = ozk::s1_split_rows(p, A, lda, M, K, e, Ap, stream);
  if (err == hipSuccess) err = ozk::s1_split_cols(p, B, ldb, K, N, f, Bp, stream);
  if (err == hipSuccess) err = ozk::flag_nonfinite(e, M, f, N, ctx->dflags, stream);
  if (err != hipSuccess) return hip_status(ctx, err);
  return s1_gemm_common(ctx, p, M, N, K, Ap, e, Bp, f, alpha, beta, nullptr, ldc, w + pl.off_z, pl.total - pl.off_z,
                        nullptr, stream, cfg, C);
}

ozk_status ozk_cgemm_3m(ozk_ctx* ctx, int s, int64_t M, int64_t N, int64_t K, const float* alpha, const float* A,
                        int64_t lda, const float* B, int64_t ldb, const float* beta, float* C, int64_t ldc, void* ws,
                        size_t ws_bytes, hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (s < 1 || s > OZK_MAX_S) return fail(ctx, OZK_ERR_UNSUPPORTED, 2);
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, M < 0 ? 3 : (N < 0 ? 4 : 5));
  if (!alpha) return fail(ctx, OZK_ERR_INVALID_ARG, 6);
  if (!A && M > 0 && K > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 7);
  if (lda < (K > 0 ? K : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 8);
  if (!B && K > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 9);
  if (ldb < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 10);
  if (!beta) return fail(ctx, OZK_ERR_INVALID_ARG, 11);
  if (!C && M > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 12);
  if (ldc < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 13);
  if (s2_long_k(K)) return fail(ctx, OZK_ERR_UNSUPPORTED, 5);
  const S2Plan pl = s2_plan(s, true, M, N, K);
  if (!ws || ws_bytes < pl.total) return fail(ctx, OZK_ERR_WORKSPACE, 14);
  if (M == 0 || N == 0) return OZK_OK;
  char* w = (char*)ws;
  int32_t* sig = (int32_t*)(w + pl.off_sig);
  int32_t* tau = (int32_t*)(w + pl.off_tau);
  int8_t* Ap = (int8_t*)(w + pl.off_a);
  int8_t* Bp = (int8_t*)(w + pl.off_b);
  int8_t* res = (int8_t*)(w + pl.off_res);
  hipError_t err = ozk::s2_split_rows(s, true, A, lda, M, K, sig, Ap, stream);
  if (err == hipSuccess) err = ozk::s2_split_cols(s, true, B, ldb, K, N, tau, Bp, stream);
  if (err == hipSuccess) err = ozk::flag_nonfinite(sig, M, tau, N, ctx->dflags, stream);
  const ozk_gemm_config cfg = config_for(ctx, OZK_OP_ZGEMM, OZK_SCHEME2, s, M, N, K);
  if (err == hipSuccess)
    err = ozk::s2_gemm_mod(s, true, M, N, K, Ap, Bp, res, stream, cfg.variant, cfg.raster, cfg.group);
  if (err == hipSuccess) err = ozk::s2_crt(s, true, M, N, res, sig, tau, alpha, beta, C, ldc, stream);
  return hip_status(ctx, err);
}

ozk_status ozk_zgemm_3m(ozk_ctx* ctx, int s, int64_t M, int64_t N, int64_t K, const double* alpha,
                        const double* A, int64_t lda, const double* B, int64_t ldb, const double* beta,
                        double* C, int64_t ldc, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (s < 1 || s > OZK_MAX_S) return fail(ctx, OZK_ERR_UNSUPPORTED, 2);
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, M < 0 ? 3 : (N < 0 ? 4 : 5));
  if (!alpha) return fail(ctx, OZK_ERR_INVALID_ARG, 6);
  if (!A && M > 0 && K > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 7);
  if (lda < (K > 0 ? K : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 8);
  if (!B && K > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 9);
  if (ldb < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 10);
  if (!beta) return fail(ctx, OZK_ERR_INVALID_ARG, 11);
  if (!C && M > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 12);
  if (ldc < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 13);
  if (s2_long_k(K)) return fail(ctx, OZK_ERR_UNSUPPORTED, 5);
  const S2Plan pl = s2_plan(s, true, M, N, K);
  if (!ws || ws_bytes < pl.total) return fail(ctx, OZK_ERR_WORKSPACE, 14);
  if (M == 0 || N == 0) return OZK_OK;
  char* w = (char*)ws;
  int32_t* sig = (int32_t*)(w + pl.off_sig);
  int32_t* tau = (int32_t*)(w + pl.off_tau);
  int8_t* Ap = (int8_t*)(w + pl.off_a);
  int8_t* Bp = (int8_t*)(w + pl.off_b);
  int8_t* res = (int8_t*)(w + pl.off_res);
  hipError_t err = ozk::s2_split_rows(s, true, A, lda, M, K, sig, Ap, stream);
  if (err == hipSuccess) err = ozk::s2_split_cols(s, true, B, ldb, K, N, tau, Bp, stream);
  if (err == hipSuccess) err = ozk::flag_nonfinite(sig, M, tau, N, ctx->dflags, stream);
  const ozk_gemm_config cfg = config_for(ctx, OZK_OP_ZGEMM, OZK_SCHEME2, s, M, N, K);
  if (err == hipSuccess)
    err = ozk::s2_gemm_mod(s, true, M, N, K, Ap, Bp, res, stream, cfg.variant, cfg.raster, cfg.group);
  if (err == hipSuccess) err = ozk::s2_crt(s, true, M, N, res, sig, tau, alpha, beta, C, ldc, stream);
  return hip_status(ctx, err);
}

}  // extern "C"

// The complex product by Scheme I and 4M (T = double: ZGEMM, float: CGEMM):
// the real embedding's pre-pass (A's rows as they are stored, B through the
// embedding kernel), the Scheme I GEMM of the M x 2K by 2K x 2N real product
// into the parts H, then the complex update.  Arguments checked by the caller.
template <typename T>
static ozk_status zgemm4m_run(ozk_ctx* ctx, int p, int64_t M, int64_t N, int64_t K, const T* alpha, const T* A,
                              int64_t lda, const T* B, int64_t ldb, const T* beta, T* C, int64_t ldc, void* ws,
                              size_t ws_bytes, hipStream_t stream, int ws_arg) {
  if (2 * N > OZK_MAX_ROWS) return fail(ctx, OZK_ERR_INVALID_ARG, 5);
  const S1ZPlan zp = s1z_plan(ctx, p, M, N, K);
  if (!ws || ws_bytes < zp.total) return fail(ctx, OZK_ERR_WORKSPACE, ws_arg);
  if (M == 0 || N == 0) return OZK_OK;
  char* w = (char*)ws;
  const S1Plan& pl = zp.s1;
  int32_t* e = (int32_t*)(w + pl.off_e);
  int32_t* f = (int32_t*)(w + pl.off_f);
  int8_t* Ap = (int8_t*)(w + pl.off_a);
  int8_t* Bp = (int8_t*)(w + pl.off_b);
  T* H = (T*)(w + zp.off_h);
  // row i of A viewed as 2K reals (re, im, re, im, ...) is row i of the embedding
  hipError_t err = ozk::s1_split_rows(p, A, 2 * lda, M, 2 * K, e, Ap, stream);
  if (err == hipSuccess) err = ozk::s1_split_cols_4m(p, B, ldb, K, N, f, Bp, stream);
  if (err == hipSuccess) err = ozk::flag_nonfinite(e, M, f, 2 * N, ctx->dflags, stream);
  if (err != hipSuccess) return hip_status(ctx, err);
  ozk_status st;
  if constexpr (sizeof(T) == 8)
    st = s1_gemm_common(ctx, p, M, 2 * N, 2 * K, Ap, e, Bp, f, 1.0, 0.0, (double*)H, 2 * N, w + pl.off_z,
                        zp.off_h - pl.off_z, nullptr, stream, zp.cfg);
  else
    st = s1_gemm_common(ctx, p, M, 2 * N, 2 * K, Ap, e, Bp, f, 1.0, 0.0, nullptr, 2 * N, w + pl.off_z,
                        zp.off_h - pl.off_z, nullptr, stream, zp.cfg, (float*)H);
  if (st != OZK_OK) return st;
  return hip_status(ctx, ozk::zaxpby(H, 2 * N, M, N, alpha, beta, C, ldc, stream));
}

extern "C" {

// Shared checks of ozk_zgemm / ozk_cgemm (argument positions of their signature).
static ozk_status check_complex_call(ozk_ctx* ctx, int scheme, int p_or_s, int64_t M, int64_t N, int64_t K,
                                     const void* alpha, const void* A, int64_t lda, const void* B, int64_t ldb,
                                     const void* beta, const void* C, int64_t ldc) {
  if (scheme != OZK_SCHEME1 && scheme != OZK_SCHEME2) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, M < 0 ? 4 : (N < 0 ? 5 : 6));
  if (!alpha) return fail(ctx, OZK_ERR_INVALID_ARG, 7);
  if (!A && M > 0 && K > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 8);
  if (lda < (K > 0 ? K : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 9);
  if (!B && K > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 10);
  if (ldb < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 11);
  if (!beta) return fail(ctx, OZK_ERR_INVALID_ARG, 12);
  if (!C && M > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 13);
  if (ldc < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 14);
  const int hi = scheme == OZK_SCHEME1 ? OZK_MAX_P : OZK_MAX_S;
  if (p_or_s < 1 || p_or_s > hi) return fail(ctx, OZK_ERR_UNSUPPORTED, 3);
  if (scheme == OZK_SCHEME2 && s2_long_k(K)) return fail(ctx, OZK_ERR_UNSUPPORTED, 6);
  return OZK_OK;
}

ozk_status ozk_zgemm(ozk_ctx* ctx, ozk_scheme scheme, int p_or_s, int64_t M, int64_t N, int64_t K,
                     const double* alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                     const double* beta, double* C, int64_t ldc, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  const ozk_status st = check_complex_call(ctx, scheme, p_or_s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  if (st != OZK_OK) return st;
  if (scheme == OZK_SCHEME2) {
    const ozk_status r = ozk_zgemm_3m(ctx, p_or_s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, ws_bytes, stream);
    if (r == OZK_ERR_WORKSPACE) ctx->last_arg = 15;
    return r;
  }
  return zgemm4m_run<double>(ctx, p_or_s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, ws_bytes, stream, 15);
}

ozk_status ozk_cgemm(ozk_ctx* ctx, ozk_scheme scheme, int p_or_s, int64_t M, int64_t N, int64_t K,
                     const float* alpha, const float* A, int64_t lda, const float* B, int64_t ldb, const float* beta,
                     float* C, int64_t ldc, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  const ozk_status st = check_complex_call(ctx, scheme, p_or_s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  if (st != OZK_OK) return st;
  if (scheme == OZK_SCHEME2) {
    const ozk_status r = ozk_cgemm_3m(ctx, p_or_s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, ws_bytes, stream);
    if (r == OZK_ERR_WORKSPACE) ctx->last_arg = 15;
    return r;
  }
  return zgemm4m_run<float>(ctx, p_or_s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, ws_bytes, stream, 15);
}

// ------------------------------------------- general layouts (ozk_gemm_ex)

}  // extern "C"

// Real product with transposed operands in binary32 (the binary64 one is
// dgemm_run): as ozk_sgemm, with a transposed operand read by the other
// pre-pass kernel (same packed layout and scales).
static ozk_status sgemm_run(ozk_ctx* ctx, ozk_scheme scheme, int p_or_s, bool trans_a, bool trans_b, int64_t M,
                            int64_t N, int64_t K, float alpha, const float* A, int64_t lda, const float* B,
                            int64_t ldb, float beta, float* C, int64_t ldc, void* ws, size_t ws_bytes,
                            hipStream_t stream, int ws_arg, bool swap_budgets) {
  char* w = (char*)ws;
  if (scheme == OZK_SCHEME2) {
    const int s = p_or_s;
    const S2Plan pl = s2_plan(s, false, M, N, K);
    if (!ws || ws_bytes < pl.total) return fail(ctx, OZK_ERR_WORKSPACE, ws_arg);
    if (M == 0 || N == 0) return OZK_OK;
    int32_t* sig = (int32_t*)(w + pl.off_sig);
    int32_t* tau = (int32_t*)(w + pl.off_tau);
    int8_t* Ap = (int8_t*)(w + pl.off_a);
    int8_t* Bp = (int8_t*)(w + pl.off_b);
    int8_t* res = (int8_t*)(w + pl.off_res);
    int ta_bits, tb_bits;
    ozk::s2_targets(s, ta_bits, tb_bits);
    if (swap_budgets) std::swap(ta_bits, tb_bits);
    hipError_t err = trans_a ? ozk::s2_split_cols(s, false, A, lda, K, M, sig, Ap, stream, ta_bits)
                             : ozk::s2_split_rows(s, false, A, lda, M, K, sig, Ap, stream, ta_bits);
    if (err == hipSuccess)
      err = trans_b ? ozk::s2_split_rows(s, false, B, ldb, N, K, tau, Bp, stream, tb_bits)
                    : ozk::s2_split_cols(s, false, B, ldb, K, N, tau, Bp, stream, tb_bits);
    if (err == hipSuccess) err = ozk::flag_nonfinite(sig, M, tau, N, ctx->dflags, stream);
    const ozk_gemm_config cfg = config_for(ctx, OZK_OP_DGEMM, OZK_SCHEME2, s, M, N, K);
    if (err == hipSuccess)
      err = ozk::s2_gemm_mod(s, false, M, N, K, Ap, Bp, res, stream, cfg.variant, cfg.raster, cfg.group);
    const float al[2] = {alpha, 0.0f}, be[2] = {beta, 0.0f};
    if (err == hipSuccess) err = ozk::s2_crt(s, false, M, N, res, sig, tau, al, be, C, ldc, stream);
    return hip_status(ctx, err);
  }
  const int p = p_or_s;
  const ozk_gemm_config cfg = config_for(ctx, OZK_OP_DGEMM, OZK_SCHEME1, p, M, N, K);
  const S1Plan pl = s1_plan(ctx, p, M, N, K, cfg.split);
  if (!ws || ws_bytes < pl.total) return fail(ctx, OZK_ERR_WORKSPACE, ws_arg);
  if (M == 0 || N == 0) return OZK_OK;
  int32_t* e = (int32_t*)(w + pl.off_e);
  int32_t* f = (int32_t*)(w + pl.off_f);
  int8_t* Ap = (int8_t*)(w + pl.off_a);
  int8_t* Bp = (int8_t*)(w + pl.off_b);
  hipError_t err = trans_a ? ozk::s1_split_cols(p, A, lda, K, M, e, Ap, stream)
                           : ozk::s1_split_rows(p, A, lda, M, K, e, Ap, stream);
  if (err == hipSuccess)
    err = trans_b ? ozk::s1_split_rows(p, B, ldb, N, K, f, Bp, stream) : ozk::s1_split_cols(p, B, ldb, K, N, f, Bp, stream);
  if (err == hipSuccess) err = ozk::flag_nonfinite(e, M, f, N, ctx->dflags, stream);
  if (err != hipSuccess) return hip_status(ctx, err);
  return s1_gemm_common(ctx, p, M, N, K, Ap, e, Bp, f, alpha, beta, nullptr, ldc, w + pl.off_z, pl.total - pl.off_z,
                        nullptr, stream, cfg, C);
}

// The 3M complex product with transposed operands (T = double: ZGEMM,
// float: CGEMM); a transposed operand is read by the other pre-pass kernel.
template <typename T>
static ozk_status zgemm3m_run(ozk_ctx* ctx, int s, bool trans_a, bool trans_b, int64_t M, int64_t N, int64_t K,
                              const T* alpha, const T* A, int64_t lda, const T* B, int64_t ldb, const T* beta, T* C,
                              int64_t ldc, void* ws, size_t ws_bytes, hipStream_t stream, int ws_arg,
                              bool swap_budgets) {
  const S2Plan pl = s2_plan(s, true, M, N, K);
  if (!ws || ws_bytes < pl.total) return fail(ctx, OZK_ERR_WORKSPACE, ws_arg);
  if (M == 0 || N == 0) return OZK_OK;
  char* w = (char*)ws;
  int32_t* sig = (int32_t*)(w + pl.off_sig);
  int32_t* tau = (int32_t*)(w + pl.off_tau);
  int8_t* Ap = (int8_t*)(w + pl.off_a);
  int8_t* Bp = (int8_t*)(w + pl.off_b);
  int8_t* res = (int8_t*)(w + pl.off_res);
  int ta_bits, tb_bits;
  ozk::s2_targets(s, ta_bits, tb_bits);
  if (swap_budgets) std::swap(ta_bits, tb_bits);
  hipError_t err = trans_a ? ozk::s2_split_cols(s, true, A, lda, K, M, sig, Ap, stream, ta_bits)
                           : ozk::s2_split_rows(s, true, A, lda, M, K, sig, Ap, stream, ta_bits);
  if (err == hipSuccess)
    err = trans_b ? ozk::s2_split_rows(s, true, B, ldb, N, K, tau, Bp, stream, tb_bits)
                  : ozk::s2_split_cols(s, true, B, ldb, K, N, tau, Bp, stream, tb_bits);
  if (err == hipSuccess) err = ozk::flag_nonfinite(sig, M, tau, N, ctx->dflags, stream);
  const ozk_gemm_config cfg = config_for(ctx, OZK_OP_ZGEMM, OZK_SCHEME2, s, M, N, K);
  if (err == hipSuccess)
    err = ozk::s2_gemm_mod(s, true, M, N, K, Ap, Bp, res, stream, cfg.variant, cfg.raster, cfg.group);
  if (err == hipSuccess) err = ozk::s2_crt(s, true, M, N, res, sig, tau, alpha, beta, C, ldc, stream);
  return hip_status(ctx, err);
}

extern "C" {

ozk_status ozk_gemm_ex(ozk_ctx* ctx, ozk_dtype dtype, ozk_layout layout, int trans_a, int trans_b, ozk_scheme scheme,
                       int p_or_s, int64_t M, int64_t N, int64_t K, const void* alpha, const void* A, int64_t lda,
                       const void* B, int64_t ldb, const void* beta, void* C, int64_t ldc, void* ws,
                       size_t ws_bytes, hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (dtype != OZK_F64 && dtype != OZK_F32 && dtype != OZK_C128 && dtype != OZK_C64)
    return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  if (layout != OZK_ROW_MAJOR && layout != OZK_COL_MAJOR) return fail(ctx, OZK_ERR_INVALID_ARG, 3);
  if (trans_a != 0 && trans_a != 1) return fail(ctx, OZK_ERR_INVALID_ARG, 4);
  if (trans_b != 0 && trans_b != 1) return fail(ctx, OZK_ERR_INVALID_ARG, 5);
  if (scheme != OZK_SCHEME1 && scheme != OZK_SCHEME2) return fail(ctx, OZK_ERR_INVALID_ARG, 6);
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, M < 0 ? 8 : (N < 0 ? 9 : 10));
  if (!alpha) return fail(ctx, OZK_ERR_INVALID_ARG, 11);
  if (!beta) return fail(ctx, OZK_ERR_INVALID_ARG, 16);
  // Stored shapes: op(A) is M x K, so A holds M x K (no transpose) or K x M;
  // each leading dimension is at least the length of a stored line (a row
  // for row-major, a column for column-major).
  const bool col = layout == OZK_COL_MAJOR;
  const int64_t a_rows = trans_a ? K : M, a_cols = trans_a ? M : K;
  const int64_t b_rows = trans_b ? N : K, b_cols = trans_b ? K : N;
  const int64_t a_line = col ? a_rows : a_cols, b_line = col ? b_rows : b_cols, c_line = col ? M : N;
  if (!A && a_rows > 0 && a_cols > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 12);
  if (lda < (a_line > 0 ? a_line : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 13);
  if (!B && b_rows > 0 && b_cols > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 14);
  if (ldb < (b_line > 0 ? b_line : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 15);
  if (!C && M > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 17);
  if (ldc < (c_line > 0 ? c_line : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 18);
  const bool cplx = dtype == OZK_C128 || dtype == OZK_C64;
  const int hi = scheme == OZK_SCHEME1 ? OZK_MAX_P : OZK_MAX_S;
  if (p_or_s < 1 || p_or_s > hi) return fail(ctx, OZK_ERR_UNSUPPORTED, 7);
  if (scheme == OZK_SCHEME2 && s2_long_k(K)) return fail(ctx, OZK_ERR_UNSUPPORTED, 10);
  // Column-major storage of X is row-major storage of X^T, and C = op(A) op(B)
  // is C^T = op(B)^T op(A)^T: the row-major product of the swapped operands,
  // each transposed exactly when the other one was.  A row of op(A) and a
  // column of op(B) keep their scales (Scheme II: each operand keeps its own
  // bit budget), so the integer sums and the results are those of the
  // row-major call -- except for the Scheme I complex product, whose 4M
  // embedding then carries the negated imaginary parts on the other operand
  // (its results are the 4M product of the transposed problem).
  int64_t m = M, n = N;
  const void *a = A, *b = B;
  int64_t la = lda, lb = ldb;
  bool ta = trans_a != 0, tb = trans_b != 0;
  if (col) {
    m = N;
    n = M;
    a = B;
    b = A;
    la = ldb;
    lb = lda;
    ta = trans_b != 0;
    tb = trans_a != 0;
  }
  switch (dtype) {
    case OZK_F64:
      return dgemm_run(ctx, scheme, p_or_s, ta, tb, m, n, K, *(const double*)alpha, (const double*)a, la,
                       (const double*)b, lb, *(const double*)beta, (double*)C, ldc, ws, ws_bytes, stream, 19, col);
    case OZK_F32:
      return sgemm_run(ctx, scheme, p_or_s, ta, tb, m, n, K, *(const float*)alpha, (const float*)a, la,
                       (const float*)b, lb, *(const float*)beta, (float*)C, ldc, ws, ws_bytes, stream, 19, col);
    default:
      break;
  }
  if (scheme == OZK_SCHEME1) {
    // 4M reads the row operand's stored rows as its real embedding and builds
    // the column operand's: transposed operands have no such kernels
    if (ta || tb) return fail(ctx, OZK_ERR_UNSUPPORTED, ta ? (col ? 5 : 4) : (col ? 4 : 5));
    if (dtype == OZK_C128)
      return zgemm4m_run<double>(ctx, p_or_s, m, n, K, (const double*)alpha, (const double*)a, la, (const double*)b,
                                 lb, (const double*)beta, (double*)C, ldc, ws, ws_bytes, stream, 19);
    return zgemm4m_run<float>(ctx, p_or_s, m, n, K, (const float*)alpha, (const float*)a, la, (const float*)b, lb,
                              (const float*)beta, (float*)C, ldc, ws, ws_bytes, stream, 19);
  }
  (void)cplx;
  if (dtype == OZK_C128)
    return zgemm3m_run<double>(ctx, p_or_s, ta, tb, m, n, K, (const double*)alpha, (const double*)a, la,
                               (const double*)b, lb, (const double*)beta, (double*)C, ldc, ws, ws_bytes, stream, 19,
                               col);
  return zgemm3m_run<float>(ctx, p_or_s, ta, tb, m, n, K, (const float*)alpha, (const float*)a, la, (const float*)b,
                            lb, (const float*)beta, (float*)C, ldc, ws, ws_bytes, stream, 19, col);
}

// The unfused Scheme II / 3M baseline: the fused path's pre-pass and CRT
// around one GEMM per modular product with INT32 planes through HBM.
static size_t s2_unfused_ws(int s, bool cplx, int64_t M, int64_t N, int64_t K, S2Plan& pl) {
  pl = s2_plan(s, cplx, M, N, K);
  return align256(pl.total) + (size_t)ozk::s2_unfused_planes_bytes(s, cplx, M, N);
}

ozk_status ozk_s2_unfused_workspace_size(ozk_ctx* ctx, int s, int complex_planes, int64_t M, int64_t N, int64_t K,
                                         size_t* bytes) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (s < 1 || s > OZK_MAX_S) return fail(ctx, OZK_ERR_UNSUPPORTED, 2);
  if (complex_planes != 0 && complex_planes != 1) return fail(ctx, OZK_ERR_INVALID_ARG, 3);
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, 4);
  if (!bytes) return fail(ctx, OZK_ERR_INVALID_ARG, 7);
  S2Plan pl;
  *bytes = s2_unfused_ws(s, complex_planes != 0, M, N, K, pl);
  return OZK_OK;
}

ozk_status ozk_s2_gemm_unfused(ozk_ctx* ctx, int s, int complex_planes, int64_t M, int64_t N, int64_t K,
                               const double* alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                               const double* beta, double* C, int64_t ldc, void* ws, size_t ws_bytes,
                               hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (s < 1 || s > OZK_MAX_S) return fail(ctx, OZK_ERR_UNSUPPORTED, 2);
  if (complex_planes != 0 && complex_planes != 1) return fail(ctx, OZK_ERR_INVALID_ARG, 3);
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, M < 0 ? 4 : (N < 0 ? 5 : 6));
  if (K > 131071) return fail(ctx, OZK_ERR_UNSUPPORTED, 6);  // |sum| <= K 2^14 < 2^31
  if (!alpha) return fail(ctx, OZK_ERR_INVALID_ARG, 7);
  if (!A && M > 0 && K > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 8);
  if (lda < (K > 0 ? K : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 9);
  if (!B && K > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 10);
  if (ldb < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 11);
  if (!beta) return fail(ctx, OZK_ERR_INVALID_ARG, 12);
  if (!C && M > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 13);
  if (ldc < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 14);
  const bool cplx = complex_planes != 0;
  S2Plan pl;
  const size_t need = s2_unfused_ws(s, cplx, M, N, K, pl);
  if (!ws || ws_bytes < need) return fail(ctx, OZK_ERR_WORKSPACE, 15);
  if (M == 0 || N == 0) return OZK_OK;
  char* w = (char*)ws;
  int32_t* sig = (int32_t*)(w + pl.off_sig);
  int32_t* tau = (int32_t*)(w + pl.off_tau);
  int8_t* Ap = (int8_t*)(w + pl.off_a);
  int8_t* Bp = (int8_t*)(w + pl.off_b);
  int8_t* res = (int8_t*)(w + pl.off_res);
  int32_t* planes = (int32_t*)(w + align256(pl.total));
  hipError_t err = ozk::s2_split_rows(s, cplx, A, lda, M, K, sig, Ap, stream);
  if (err == hipSuccess) err = ozk::s2_split_cols(s, cplx, B, ldb, K, N, tau, Bp, stream);
  if (err == hipSuccess) err = ozk::flag_nonfinite(sig, M, tau, N, ctx->dflags, stream);
  if (err == hipSuccess) err = ozk::s2_gemm_mod_unfused(s, cplx, M, N, K, Ap, Bp, planes, res, stream);
  const double al[2] = {alpha[0], cplx ? alpha[1] : 0.0}, be[2] = {beta[0], cplx ? beta[1] : 0.0};
  if (err == hipSuccess) err = ozk::s2_crt(s, cplx, M, N, res, sig, tau, al, be, C, ldc, stream);
  return hip_status(ctx, err);
}

ozk_status ozk_s2_split_rows(ozk_ctx* ctx, int s, int complex_planes, int64_t rows, int64_t K,
                             const double* X, int64_t ldx, int32_t* sigma, int8_t* packed,
                             hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (s < 1 || s > OZK_MAX_S) return fail(ctx, OZK_ERR_UNSUPPORTED, 2);
  if (complex_planes != 0 && complex_planes != 1) return fail(ctx, OZK_ERR_INVALID_ARG, 3);
  if (bad_rows(rows)) return fail(ctx, OZK_ERR_INVALID_ARG, 4);
  if (K < 0 || K > ((int64_t)1 << 40)) return fail(ctx, OZK_ERR_INVALID_ARG, 5);
  if (s2_long_k(K)) return fail(ctx, OZK_ERR_UNSUPPORTED, 5);
  if (!X && rows > 0 && K > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 6);
  if (ldx < (K > 0 ? K : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 7);
  if (!sigma && rows > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 8);
  if (!packed && rows > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 9);
  return hip_status(ctx, ozk::s2_split_rows(s, complex_planes != 0, X, ldx, rows, K, sigma, packed, stream));
}

ozk_status ozk_s2_split_cols(ozk_ctx* ctx, int s, int complex_planes, int64_t K, int64_t cols,
                             const double* X, int64_t ldx, int32_t* tau, int8_t* packed,
                             hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (s < 1 || s > OZK_MAX_S) return fail(ctx, OZK_ERR_UNSUPPORTED, 2);
  if (complex_planes != 0 && complex_planes != 1) return fail(ctx, OZK_ERR_INVALID_ARG, 3);
  if (K < 0 || K > ((int64_t)1 << 40)) return fail(ctx, OZK_ERR_INVALID_ARG, 4);
  if (s2_long_k(K)) return fail(ctx, OZK_ERR_UNSUPPORTED, 4);
  if (bad_rows(cols)) return fail(ctx, OZK_ERR_INVALID_ARG, 5);
  if (!X && cols > 0 && K > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 6);
  if (ldx < (cols > 0 ? cols : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 7);
  if (!tau && cols > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 8);
  if (!packed && cols > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 9);
  return hip_status(ctx, ozk::s2_split_cols(s, complex_planes != 0, X, ldx, K, cols, tau, packed, stream));
}

ozk_status ozk_s2_gemm_mod(ozk_ctx* ctx, int s, int complex_planes, int64_t M, int64_t N, int64_t K,
                           const int8_t* packedA, const int8_t* packedB, int8_t* Cres, hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (s < 1 || s > OZK_MAX_S) return fail(ctx, OZK_ERR_UNSUPPORTED, 2);
  if (complex_planes != 0 && complex_planes != 1) return fail(ctx, OZK_ERR_INVALID_ARG, 3);
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, 4);
  if (M > 0 && N > 0 && (!packedA || !packedB || !Cres)) return fail(ctx, OZK_ERR_INVALID_ARG, 7);
  const ozk_gemm_config cfg =
      config_for(ctx, complex_planes ? OZK_OP_ZGEMM : OZK_OP_DGEMM, OZK_SCHEME2, s, M, N, K);
  return hip_status(ctx, ozk::s2_gemm_mod(s, complex_planes != 0, M, N, K, packedA, packedB, Cres, stream,
                                          cfg.variant, cfg.raster, cfg.group));
}

ozk_status ozk_s2_crt(ozk_ctx* ctx, int s, int complex_planes, int64_t M, int64_t N, const int8_t* Cres,
                      const int32_t* sigma, const int32_t* tau, const double* alpha, const double* beta,
                      double* C, int64_t ldc, hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (s < 1 || s > OZK_MAX_S) return fail(ctx, OZK_ERR_UNSUPPORTED, 2);
  if (complex_planes != 0 && complex_planes != 1) return fail(ctx, OZK_ERR_INVALID_ARG, 3);
  if (bad_rows(M)) return fail(ctx, OZK_ERR_INVALID_ARG, 4);
  if (bad_rows(N)) return fail(ctx, OZK_ERR_INVALID_ARG, 5);
  if (M > 0 && N > 0 && (!Cres || !sigma || !tau || !C)) return fail(ctx, OZK_ERR_INVALID_ARG, 6);
  if (!alpha) return fail(ctx, OZK_ERR_INVALID_ARG, 9);
  if (!beta) return fail(ctx, OZK_ERR_INVALID_ARG, 10);
  if (ldc < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 12);
  return hip_status(ctx, ozk::s2_crt(s, complex_planes != 0, M, N, Cres, sigma, tau, alpha, beta, C, ldc, stream));
}

ozk_status ozk_selector_load(ozk_ctx* ctx, const float* params, size_t n, const float* thresholds, int margin) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (!params || n != OZK_SELECTOR_PARAMS) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  if (!thresholds) return fail(ctx, OZK_ERR_INVALID_ARG, 4);
  for (int i = 0; i < OZK_SELECTOR_HEADS; ++i)
    if (!(thresholds[i] > 0.f && thresholds[i] < 1.f)) return fail(ctx, OZK_ERR_INVALID_ARG, 4);
  if (margin < 0 || margin > 8) return fail(ctx, OZK_ERR_INVALID_ARG, 5);
  if (!ctx->sel_w && hipMalloc(&ctx->sel_w, sizeof(float) * OZK_SELECTOR_PARAMS) != hipSuccess) {
    ctx->sel_w = nullptr;
    return fail(ctx, OZK_ERR_HIP, 0);
  }
  if (hipMemcpy(ctx->sel_w, params, sizeof(float) * OZK_SELECTOR_PARAMS, hipMemcpyHostToDevice) != hipSuccess)
    return fail(ctx, OZK_ERR_HIP, 0);
  for (int i = 0; i < OZK_SELECTOR_HEADS; ++i) ctx->sel_thr[i] = thresholds[i];
  ctx->sel_margin = margin;
  return OZK_OK;
}

static bool bad_tol(double tol) { return !(tol > 0.0 && tol < 1.0); }

ozk_status ozk_select(ozk_ctx* ctx, double tol, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                      const double* B, int64_t ldb, int32_t* e, int32_t* f, int32_t* counters, int32_t* info,
                      float* features, hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (bad_tol(tol)) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, 3);
  if (!A && M > 0 && K > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 6);
  if (lda < (K > 0 ? K : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 7);
  if (!B && K > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 8);
  if (ldb < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 9);
  if ((!e && M > 0) || (!f && N > 0)) return fail(ctx, OZK_ERR_INVALID_ARG, 10);
  if (!counters) return fail(ctx, OZK_ERR_INVALID_ARG, 12);
  if (!info) return fail(ctx, OZK_ERR_INVALID_ARG, 13);
  hipError_t err = ozk::sel_features(A, lda, M, B, ldb, N, K, e, f, counters, stream);
  if (err == hipSuccess)
    err = ozk::sel_infer(counters, ctx->sel_w, ctx->sel_thr, ctx->sel_margin, tol, K, info, features, stream);
  return hip_status(ctx, err);
}

ozk_status ozk_dgemm_auto(ozk_ctx* ctx, double tol, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                          int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc, void* ws,
                          size_t ws_bytes, int32_t* info, hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (bad_tol(tol)) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, M < 0 ? 3 : (N < 0 ? 4 : 5));
  if (!A && M > 0 && K > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 7);
  if (lda < (K > 0 ? K : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 8);
  if (!B && K > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 9);
  if (ldb < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 10);
  if (!C && M > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 12);
  if (ldc < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 13);
  if (s2_long_k(K)) return fail(ctx, OZK_ERR_UNSUPPORTED, 5);  // Scheme II may be chosen
  const AutoPlan ap = auto_plan(ctx, M, N, K);
  if (!ws || ws_bytes < ap.total) return fail(ctx, OZK_ERR_WORKSPACE, 14);
  if (M == 0 || N == 0) return OZK_OK;
  char* w = (char*)ws;
  int32_t* cnt = (int32_t*)(w + ap.off_cnt);
  int32_t* inf = info ? info : (int32_t*)(w + ap.off_info);
  // statistics (also the Scheme I exponents) and the decision
  const S1Plan& p1 = ap.s1;
  int32_t* e = (int32_t*)(w + p1.off_e);
  int32_t* f = (int32_t*)(w + p1.off_f);
  hipError_t err = ozk::sel_features(A, lda, M, B, ldb, N, K, e, f, cnt, stream);
  if (err == hipSuccess)
    err = ozk::sel_infer(cnt, ctx->sel_w, ctx->sel_thr, ctx->sel_margin, tol, K, inf, nullptr, stream);
  if (err == hipSuccess) err = ozk::flag_nonfinite(e, M, f, N, ctx->dflags, stream);
  if (err == hipSuccess) err = ozk::flag_decision(inf, ctx->dflags, stream);
  // Scheme I at the chosen p (every kernel returns when Scheme II was chosen)
  int8_t* Ap = (int8_t*)(w + p1.off_a);
  int8_t* Bp = (int8_t*)(w + p1.off_b);
  if (err == hipSuccess) err = ozk::s1_slice_auto(inf, A, lda, M, B, ldb, N, K, e, f, Ap, Bp, stream);
  if (err == hipSuccess) {
    ozk::S1GemmArgs g;
    g.M = M;
    g.N = N;
    g.Ap = Ap;
    g.Bp = Bp;
    g.nchunk = p1.nchunk;
    g.steps_per_split = p1.nsplit > 1 ? p1.steps_per_split : (p1.nchunk > 0 ? p1.nchunk : 1);
    g.nsplit = p1.nsplit;
    g.e = e;
    g.f = f;
    g.alpha = alpha;
    g.beta = beta;
    g.C = C;
    g.ldc = ldc;
    g.zpart = p1.nsplit > 1 ? (int64_t*)(w + p1.off_z) : nullptr;
    g.diag = nullptr;
    int cfg[OZK_MAX_P][3];  // the tuned (or default) tiling of each slice count's size class
    for (int p = 1; p <= OZK_MAX_P; ++p) {
      const ozk_gemm_config c = config_for(ctx, OZK_OP_DGEMM, OZK_SCHEME1, p, M, N, K);
      cfg[p - 1][0] = c.variant;
      cfg[p - 1][1] = c.raster;
      cfg[p - 1][2] = c.group;
    }
    err = ozk::s1_gemm_auto(inf, g, cfg, stream);
  }
  // Scheme II at the chosen s (every kernel returns when Scheme I was chosen)
  const S2Plan& p2 = ap.s2;
  int32_t* sig = (int32_t*)(w + p2.off_sig);
  int32_t* tau = (int32_t*)(w + p2.off_tau);
  int8_t* Ar = (int8_t*)(w + p2.off_a);
  int8_t* Br = (int8_t*)(w + p2.off_b);
  int8_t* res = (int8_t*)(w + p2.off_res);
  const double al[2] = {alpha, 0.0}, be[2] = {beta, 0.0};
  if (err == hipSuccess) err = ozk::s2_split_rows_auto(inf, false, A, lda, M, K, sig, Ar, stream);
  if (err == hipSuccess) err = ozk::s2_split_cols_auto(inf, false, B, ldb, K, N, tau, Br, stream);
  if (err == hipSuccess) err = ozk::s2_gemm_mod_auto(inf, false, M, N, K, Ar, Br, res, stream);
  if (err == hipSuccess) err = ozk::s2_crt_auto(inf, false, M, N, res, sig, tau, al, be, C, ldc, stream);
  return hip_status(ctx, err);
}

ozk_status ozk_zgemm_auto(ozk_ctx* ctx, double tol, int64_t M, int64_t N, int64_t K, const double* alpha,
                          const double* A, int64_t lda, const double* B, int64_t ldb, const double* beta, double* C,
                          int64_t ldc, void* ws, size_t ws_bytes, int32_t* info, hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (bad_tol(tol)) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, M < 0 ? 3 : (N < 0 ? 4 : 5));
  if (!alpha) return fail(ctx, OZK_ERR_INVALID_ARG, 6);
  if (!A && M > 0 && K > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 7);
  if (lda < (K > 0 ? K : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 8);
  if (!B && K > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 9);
  if (ldb < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 10);
  if (!beta) return fail(ctx, OZK_ERR_INVALID_ARG, 11);
  if (!C && M > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 12);
  if (ldc < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 13);
  if (s2_long_k(K)) return fail(ctx, OZK_ERR_UNSUPPORTED, 5);
  const S2Plan pl = s2_plan(OZK_MAX_S, true, M, N, K);  // per-modulus planes do not depend on s
  const size_t off_cnt = align256(pl.total), off_info = off_cnt + 256;
  if (!ws || ws_bytes < off_cnt + 512) return fail(ctx, OZK_ERR_WORKSPACE, 14);
  if (M == 0 || N == 0) return OZK_OK;
  char* w = (char*)ws;
  int32_t* sig = (int32_t*)(w + pl.off_sig);
  int32_t* tau = (int32_t*)(w + pl.off_tau);
  int8_t* Ap = (int8_t*)(w + pl.off_a);
  int8_t* Bp = (int8_t*)(w + pl.off_b);
  int8_t* res = (int8_t*)(w + pl.off_res);
  int32_t* cnt = (int32_t*)(w + off_cnt);
  int32_t* inf = info ? info : (int32_t*)(w + off_info);
  // statistics (tau serves as the column-exponent scratch) and the decision
  hipError_t err = ozk::zsel_features(A, lda, M, B, ldb, N, K, tau, cnt, stream);
  if (err == hipSuccess) err = ozk::zsel_decide(cnt, tol, K, inf, stream);
  if (err == hipSuccess) err = ozk::flag_decision(inf, ctx->dflags, stream);
  if (err == hipSuccess) err = ozk::s2_split_rows_auto(inf, true, A, lda, M, K, sig, Ap, stream);
  if (err == hipSuccess) err = ozk::s2_split_cols_auto(inf, true, B, ldb, K, N, tau, Bp, stream);
  if (err == hipSuccess) err = ozk::flag_nonfinite(sig, M, tau, N, ctx->dflags, stream);
  if (err == hipSuccess) err = ozk::s2_gemm_mod_auto(inf, true, M, N, K, Ap, Bp, res, stream);
  if (err == hipSuccess) err = ozk::s2_crt_auto(inf, true, M, N, res, sig, tau, alpha, beta, C, ldc, stream);
  return hip_status(ctx, err);
}

ozk_status ozk_mlp_forward(ozk_ctx* ctx, const float* params, const float* X, int n, float* logits,
                           hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (!params) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  if (n < 0) return fail(ctx, OZK_ERR_INVALID_ARG, 4);
  if (n > 0 && (!X || !logits)) return fail(ctx, OZK_ERR_INVALID_ARG, 3);
  return hip_status(ctx, ozk::mlp_forward(params, X, n, logits, stream));
}

ozk_status ozk_mlp_grad(ozk_ctx* ctx, const float* params, const float* X, const float* Y, int n, float* grad,
                        float* loss, hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (!params) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  if (n < 0) return fail(ctx, OZK_ERR_INVALID_ARG, 5);
  if (n > 0 && (!X || !Y)) return fail(ctx, OZK_ERR_INVALID_ARG, 3);
  if (!grad || !loss) return fail(ctx, OZK_ERR_INVALID_ARG, 6);
  return hip_status(ctx, ozk::mlp_grad(params, X, Y, n, grad, loss, stream));
}

ozk_status ozk_mlp_adam(ozk_ctx* ctx, float* params, const float* grad, float* m, float* v, int step, float lr,
                        hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (!params || !grad || !m || !v) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  if (step < 1) return fail(ctx, OZK_ERR_INVALID_ARG, 6);
  if (!(lr > 0.f)) return fail(ctx, OZK_ERR_INVALID_ARG, 7);
  return hip_status(ctx, ozk::mlp_adam(params, grad, m, v, step, lr, stream));
}

ozk_status ozk_ref_dd(ozk_ctx* ctx, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, const double* B,
                      int64_t ldb, int64_t n, const int64_t* rows, const int64_t* cols, double* hi, double* lo,
                      double* absab, hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  if (lda < (K > 0 ? K : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 6);
  if (ldb < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 8);
  if (n < 0) return fail(ctx, OZK_ERR_INVALID_ARG, 9);
  if (n > 0 && (!A || !B || !rows || !cols || !hi || !lo || !absab)) return fail(ctx, OZK_ERR_INVALID_ARG, 10);
  return hip_status(ctx, ozk::ref_dd(M, N, K, A, lda, B, ldb, n, rows, cols, hi, lo, absab, stream));
}

struct ozk_batch_plan {
  int device = 0;
  ozk_op op = OZK_OP_DGEMM;
  ozk_scheme scheme = OZK_SCHEME2;
  int s = 0;
  int count = 0;
  int ncu = 256;
  void* dev = nullptr;  // device tables
  ozk::BatchDev bd{};
  ozk::BatchTotals tot{};
  size_t ws_bytes = 0;
  int grid_small = 1, grid_large = 1;
  // host state for re-planning the tile of each problem
  std::vector<ozk::BatchProb> prob;
  std::vector<uint8_t> large;  // 1: the problem's items take the 128 x 128 tile
  size_t hint_cap = 0;         // entries of each item hint array on the device
  struct ItemTables {          // device regions of one tile's item chunks (ozk::BatchItems)
    int64_t* start = nullptr;
    int32_t* hint = nullptr;
    int32_t* prob = nullptr;
    int64_t* tile0 = nullptr;
    int64_t* queue = nullptr;
  } tab[2];                    // [0] small tile, [1] large tile
};

namespace {

// The batched op code whose table entries hold the batch tile of a size class.
int batched_op(ozk_op op) { return op == OZK_OP_ZGEMM ? OZK_OP_ZGEMM_BATCHED : OZK_OP_DGEMM_BATCHED; }

// Coarse index of a prefix array: hint[b] = the problem holding unit min(64 b, total - 1).
std::vector<int32_t> unit_hints(const std::vector<int64_t>& start, int count) {
  const int64_t tot = start[count];
  std::vector<int32_t> h((size_t)((tot >> ozk::OZK_BATCH_HINT_SHIFT) + 2), 0);
  int i = 0;
  for (size_t b = 0; b < h.size(); ++b) {
    const int64_t x = std::min<int64_t>((int64_t)b << ozk::OZK_BATCH_HINT_SHIFT, tot > 0 ? tot - 1 : 0);
    while (i + 1 < count && start[i + 1] <= x) ++i;  // the largest i with start[i] <= x
    h[b] = i;
  }
  return h;
}

// The item chunks and queues of both tiles (ozk::BatchItems) from pl->large,
// uploaded into the plan's device regions, and the grids of the two
// persistent launches.  A problem whose items carry more than a quarter of
// one queue's share of the tile's INT8 work is cut into up to
// OZK_BATCH_QUEUES chunks of consecutive tiles; the chunks, the most work
// first, each go to the queue with the least work so far (longest processing
// time first); a queue then runs its chunks by decreasing K, so that its
// longest items start first.
hipError_t upload_items(ozk_batch_plan* pl) {
  constexpr int Q = ozk::OZK_BATCH_QUEUES;
  const int count = pl->count;
  const bool cplx = pl->op == OZK_OP_ZGEMM;
  struct Chunk {
    int prob;
    int64_t tile0, n, kp;
  };
  for (int kind = 0; kind < 2; ++kind) {
    auto tiles = [&](int i) {
      const ozk::BatchProb& q = pl->prob[i];
      return (pl->large[i] == kind && q.tiles > 0) ? ozk::s2_tile_count(cplx, kind == 1, q.M, q.N) : (int64_t)0;
    };
    auto kp = [&](int i) { return pl->prob[i].Kp > 0 ? pl->prob[i].Kp : (int64_t)1; };  // K = 0 items still store
    double total = 0.0;
    for (int i = 0; i < count; ++i) total += (double)tiles(i) * (double)kp(i);
    std::vector<Chunk> chunks;
    for (int i = 0; i < count; ++i) {
      const int64_t t = tiles(i);
      if (t == 0) continue;
      const double w = (double)t * (double)kp(i);
      int64_t c = (int64_t)std::ceil(w * 4.0 * Q / total);
      c = std::max<int64_t>(1, std::min<int64_t>(c, std::min<int64_t>(t, Q)));
      for (int64_t j = 0; j < c; ++j) chunks.push_back({i, t * j / c, t * (j + 1) / c - t * j / c, kp(i)});
    }
    std::vector<int> by_work(chunks.size());
    std::iota(by_work.begin(), by_work.end(), 0);
    std::stable_sort(by_work.begin(), by_work.end(), [&](int a, int b) {
      return chunks[a].n * chunks[a].kp > chunks[b].n * chunks[b].kp;
    });
    std::vector<std::vector<int>> queue(Q);
    std::vector<double> load(Q, 0.0);
    for (int c : by_work) {
      const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      queue[x].push_back(c);
      load[x] += (double)chunks[c].n * (double)chunks[c].kp;
    }
    std::vector<int64_t> start(1, 0), tile0, qoff(Q + 1, 0);
    std::vector<int32_t> prob;
    int64_t qmax = 0;
    for (int x = 0; x < Q; ++x) {
      std::stable_sort(queue[x].begin(), queue[x].end(), [&](int a, int b) { return chunks[a].kp > chunks[b].kp; });
      qoff[x] = start.back();
      for (int c : queue[x]) {
        prob.push_back(chunks[c].prob);
        tile0.push_back(chunks[c].tile0);
        start.push_back(start.back() + chunks[c].n);
      }
      qmax = std::max<int64_t>(qmax, start.back() - qoff[x]);
    }
    qoff[Q] = start.back();
    const int nchunk = (int)prob.size();
    if (nchunk > Q * (count > 0 ? count : 1)) return hipErrorInvalidValue;
    const std::vector<int32_t> hint = unit_hints(start, nchunk);
    if (hint.size() > pl->hint_cap) return hipErrorInvalidValue;
    const ozk_batch_plan::ItemTables& d = pl->tab[kind];
    hipError_t e = hipMemcpy(d.start, start.data(), sizeof(int64_t) * start.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d.hint, hint.data(), sizeof(int32_t) * hint.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && nchunk > 0)
      e = hipMemcpy(d.prob, prob.data(), sizeof(int32_t) * nchunk, hipMemcpyHostToDevice);
    if (e == hipSuccess && nchunk > 0)
      e = hipMemcpy(d.tile0, tile0.data(), sizeof(int64_t) * nchunk, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d.queue, qoff.data(), sizeof(int64_t) * (Q + 1), hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    // resident workgroups, a multiple of Q, and no more than the longest queue needs
    const int64_t slots = (int64_t)pl->ncu * ozk::s2_batch_gemm_blocks_per_cu(cplx, kind == 1);
    const int64_t n = start.back();
    const int grid = (int)std::max<int64_t>(Q, std::min<int64_t>(slots / Q, qmax) * Q);
    const ozk::BatchItems items{{d.start, d.hint}, d.prob, d.tile0, d.queue};
    if (kind) {
      pl->tot.items_l = n;
      pl->grid_large = grid;
      pl->bd.items_l = items;
    } else {
      pl->tot.items = n;
      pl->grid_small = grid;
      pl->bd.items = items;
    }
  }
  return hipSuccess;
}

void free_plan(ozk_batch_plan* pl) {
  if (!pl) return;
  if (pl->dev) (void)hipFree(pl->dev);
  delete pl;
}

}  // namespace

ozk_status ozk_batch_plan_create(ozk_ctx* ctx, ozk_op op, ozk_scheme scheme, int p_or_s, int count,
                                 const ozk_gemm_desc* descs, ozk_batch_plan** plan, size_t* ws_bytes) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (!plan) return fail(ctx, OZK_ERR_INVALID_ARG, 7);
  *plan = nullptr;
  if (op != OZK_OP_DGEMM && op != OZK_OP_ZGEMM) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  if (scheme != OZK_SCHEME2) return fail(ctx, OZK_ERR_UNSUPPORTED, 3);
  if (p_or_s < 1 || p_or_s > OZK_MAX_S) return fail(ctx, OZK_ERR_UNSUPPORTED, 4);
  if (count < 0) return fail(ctx, OZK_ERR_INVALID_ARG, 5);
  if (count > 0 && !descs) return fail(ctx, OZK_ERR_INVALID_ARG, 6);
  const bool cplx = op == OZK_OP_ZGEMM;
  const int s = p_or_s;
  for (int i = 0; i < count; ++i) {
    const ozk_gemm_desc& d = descs[i];
    if (bad_dims(d.M, d.N, d.K) || d.lda < (d.K > 0 ? d.K : 1) || d.ldb < (d.N > 0 ? d.N : 1) ||
        d.ldc < (d.N > 0 ? d.N : 1) || (!d.A && d.M > 0 && d.K > 0) || (!d.B && d.K > 0 && d.N > 0) ||
        (!d.C && d.M > 0 && d.N > 0))
      return fail(ctx, OZK_ERR_INVALID_ARG, 6);
    if (s2_long_k(d.K)) return fail(ctx, OZK_ERR_UNSUPPORTED, 6);
  }
  ozk_batch_plan* pl = new (std::nothrow) ozk_batch_plan();
  if (!pl) return fail(ctx, OZK_ERR_HIP, 0);
  pl->device = ctx->device;
  pl->op = op;
  pl->scheme = scheme;
  pl->s = s;
  pl->count = count;
  pl->prob.resize(count);
  pl->large.assign(count, 0);
  size_t o = 0;
  int64_t max_items = 0;
  for (int i = 0; i < count; ++i) {
    const ozk_gemm_desc& d = descs[i];
    ozk::BatchProb& q = pl->prob[i];
    q.M = d.M;
    q.N = d.N;
    q.K = d.K;
    q.Kp = round_up(d.K, OZK_K_CHUNK);
    q.ra = round_up(d.M, ozk::OZK_BATCH_ROW_ALIGN);
    q.rb = round_up(d.N, ozk::OZK_BATCH_ROW_ALIGN);
    q.tiles = (d.M > 0 && d.N > 0) ? 1 : 0;  // a live problem
    q.A = d.A;
    q.lda = d.lda;
    q.B = d.B;
    q.ldb = d.ldb;
    q.C = d.C;
    q.ldc = d.ldc;
    q.a_re = d.alpha[0];
    q.a_im = cplx ? d.alpha[1] : 0.0;
    q.b_re = d.beta[0];
    q.b_im = cplx ? d.beta[1] : 0.0;
    q.off_sig = o; o = align256(o + 4 * (size_t)(d.M > 0 ? d.M : 1));
    q.off_tau = o; o = align256(o + 4 * (size_t)(d.N > 0 ? d.N : 1));
    q.off_a = o; o = align256(o + (size_t)q.ra * q.Kp * s * (cplx ? 3 : 1));
    q.off_b = o; o = align256(o + (size_t)q.rb * q.Kp * s * (cplx ? 3 : 1));
    q.ldr = round_up(d.N, 4);  // whole 4-byte residue words per row
    q.off_res = o; o = align256(o + (size_t)s * (cplx ? 2 : 1) * d.M * q.ldr);
    if (q.tiles) {
      max_items += ozk::s2_tile_count(cplx, false, q.M, q.N);  // the small tile gives the most items
      // the tile of this size class: the tuned table's choice (variant 1: the
      // large tile), else the large tile once both sides reach 256
      auto it = ctx->configs.find(cfg_key(batched_op(op), OZK_SCHEME2, s, d.M, d.N, d.K));
      pl->large[i] = it != ctx->configs.end() ? (it->second.cfg.variant == 1) : (d.M >= 256 && d.N >= 256);
    }
  }
  std::vector<int64_t> rows(count + 1, 0), cols(count + 1, 0), split(count + 1, 0), crt(count + 1, 0);
  for (int i = 0; i < count; ++i) {
    const ozk::BatchProb& q = pl->prob[i];
    const bool live = q.tiles > 0;
    rows[i + 1] = rows[i] + (live ? ozk::s2_split_rows_blocks(q.ra) : 0);
    cols[i + 1] = cols[i] + (live ? ozk::s2_batch_col_blocks(cplx, q.K, q.N) : 0);
    split[i + 1] = split[i] + (live ? ozk::s2_split_cols_blocks(q.rb, q.Kp) : 0);
    crt[i + 1] = crt[i] + (live ? (q.M * q.N + 255) / 256 : 0);
  }
  pl->ws_bytes = o > 0 ? o : 256;
  pl->tot = {rows[count], cols[count], split[count], 0, 0, crt[count]};
  const std::vector<int32_t> h_rows = unit_hints(rows, count), h_cols = unit_hints(cols, count),
                             h_split = unit_hints(split, count), h_crt = unit_hints(crt, count);
  pl->hint_cap = (size_t)((max_items >> ozk::OZK_BATCH_HINT_SHIFT) + 2);
  // device tables: problems, four prefix arrays with their hints, and for each
  // tile the item chunks (prefix array, hints, problem, first tile) and queues
  const size_t nprob = sizeof(ozk::BatchProb) * (count > 0 ? count : 1);
  const size_t npre = sizeof(int64_t) * (count + 1);
  const size_t nchk = (size_t)ozk::OZK_BATCH_QUEUES * (count > 0 ? count : 1);  // chunks per tile at most
  const size_t nhcap = sizeof(int32_t) * pl->hint_cap;
  const size_t nqueue = sizeof(int64_t) * (ozk::OZK_BATCH_QUEUES + 1);
  size_t nhint = 0;
  for (const auto* h : {&h_rows, &h_cols, &h_split, &h_crt}) nhint += align256(sizeof(int32_t) * h->size());
  const size_t per_tile = align256(sizeof(int64_t) * (nchk + 1)) + align256(nhcap) + align256(sizeof(int32_t) * nchk) +
                          align256(sizeof(int64_t) * nchk) + align256(nqueue);
  const size_t total = align256(nprob) + 4 * align256(npre) + nhint + 2 * per_tile;
  if (hipMalloc(&pl->dev, total) != hipSuccess) {
    pl->dev = nullptr;
    free_plan(pl);
    return fail(ctx, OZK_ERR_HIP, 0);
  }
  char* base = (char*)pl->dev;
  size_t off = 0;
  bool ok = true;
  auto put = [&](const void* src, size_t bytes, size_t room) -> void* {
    void* dst = base + off;
    if (bytes && hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) ok = false;
    off += align256(room > 0 ? room : 1);
    return dst;
  };
  void* pp = put(pl->prob.data(), sizeof(ozk::BatchProb) * count, nprob);
  void* r1 = put(rows.data(), npre, npre);
  void* r2 = put(cols.data(), npre, npre);
  void* r3 = put(split.data(), npre, npre);
  void* r5 = put(crt.data(), npre, npre);
  void* q1 = put(h_rows.data(), sizeof(int32_t) * h_rows.size(), sizeof(int32_t) * h_rows.size());
  void* q2 = put(h_cols.data(), sizeof(int32_t) * h_cols.size(), sizeof(int32_t) * h_cols.size());
  void* q3 = put(h_split.data(), sizeof(int32_t) * h_split.size(), sizeof(int32_t) * h_split.size());
  void* q5 = put(h_crt.data(), sizeof(int32_t) * h_crt.size(), sizeof(int32_t) * h_crt.size());
  for (ozk_batch_plan::ItemTables& t : pl->tab) {
    t.start = (int64_t*)put(nullptr, 0, sizeof(int64_t) * (nchk + 1));
    t.hint = (int32_t*)put(nullptr, 0, nhcap);
    t.prob = (int32_t*)put(nullptr, 0, sizeof(int32_t) * nchk);
    t.tile0 = (int64_t*)put(nullptr, 0, sizeof(int64_t) * nchk);
    t.queue = (int64_t*)put(nullptr, 0, nqueue);
  }
  pl->bd.prob = (const ozk::BatchProb*)pp;
  pl->bd.rows = {(const int64_t*)r1, (const int32_t*)q1};
  pl->bd.cols = {(const int64_t*)r2, (const int32_t*)q2};
  pl->bd.split = {(const int64_t*)r3, (const int32_t*)q3};
  pl->bd.crt = {(const int64_t*)r5, (const int32_t*)q5};
  pl->bd.count = count;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) pl->ncu = prop.multiProcessorCount;
  if (!ok || upload_items(pl) != hipSuccess) {
    free_plan(pl);
    return fail(ctx, OZK_ERR_HIP, 0);
  }
  *plan = pl;
  if (ws_bytes) *ws_bytes = pl->ws_bytes;
  return OZK_OK;
}

ozk_status ozk_gemm_batched(ozk_ctx* ctx, const ozk_batch_plan* plan, void* ws, size_t ws_bytes,
                            hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (!plan) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  if (!ws || ws_bytes < plan->ws_bytes) return fail(ctx, OZK_ERR_WORKSPACE, 3);
  if (plan->count == 0) return OZK_OK;
  hipError_t err = ozk::s2_batched(plan->s, plan->op == OZK_OP_ZGEMM, plan->bd, plan->tot, (int8_t*)ws,
                                   plan->grid_small, plan->grid_large, stream);
  if (err == hipSuccess) err = ozk::flag_batch(plan->bd, (const int8_t*)ws, ctx->dflags, stream);
  return hip_status(ctx, err);
}

ozk_status ozk_batch_plan_destroy(ozk_batch_plan* plan) {
  free_plan(plan);
  return OZK_OK;
}

ozk_status ozk_batch_plan_tiles(const ozk_batch_plan* plan, int count, int32_t* large) {
  if (!plan || count != plan->count || (count > 0 && !large)) return OZK_ERR_INVALID_ARG;
  for (int i = 0; i < count; ++i) large[i] = plan->large[i];
  return OZK_OK;
}

ozk_status ozk_tune_batch(ozk_ctx* ctx, ozk_batch_plan* plan, void* ws, size_t ws_bytes, int reps,
                          hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (!plan) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  if (!ws || ws_bytes < plan->ws_bytes) return fail(ctx, OZK_ERR_WORKSPACE, 3);
  if (reps < 1 || reps > 100) return fail(ctx, OZK_ERR_INVALID_ARG, 5);
  if (plan->count == 0) return OZK_OK;
  const bool cplx = plan->op == OZK_OP_ZGEMM;
  int8_t* w = (int8_t*)ws;
  hipError_t err = ozk::s2_batched_prepass(plan->s, cplx, plan->bd, plan->tot, w, stream);
  // size classes of the live problems, the most INT8 work first
  std::map<ozk_cfg_key, std::vector<int>> cls;
  std::map<ozk_cfg_key, double> work;
  for (int i = 0; i < plan->count; ++i) {
    const ozk::BatchProb& q = plan->prob[i];
    if (!q.tiles) continue;
    const ozk_cfg_key k = cfg_key(batched_op(plan->op), OZK_SCHEME2, plan->s, q.M, q.N, q.K);
    cls[k].push_back(i);
    work[k] += (double)q.M * q.N * (q.K > 0 ? q.K : 1);
  }
  std::vector<ozk_cfg_key> keys;
  for (const auto& kv : cls) keys.push_back(kv.first);
  std::stable_sort(keys.begin(), keys.end(), [&](const ozk_cfg_key& a, const ozk_cfg_key& b) { return work[a] > work[b]; });
  // the GEMM step of the batch with the tiles `t`
  auto time_tiles = [&](const std::vector<uint8_t>& t, float* ms) {
    plan->large = t;
    hipError_t e = upload_items(plan);
    if (e == hipSuccess)
      e = time_median(stream, reps, [&] {
        return ozk::s2_batched_gemm(plan->s, cplx, plan->bd, plan->tot, w, plan->grid_small, plan->grid_large,
                                    stream);
      }, ms);
    return e;
  };
  // start from the fastest of the plan's tiles, all small and all large (the
  // two tiles run as two launches one after the other, so a class's best
  // tile depends on what the others use)
  std::vector<uint8_t> cur = plan->large;
  float cur_ms = 0.f;
  if (err == hipSuccess) err = time_tiles(cur, &cur_ms);
  for (uint8_t kind = 0; kind < 2 && err == hipSuccess; ++kind) {
    std::vector<uint8_t> t(plan->count, kind);
    float ms = 0.f;
    err = time_tiles(t, &ms);
    if (err == hipSuccess && ms < cur_ms) {
      cur = t;
      cur_ms = ms;
    }
  }
  // then greedy over the classes: each takes the tile with the faster GEMM
  // step, the others keeping their current choice
  for (const ozk_cfg_key& k : keys) {
    if (err != hipSuccess) break;
    const uint8_t had = cur[cls[k].front()];
    std::vector<uint8_t> t = cur;
    for (int i : cls[k]) t[i] = (uint8_t)(1 - had);
    float ms = 0.f;
    err = time_tiles(t, &ms);
    if (err == hipSuccess && ms < cur_ms) {
      cur = t;
      cur_ms = ms;
    }
  }
  plan->large = cur;
  for (const ozk_cfg_key& k : keys) ctx->configs[k] = ozk_cfg_entry{ozk_gemm_config{cur[cls[k].front()], 0, 4, 1}, cur_ms};
  // the chosen tiles, and the batch computed with them
  if (err == hipSuccess) err = upload_items(plan);
  if (err == hipSuccess)
    err = ozk::s2_batched_gemm(plan->s, cplx, plan->bd, plan->tot, w, plan->grid_small, plan->grid_large, stream);
  if (err == hipSuccess) err = ozk::s2_batched_crt(plan->s, cplx, plan->bd, plan->tot, w, stream);
  if (err == hipSuccess) err = hipStreamSynchronize(stream);
  return hip_status(ctx, err);
}

// ------------------------------------------------------------- autotuner

static ozk_status check_target(ozk_ctx* ctx, int op, int scheme, int p_or_s) {
  if (op != OZK_OP_DGEMM && op != OZK_OP_ZGEMM && op != OZK_OP_DGEMM_BATCHED && op != OZK_OP_ZGEMM_BATCHED)
    return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  if (scheme != OZK_SCHEME1 && scheme != OZK_SCHEME2) return fail(ctx, OZK_ERR_INVALID_ARG, 3);
  if (scheme == OZK_SCHEME1 && op != OZK_OP_DGEMM) return fail(ctx, OZK_ERR_UNSUPPORTED, 3);
  const int hi = scheme == OZK_SCHEME1 ? OZK_MAX_P : OZK_MAX_S;
  if (p_or_s < 1 || p_or_s > hi) return fail(ctx, OZK_ERR_UNSUPPORTED, 4);
  return OZK_OK;
}

// Largest K split the tuner tries: the 128-bit partials of all runs stay
// within 256 MiB, at most 8 runs and at most one run per K step.
static int tune_max_split(int64_t M, int64_t N, int64_t K) {
  const int64_t nchunk = round_up(K, OZK_K_CHUNK) / OZK_K_CHUNK;
  int s = 1;
  while (s < 8 && 2 * s <= nchunk && 16 * (2 * s) * M * N <= ((int64_t)256 << 20)) s *= 2;
  return s;
}

ozk_status ozk_config_set(ozk_ctx* ctx, ozk_op op, ozk_scheme scheme, int p_or_s, int64_t M, int64_t N, int64_t K,
                          const ozk_gemm_config* cfg) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  ozk_status st = check_target(ctx, op, scheme, p_or_s);
  if (st != OZK_OK) return st;
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, 5);
  if (!cfg || !valid_config(scheme, *cfg)) return fail(ctx, OZK_ERR_INVALID_ARG, 8);
  if ((op == OZK_OP_DGEMM_BATCHED || op == OZK_OP_ZGEMM_BATCHED) && cfg->variant > 1)
    return fail(ctx, OZK_ERR_INVALID_ARG, 8);  // batch tiles: 0 small, 1 large
  ozk_gemm_config c = *cfg;
  if (scheme == OZK_SCHEME2) c.split = 1;
  ctx->configs[cfg_key(op, scheme, p_or_s, M, N, K)] = ozk_cfg_entry{c, 0.f};
  return OZK_OK;
}

ozk_status ozk_config_get(ozk_ctx* ctx, ozk_op op, ozk_scheme scheme, int p_or_s, int64_t M, int64_t N, int64_t K,
                          ozk_gemm_config* cfg, int* found, float* ms) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  ozk_status st = check_target(ctx, op, scheme, p_or_s);
  if (st != OZK_OK) return st;
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, 5);
  if (!cfg) return fail(ctx, OZK_ERR_INVALID_ARG, 8);
  auto it = ctx->configs.find(cfg_key(op, scheme, p_or_s, M, N, K));
  const bool have = it != ctx->configs.end();
  *cfg = have ? it->second.cfg : default_config();
  if (found) *found = have ? 1 : 0;
  if (ms) *ms = have ? it->second.ms : 0.f;
  return OZK_OK;
}

ozk_status ozk_config_clear(ozk_ctx* ctx) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  ctx->configs.clear();
  return OZK_OK;
}

static const char* const CFG_FIELDS[] = {"op", "scheme", "p_or_s", "m_class", "n_class", "k_class",
                                         "variant", "raster", "group", "split"};

ozk_status ozk_config_save(ozk_ctx* ctx, const char* path) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (!path) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  FILE* fh = fopen(path, "w");
  if (!fh) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  fprintf(fh, "{\"format\": \"ozk-gemm-configs-1\", \"entries\": [");
  bool first = true;
  for (const auto& kv : ctx->configs) {
    const ozk_cfg_key& k = kv.first;
    const ozk_gemm_config& c = kv.second.cfg;
    const int v[10] = {k.op, k.scheme, k.p_or_s, k.mb, k.nb, k.kb, c.variant, c.raster, c.group, c.split};
    fprintf(fh, "%s\n  {", first ? "" : ",");
    for (int i = 0; i < 10; ++i) fprintf(fh, "\"%s\": %d, ", CFG_FIELDS[i], v[i]);
    fprintf(fh, "\"ms\": %.6g}", (double)kv.second.ms);
    first = false;
  }
  fprintf(fh, "\n]}\n");
  const bool ok = fclose(fh) == 0;
  return ok ? OZK_OK : fail(ctx, OZK_ERR_INVALID_ARG, 2);
}

// Reads what ozk_config_save writes: every {...} inside the entries list
// with the ten integer fields (and "ms"); entries are added to the table.
ozk_status ozk_config_load(ozk_ctx* ctx, const char* path) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  if (!path) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  FILE* fh = fopen(path, "r");
  if (!fh) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof buf, fh)) > 0) text.append(buf, n);
  fclose(fh);
  const size_t list = text.find("\"entries\"");
  if (list == std::string::npos) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
  std::map<ozk_cfg_key, ozk_cfg_entry> add;
  size_t pos = text.find('[', list);
  while (pos != std::string::npos) {
    const size_t open = text.find('{', pos);
    if (open == std::string::npos) break;
    const size_t close = text.find('}', open);
    if (close == std::string::npos) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
    const std::string obj = text.substr(open, close - open);
    long v[10];
    for (int i = 0; i < 10; ++i) {
      const std::string key = std::string("\"") + CFG_FIELDS[i] + "\"";
      const size_t at = obj.find(key);
      if (at == std::string::npos) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
      const size_t colon = obj.find(':', at + key.size());
      if (colon == std::string::npos) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
      char* end = nullptr;
      v[i] = strtol(obj.c_str() + colon + 1, &end, 10);
      if (end == obj.c_str() + colon + 1) return fail(ctx, OZK_ERR_INVALID_ARG, 2);
    }
    double ms = 0.0;
    const size_t at = obj.find("\"ms\"");
    if (at != std::string::npos) ms = strtod(obj.c_str() + obj.find(':', at) + 1, nullptr);
    const ozk_gemm_config c{(int)v[6], (int)v[7], (int)v[8], (int)v[9]};
    ozk_ctx probe;
    const bool batched = v[0] == OZK_OP_DGEMM_BATCHED || v[0] == OZK_OP_ZGEMM_BATCHED;
    if (check_target(&probe, (int)v[0], (int)v[1], (int)v[2]) != OZK_OK || !valid_config((int)v[1], c) ||
        (batched && c.variant > 1) ||
        v[3] < 0 || v[3] > 62 || v[4] < 0 || v[4] > 62 || v[5] < 0 || v[5] > 62)
      return fail(ctx, OZK_ERR_INVALID_ARG, 2);
    add[ozk_cfg_key{(int)v[0], (int)v[1], (int)v[2], (int)v[3], (int)v[4], (int)v[5]}] = ozk_cfg_entry{c, (float)ms};
    pos = close + 1;
  }
  for (const auto& kv : add) ctx->configs[kv.first] = kv.second;
  return OZK_OK;
}

ozk_status ozk_tune_workspace_size(ozk_ctx* ctx, ozk_op op, ozk_scheme scheme, int p_or_s, int64_t M, int64_t N,
                                   int64_t K, size_t* bytes) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  ozk_status st = check_target(ctx, op, scheme, p_or_s);
  if (st != OZK_OK) return st;
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, 5);
  if (!bytes) return fail(ctx, OZK_ERR_INVALID_ARG, 8);
  if (scheme == OZK_SCHEME1)
    *bytes = s1_plan(ctx, p_or_s, M, N, K, tune_max_split(M, N, K)).total;
  else
    *bytes = s2_plan(p_or_s, op == OZK_OP_ZGEMM, M, N, K).total;
  return OZK_OK;
}

ozk_status ozk_tune(ozk_ctx* ctx, ozk_op op, ozk_scheme scheme, int p_or_s, int64_t M, int64_t N, int64_t K,
                    const double* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc, void* ws,
                    size_t ws_bytes, int reps, ozk_gemm_config* best, float* best_ms, hipStream_t stream) {
  if (!ctx) return OZK_ERR_INVALID_ARG;
  ctx->last_arg = 0;
  ozk_status st = check_target(ctx, op, scheme, p_or_s);
  if (st != OZK_OK) return st;
  if (bad_dims(M, N, K)) return fail(ctx, OZK_ERR_INVALID_ARG, 5);
  const int64_t ew = op == OZK_OP_ZGEMM ? 2 : 1;  // doubles per element
  if (!A && M > 0 && K > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 8);
  if (lda < (K > 0 ? K : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 9);
  if (!B && K > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 10);
  if (ldb < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 11);
  if (!C && M > 0 && N > 0) return fail(ctx, OZK_ERR_INVALID_ARG, 12);
  if (ldc < (N > 0 ? N : 1)) return fail(ctx, OZK_ERR_INVALID_ARG, 13);
  if (reps < 1 || reps > 1000) return fail(ctx, OZK_ERR_INVALID_ARG, 16);
  (void)ew;
  const ozk_cfg_key key = cfg_key(op, scheme, p_or_s, M, N, K);
  ozk_gemm_config top = default_config();
  float top_ms = 0.f;
  hipError_t err = hipSuccess;
  char* w = (char*)ws;
  if (scheme == OZK_SCHEME1) {
    const int p = p_or_s;
    const S1Plan base = s1_plan(ctx, p, M, N, K, 1);
    if (!ws || ws_bytes < base.total) return fail(ctx, OZK_ERR_WORKSPACE, 15);
    if (M > 0 && N > 0) {
      int32_t* e = (int32_t*)(w + base.off_e);
      int32_t* f = (int32_t*)(w + base.off_f);
      int8_t* Ap = (int8_t*)(w + base.off_a);
      int8_t* Bp = (int8_t*)(w + base.off_b);
      err = ozk::s1_split_rows(p, A, lda, M, K, e, Ap, stream);
      if (err == hipSuccess) err = ozk::s1_split_cols(p, B, ldb, K, N, f, Bp, stream);
      const int max_split = tune_max_split(M, N, K);
      float top_t = 0.f;
      bool have = false;
      for (int v = 0; v < OZK_S1_VARIANTS && err == hipSuccess; ++v)
        for (int raster = 0; raster < 2 && err == hipSuccess; ++raster)
          for (int group : {2, 4, 8, 16})
            for (int split = 1; split <= max_split && err == hipSuccess; split *= 2) {
              const S1Plan pl = s1_plan(ctx, p, M, N, K, split);
              if (pl.total > ws_bytes) continue;
              if (split > 1 && pl.nsplit == base.nsplit) continue;  // no change from split 1
              ozk::S1GemmArgs g;
              g.M = M;
              g.N = N;
              g.Ap = Ap;
              g.Bp = Bp;
              g.nchunk = pl.nchunk;
              g.steps_per_split = pl.nsplit > 1 ? pl.steps_per_split : (pl.nchunk > 0 ? pl.nchunk : 1);
              g.nsplit = pl.nsplit;
              g.e = e;
              g.f = f;
              g.alpha = 1.0;
              g.beta = 0.0;
              g.C = C;
              g.ldc = ldc;
              g.zpart = pl.nsplit > 1 ? (int64_t*)(w + pl.off_z) : nullptr;
              g.diag = nullptr;
              g.variant = v;
              g.raster = raster;
              g.group = group;
              float t = 0.f;
              err = time_median(stream, reps, [&]() { return ozk::s1_gemm(p, g, stream); }, &t);
              if (err == hipSuccess && (!have || t < top_t)) {
                have = true;
                top_t = t;
                top = ozk_gemm_config{v, raster, group, split};
              }
            }
      top_ms = top_t;
      if (err == hipSuccess) {  // leave C = A B from the chosen configuration
        ctx->configs[key] = ozk_cfg_entry{top, top_ms};
        const S1Plan pl = s1_plan(ctx, p, M, N, K, top.split);
        st = s1_gemm_common(ctx, p, M, N, K, Ap, e, Bp, f, 1.0, 0.0, C, ldc, w + pl.off_z, pl.total - pl.off_z,
                            nullptr, stream, top);
        if (st != OZK_OK) return st;
      }
    } else {
      ctx->configs[key] = ozk_cfg_entry{top, 0.f};
    }
  } else {
    const int s = p_or_s;
    const bool cplx = op == OZK_OP_ZGEMM;
    if (s2_long_k(K)) return fail(ctx, OZK_ERR_UNSUPPORTED, 7);
    const S2Plan pl = s2_plan(s, cplx, M, N, K);
    if (!ws || ws_bytes < pl.total) return fail(ctx, OZK_ERR_WORKSPACE, 15);
    if (M > 0 && N > 0) {
      int32_t* sig = (int32_t*)(w + pl.off_sig);
      int32_t* tau = (int32_t*)(w + pl.off_tau);
      int8_t* Ap = (int8_t*)(w + pl.off_a);
      int8_t* Bp = (int8_t*)(w + pl.off_b);
      int8_t* res = (int8_t*)(w + pl.off_res);
      err = ozk::s2_split_rows(s, cplx, A, lda, M, K, sig, Ap, stream);
      if (err == hipSuccess) err = ozk::s2_split_cols(s, cplx, B, ldb, K, N, tau, Bp, stream);
      float top_t = 0.f;
      bool have = false;
      for (int v = 0; v < OZK_S2_VARIANTS && err == hipSuccess; ++v)
        for (int raster = 0; raster < 2 && err == hipSuccess && v != OZK_S2_FUSED_CRT; ++raster)
          for (int group : {2, 4, 8, 16}) {
            float t = 0.f;
            err = time_median(
                stream, reps, [&]() { return ozk::s2_gemm_mod(s, cplx, M, N, K, Ap, Bp, res, stream, v, raster, group); },
                &t);
            if (err == hipSuccess && (!have || t < top_t)) {
              have = true;
              top_t = t;
              top = ozk_gemm_config{v, raster, group, 1};
            }
          }
      top_ms = top_t;
      if (err == hipSuccess) {
        ctx->configs[key] = ozk_cfg_entry{top, top_ms};
        err = ozk::s2_gemm_mod(s, cplx, M, N, K, Ap, Bp, res, stream, top.variant, top.raster, top.group);
        const double one[2] = {1.0, 0.0}, zero[2] = {0.0, 0.0};
        if (err == hipSuccess) err = ozk::s2_crt(s, cplx, M, N, res, sig, tau, one, zero, C, ldc, stream);
      }
    } else {
      ctx->configs[key] = ozk_cfg_entry{top, 0.f};
    }
  }
  if (err != hipSuccess) return hip_status(ctx, err);
  if (best) *best = top;
  if (best_ms) *best_ms = top_ms;
  return OZK_OK;
}

}  // extern "C"
