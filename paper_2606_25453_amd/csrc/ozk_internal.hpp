// Host-side declarations shared by the kernel files and the C ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "ozk.h"

namespace ozk {

static inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

struct S1GemmArgs {
  int64_t M, N;
  const int8_t* Ap;
  const int8_t* Bp;
  int64_t nchunk;           // K steps of 32 in the packed operands
  int64_t steps_per_split;  // K steps per K run (overflow-free)
  int64_t nsplit;           // number of K runs
  const int32_t* e;
  const int32_t* f;
  double alpha, beta;
  double* C;
  int64_t ldc;
  int64_t* zpart;  // nsplit x M x N x 2 int64 when nsplit > 1
  float* C32 = nullptr;  // binary32 output instead of C (alpha, beta then hold binary32 values)
  int32_t* diag;   // p x M x N int32 for the check entry point, else null
  int variant = 0;  // tile variant (0 .. OZK_S1_VARIANTS - 1)
  int raster = 0;   // 0: XCD-aware tile order, 1: plain
  int group = 4;    // tile rows per raster group
};

hipError_t s1_split_rows(int p, const double* X, int64_t ldx, int64_t rows, int64_t K, int32_t* e,
                         int8_t* packed, hipStream_t st);
hipError_t s1_split_cols(int p, const double* X, int64_t ldx, int64_t K, int64_t cols, int32_t* f,
                         int8_t* packed, hipStream_t st);
// binary32 operands (each entry widened exactly to binary64 on load)
hipError_t s1_split_rows(int p, const float* X, int64_t ldx, int64_t rows, int64_t K, int32_t* e,
                         int8_t* packed, hipStream_t st);
hipError_t s1_split_cols(int p, const float* X, int64_t ldx, int64_t K, int64_t cols, int32_t* f,
                         int8_t* packed, hipStream_t st);
hipError_t s1_gemm(int p, const S1GemmArgs& g, hipStream_t st);
// The 4M complex column operand: the slices and column exponents of the real
// 2K x 2N embedding of complex B (K x N, interleaved, ldx in complex
// elements); f has 2N entries and the packed operand 2N columns of 2K.
hipError_t s1_split_cols_4m(int p, const double* X, int64_t ldx, int64_t K, int64_t N, int32_t* f, int8_t* packed,
                            hipStream_t st);
hipError_t s1_split_cols_4m(int p, const float* X, int64_t ldx, int64_t K, int64_t N, int32_t* f, int8_t* packed,
                            hipStream_t st);
// Complex update C = alpha H + beta C from the (Re, Im) pairs of H (M x 2N,
// row stride ldh), with the fixed FMA sequence; alpha, beta host {re, im}.
hipError_t zaxpby(const double* H, int64_t ldh, int64_t M, int64_t N, const double* alpha, const double* beta,
                  double* C, int64_t ldc, hipStream_t st);
hipError_t zaxpby(const float* H, int64_t ldh, int64_t M, int64_t N, const float* alpha, const float* beta,
                  float* C, int64_t ldc, hipStream_t st);
// The unfused baseline (one GEMM per slice pair, INT32 planes through HBM,
// then the exact reconstruction); K <= 131071 keeps each plane exact.
int64_t s1_unfused_planes_bytes(int p, int64_t M, int64_t N);
hipError_t s1_gemm_unfused(int p, int64_t M, int64_t N, int64_t K, const int8_t* Ap, const int32_t* e,
                           const int8_t* Bp, const int32_t* f, double alpha, double beta, double* C, int64_t ldc,
                           int32_t* planes, hipStream_t st);
// slice count read from device memory (selector output)
hipError_t s1_slice_auto(const int32_t* p_dev, const double* A, int64_t lda, int64_t M, const double* B, int64_t ldb,
                         int64_t N, int64_t K, const int32_t* e, const int32_t* f, int8_t* Ap, int8_t* Bp,
                         hipStream_t st);
// cfg[p - 1] = {variant, raster, group} of the kernel for slice count p
hipError_t s1_gemm_auto(const int32_t* p_dev, const S1GemmArgs& g, const int (*cfg)[3], hipStream_t st);

// Packed rows of a batched problem are padded to 128 (both batch GEMM tiles,
// a multiple of the 16-row and 64-column pre-pass blocks), not to
// OZK_ROW_ALIGN: small problems then carry far fewer padding rows, and the
// tile of a problem can change without a new layout.
constexpr int OZK_BATCH_ROW_ALIGN = 128;

// One problem of a batch; workspace parts are byte offsets from the
// workspace base passed to each launch.
struct BatchProb {
  int64_t M, N, K, Kp, ra, rb, tiles;
  int64_t ldr;  // row stride of the problem's residue planes: N rounded up to 4
  const double* A;
  int64_t lda;
  const double* B;
  int64_t ldb;
  double* C;
  int64_t ldc;
  double a_re, a_im, b_re, b_im;
  int64_t off_sig, off_tau, off_a, off_b, off_res;
};

// Work units of one batched step: the prefix sums of the units of every
// problem (count + 1 entries, from 0) and a coarse index, hint[b] = the
// problem holding unit min(64 b, total - 1) (total / 64 + 2 entries), so that
// a unit's problem is a binary search over the few problems between two
// hints instead of over the whole table.
constexpr int OZK_BATCH_HINT_SHIFT = 6;

struct BatchUnits {
  const int64_t* start;
  const int32_t* hint;
};

// GEMM items (output tiles of a problem, all moduli each) of one batch tile,
// in the order of the persistent launch.  Items come in chunks, runs of
// consecutive output tiles of one problem, and the chunks in
// OZK_BATCH_QUEUES queues of about equal INT8 work: queue x holds the items
// [queue[x], queue[x + 1]) and is run by the workgroups w with
// w % OZK_BATCH_QUEUES == x.  Workgroups are dispatched to the eight XCDs in
// turn, so a queue is one XCD's and the tiles of a chunk share its L2.
constexpr int OZK_BATCH_QUEUES = 8;

struct BatchItems {
  BatchUnits chunks;     // item prefix sums over the chunks, queue by queue
  const int32_t* prob;   // chunk -> problem
  const int64_t* tile0;  // chunk -> its first output tile within the problem
  const int64_t* queue;  // OZK_BATCH_QUEUES + 1 item offsets
};

// Device view of a batch plan: the problem table and the work units of each
// step.
struct BatchDev {
  const BatchProb* prob;
  BatchUnits rows;     // row blocks of 16 rows (pre-pass of A)
  BatchUnits cols;     // column blocks of 32 (column scales of B)
  BatchUnits split;    // (64-column block, K chunk) pairs (residues of B)
  BatchItems items;    // GEMM items of the small-tile problems
  BatchItems items_l;  // the same for the large-tile problems
  BatchUnits crt;      // output blocks of 256 (CRT)
  int count;
};

struct BatchTotals {
  int64_t rows, cols, split, items, items_l, crt;
};

hipError_t s2_batched(int s, bool cplx, const BatchDev& bd, const BatchTotals& tot, int8_t* ws, int grid_small,
                      int grid_large, hipStream_t st);
// the steps of s2_batched on their own (the tuner times the GEMM step)
hipError_t s2_batched_prepass(int s, bool cplx, const BatchDev& bd, const BatchTotals& tot, int8_t* ws,
                              hipStream_t st);
hipError_t s2_batched_gemm(int s, bool cplx, const BatchDev& bd, const BatchTotals& tot, int8_t* ws, int grid_small,
                           int grid_large, hipStream_t st);
hipError_t s2_batched_crt(int s, bool cplx, const BatchDev& bd, const BatchTotals& tot, int8_t* ws, hipStream_t st);
int s2_batch_gemm_blocks_per_cu(bool cplx, bool large);
int64_t s2_tile_count(bool cplx, bool large, int64_t M, int64_t N);
int64_t s2_split_rows_blocks(int64_t rows_packed);             // workgroups of the row residue pass
int64_t s2_split_cols_blocks(int64_t cols_packed, int64_t Kp);  // workgroups of the column residue pass
int64_t s2_batch_col_blocks(bool cplx, int64_t K, int64_t cols);  // workgroups of the batched column-scale pass

void s2_targets(int s, int& ta, int& tb);

// Scheme II bit budgets T_A, T_B for every modulus count (index s, 1..20).
struct S2Budgets {
  int ta[OZK_MAX_S + 1];
  int tb[OZK_MAX_S + 1];
};
S2Budgets s2_budgets();

// The real Scheme II steps with the modulus count read from device memory
// (info[4] == 2 selects them and info[5] holds s; every kernel returns at
// once otherwise).  The packed operands and residues use the layouts of
// s = OZK_MAX_S (per-modulus planes do not depend on s).  The CRT constants
// of every s live in constant memory, written by s2_upload_crt_tables on the
// current device (once per context, before any auto call).
hipError_t s2_upload_crt_tables();
hipError_t s2_split_rows_auto(const int32_t* info, bool cplx, const double* X, int64_t ldx, int64_t rows, int64_t K,
                              int32_t* sigma, int8_t* packed, hipStream_t st);
hipError_t s2_split_cols_auto(const int32_t* info, bool cplx, const double* X, int64_t ldx, int64_t K, int64_t cols,
                              int32_t* tau, int8_t* packed, hipStream_t st);
hipError_t s2_gemm_mod_auto(const int32_t* info, bool cplx, int64_t M, int64_t N, int64_t K, const int8_t* Ap,
                            const int8_t* Bp, int8_t* out, hipStream_t st);
// alpha, beta: host {re, im} (the imaginary parts unused for real products)
hipError_t s2_crt_auto(const int32_t* info, bool cplx, int64_t M, int64_t N, const int8_t* res, const int32_t* sigma,
                       const int32_t* tau, const double* alpha, const double* beta, double* C, int64_t ldc,
                       hipStream_t st);

// Statistics of a complex product for the automatic ZGEMM: the largest
// exponent deficit of a nonzero real or imaginary part below its row's
// (column's) largest part exponent, for the rows of A and the columns of B
// (counters [32] and [33]; [0, 32) zeroed), and the decision info of the
// Scheme II a-priori bound (3M; the deficits relative to the complex entry
// exponent max(expo re, expo im) + 1 are one more).
hipError_t zsel_features(const double* A, int64_t lda, int64_t M, const double* B, int64_t ldb, int64_t N, int64_t K,
                         int32_t* f_scratch, int32_t* cnt, hipStream_t st);
hipError_t zsel_decide(const int32_t* cnt, double tol, int64_t K, int32_t* info, hipStream_t st);

hipError_t sel_features(const double* A, int64_t lda, int64_t M, const double* B, int64_t ldb, int64_t N, int64_t K,
                        int32_t* e, int32_t* f, int32_t* cnt, hipStream_t st);
hipError_t sel_infer(const int32_t* cnt, const float* w, const float* thresholds, int margin, double tol, int64_t K,
                     int32_t* info, float* feat, hipStream_t st);
hipError_t mlp_forward(const float* w, const float* X, int n, float* logits, hipStream_t st);
hipError_t mlp_grad(const float* w, const float* X, const float* Y, int n, float* grad, float* loss, hipStream_t st);
hipError_t mlp_adam(float* w, const float* g, float* m, float* v, int step, float lr, hipStream_t st);
hipError_t ref_dd(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, const double* B, int64_t ldb,
                  int64_t n, const int64_t* rows, const int64_t* cols, double* hi, double* lo, double* absab,
                  hipStream_t st);
hipError_t s2_split_rows(int s, bool cplx, const double* X, int64_t ldx, int64_t rows, int64_t K, int32_t* sigma,
                         int8_t* packed, hipStream_t st, int budget = -1);
hipError_t s2_split_cols(int s, bool cplx, const double* X, int64_t ldx, int64_t K, int64_t cols, int32_t* tau,
                         int8_t* packed, hipStream_t st, int budget = -1);
hipError_t s2_gemm_mod(int s, bool cplx, int64_t M, int64_t N, int64_t K, const int8_t* Ap, const int8_t* Bp,
                       int8_t* out, hipStream_t st, int variant = 0, int raster = 0, int group = 4);
hipError_t s2_crt(int s, bool cplx, int64_t M, int64_t N, const int8_t* res, const int32_t* sigma,
                  const int32_t* tau, const double* alpha, const double* beta, double* C, int64_t ldc,
                  hipStream_t st);
// budget: the bit budget of the scale (default: T_A for the row pass, T_B for
// the column pass; a transposed operand takes the other pass with its own).
// binary32 operands (widened exactly on load) and binary32 results
hipError_t s2_split_rows(int s, bool cplx, const float* X, int64_t ldx, int64_t rows, int64_t K, int32_t* sigma,
                         int8_t* packed, hipStream_t st, int budget = -1);
hipError_t s2_split_cols(int s, bool cplx, const float* X, int64_t ldx, int64_t K, int64_t cols, int32_t* tau,
                         int8_t* packed, hipStream_t st, int budget = -1);
hipError_t s2_crt(int s, bool cplx, int64_t M, int64_t N, const int8_t* res, const int32_t* sigma,
                  const int32_t* tau, const float* alpha, const float* beta, float* C, int64_t ldc,
                  hipStream_t st);
// The unfused Scheme II / 3M baseline: one INT8 GEMM per modular product
// writing INT32 planes (s x M x N, 3M: 3s), then the reduction to the
// residue planes of s2_gemm_mod (K <= 131071).
int64_t s2_unfused_planes_bytes(int s, bool cplx, int64_t M, int64_t N);
hipError_t s2_gemm_mod_unfused(int s, bool cplx, int64_t M, int64_t N, int64_t K, const int8_t* Ap, const int8_t* Bp,
                               int32_t* planes, int8_t* out, hipStream_t st);
// GEMM and CRT in one kernel (real products; no residue planes).
hipError_t s2_gemm_crt(int s, int64_t M, int64_t N, int64_t K, const int8_t* Ap, const int8_t* Bp,
                       const int32_t* sigma, const int32_t* tau, double alpha, double beta, double* C, int64_t ldc,
                       int raster, int group, hipStream_t st);

// Condition flags (flags.hip): OR bits into the context's device word.
hipError_t flag_nonfinite(const int32_t* a, int64_t na, const int32_t* b, int64_t nb, uint32_t* flags,
                          hipStream_t st);
hipError_t flag_batch(const BatchDev& bd, const int8_t* ws, uint32_t* flags, hipStream_t st);
hipError_t flag_decision(const int32_t* info, uint32_t* flags, hipStream_t st);
hipError_t flag_take(uint32_t* flags, uint32_t* out, hipStream_t st);

// Raise the dynamic LDS limit of kernel `fn` to `bytes` on the current
// device, once per device (`done` holds one bit per device ordinal < 64 and
// is safe to share between host threads; devices beyond 64 set it on every
// launch).
inline hipError_t lds_limit(const void* fn, int bytes, std::atomic<uint64_t>& done) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const uint64_t bit = dev >= 0 && dev < 64 ? (uint64_t)1 << dev : 0;
  if (bit && (done.load(std::memory_order_acquire) & bit)) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess && bit) done.fetch_or(bit, std::memory_order_acq_rel);
  return e;
}

}  // namespace ozk
