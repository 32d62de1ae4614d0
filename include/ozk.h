/*
 * ozk.h -- C ABI of an FP64 / complex128 GEMM library that emulates the
 * products on INT8 matrix cores (AMD MI355X, gfx950) with the Ozaki schemes.
 *
 * Paper: "EmuGEMM: Fused Tensor Core Kernels for Precision Emulation in Matrix
 * Multiplication".  Problem statement C = A B with A in R^{MxK},
 * B in R^{KxN} (Sec. II-B); this library computes C = alpha*A*B + beta*C.
 *
 * Conventions for every call
 * --------------------------
 * - Matrices are row-major (C order, as in PyTorch) with leading dimensions
 *   in elements: A(i,k) = A[i*lda + k], B(k,j) = B[k*ldb + j],
 *   C(i,j) = C[i*ldc + j].  Complex matrices are interleaved (re, im) pairs
 *   (std::complex<double> / torch.complex128) and leading dimensions count
 *   complex elements.
 * - Every pointer argument except the context is a DEVICE pointer owned by
 *   the caller.  The library never allocates or frees per call, never
 *   synchronises the stream and never reads device data on the host, so
 *   calls may be captured into a HIP graph.  All work is enqueued on
 *   `stream` (0 = the null stream).
 * - Arguments are validated synchronously; on failure nothing is enqueued
 *   and the status says why (ozk_last_arg() names the 1-based position of
 *   the offending argument).  No exception or abort crosses the ABI.
 * - beta == 0 means C is not read (BLAS convention).  M, N or K == 0 are
 *   valid: with K == 0 the product is exactly zero.  M and N (rows and
 *   columns of packed operands) are at most OZK_MAX_ROWS = 2^24, K at most
 *   2^40; larger sizes return OZK_ERR_INVALID_ARG.
 * - Scheme II (and every call that may run it) takes K <= OZK_S2_MAX_K =
 *   2^22: its row/column scales come from an exact integer bound on the 2-norm
 *   that adds up to 2^40 per entry in 64-bit integers, which stays exact for
 *   K < 2^23.  Longer K returns OZK_ERR_UNSUPPORTED.
 * - A row of A or a column of B that holds a NaN or an infinity yields NaN
 *   in the corresponding row/column of alpha*A*B (the paper does not define
 *   this case); finite rows and columns are unaffected.
 *
 * Packed operand layouts (workspace contents, documented so that each step
 * can be called and checked on its own)
 * ------------------------------------------------------------------------
 * OZK_ROW_ALIGN = 256: packed operands hold Rp = roundup(rows, 256) rows;
 * the rows past `rows` are zero.  K is padded with zeros to
 * Kp = roundup(K, 32) (OZK_K_CHUNK).
 *
 * Scheme I packed operand (Sec. III-A, Eq. 11, with t_K = 32): the
 *   interleaved matrix A^ (rows x p K, 32-wide column blocks cycling through
 *   the slices: block j = c p + t holds slice t of k = 32c .. 32c+31) stored
 *   block-column by block-column, each block a contiguous Rp x 32 slab:
 *   P[c][t][r][kk] = slice t of row r at k = 32c + kk,   int8,
 *   byte offset ((c p + t) Rp + r) 32 + kk,  c < Kp/32, t < p, r < Rp.
 *   The "rows" of B's packed operand are the COLUMNS of B (B is transposed
 *   so that both operands are contiguous along k).
 *   Slice format: with e the row (column) exponent -- the smallest e with
 *   |x| < 2^e over the row's nonzero entries -- and X = floor(x 2^(8p-2-e)
 *   + 1/2), the slices are the balanced base-256 digits of X: slice t in
 *   [-128, 127] (slice 0 in [-64, 64]) with x ~ 2^e sum_t slice_t 2^(-6-8t).
 *
 * Scheme II packed operand (Sec. II-C.2, Eq. 5): per modulus l one packed
 *   operand in the Scheme I layout with a single slice,
 *   R[l][c][r][kk] = smod(trunc(x 2^sigma_r), m_l) at k = 32c + kk, int8,
 *   smod(x, m) the representative in [-floor(m/2), ceil(m/2)-1]; moduli
 *   m_l = 256, 255, 253, 251, 247, 241, ... (greedy pairwise coprime).
 *   3M complex: per modulus a packed operand with three slices,
 *   R[l][c][q][r][kk], q = 0 the real part, 1 the imaginary part,
 *   2 smod(real + imaginary).
 *   The row (column) scale sigma is shared by both parts; rows past `rows`
 *   and k past K are zero.
 *
 * Exponent sentinels in the int32 scale vectors: OZK_EXP_ZERO marks a row
 * (column) with no nonzero entry, OZK_EXP_NONFINITE one with a NaN or inf.
 */
#ifndef OZK_H
#define OZK_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OZK_ROW_ALIGN 256
#define OZK_K_CHUNK 32
#define OZK_EXP_ZERO (-100000)
#define OZK_EXP_NONFINITE 100000
#define OZK_MAX_P 8
#define OZK_MAX_S 20
#define OZK_MAX_ROWS 16777216       /* 2^24: largest M, N (32-bit packed offsets) */
#define OZK_S2_MAX_K 4194304        /* 2^22: longest K of a Scheme II product (see below) */
#define OZK_S1_VARIANTS 4           /* Scheme I GEMM tile variants */
#define OZK_S2_VARIANTS 7           /* Scheme II GEMM variants (4: fused CRT) */
#define OZK_S2_FUSED_CRT 4          /* Scheme II variant with the CRT fused into the GEMM (real only) */
#define OZK_NOALLOC_SCRATCH_BYTES 67108864  /* 64 MiB: the fixed buffer of ozk_dgemm_noalloc */
#define OZK_SELECTOR_PARAMS 8220   /* float32 parameters of the selector MLP */
#define OZK_SELECTOR_HEADS 28      /* ordinal heads: 8 for p, 20 for s */
#define OZK_SELECTOR_COUNTERS 34   /* int32 feature counters */
#define OZK_SELECTOR_INFO 8        /* int32 decision entries */

/* Condition bits of a context's flag word (ozk_get_flags). */
#define OZK_FLAG_NONFINITE 1u          /* an input row of A or column of B held a NaN or an infinity */
#define OZK_FLAG_SELECTOR_FALLBACK 2u  /* an automatic call decided by the a-priori bound alone */
#define OZK_FLAG_SCHEME2_CHOSEN 4u     /* an automatic call found no slice count <= 8 enough: Scheme II ran */
#define OZK_FLAG_S_UNPROVEN 8u         /* ... with s = 20, no modulus count <= 20 proven enough */

typedef struct ozk_ctx ozk_ctx;

typedef enum {
  OZK_OK = 0,
  OZK_ERR_INVALID_ARG = -1, /* bad pointer, dimension, leading dimension */
  OZK_ERR_UNSUPPORTED = -2, /* p outside [1, 8], s outside [1, 20], ... */
  OZK_ERR_WORKSPACE = -3,   /* workspace missing or too small */
  OZK_ERR_HIP = -4          /* a HIP runtime call failed */
} ozk_status;

typedef enum { OZK_SCHEME1 = 1, OZK_SCHEME2 = 2 } ozk_scheme;
/* Element types of ozk_gemm_ex: binary64, binary32, and complex numbers of
 * them (interleaved re, im). */
typedef enum { OZK_F64 = 0, OZK_F32 = 1, OZK_C128 = 2, OZK_C64 = 3 } ozk_dtype;
/* Storage of every matrix of an ozk_gemm_ex call. */
typedef enum { OZK_ROW_MAJOR = 0, OZK_COL_MAJOR = 1 } ozk_layout;
/* Operations.  The _BATCHED codes only key the tuned table's entries that
 * choose the GEMM tile of a batched problem's size class (see
 * ozk_batch_plan_create). */
typedef enum {
  OZK_OP_DGEMM = 0,
  OZK_OP_ZGEMM = 1,
  OZK_OP_DGEMM_BATCHED = 2,
  OZK_OP_ZGEMM_BATCHED = 3
} ozk_op;

/* ---------------------------------------------------------------- context */

/* Create a context bound to HIP device `device` (made current on the calling
 * thread).  The context owns only small constant tables.  One context per
 * host thread; a context may be used with any stream of its device. */
ozk_status ozk_create(ozk_ctx** ctx, int device);
/* Destroy a context (NULL is accepted).  Work already enqueued must have
 * completed. */
ozk_status ozk_destroy(ozk_ctx* ctx);
/* 1-based position of the argument that made the last call on this context
 * fail with OZK_ERR_INVALID_ARG / UNSUPPORTED / WORKSPACE; 0 otherwise. */
int ozk_last_arg(const ozk_ctx* ctx);
/* Static description of a status code. */
const char* ozk_status_string(ozk_status s);
/* Library version, "major.minor.patch". */
const char* ozk_version(void);
/* Testing hook: make every Scheme I call on this context fold its K runs
 * every k values of K instead of every ozk_s1_k_split(p) (whichever is
 * shorter), which exercises the exact 128-bit fold on small problems.  k is
 * 0 (back to the default) or a positive multiple of OZK_K_CHUNK; anything
 * else returns OZK_ERR_INVALID_ARG (arg 2).  Query workspace sizes after
 * setting it. */
ozk_status ozk_set_k_split(ozk_ctx* ctx, int64_t k);

/* Conditions found on the device, which no synchronous status can report
 * because the library never reads device data on the host (the paper
 * defines none of them: they are this library's): every whole call (DGEMM,
 * SGEMM, ZGEMM, CGEMM, the unfused, transposed, allocation-free, automatic
 * and batched calls) ORs bits into a device flag word of its context, on
 * its stream, after its pre-pass:
 *   OZK_FLAG_NONFINITE         a row of A or a column of B held a NaN or an
 *                              infinity (its row / column of the result is
 *                              NaN; the other outputs are unaffected);
 *   OZK_FLAG_SELECTOR_FALLBACK an automatic call (ozk_dgemm_auto,
 *                              ozk_zgemm_auto) decided by the a-priori bound
 *                              alone: no network loaded, or its features
 *                              outside the network's training range;
 *   OZK_FLAG_SCHEME2_CHOSEN    an automatic DGEMM found no slice count up to
 *                              8 that meets the tolerance and ran Scheme II
 *                              (Scheme I "infeasible");
 *   OZK_FLAG_S_UNPROVEN        an automatic call ran Scheme II with s = 20
 *                              although no modulus count up to 20 is proven
 *                              to meet the tolerance.
 * ozk_get_flags waits for the work enqueued on `stream` (hipStreamSynchronize),
 * then atomically takes the word, clearing it, and stores it in *flags (a
 * HOST pointer): the OR of the conditions raised since the context was
 * created or its flags were last taken, by every call whose work has
 * completed.  Work on other streams still running may raise bits after the
 * take; they are kept for the next one.  Synchronises, so it must not be
 * captured into a graph.  Errors: OZK_ERR_INVALID_ARG (arg 3) for a null
 * flags pointer, OZK_ERR_HIP. */
ozk_status ozk_get_flags(ozk_ctx* ctx, hipStream_t stream, uint32_t* flags);

/* ---------------------------------------------------------- sizes / layout */

/* Bytes of a Scheme I packed operand with `rows` rows, contraction length K
 * and p slices: roundup(rows, 256) * roundup(K, 32) * p. */
size_t ozk_s1_packed_bytes(int64_t rows, int64_t K, int p);
/* Bytes of a Scheme II packed operand: s * roundup(rows,256) * roundup(K,32)
 * * (3 if complex else 1). */
size_t ozk_s2_packed_bytes(int64_t rows, int64_t K, int s, int complex_planes);
/* Longest K run whose Scheme I INT32 diagonals cannot overflow
 * (|slice_0| <= 64, |slice_t| <= 128 bound diagonal d by max(2^12, d 2^14)
 * per k), rounded down to a multiple of 32. */
int64_t ozk_s1_k_split(int p);

/* Workspace bytes ozk_dgemm / ozk_zgemm_3m need for this problem.  For
 * Scheme I it holds the scale vectors, the two packed operands and, when K
 * exceeds ozk_s1_k_split(p), 16 bytes per output per K run; for Scheme II
 * the scales, the residue planes and s (or 2s for complex) int8 output
 * residue planes.  Scheme I with p_or_s = 0: the size ozk_dgemm_auto needs
 * (room for p = 8 plus the selector counters).  OZK_OP_ZGEMM with Scheme I:
 * the 4M workspace of ozk_zgemm / ozk_cgemm; with Scheme II and p_or_s = 0:
 * the workspace of ozk_zgemm_auto. */
ozk_status ozk_workspace_size(ozk_ctx* ctx, ozk_op op, ozk_scheme scheme,
                              int64_t M, int64_t N, int64_t K, int p_or_s,
                              size_t* bytes);

/* ------------------------------------------------------------ whole calls */

/* C = alpha*A*B + beta*C in FP64, emulated with Scheme I (p = slices per
 * operand, 1..8; Sec. II-C.1, Sec. III) or Scheme II (p_or_s = number of
 * moduli, 1..20; Sec. II-C.2, Sec. IV-A).  Runs the pre-pass, the fused
 * GEMM and the epilogue (CRT for Scheme II) on `stream`.  `ws` must hold
 * ozk_workspace_size(..) bytes. */
ozk_status ozk_dgemm(ozk_ctx* ctx, ozk_scheme scheme, int p_or_s, int64_t M,
                     int64_t N, int64_t K, double alpha, const double* A,
                     int64_t lda, const double* B, int64_t ldb, double beta,
                     double* C, int64_t ldc, void* ws, size_t ws_bytes,
                     hipStream_t stream);

/* ozk_dgemm for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation, argument meanings, layouts and errors as ozk_dgemm,
 * bit-identical results, but no workspace argument.  The workspace ozk_dgemm
 * would take lives in a fixed buffer of OZK_NOALLOC_SCRATCH_BYTES (64 MiB)
 * inside the library, a static device array of which every device the
 * library runs on holds its own copy until the process ends; its address is
 * looked up once per device when a context is created.  Problems whose
 * ozk_workspace_size(ctx, OZK_OP_DGEMM, scheme, M, N, K, p_or_s) exceeds the
 * buffer return OZK_ERR_WORKSPACE (ozk_last_arg() = 4) before anything is
 * enqueued; e.g. Scheme I at p = 7 fits up to M = N = K = 2048.  The call
 * allocates and frees nothing, and needs no zeroed memory (every kernel
 * initialises what it accumulates into).  All calls on one device share the
 * buffer and it keeps the last call's contents: calls that overlap on one
 * device (other streams, other host threads) race and must be ordered by
 * the caller, e.g. by issuing them on one stream. */
ozk_status ozk_dgemm_noalloc(ozk_ctx* ctx, ozk_scheme scheme, int p_or_s,
                             int64_t M, int64_t N, int64_t K, double alpha,
                             const double* A, int64_t lda, const double* B,
                             int64_t ldb, double beta, double* C, int64_t ldc,
                             hipStream_t stream);

/* ozk_dgemm with transposed operands: C = alpha*op(A)*op(B) + beta*C where
 * op(A) = A (trans_a = 0: A stored M x K, lda >= K) or A^T (trans_a = 1: A
 * stored K x M, lda >= M), and op(B) = B (trans_b = 0: B stored K x N,
 * ldb >= N) or B^T (trans_b = 1: B stored N x K, ldb >= K), all row-major.
 * A transposed operand is read by the other pre-pass kernel (the column
 * pass for A^T, the row pass for B^T), which writes the same packed layout
 * and scales, so the result is bit-identical to ozk_dgemm on the explicit
 * transposes.  Both schemes; workspace as ozk_dgemm.  Errors as ozk_dgemm,
 * with the argument indices of this signature (trans flags other than 0 or
 * 1: OZK_ERR_INVALID_ARG, arg 4 or 5; workspace: arg 19). */
ozk_status ozk_dgemm_t(ozk_ctx* ctx, ozk_scheme scheme, int p_or_s, int trans_a,
                       int trans_b, int64_t M, int64_t N, int64_t K,
                       double alpha, const double* A, int64_t lda,
                       const double* B, int64_t ldb, double beta, double* C,
                       int64_t ldc, void* ws, size_t ws_bytes,
                       hipStream_t stream);

/* The general form of the whole calls: C = alpha*op(A)*op(B) + beta*C for
 * every element type, both storage orders and transposed operands (the
 * paper's problem statement, Sec. II-B, with the BLAS options; non-square
 * shapes are untested in the paper, Sec. V-G).  op(X) = X (trans = 0) or
 * X^T (trans = 1; no conjugation), op(A) is M x K and op(B) K x N; A is
 * stored M x K (trans_a = 0) or K x M, B is stored K x N (trans_b = 0) or
 * N x K, C is M x N, all in `layout`, with leading dimensions in elements
 * (complex elements for complex types) at least the length of a stored row
 * (row-major) or column (column-major).  alpha, beta: HOST pointers to one
 * value of the element's real type (F64, F32) or to {re, im} (C128, C64).
 * A column-major problem is run as the row-major product C^T = op(B)^T
 * op(A)^T of the same memory (the operands swap, each transposed exactly
 * when the other one was), and a transposed operand is read by the other
 * pre-pass kernel: each row of op(A) and each column of op(B) keeps its
 * scale (and, Scheme II, its bit budget), the integer sums are the same, so
 * results are bit-identical to ozk_dgemm / ozk_sgemm / ozk_zgemm /
 * ozk_cgemm on the explicit row-major operands.  One exception: the Scheme
 * I complex product of column-major operands is the 4M product of the
 * transposed problem, B^T A^T, whose embedding negates the imaginary parts
 * of A instead of B; Scheme I drops slice pairs of the balanced digits,
 * whose expansion of -x is not the negated expansion of x, so its last bits
 * differ from the row-major call while the error bound is the same.
 * Schemes and counts as those calls; Scheme I complex (4M) takes no
 * transposed operand (OZK_ERR_UNSUPPORTED, arg 4 or 5: its embedding is
 * built from stored rows of op(A) and columns of op(B)).  Workspace:
 * ozk_workspace_size(ctx, F64/F32 -> OZK_OP_DGEMM, C128/C64 -> OZK_OP_ZGEMM,
 * scheme, M', N', K, p_or_s) with (M', N') = (M, N) for row-major and
 * (N, M) for column-major storage.  Device pointers, caller-owned memory,
 * asynchronous on `stream`.  Errors: OZK_ERR_INVALID_ARG with the argument
 * index (2 dtype, 3 layout, 4-5 trans, 6 scheme, 8-10 sizes, 11 alpha,
 * 12-15 A, B, 16 beta, 17-18 C), OZK_ERR_UNSUPPORTED (arg 7) for a count out
 * of range, OZK_ERR_WORKSPACE (arg 19). */
ozk_status ozk_gemm_ex(ozk_ctx* ctx, ozk_dtype dtype, ozk_layout layout,
                       int trans_a, int trans_b, ozk_scheme scheme,
                       int p_or_s, int64_t M, int64_t N, int64_t K,
                       const void* alpha, const void* A, int64_t lda,
                       const void* B, int64_t ldb, const void* beta, void* C,
                       int64_t ldc, void* ws, size_t ws_bytes,
                       hipStream_t stream);

/* The unfused Scheme I baseline, as an ablation of the fused kernel (the
 * naive scheme of the paper's traffic model, Sec. III, Eq. 9): the same
 * pre-pass as ozk_dgemm, then one INT8 GEMM per slice pair (t, u), t + u < p,
 * each writing its INT32 result to HBM, then a pass that reads the
 * p(p+1)/2 planes back, forms Z exactly and rounds once.  The result is
 * bit-identical to ozk_dgemm(OZK_SCHEME1, p); only the INT32 round trip
 * (4 p(p+1) M N bytes written and read) and the p(p+1)/2 operand passes
 * differ.  1 <= p <= 8, K <= 131071 (|sum| <= K 2^14 keeps each INT32 plane exact).
 * Workspace: ozk_s1_unfused_workspace_size bytes (the packed operands plus
 * 2 p(p+1) M N bytes of planes).  Device pointers, caller-owned memory,
 * asynchronous on `stream`; errors as ozk_dgemm (OZK_ERR_UNSUPPORTED, arg 5,
 * for K > 131071). */
ozk_status ozk_s1_unfused_workspace_size(ozk_ctx* ctx, int p, int64_t M,
                                         int64_t N, int64_t K, size_t* bytes);
ozk_status ozk_s1_dgemm_unfused(ozk_ctx* ctx, int p, int64_t M, int64_t N,
                                int64_t K, double alpha, const double* A,
                                int64_t lda, const double* B, int64_t ldb,
                                double beta, double* C, int64_t ldc, void* ws,
                                size_t ws_bytes, hipStream_t stream);

/* Emulated SGEMM, C = alpha*A*B + beta*C in binary32 (the paper's FP32-level
 * operating points: Scheme I with p = 1..4, Scheme II with s = 8..11;
 * Sec. V-D).  A (M x K, lda) and B (K x N, ldb) are row-major binary32,
 * widened exactly to binary64 for the exponent, slice and residue steps, so
 * the slices or residues, the INT32 products and the exact integer result
 * Z are those of ozk_dgemm on the widened operands; the one rounding of
 * Z 2^E goes to binary32 (round to nearest even, gradual underflow,
 * overflow to infinity), then C = alpha*h (beta == 0, C not read) or
 * fmaf(alpha, h, beta*C), in binary32.  Non-finite rows of A or columns of
 * B give NaN.  Scheme I: 1 <= p_or_s <= 8; Scheme II: 1 <= p_or_s <= 20
 * (with the separate CRT kernel whatever the configuration).  The
 * workspace is that of ozk_dgemm with the same scheme and count
 * (ozk_workspace_size(ctx, OZK_OP_DGEMM, scheme, M, N, K, p_or_s)), and the
 * GEMM step takes the DGEMM configuration of the size class.  Device
 * pointers; the caller owns all memory; asynchronous on `stream`.  Errors:
 * OZK_ERR_INVALID_ARG with the argument index for a bad scheme, sizes,
 * leading dimensions or null pointers, OZK_ERR_UNSUPPORTED (arg 3) for a
 * count out of range, OZK_ERR_WORKSPACE (arg 15). */
ozk_status ozk_sgemm(ozk_ctx* ctx, ozk_scheme scheme, int p_or_s, int64_t M,
                     int64_t N, int64_t K, float alpha, const float* A,
                     int64_t lda, const float* B, int64_t ldb, float beta,
                     float* C, int64_t ldc, void* ws, size_t ws_bytes,
                     hipStream_t stream);

/* Emulated CGEMM by Scheme II and 3M, binary32 complex (interleaved re, im;
 * torch.complex64) in and out: ozk_zgemm_3m on the exactly widened operands
 * with the final roundings to binary32 and the complex alpha/beta update of
 * ozk_zgemm_3m's fixed FMA sequence in binary32 (fmaf).  alpha and beta
 * point to {re, im} on the host.  Workspace ozk_workspace_size(ctx,
 * OZK_OP_ZGEMM, OZK_SCHEME2, M, N, K, s); the GEMM step takes the ZGEMM
 * configuration.  Errors as ozk_zgemm_3m. */
ozk_status ozk_cgemm_3m(ozk_ctx* ctx, int s, int64_t M, int64_t N, int64_t K,
                        const float* alpha, const float* A, int64_t lda,
                        const float* B, int64_t ldb, const float* beta,
                        float* C, int64_t ldc, void* ws, size_t ws_bytes,
                        hipStream_t stream);

/* C = alpha*A*B + beta*C in complex128 with Scheme II and the 3M identity
 * (Sec. IV-B, Eq. 16): three modular products per modulus, exact.  alpha and
 * beta are HOST arrays {re, im}; beta == 0 (both parts) means C is not read.
 * The update is out_re = fma(a_re, h_re, fma(-a_im, h_im, bc_re)),
 * out_im = fma(a_re, h_im, fma(a_im, h_re, bc_im)) with
 * bc = (fma(b_re, c_re, -(b_im c_im)), fma(b_re, c_im, b_im c_re)). */
ozk_status ozk_zgemm_3m(ozk_ctx* ctx, int s, int64_t M, int64_t N, int64_t K,
                        const double* alpha, const double* A, int64_t lda,
                        const double* B, int64_t ldb, const double* beta,
                        double* C, int64_t ldc, void* ws, size_t ws_bytes,
                        hipStream_t stream);

/* Complex GEMM, C = alpha*A*B + beta*C, by either scheme (ZGEMM: complex128,
 * CGEMM: complex64 in and out; interleaved (re, im); leading dimensions in
 * complex elements; alpha and beta are HOST arrays {re, im}).
 *   OZK_SCHEME2: Scheme II with 3M (exactly ozk_zgemm_3m / ozk_cgemm_3m;
 *     p_or_s = s moduli, 1..20).
 *   OZK_SCHEME1: Scheme I with the 4M formulation (Sec. IV-B names 4M as the
 *     standard four-product form; Sec. V-D reports Scheme I complex GEMMs):
 *     the four real products Re A Re B, Im A Im B, Re A Im B, Im A Re B and
 *     the subtraction and addition that combine them are one Scheme I
 *     product of real embeddings, A' = (M x 2K: row i holds Re a_ik, Im a_ik
 *     for k = 0..K-1, i.e. A as stored viewed as reals) and B'' (2K x 2N: row
 *     2k holds (Re b_kj, Im b_kj) at columns (2j, 2j+1), row 2k+1 holds
 *     (-Im b_kj, Re b_kj)), whose product's columns 2j and 2j+1 are Re and
 *     Im of (AB)_ij.  So each part is formed exactly in integers and rounded
 *     once; a row of A has one exponent for both parts, and so has a column
 *     of B.  p_or_s = p slices, 1..8; the INT8 work is 4 p(p+1) MNK.  The
 *     GEMM step takes the DGEMM configuration of the embedded size class
 *     (M, 2N, 2K); it writes the M x 2N real parts to the workspace and a
 *     final pass applies the complex update with the fixed FMA sequence of
 *     ozk_zgemm_3m (in binary32 for CGEMM, whose operands are widened
 *     exactly and whose parts are rounded once to binary32).  N <= 2^23.
 * Workspace: ozk_workspace_size(ctx, OZK_OP_ZGEMM, scheme, M, N, K, p_or_s)
 * bytes (Scheme I: the Scheme I workspace of the embedded product plus
 * 16 MN bytes).  Device pointers, caller-owned memory, asynchronous on
 * `stream`.  Errors: OZK_ERR_INVALID_ARG with the argument index (2 scheme,
 * 4-6 sizes, 7 alpha, 8-11 A, B, 12 beta, 13-14 C), OZK_ERR_UNSUPPORTED
 * (arg 3) for a count out of range, OZK_ERR_WORKSPACE (arg 15). */
ozk_status ozk_zgemm(ozk_ctx* ctx, ozk_scheme scheme, int p_or_s, int64_t M,
                     int64_t N, int64_t K, const double* alpha,
                     const double* A, int64_t lda, const double* B,
                     int64_t ldb, const double* beta, double* C, int64_t ldc,
                     void* ws, size_t ws_bytes, hipStream_t stream);
ozk_status ozk_cgemm(ozk_ctx* ctx, ozk_scheme scheme, int p_or_s, int64_t M,
                     int64_t N, int64_t K, const float* alpha, const float* A,
                     int64_t lda, const float* B, int64_t ldb,
                     const float* beta, float* C, int64_t ldc, void* ws,
                     size_t ws_bytes, hipStream_t stream);

/* The unfused Scheme II baseline, as an ablation of the fused kernels (the
 * naive forms of the paper's traffic models: Sec. IV-A, Eq. 14 for real
 * products and Sec. IV-B, Eq. 17 for 3M): the same pre-pass and CRT as
 * ozk_dgemm(OZK_SCHEME2, s) (complex_planes = 0) or ozk_zgemm_3m
 * (complex_planes = 1), but every modular product -- one per modulus, or
 * T1, T2, T3 per modulus for 3M -- is an INT8 GEMM writing its INT32
 * result to HBM, and a pass reads the planes back and reduces them mod m
 * (3M: forms smod(T1 - T2) and smod(T3 - T1 - T2)) into the residue planes
 * the CRT reads.  Bit-identical to the fused call; only the INT32 round trip
 * (4 MN bytes per product, written and read) differs.  X, C real (FP64) or
 * complex (interleaved complex128) by complex_planes; alpha, beta HOST
 * arrays {re, im} (the imaginary part ignored for real data).
 * 1 <= s <= 20, K <= 131071 (|sum| <= K 2^14 keeps each INT32 plane exact;
 * longer K returns OZK_ERR_UNSUPPORTED, arg 6).  Workspace:
 * ozk_s2_unfused_workspace_size bytes (the fused call's workspace plus
 * 4 s MN bytes of planes, 12 s MN for 3M).  Errors as ozk_zgemm. */
ozk_status ozk_s2_unfused_workspace_size(ozk_ctx* ctx, int s, int complex_planes,
                                         int64_t M, int64_t N, int64_t K,
                                         size_t* bytes);
ozk_status ozk_s2_gemm_unfused(ozk_ctx* ctx, int s, int complex_planes,
                               int64_t M, int64_t N, int64_t K,
                               const double* alpha, const double* A,
                               int64_t lda, const double* B, int64_t ldb,
                               const double* beta, double* C, int64_t ldc,
                               void* ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------ Scheme I, step by step */

/* Pre-pass for a row operand (A): e[i] = row exponent (smallest e with
 * |a_ik| < 2^e, or a sentinel) for i < rows, and the packed slices P
 * (ozk_s1_packed_bytes(rows, K, p) bytes, layout above).  Sec. II-C.1 Eq. 1,
 * Sec. III-A Eq. 11. */
ozk_status ozk_s1_split_rows(ozk_ctx* ctx, int p, int64_t rows, int64_t K,
                             const double* X, int64_t ldx, int32_t* e,
                             int8_t* packed, hipStream_t stream);
/* The same for a column operand (B, K x cols): f[j] = column exponent, and
 * the packed slices of B transposed. */
ozk_status ozk_s1_split_cols(ozk_ctx* ctx, int p, int64_t K, int64_t cols,
                             const double* X, int64_t ldx, int32_t* f,
                             int8_t* packed, hipStream_t stream);
/* Fused Scheme I GEMM (Sec. III-B, Alg. 1): all p(p+1)/2 slice-pair INT8
 * products accumulated into p INT32 diagonals that stay in registers; the
 * epilogue forms the exact integer Z = sum_d 2^(8(p-1-d)) C_d and writes
 * RN(Z 2^(e_i + f_j - 12 - 8(p-1))) through alpha/beta.  When K exceeds
 * ozk_s1_k_split(p) the K runs are folded exactly through `ws` (16 bytes per
 * output per run; pass NULL/0 otherwise). */
ozk_status ozk_s1_gemm(ozk_ctx* ctx, int p, int64_t M, int64_t N, int64_t K,
                       const int8_t* packedA, const int32_t* e,
                       const int8_t* packedB, const int32_t* f, double alpha,
                       double beta, double* C, int64_t ldc, void* ws,
                       size_t ws_bytes, hipStream_t stream);
/* Check entry point: the raw INT32 diagonals C_d (Eq. 2) of the fused
 * kernel, Cd[d][i][j] (int32, M x N per diagonal, row-major).  Requires
 * K <= ozk_s1_k_split(p). */
ozk_status ozk_s1_diagonals(ozk_ctx* ctx, int p, int64_t M, int64_t N,
                            int64_t K, const int8_t* packedA,
                            const int8_t* packedB, int32_t* Cd,
                            hipStream_t stream);

/* ----------------------------------------------- Scheme II, step by step */

/* Pre-pass for a row operand: sigma[i] (power-of-two row scale exponent,
 * chosen from an exact bound on the row's 2-norm so that the CRT exactness
 * condition 2 sum |a'||b'| < P holds, Sec. II-C.2) and the s residue planes.
 * complex_planes = 1: X is complex (interleaved) and three planes per
 * modulus are written (real, imaginary, their sum mod m) with one shared
 * sigma per row (Sec. IV-B). */
ozk_status ozk_s2_split_rows(ozk_ctx* ctx, int s, int complex_planes,
                             int64_t rows, int64_t K, const double* X,
                             int64_t ldx, int32_t* sigma, int8_t* packed,
                             hipStream_t stream);
/* The same for a column operand (B, K x cols), transposed on the fly. */
ozk_status ozk_s2_split_cols(ozk_ctx* ctx, int s, int complex_planes,
                             int64_t K, int64_t cols, const double* X,
                             int64_t ldx, int32_t* tau, int8_t* packed,
                             hipStream_t stream);
/* Per-modulus INT8 GEMM with the modular reduction fused into the epilogue
 * (Sec. IV-A, Eqs. 6-7): Cres[l][i][j] = smod(sum_k R_l[i][k] S_l[j][k], m_l)
 * (int8, s planes of M x N).  complex_planes = 1: 3M (Sec. IV-B, Eq. 16),
 * Cres[l][0] = smod(T1 - T2), Cres[l][1] = smod(T3 - T1 - T2), 2s planes.
 * Any K: the INT32 accumulators are reduced by multiples of m_l every
 * 131040 values of k, which leaves their residues unchanged. */
ozk_status ozk_s2_gemm_mod(ozk_ctx* ctx, int s, int complex_planes, int64_t M,
                           int64_t N, int64_t K, const int8_t* packedA,
                           const int8_t* packedB, int8_t* Cres,
                           hipStream_t stream);
/* CRT recombination and inverse scaling (Eq. 8): Z = smod(sum_l
 * (P/m_l) q_l Cres_l, P) in multiword integers, h = RN(Z 2^(-sigma_i -
 * tau_j)), then the alpha/beta update (real: alpha[0], beta[0]; complex:
 * the fma sequence of ozk_zgemm_3m).  alpha, beta are HOST arrays. */
ozk_status ozk_s2_crt(ozk_ctx* ctx, int s, int complex_planes, int64_t M,
                      int64_t N, const int8_t* Cres, const int32_t* sigma,
                      const int32_t* tau, const double* alpha,
                      const double* beta, double* C, int64_t ldc,
                      hipStream_t stream);

/* ---------------------------------- learned slice / modulus count selector */
/* The paper's implementation has no automatic precision selection (it is
 * named as missing, Sec. VI); this library predicts the smallest Scheme I
 * slice count p and the smallest Scheme II modulus count s meeting a
 * componentwise tolerance with a small MLP (34 -> 64 -> 64 -> 28, ReLU; 8
 * ordinal heads "p > t", t = 1..8, then 20 heads "s > t", t = 1..20) from
 * exponent statistics gathered on the device, each bounded by an a-priori
 * error bound.
 *
 * Parameter layout (float32, OZK_SELECTOR_PARAMS values, weights [in][out]):
 * W1[34][64], b1[64], W2[64][64], b2[64], W3[64][28], b3[28].
 * Features: for A's rows and B's columns, the fractions of nonzero entries
 * whose exponent deficit e_i - expo(a_ik) falls in the bins [0] [1] [2] [3]
 * [4,6) [6,8) [8,12) [12,16) [16,24) [24,32) [32,48) [48,64) [64,96)
 * [96,128) [128,256) [256,inf); then log2(K)/14 and -log10(tol)/16.
 * Counters (int32, OZK_SELECTOR_COUNTERS): 16 + 16 bin counts, the largest
 * deficit of A, of B.  Decision, with thr_h the per-head thresholds:
 * p_net = 1 + #{t <= 8 : sigmoid(z_t) > thr_t} + margin (at most 9),
 * s_net = 1 + #{t <= 20 : sigmoid(z_{8+t}) > thr_{8+t}} + margin (at most
 * 21); p_bound (s_bound) = the smallest p (s) whose a-priori bound is <= tol
 * (9, resp. 21, if none); p = min(p_net, p_bound) and s = min(s_net,
 * s_bound), or the bounds alone when no network is loaded or the features
 * are outside the training range (K > 16384, tol outside [1e-16, 1e-5], any
 * entry in the last deficit bin).  p <= 8: Scheme I with p slices.  p = 9
 * (no slice count up to 8 is enough): Scheme II with s moduli (the Scheme II
 * bound uses the norm-bound scales, Sec. II-C.2), or s = 20 when s = 21.
 * info (device int32[OZK_SELECTOR_INFO]): [0] Scheme I slices (0 when
 * Scheme II is chosen), [1] p_net (0 without network), [2] p_bound,
 * [3] 1 if out of range, [4] scheme (1 or 2), [5] Scheme II moduli (0 with
 * Scheme I), [6] s_bound (21 if none up to 20), [7] s_net (0 without
 * network). */

/* Load selector parameters (HOST float array of OZK_SELECTOR_PARAMS) and the
 * OZK_SELECTOR_HEADS decision thresholds (HOST floats, each in (0, 1)) into
 * the context (the parameters are copied to device memory owned by the
 * context).  margin: 0..8 counts added to p_net and s_net.  Errors:
 * OZK_ERR_INVALID_ARG (arg 2 parameters, 4 thresholds, 5 margin). */
ozk_status ozk_selector_load(ozk_ctx* ctx, const float* params, size_t n,
                             const float* thresholds, int margin);
/* Exponent statistics and the selector decision for C = A B, all on the
 * device: e[M], f[N] (the Scheme I row/column exponents), counters,
 * info[OZK_SELECTOR_INFO] and, if features is not NULL, the 34 features
 * (float32). */
ozk_status ozk_select(ozk_ctx* ctx, double tol, int64_t M, int64_t N,
                      int64_t K, const double* A, int64_t lda, const double* B,
                      int64_t ldb, int32_t* e, int32_t* f, int32_t* counters,
                      int32_t* info, float* features, hipStream_t stream);
/* DGEMM with the scheme and the slice or modulus count chosen on the device
 * for the componentwise tolerance `tol` (the decision above): the kernels of
 * both schemes are enqueued and those not chosen return at once, so there is
 * no host round trip and the call can be captured into a graph.  ws must
 * hold ozk_workspace_size(ctx, OZK_OP_DGEMM, OZK_SCHEME1, M, N, K, 0) bytes
 * (room for either scheme); info (device int32[OZK_SELECTOR_INFO], may be
 * NULL) receives the decision. */
ozk_status ozk_dgemm_auto(ozk_ctx* ctx, double tol, int64_t M, int64_t N,
                          int64_t K, double alpha, const double* A,
                          int64_t lda, const double* B, int64_t ldb,
                          double beta, double* C, int64_t ldc, void* ws,
                          size_t ws_bytes, int32_t* info, hipStream_t stream);

/* ZGEMM (complex128, interleaved; alpha, beta HOST {re, im}) with the
 * modulus count chosen on the device for the componentwise tolerance `tol`
 * (the complex E_cw: the real and imaginary parts scaled by the magnitude
 * sums of the products forming them): Scheme II with 3M (Sec. IV-B) at the
 * smallest s whose a-priori bound meets tol -- the Scheme II bound above
 * with the largest deficits of the real and imaginary parts below the
 * largest part exponent of their row of A (column of B), plus one (the
 * shared per-row scale is taken from |re| + |im|) -- or s = 20 when none is
 * proven (OZK_FLAG_S_UNPROVEN).  The network is trained on real products
 * and is not used, so the call raises OZK_FLAG_SELECTOR_FALLBACK.  Every
 * kernel reads s from the device; no host round trip, graph-capturable.
 * ws: ozk_workspace_size(ctx, OZK_OP_ZGEMM, OZK_SCHEME2, M, N, K, 0) bytes;
 * info (device int32[OZK_SELECTOR_INFO], may be NULL): [4] = 2, [5] s,
 * [6] the bound's s (21 if none), the other entries 0 (and [2] 9).
 * Errors as ozk_zgemm_3m (arg 2 a tolerance outside (0, 1), workspace 14). */
ozk_status ozk_zgemm_auto(ozk_ctx* ctx, double tol, int64_t M, int64_t N,
                          int64_t K, const double* alpha, const double* A,
                          int64_t lda, const double* B, int64_t ldb,
                          const double* beta, double* C, int64_t ldc,
                          void* ws, size_t ws_bytes, int32_t* info,
                          hipStream_t stream);

/* Training kernels of the selector network (device float32 arrays; X is
 * n x 34, Y n x 28 ordinal targets, logits n x 28).  ozk_mlp_grad writes the
 * gradient of the mean binary cross-entropy into grad (OZK_SELECTOR_PARAMS)
 * and the loss into *loss; ozk_mlp_adam applies one bias-corrected Adam
 * step (beta1 0.9, beta2 0.999, eps 1e-8; step counts from 1). */
ozk_status ozk_mlp_forward(ozk_ctx* ctx, const float* params, const float* X,
                           int n, float* logits, hipStream_t stream);
ozk_status ozk_mlp_grad(ozk_ctx* ctx, const float* params, const float* X,
                        const float* Y, int n, float* grad, float* loss,
                        hipStream_t stream);
ozk_status ozk_mlp_adam(ozk_ctx* ctx, float* params, const float* grad,
                        float* m, float* v, int step, float lr,
                        hipStream_t stream);
/* Check tool: double-double dot products of the n outputs (rows[i],
 * cols[i]) of A B (device index arrays): hi + lo to about 2^-104 relative
 * per term, absab = sum_k |a||b| (for componentwise errors).  An index
 * outside [0, M) x [0, N) yields NaN in all three outputs. */
ozk_status ozk_ref_dd(ozk_ctx* ctx, int64_t M, int64_t N, int64_t K,
                      const double* A, int64_t lda, const double* B,
                      int64_t ldb, int64_t n, const int64_t* rows,
                      const int64_t* cols, double* hi, double* lo,
                      double* absab, hipStream_t stream);

/* ------------------------------------------------- batches of problems */

/* One problem of a batch: C = alpha*A*B + beta*C with the same conventions
 * as the single calls (device pointers, row-major, leading dimensions in
 * elements; complex data interleaved).  alpha/beta are {re, im}; DGEMM uses
 * the real parts. */
typedef struct ozk_gemm_desc {
  int64_t M, N, K;
  const double* A;
  int64_t lda;
  const double* B;
  int64_t ldb;
  double* C;
  int64_t ldc;
  double alpha[2];
  double beta[2];
} ozk_gemm_desc;

typedef struct ozk_batch_plan ozk_batch_plan;

/* Plan a batch of `count` uneven problems (descs is a HOST array; the
 * pointers inside are kept and used by every ozk_gemm_batched call).  This
 * is the only step that allocates: a small device table with the problem
 * list, per-step prefix sums of the work units and, for each of the two
 * GEMM tiles, the order of its work items (problems by decreasing K, so the
 * longest items start first).  Each problem's GEMM items take one of two
 * tiles: 64 x 64 (several workgroups per CU hide the latency of short
 * items) or 128 x 128 (fewer LDS bytes per MFMA).  The tile of a problem is
 * the context table's entry for its size class under op
 * OZK_OP_DGEMM_BATCHED / OZK_OP_ZGEMM_BATCHED (variant 0 small, 1 large;
 * written by ozk_tune_batch, ozk_config_set or ozk_config_load), or, for a
 * class without an entry, the large tile when M and N are both at least 256.
 * *ws_bytes receives the workspace every call needs.  Supported: Scheme II
 * real DGEMM (op OZK_OP_DGEMM) and 3M ZGEMM (op OZK_OP_ZGEMM), 1 <= s <= 20;
 * other combinations return OZK_ERR_UNSUPPORTED.  Not in the paper: its
 * problems are single square GEMMs (Sec. V-B). */
ozk_status ozk_batch_plan_create(ozk_ctx* ctx, ozk_op op, ozk_scheme scheme,
                                 int p_or_s, int count,
                                 const ozk_gemm_desc* descs,
                                 ozk_batch_plan** plan, size_t* ws_bytes);
/* Run a planned batch on `stream`: one launch per step for all problems
 * (pre-pass of the rows, column scales, column residues, a persistent
 * INT8 GEMM over every (problem, modulus, tile) item, CRT).  No allocation,
 * no host synchronisation, no memset: the sequence can be captured into a
 * HIP graph and replayed. */
ozk_status ozk_gemm_batched(ozk_ctx* ctx, const ozk_batch_plan* plan, void* ws,
                            size_t ws_bytes, hipStream_t stream);
/* Free a plan (NULL accepted); work using it must have completed. */
ozk_status ozk_batch_plan_destroy(ozk_batch_plan* plan);
/* The tile of each problem of a plan: large[i] = 1 for 128 x 128, 0 for
 * 64 x 64 (HOST array of count = the plan's problem count). */
ozk_status ozk_batch_plan_tiles(const ozk_batch_plan* plan, int count,
                                int32_t* large);
/* Autotune a plan's tiles on its own problems (the paper tunes its kernel
 * parameters, Sec. V-A; its problems are not batched): run the pre-pass,
 * time the whole GEMM step (median of `reps` after one warm-up, HIP events)
 * with the plan's tiles, with every problem on the small tile and with
 * every problem on the large one, start from the fastest, then, size class
 * by size class in decreasing INT8 work, move the class's problems to the
 * other tile when that makes the whole step faster, and store each class's
 * tile in the context table (op OZK_OP_DGEMM_BATCHED /
 * OZK_OP_ZGEMM_BATCHED, variant 0 or 1, with the step time), where later
 * plans of the context find it.  The plan is
 * updated in place and the batch is computed with the chosen tiles.  Every
 * tile computes the same integers, so results do not depend on the choice.
 * Synchronises the stream (not graph-capturable).  Errors:
 * OZK_ERR_INVALID_ARG (arg 2 plan, 5 reps outside 1..100),
 * OZK_ERR_WORKSPACE (arg 3). */
ozk_status ozk_tune_batch(ozk_ctx* ctx, ozk_batch_plan* plan, void* ws,
                          size_t ws_bytes, int reps, hipStream_t stream);

/* -------------------------------------------------------- autotuner */
/* A GEMM configuration.  The paper picks its kernel parameters (M stacking,
 * N tile, swizzle, buffering stages; Table I) with an autotuner (Sec. V-A);
 * here the INT8 GEMM step of each
 * call takes its configuration from a per-context table keyed by the size
 * class (op, scheme, p or s, and ceil(log2) of M, N and K), filled by
 * ozk_tune, ozk_config_set or ozk_config_load; classes without an entry use
 * the default {0, 0, 4, 1}.  Every configuration computes the same integers,
 * so results are bit-identical whichever is used; only the time differs.
 *   variant: tile variant, Scheme I 0 .. OZK_S1_VARIANTS-1 (bit 1: the other
 *            wave-tile orientation, 128x64 <-> 128x128 for p <= 4 and
 *            128x64 <-> 64x128 for p >= 5; bit 0: one LDS stage fewer),
 *            Scheme II 0 .. OZK_S2_VARIANTS-1 (bit 1: the large tile,
 *            256x128 real (variant 3: 256x256), 128x128 3M, instead of
 *            128x128 / 128x64, taken only while K <= 131040 and replaced by
 *            the base tile beyond; bit 0: the other LDS staging depth: K
 *            chunks per stage and stages 2 x 4 (variant 0), 1 x 4 (1),
 *            2 x 4 or 3M 1 x 4 (2), 2 x 3 (3)); variants 5 and 6: the large
 *            tiles with other stagings (real 256x128 with 4 x 2, 256x256 with
 *            3 x 2; 3M 128x128 with 2 x 3, 1 x 6), replaced by variants 1 and
 *            0 beyond K = 131040; variant OZK_S2_FUSED_CRT (4)
 *            fuses the CRT into the GEMM of a real product (64x64 tiles
 *            running all s moduli, the CRT sums in registers, C written
 *            directly, no residue planes; the paper keeps the CRT in a
 *            kernel of its own for the register budget, Sec. IV-C) -- 3M
 *            products and the step entry points run variant 0 in its place,
 *            and ozk_tune does not try it;
 *   raster:  0 = tiles of one XCD form a compact block, 1 = dispatch order;
 *   group:   tile rows per raster group, 1 .. 64;
 *   split:   Scheme I only: at least this many K runs (their 128-bit partial
 *            sums are folded exactly; the workspace grows by 16*split*M*N
 *            bytes), 1 .. 64; Scheme II stores 1.
 * The table is host state of the context (not thread-safe: one context per
 * host thread).  ozk_workspace_size reflects the configuration of the size
 * class, so query it after tuning or setting. */
typedef struct ozk_gemm_config {
  int variant;
  int raster;
  int group;
  int split;
} ozk_gemm_config;

/* Store cfg for the size class of (M, N, K).  Scheme I needs op DGEMM. */
ozk_status ozk_config_set(ozk_ctx* ctx, ozk_op op, ozk_scheme scheme,
                          int p_or_s, int64_t M, int64_t N, int64_t K,
                          const ozk_gemm_config* cfg);
/* The configuration calls of this size class use (*found = 1 and *ms the
 * tuned time if an entry exists, else the default and *found = 0); found
 * and ms may be NULL. */
ozk_status ozk_config_get(ozk_ctx* ctx, ozk_op op, ozk_scheme scheme,
                          int p_or_s, int64_t M, int64_t N, int64_t K,
                          ozk_gemm_config* cfg, int* found, float* ms);
ozk_status ozk_config_clear(ozk_ctx* ctx);
/* Write / merge the table as JSON (a host file path). */
ozk_status ozk_config_save(ozk_ctx* ctx, const char* path);
ozk_status ozk_config_load(ozk_ctx* ctx, const char* path);
/* Workspace ozk_tune needs to try every candidate (smaller workspaces skip
 * the K splits that do not fit). */
ozk_status ozk_tune_workspace_size(ozk_ctx* ctx, ozk_op op, ozk_scheme scheme,
                                   int p_or_s, int64_t M, int64_t N, int64_t K,
                                   size_t* bytes);
/* Tune the size class of (M, N, K) on these operands: run the pre-pass
 * once, time the INT8 GEMM step (with the K-run fold) of every candidate
 * configuration -- variants x rasters x groups {2, 4, 8, 16} x K splits 1, 2, 4, 8
 * (Scheme I, while the partial sums fit 256 MiB) -- as the median of `reps`
 * runs after one warm-up, store the fastest in the table, and leave
 * C = A B (alpha 1, beta 0) computed with it.  Complex operands (ZGEMM,
 * Scheme II) are interleaved.  Unlike the other calls this one synchronises
 * the stream (HIP events) and must not be captured into a graph. */
ozk_status ozk_tune(ozk_ctx* ctx, ozk_op op, ozk_scheme scheme, int p_or_s,
                    int64_t M, int64_t N, int64_t K, const double* A,
                    int64_t lda, const double* B, int64_t ldb, double* C,
                    int64_t ldc, void* ws, size_t ws_bytes, int reps,
                    ozk_gemm_config* best, float* best_ms, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* OZK_H */
