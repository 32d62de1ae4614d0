// Ozaki Scheme I on gfx950 INT8 MFMA (paper Sec. II-C.1 and Sec. III).
//
//   k_s1_split_rows   row exponents + balanced 8-bit slices of a row operand,
//                     written in the interleaved packed layout (Eq. 11)
//   k_s1_exp_cols     column exponents of a column operand (atomic max)
//   k_s1_split_cols   slices of a column operand, transposed on the fly
//   k_s1_gemm         fused kernel (s1_gemm.hpp, instantiated per p in
//                     s1_gemm_inst.hip): p(p+1)/2 slice-pair MFMAs per K step
//                     into p INT32 diagonals kept in registers (Alg. 1), then
//                     the exact integer shift-reduce and one rounding per output
//   k_s1_fold         exact sum of the per-K-run 128-bit partials (long K)
#include "ozk_device.hpp"
#include "ozk_internal.hpp"
#include "s1_gemm.hpp"

namespace ozk {

// ---------------------------------------------------------------- pre-pass

// Balanced base-256 digits of X = floor(x 2^(8p-2-e) + 1/2): digit t is
// written to byte t of `out` (p bytes).
template <int P>
__device__ __forceinline__ void s1_digits(double x, int e, int8_t (&out)[P]) {
  int64_t X = 0;
  if (e != OZK_EXP_ZERO && e != OZK_EXP_NONFINITE) X = round_half_up_scaled(x, 8 * P - 2 - e);
#pragma unroll
  for (int t = P - 1; t >= 1; --t) {
    const int64_t d = ((X + 128) & 255) - 128;
    out[t] = (int8_t)d;
    X = (X - d) >> 8;  // exact
  }
  out[0] = (int8_t)X;
}

// Slices of packed row r whose exponent is e: each lane turns 4 consecutive
// k into p digits and stores 4 bytes per slice at packed[k/32][t][r][k%32].
// Rows past `rows` and k past K are zero.
template <int P>
__device__ __forceinline__ void s1_slice_row(const double* __restrict__ xr, int64_t r, int64_t rows, int64_t K,
                                             int64_t Kp, int64_t rows_packed, int e, int8_t* __restrict__ packed) {
  const int lane = threadIdx.x & 63;
#pragma unroll 4
  for (int64_t k0 = (int64_t)lane * 4; k0 < Kp; k0 += 256) {
    uint32_t word[P];
#pragma unroll
    for (int t = 0; t < P; ++t) word[t] = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t k = k0 + j;
      const double v = (r < rows && k < K) ? xr[k] : 0.0;
      int8_t d[P];
      s1_digits<P>(v, e, d);
#pragma unroll
      for (int t = 0; t < P; ++t) word[t] |= (uint32_t)(uint8_t)d[t] << (8 * j);
    }
    const int64_t c = k0 / OZK_K_CHUNK, kk = k0 % OZK_K_CHUNK;
#pragma unroll
    for (int t = 0; t < P; ++t)
      *reinterpret_cast<uint32_t*>(packed + ((c * P + t) * rows_packed + r) * OZK_K_CHUNK + kk) = word[t];
  }
}

// One wave per packed row: the row exponent (wave max), then the slices.
template <int P>
__global__ __launch_bounds__(256) void k_s1_split_rows(const double* __restrict__ X, int64_t ldx,
                                                       int64_t rows, int64_t K, int64_t Kp,
                                                       int64_t rows_packed, int32_t* __restrict__ e_out,
                                                       int8_t* __restrict__ packed) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= rows_packed) return;
  int e = OZK_EXP_ZERO;
  const double* xr = X + r * ldx;
  if (r < rows) {
#pragma unroll 8
    for (int64_t k = lane; k < K; k += 64) {
      const int ek = expo_of(xr[k]);
      e = ek > e ? ek : e;
    }
    e = wave_max(e);
    if (lane == 0) e_out[r] = e;
  }
  s1_slice_row<P>(xr, r, rows, K, Kp, rows_packed, e, packed);
}

// Slices with p and the row exponents read from device memory (the slice
// count chosen on the device by the selector).
__global__ __launch_bounds__(256) void k_s1_slice_rows_auto(const double* __restrict__ X, int64_t ldx, int64_t rows,
                                                            int64_t K, int64_t Kp, int64_t rows_packed,
                                                            const int32_t* __restrict__ e_in,
                                                            const int32_t* __restrict__ p_dev,
                                                            int8_t* __restrict__ packed) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= rows_packed || *p_dev < 1) return;  // p = 0: Scheme II was chosen
  const int e = r < rows ? e_in[r] : OZK_EXP_ZERO;
  const double* xr = X + r * ldx;
  switch (*p_dev) {
    case 1: s1_slice_row<1>(xr, r, rows, K, Kp, rows_packed, e, packed); break;
    case 2: s1_slice_row<2>(xr, r, rows, K, Kp, rows_packed, e, packed); break;
    case 3: s1_slice_row<3>(xr, r, rows, K, Kp, rows_packed, e, packed); break;
    case 4: s1_slice_row<4>(xr, r, rows, K, Kp, rows_packed, e, packed); break;
    case 5: s1_slice_row<5>(xr, r, rows, K, Kp, rows_packed, e, packed); break;
    case 6: s1_slice_row<6>(xr, r, rows, K, Kp, rows_packed, e, packed); break;
    case 7: s1_slice_row<7>(xr, r, rows, K, Kp, rows_packed, e, packed); break;
    default: s1_slice_row<8>(xr, r, rows, K, Kp, rows_packed, e, packed); break;
  }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Column exponents: thread j scans a run of 256 rows of column j.
__global__ __launch_bounds__(256) void k_s1_exp_cols(const double* __restrict__ X, int64_t ldx,
                                                     int64_t K, int64_t cols, int32_t* __restrict__ f) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= cols) return;
  const int64_t k0 = (int64_t)blockIdx.y * 256;
  const int64_t k1 = k0 + 256 < K ? k0 + 256 : K;
  int e = OZK_EXP_ZERO;
#pragma unroll 8
  for (int64_t k = k0; k < k1; ++k) {
    const int ek = expo_of(X[k * ldx + j]);
    e = ek > e ? ek : e;
  }
  if (e != OZK_EXP_ZERO) atomicMax(&f[j], e);
}

// Column operand slices: thread (j, c) turns the 32 k of chunk c of column j
// into p x 32 digits and stores 32 bytes per slice at packed[c][t][j][:]
// (consecutive threads write consecutive 32-byte lines).
template <int P>
__device__ __forceinline__ void s1_slice_col(const double* __restrict__ X, int64_t ldx, int64_t K, int64_t cols,
                                             int64_t cols_packed, const int32_t* __restrict__ f,
                                             int8_t* __restrict__ packed, int64_t j, int64_t c) {
  const int e = j < cols ? f[j] : OZK_EXP_ZERO;
  uint32_t word[P][8];
#pragma unroll
  for (int t = 0; t < P; ++t)
#pragma unroll
    for (int w = 0; w < 8; ++w) word[t][w] = 0;
#pragma unroll
  for (int kk = 0; kk < OZK_K_CHUNK; ++kk) {
    const int64_t k = c * OZK_K_CHUNK + kk;
    const double v = (j < cols && k < K) ? X[k * ldx + j] : 0.0;
    int8_t d[P];
    s1_digits<P>(v, e, d);
#pragma unroll
    for (int t = 0; t < P; ++t) word[t][kk / 4] |= (uint32_t)(uint8_t)d[t] << (8 * (kk % 4));
  }
#pragma unroll
  for (int t = 0; t < P; ++t) {
    uint4* q = reinterpret_cast<uint4*>(packed + ((c * P + t) * cols_packed + j) * OZK_K_CHUNK);
    q[0] = make_uint4(word[t][0], word[t][1], word[t][2], word[t][3]);
    q[1] = make_uint4(word[t][4], word[t][5], word[t][6], word[t][7]);
  }
}

template <int P>
__global__ __launch_bounds__(256) void k_s1_split_cols(const double* __restrict__ X, int64_t ldx,
                                                       int64_t K, int64_t cols, int64_t Kp,
                                                       int64_t cols_packed, const int32_t* __restrict__ f,
                                                       int8_t* __restrict__ packed) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= cols_packed) return;
  s1_slice_col<P>(X, ldx, K, cols, cols_packed, f, packed, j, blockIdx.y);
}

__global__ __launch_bounds__(256) void k_s1_split_cols_auto(const double* __restrict__ X, int64_t ldx, int64_t K,
                                                            int64_t cols, int64_t Kp, int64_t cols_packed,
                                                            const int32_t* __restrict__ f,
                                                            const int32_t* __restrict__ p_dev,
                                                            int8_t* __restrict__ packed) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= cols_packed || *p_dev < 1) return;  // p = 0: Scheme II was chosen
  const int64_t c = blockIdx.y;
  switch (*p_dev) {
    case 1: s1_slice_col<1>(X, ldx, K, cols, cols_packed, f, packed, j, c); break;
    case 2: s1_slice_col<2>(X, ldx, K, cols, cols_packed, f, packed, j, c); break;
    case 3: s1_slice_col<3>(X, ldx, K, cols, cols_packed, f, packed, j, c); break;
    case 4: s1_slice_col<4>(X, ldx, K, cols, cols_packed, f, packed, j, c); break;
    case 5: s1_slice_col<5>(X, ldx, K, cols, cols_packed, f, packed, j, c); break;
    case 6: s1_slice_col<6>(X, ldx, K, cols, cols_packed, f, packed, j, c); break;
    case 7: s1_slice_col<7>(X, ldx, K, cols, cols_packed, f, packed, j, c); break;
    default: s1_slice_col<8>(X, ldx, K, cols, cols_packed, f, packed, j, c); break;
  }
}

// Exact fold of the K-run partials followed by the single rounding.
__global__ __launch_bounds__(256) void k_s1_fold(const int64_t* __restrict__ zpart, int nsplit, int M, int N,
                                                 int p, const int32_t* __restrict__ p_dev,
                                                 const int32_t* __restrict__ e_row,
                                                 const int32_t* __restrict__ f_col, double alpha,
                                                 double beta, double* __restrict__ C, int64_t ldc) {
  if (p_dev) p = *p_dev;
  if (p < 1) return;  // Scheme II was chosen
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)M * N) return;
  const int64_t row = idx / N, col = idx % N;
  i128 Z = 0;
  for (int z = 0; z < nsplit; ++z) {
    const int64_t* zp = zpart + 2 * ((int64_t)z * M * N + idx);
    Z += ((i128)zp[1] << 64) | (i128)(uint64_t)zp[0];
  }
  const int er = e_row[row], fc = f_col[col];
  double h;
  if (er == OZK_EXP_NONFINITE || fc == OZK_EXP_NONFINITE) h = __builtin_nan("");
  else if (er == OZK_EXP_ZERO || fc == OZK_EXP_ZERO) h = 0.0;
  else h = round_scaled(Z, er + fc - 12 - 8 * (p - 1));
  double* cp = C + row * ldc + col;
  *cp = axpby(alpha, h, beta, cp);
}

// ------------------------------------------------------------- launchers

template <int P>
static hipError_t launch_split_rows(const double* X, int64_t ldx, int64_t rows, int64_t K, int32_t* e,
                                    int8_t* packed, hipStream_t st) {
  const int64_t rp = round_up(rows, OZK_ROW_ALIGN), kp = round_up(K, OZK_K_CHUNK);
  if (rp == 0) return hipSuccess;  // with K == 0 the launch still writes the exponents
  hipLaunchKernelGGL(k_s1_split_rows<P>, dim3((unsigned)(rp / 4)), dim3(256), 0, st, X, ldx, rows, K, kp, rp, e,
                     packed);
  return hipGetLastError();
}

template <int P>
static hipError_t launch_split_cols(const double* X, int64_t ldx, int64_t K, int64_t cols, int32_t* f,
                                    int8_t* packed, hipStream_t st) {
  const int64_t cp = round_up(cols, OZK_ROW_ALIGN), kp = round_up(K, OZK_K_CHUNK);
  if (cols > 0) {
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((cols + 255) / 256)), dim3(256), 0, st, f, cols,
                       (int32_t)OZK_EXP_ZERO);
    if (K > 0)
      hipLaunchKernelGGL(k_s1_exp_cols, dim3((unsigned)((cols + 255) / 256), (unsigned)((K + 255) / 256)),
                         dim3(256), 0, st, X, ldx, K, cols, f);
  }
  if (cp > 0 && kp > 0)
    hipLaunchKernelGGL(k_s1_split_cols<P>, dim3((unsigned)(cp / 256), (unsigned)(kp / OZK_K_CHUNK)), dim3(256),
                       0, st, X, ldx, K, cols, kp, cp, f, packed);
  return hipGetLastError();
}

hipError_t s1_split_rows(int p, const double* X, int64_t ldx, int64_t rows, int64_t K, int32_t* e,
                         int8_t* packed, hipStream_t st) {
  switch (p) {
    case 1: return launch_split_rows<1>(X, ldx, rows, K, e, packed, st);
    case 2: return launch_split_rows<2>(X, ldx, rows, K, e, packed, st);
    case 3: return launch_split_rows<3>(X, ldx, rows, K, e, packed, st);
    case 4: return launch_split_rows<4>(X, ldx, rows, K, e, packed, st);
    case 5: return launch_split_rows<5>(X, ldx, rows, K, e, packed, st);
    case 6: return launch_split_rows<6>(X, ldx, rows, K, e, packed, st);
    case 7: return launch_split_rows<7>(X, ldx, rows, K, e, packed, st);
    case 8: return launch_split_rows<8>(X, ldx, rows, K, e, packed, st);
  }
  return hipErrorInvalidValue;
}

hipError_t s1_split_cols(int p, const double* X, int64_t ldx, int64_t K, int64_t cols, int32_t* f,
                         int8_t* packed, hipStream_t st) {
  switch (p) {
    case 1: return launch_split_cols<1>(X, ldx, K, cols, f, packed, st);
    case 2: return launch_split_cols<2>(X, ldx, K, cols, f, packed, st);
    case 3: return launch_split_cols<3>(X, ldx, K, cols, f, packed, st);
    case 4: return launch_split_cols<4>(X, ldx, K, cols, f, packed, st);
    case 5: return launch_split_cols<5>(X, ldx, K, cols, f, packed, st);
    case 6: return launch_split_cols<6>(X, ldx, K, cols, f, packed, st);
    case 7: return launch_split_cols<7>(X, ldx, K, cols, f, packed, st);
    case 8: return launch_split_cols<8>(X, ldx, K, cols, f, packed, st);
  }
  return hipErrorInvalidValue;
}

static hipError_t gemm_launch(int p, int out, const S1GemmArgs& g, const int32_t* p_dev, hipStream_t st) {
  switch (p) {
    case 1: return s1_gemm_launch<1>(out, g, p_dev, st);
    case 2: return s1_gemm_launch<2>(out, g, p_dev, st);
    case 3: return s1_gemm_launch<3>(out, g, p_dev, st);
    case 4: return s1_gemm_launch<4>(out, g, p_dev, st);
    case 5: return s1_gemm_launch<5>(out, g, p_dev, st);
    case 6: return s1_gemm_launch<6>(out, g, p_dev, st);
    case 7: return s1_gemm_launch<7>(out, g, p_dev, st);
    case 8: return s1_gemm_launch<8>(out, g, p_dev, st);
  }
  return hipErrorInvalidValue;
}

static hipError_t launch_fold(int p, const int32_t* p_dev, const S1GemmArgs& g, hipStream_t st) {
  const int64_t n = g.M * g.N;
  hipLaunchKernelGGL(k_s1_fold, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g.zpart, (int)g.nsplit,
                     (int)g.M, (int)g.N, p, p_dev, g.e, g.f, g.alpha, g.beta, g.C, g.ldc);
  return hipGetLastError();
}

hipError_t s1_gemm(int p, const S1GemmArgs& g, hipStream_t st) {
  if (g.M == 0 || g.N == 0) return hipSuccess;
  if (g.diag) return gemm_launch(p, S1_OUT_DIAG, g, nullptr, st);
  if (g.nsplit > 1) {
    hipError_t err = gemm_launch(p, S1_OUT_PARTIAL, g, nullptr, st);
    return err == hipSuccess ? launch_fold(p, nullptr, g, st) : err;
  }
  return gemm_launch(p, S1_OUT_FINAL, g, nullptr, st);
}

// ---------------------------------------------------- slice count on device

hipError_t s1_slice_auto(const int32_t* p_dev, const double* A, int64_t lda, int64_t M, const double* B, int64_t ldb,
                         int64_t N, int64_t K, const int32_t* e, const int32_t* f, int8_t* Ap, int8_t* Bp,
                         hipStream_t st) {
  const int64_t ra = round_up(M, OZK_ROW_ALIGN), rb = round_up(N, OZK_ROW_ALIGN), kp = round_up(K, OZK_K_CHUNK);
  if (ra > 0 && kp > 0)
    hipLaunchKernelGGL(k_s1_slice_rows_auto, dim3((unsigned)(ra / 4)), dim3(256), 0, st, A, lda, M, K, kp, ra, e,
                       p_dev, Ap);
  if (rb > 0 && kp > 0)
    hipLaunchKernelGGL(k_s1_split_cols_auto, dim3((unsigned)(rb / 256), (unsigned)(kp / OZK_K_CHUNK)), dim3(256), 0,
                       st, B, ldb, K, N, kp, rb, f, p_dev, Bp);
  return hipGetLastError();
}

// Every fixed-p kernel is launched; each returns at once unless p_dev holds
// its slice count, so the chosen p runs with its own tiling and no host
// round trip.
static hipError_t launch_gemm_all(int out, const int32_t* p_dev, const S1GemmArgs& g, hipStream_t st) {
  hipError_t err = hipSuccess;
  for (int p = 1; p <= OZK_MAX_P && err == hipSuccess; ++p) err = gemm_launch(p, out, g, p_dev, st);
  return err;
}

hipError_t s1_gemm_auto(const int32_t* p_dev, const S1GemmArgs& g, hipStream_t st) {
  if (g.M == 0 || g.N == 0) return hipSuccess;
  if (g.nsplit <= 1) return launch_gemm_all(S1_OUT_FINAL, p_dev, g, st);
  hipError_t err = launch_gemm_all(S1_OUT_PARTIAL, p_dev, g, st);
  return err == hipSuccess ? launch_fold(OZK_MAX_P, p_dev, g, st) : err;
}

}  // namespace ozk
