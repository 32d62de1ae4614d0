// Ozaki Scheme I on gfx950 INT8 MFMA (paper Sec. II-C.1 and Sec. III).
//
//   k_s1_split_rows   row exponents + balanced 8-bit slices of a row operand,
//                     written in the interleaved packed layout (Eq. 11)
//   k_s1_exp_cols     column exponents of a column operand (atomic max)
//   k_s1_split_cols   slices of a column operand, transposed on the fly
//   k_s1_gemm         fused kernel: p(p+1)/2 slice-pair MFMAs per K step into
//                     p INT32 diagonals kept in registers (Alg. 1), then the
//                     exact integer shift-reduce and one rounding per output
//   k_s1_fold         exact sum of the per-K-run 128-bit partials (long K)
#include "mfma_gemm.hpp"
#include "ozk_device.hpp"
#include "ozk_internal.hpp"

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
  if (r >= rows_packed) return;
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
  if (j >= cols_packed) return;
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

// ------------------------------------------------------------- fused GEMM

template <int P>
struct S1Cfg {
  // p <= 4: 2 x 2 MFMA tiles per wave (128 x 128 workgroup tile, 16p*4 acc
  // registers); p >= 5: 2 x 1 (128 x 64).  Stages: as many as fit 160 KB.
  static constexpr int TM = 2;
  static constexpr int TN = P <= 4 ? 2 : 1;
  static constexpr int NS = P <= 2 ? 4 : 3;
};

enum S1Out { S1_OUT_FINAL = 0, S1_OUT_PARTIAL = 1, S1_OUT_DIAG = 2 };

struct S1KArgs {
  const int8_t* Ap;
  const int8_t* Bp;
  int64_t rows_a, rows_b, nchunk_total, steps_per_split;
  int M, N;
  const int32_t* e_row;
  const int32_t* f_col;
  double alpha, beta;
  double* C;
  int64_t ldc;
  int64_t* zpart;
  int32_t* diag;
};

// One output tile (workgroup tile index `tile`, K run z): the triangular
// MFMA accumulation, then the epilogue selected by OUT.
template <int P, int OUT, int TM, int TN, int NS>
__device__ __forceinline__ void s1_gemm_tile(const S1KArgs& g, int64_t tile, int64_t z, int8_t* lds) {
  using T = GemmTile<P, TM, TN, NS>;
  const int64_t M = g.M, N = g.N;
  const int64_t tiles_m = (M + T::BM - 1) / T::BM, tiles_n = (N + T::BN - 1) / T::BN;
  int64_t tm, tn;
  tile_of(tile, tiles_m, tiles_n, tm, tn);
  const int64_t m0 = tm * T::BM, n0 = tn * T::BN;
  const int64_t step0 = z * g.steps_per_split;
  int64_t nsteps = g.nchunk_total - step0;
  if (nsteps > g.steps_per_split) nsteps = g.steps_per_split;

  v16i acc[P][TM][TN];
  zero_acc<P, TM, TN>(acc);
  gemm_tile_accumulate<P, TM, TN, NS, TRIANGULAR>(g.Ap, g.Bp, g.rows_a, g.rows_b, m0, n0, step0, nsteps, lds, acc);

  for_each_output<P, TM, TN>(acc, m0, n0, M, N, [&](int64_t row, int64_t col, const int* vals) {
    if (OUT == S1_OUT_DIAG) {
#pragma unroll
      for (int d = 0; d < P; ++d) g.diag[((int64_t)d * M + row) * N + col] = vals[d];
      return;
    }
    i128 Z = 0;
#pragma unroll
    for (int d = 0; d < P; ++d) Z += (i128)vals[d] << (8 * (P - 1 - d));
    if (OUT == S1_OUT_PARTIAL) {
      int64_t* zp = g.zpart + 2 * ((z * M + row) * N + col);
      zp[0] = (int64_t)(uint64_t)(u128)Z;
      zp[1] = (int64_t)(Z >> 64);
      return;
    }
    const int er = g.e_row[row], fc = g.f_col[col];
    double h;
    if (er == OZK_EXP_NONFINITE || fc == OZK_EXP_NONFINITE) h = __builtin_nan("");
    else if (er == OZK_EXP_ZERO || fc == OZK_EXP_ZERO) h = 0.0;
    else h = round_scaled(Z, er + fc - 12 - 8 * (P - 1));
    double* cp = g.C + row * g.ldc + col;
    *cp = axpby(g.alpha, h, g.beta, cp);
  });
}

template <int P, int OUT>
__global__ __launch_bounds__(256, 1) void k_s1_gemm(S1KArgs g) {
  using Cfg = S1Cfg<P>;
  extern __shared__ __attribute__((aligned(1024))) int8_t lds[];
  s1_gemm_tile<P, OUT, Cfg::TM, Cfg::TN, Cfg::NS>(g, blockIdx.x, blockIdx.z, lds);
}

// The slice count read from device memory: one tiling for every p (128 x 64,
// 3 stages, LDS sized for p = 8).
constexpr int S1_AUTO_TM = 2, S1_AUTO_TN = 1, S1_AUTO_NS = 3;
using S1AutoTile = GemmTile<8, S1_AUTO_TM, S1_AUTO_TN, S1_AUTO_NS>;

template <int OUT>
__global__ __launch_bounds__(256, 1) void k_s1_gemm_auto(S1KArgs g, const int32_t* __restrict__ p_dev) {
  extern __shared__ __attribute__((aligned(1024))) int8_t lds[];
  const int64_t tile = blockIdx.x, z = blockIdx.z;
  switch (*p_dev) {
    case 1: s1_gemm_tile<1, OUT, S1_AUTO_TM, S1_AUTO_TN, S1_AUTO_NS>(g, tile, z, lds); break;
    case 2: s1_gemm_tile<2, OUT, S1_AUTO_TM, S1_AUTO_TN, S1_AUTO_NS>(g, tile, z, lds); break;
    case 3: s1_gemm_tile<3, OUT, S1_AUTO_TM, S1_AUTO_TN, S1_AUTO_NS>(g, tile, z, lds); break;
    case 4: s1_gemm_tile<4, OUT, S1_AUTO_TM, S1_AUTO_TN, S1_AUTO_NS>(g, tile, z, lds); break;
    case 5: s1_gemm_tile<5, OUT, S1_AUTO_TM, S1_AUTO_TN, S1_AUTO_NS>(g, tile, z, lds); break;
    case 6: s1_gemm_tile<6, OUT, S1_AUTO_TM, S1_AUTO_TN, S1_AUTO_NS>(g, tile, z, lds); break;
    case 7: s1_gemm_tile<7, OUT, S1_AUTO_TM, S1_AUTO_TN, S1_AUTO_NS>(g, tile, z, lds); break;
    default: s1_gemm_tile<8, OUT, S1_AUTO_TM, S1_AUTO_TN, S1_AUTO_NS>(g, tile, z, lds); break;
  }
}

// Exact fold of the K-run partials followed by the single rounding.
__global__ __launch_bounds__(256) void k_s1_fold(const int64_t* __restrict__ zpart, int nsplit, int M, int N,
                                                 int p, const int32_t* __restrict__ p_dev,
                                                 const int32_t* __restrict__ e_row,
                                                 const int32_t* __restrict__ f_col, double alpha,
                                                 double beta, double* __restrict__ C, int64_t ldc) {
  if (p_dev) p = *p_dev;
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

static S1KArgs kargs_of(const S1GemmArgs& g) {
  S1KArgs k;
  k.Ap = g.Ap;
  k.Bp = g.Bp;
  k.rows_a = round_up(g.M, OZK_ROW_ALIGN);
  k.rows_b = round_up(g.N, OZK_ROW_ALIGN);
  k.nchunk_total = g.nchunk;
  k.steps_per_split = g.steps_per_split;
  k.M = (int)g.M;
  k.N = (int)g.N;
  k.e_row = g.e;
  k.f_col = g.f;
  k.alpha = g.alpha;
  k.beta = g.beta;
  k.C = g.C;
  k.ldc = g.ldc;
  k.zpart = g.zpart;
  k.diag = g.diag;
  return k;
}

template <int P, int OUT>
static hipError_t launch_gemm_p(const S1GemmArgs& g, hipStream_t st) {
  using Cfg = S1Cfg<P>;
  using T = GemmTile<P, Cfg::TM, Cfg::TN, Cfg::NS>;
  auto kern = k_s1_gemm<P, OUT>;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, T::LDS_BYTES);
    if (err != hipSuccess) return err;
    attr_set = true;
  }
  const int64_t tiles = ((g.M + T::BM - 1) / T::BM) * ((g.N + T::BN - 1) / T::BN);
  const dim3 grid((unsigned)tiles, 1, (unsigned)g.nsplit);
  hipLaunchKernelGGL(kern, grid, dim3(256), T::LDS_BYTES, st, kargs_of(g));
  return hipGetLastError();
}

template <int OUT>
static hipError_t launch_gemm_out(int p, const S1GemmArgs& g, hipStream_t st) {
  switch (p) {
    case 1: return launch_gemm_p<1, OUT>(g, st);
    case 2: return launch_gemm_p<2, OUT>(g, st);
    case 3: return launch_gemm_p<3, OUT>(g, st);
    case 4: return launch_gemm_p<4, OUT>(g, st);
    case 5: return launch_gemm_p<5, OUT>(g, st);
    case 6: return launch_gemm_p<6, OUT>(g, st);
    case 7: return launch_gemm_p<7, OUT>(g, st);
    case 8: return launch_gemm_p<8, OUT>(g, st);
  }
  return hipErrorInvalidValue;
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

hipError_t s1_gemm(int p, const S1GemmArgs& g, hipStream_t st) {
  if (g.M == 0 || g.N == 0) return hipSuccess;
  if (g.diag) return launch_gemm_out<S1_OUT_DIAG>(p, g, st);
  if (g.nsplit > 1) {
    hipError_t err = launch_gemm_out<S1_OUT_PARTIAL>(p, g, st);
    if (err != hipSuccess) return err;
    const int64_t n = g.M * g.N;
    hipLaunchKernelGGL(k_s1_fold, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g.zpart, (int)g.nsplit,
                       (int)g.M, (int)g.N, p, (const int32_t*)nullptr, g.e, g.f, g.alpha, g.beta, g.C, g.ldc);
    return hipGetLastError();
  }
  return launch_gemm_out<S1_OUT_FINAL>(p, g, st);
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

hipError_t s1_gemm_auto(const int32_t* p_dev, const S1GemmArgs& g, hipStream_t st) {
  if (g.M == 0 || g.N == 0) return hipSuccess;
  using T = S1AutoTile;
  static bool attr[2] = {false, false};
  const bool part = g.nsplit > 1;
  if (!attr[part]) {
    hipError_t err = part ? hipFuncSetAttribute(reinterpret_cast<const void*>(k_s1_gemm_auto<S1_OUT_PARTIAL>),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, T::LDS_BYTES)
                          : hipFuncSetAttribute(reinterpret_cast<const void*>(k_s1_gemm_auto<S1_OUT_FINAL>),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, T::LDS_BYTES);
    if (err != hipSuccess) return err;
    attr[part] = true;
  }
  const int64_t tiles = ((g.M + T::BM - 1) / T::BM) * ((g.N + T::BN - 1) / T::BN);
  const dim3 grid((unsigned)tiles, 1, (unsigned)g.nsplit);
  if (!part) {
    hipLaunchKernelGGL(k_s1_gemm_auto<S1_OUT_FINAL>, grid, dim3(256), T::LDS_BYTES, st, kargs_of(g), p_dev);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_s1_gemm_auto<S1_OUT_PARTIAL>, grid, dim3(256), T::LDS_BYTES, st, kargs_of(g), p_dev);
  const int64_t n = g.M * g.N;
  hipLaunchKernelGGL(k_s1_fold, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g.zpart, (int)g.nsplit,
                     (int)g.M, (int)g.N, 8, p_dev, g.e, g.f, g.alpha, g.beta, g.C, g.ldc);
  return hipGetLastError();
}

}  // namespace ozk
