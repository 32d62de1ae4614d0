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

// One wave per packed row.  Pass 1: exponent of the row (wave max).  Pass 2:
// each lane turns 4 consecutive k into p digits and stores 4 bytes per
// slice at packed[k/32][t][r][k%32].  Rows past `rows` and k past K are zero.
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
__global__ __launch_bounds__(256) void k_s1_split_cols(const double* __restrict__ X, int64_t ldx,
                                                       int64_t K, int64_t cols, int64_t Kp,
                                                       int64_t cols_packed, const int32_t* __restrict__ f,
                                                       int8_t* __restrict__ packed) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (j >= cols_packed) return;
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

template <int P, int OUT>
__global__ __launch_bounds__(256, 1) void k_s1_gemm(
    const int8_t* __restrict__ Ap, const int8_t* __restrict__ Bp, int64_t rows_a, int64_t rows_b,
    int64_t nchunk_total, int64_t steps_per_split, int M, int N, const int32_t* __restrict__ e_row,
    const int32_t* __restrict__ f_col, double alpha, double beta, double* __restrict__ C, int64_t ldc,
    int64_t* __restrict__ zpart, int32_t* __restrict__ diag) {
  using Cfg = S1Cfg<P>;
  constexpr int TM = Cfg::TM, TN = Cfg::TN, NS = Cfg::NS;
  using T = GemmTile<P, TM, TN, NS>;
  extern __shared__ __attribute__((aligned(1024))) int8_t lds[];
  const int64_t tiles_m = (M + T::BM - 1) / T::BM, tiles_n = (N + T::BN - 1) / T::BN;
  int64_t tm, tn;
  tile_of(blockIdx.x, tiles_m, tiles_n, tm, tn);
  const int64_t m0 = tm * T::BM, n0 = tn * T::BN;
  const int64_t step0 = (int64_t)blockIdx.z * steps_per_split;
  int64_t nsteps = nchunk_total - step0;
  if (nsteps > steps_per_split) nsteps = steps_per_split;

  v16i acc[P][TM][TN];
  zero_acc<P, TM, TN>(acc);
  gemm_tile_accumulate<P, TM, TN, NS, TRIANGULAR>(Ap, Bp, rows_a, rows_b, m0, n0, step0, nsteps, lds, acc);

  for_each_output<P, TM, TN>(acc, m0, n0, M, N, [&](int64_t row, int64_t col, const int* vals) {
    if (OUT == S1_OUT_DIAG) {
#pragma unroll
      for (int d = 0; d < P; ++d) diag[((int64_t)d * M + row) * N + col] = vals[d];
      return;
    }
    i128 Z = 0;
#pragma unroll
    for (int d = 0; d < P; ++d) Z += (i128)vals[d] << (8 * (P - 1 - d));
    if (OUT == S1_OUT_PARTIAL) {
      int64_t* zp = zpart + 2 * (((int64_t)blockIdx.z * M + row) * N + col);
      zp[0] = (int64_t)(uint64_t)(u128)Z;
      zp[1] = (int64_t)(Z >> 64);
      return;
    }
    const int er = e_row[row], fc = f_col[col];
    double h;
    if (er == OZK_EXP_NONFINITE || fc == OZK_EXP_NONFINITE) h = __builtin_nan("");
    else if (er == OZK_EXP_ZERO || fc == OZK_EXP_ZERO) h = 0.0;
    else h = round_scaled(Z, er + fc - 12 - 8 * (P - 1));
    double* cp = C + row * ldc + col;
    *cp = axpby(alpha, h, beta, cp);
  });
}

// Exact fold of the K-run partials followed by the single rounding.
__global__ __launch_bounds__(256) void k_s1_fold(const int64_t* __restrict__ zpart, int nsplit, int M, int N,
                                                 int p, const int32_t* __restrict__ e_row,
                                                 const int32_t* __restrict__ f_col, double alpha,
                                                 double beta, double* __restrict__ C, int64_t ldc) {
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
  hipLaunchKernelGGL(kern, grid, dim3(256), T::LDS_BYTES, st, g.Ap, g.Bp, round_up(g.M, OZK_ROW_ALIGN),
                     round_up(g.N, OZK_ROW_ALIGN), g.nchunk, g.steps_per_split, (int)g.M, (int)g.N, g.e, g.f,
                     g.alpha, g.beta, g.C, g.ldc, g.zpart, g.diag);
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
                       (int)g.M, (int)g.N, p, g.e, g.f, g.alpha, g.beta, g.C, g.ldc);
    return hipGetLastError();
  }
  return launch_gemm_out<S1_OUT_FINAL>(p, g, st);
}

}  // namespace ozk
