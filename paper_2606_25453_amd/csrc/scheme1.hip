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
// slice at packed[r][k/32][t][k%32].  Rows past `rows` and k past K are zero.
template <int P>
__global__ __launch_bounds__(256) void k_s1_split_rows(const double* __restrict__ X, int64_t ldx,
                                                       int64_t rows, int64_t K, int64_t Kp,
                                                       int64_t rows_packed, int32_t* __restrict__ e_out,
                                                       int8_t* __restrict__ packed) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= rows_packed) return;
  const int64_t nchunk = Kp / OZK_K_CHUNK;
  int8_t* prow = packed + r * nchunk * (P * OZK_K_CHUNK);
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
      *reinterpret_cast<uint32_t*>(prow + (c * P + t) * OZK_K_CHUNK + kk) = word[t];
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
// into p x 32 digits and stores 32 bytes per slice at packed[j][c][t][:].
template <int P>
__global__ __launch_bounds__(256) void k_s1_split_cols(const double* __restrict__ X, int64_t ldx,
                                                       int64_t K, int64_t cols, int64_t Kp,
                                                       int64_t cols_packed, const int32_t* __restrict__ f,
                                                       int8_t* __restrict__ packed) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (j >= cols_packed) return;
  const int64_t nchunk = Kp / OZK_K_CHUNK;
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
  int8_t* dst = packed + (j * nchunk + c) * (P * OZK_K_CHUNK);
#pragma unroll
  for (int t = 0; t < P; ++t) {
    uint4* q = reinterpret_cast<uint4*>(dst + t * OZK_K_CHUNK);
    q[0] = make_uint4(word[t][0], word[t][1], word[t][2], word[t][3]);
    q[1] = make_uint4(word[t][4], word[t][5], word[t][6], word[t][7]);
  }
}

// ------------------------------------------------------------- fused GEMM

// Workgroup of 4 waves in a 2 x 2 grid; each wave owns a (32 TM) x (32 TN)
// block of the output and P INT32 accumulators (diagonals) per 32 x 32 tile.
// Per K step of 32 the workgroup stages BM x (P x 32) bytes of A and
// BN x (P x 32) bytes of B in LDS (two buffers, one barrier per step), each
// wave reads its P A-fragments and P B-fragments once and issues the
// P(P+1)/2 x TM x TN triangular MFMAs.
template <int P, int TM, int TN>
struct S1Tile {
  static constexpr int BM = 64 * TM;
  static constexpr int BN = 64 * TN;
  static constexpr int ROW_BYTES = P * OZK_K_CHUNK;   // one K step of one row
  static constexpr int LDS_STRIDE = ROW_BYTES + 16;   // 16 B pad: conflict-free b128 reads
  static constexpr int PIECES = (BM + BN) * ROW_BYTES / 16;
  static constexpr int PIECES_PER_THREAD = (PIECES + 255) / 256;
  static constexpr int LDS_BUF = (BM + BN) * LDS_STRIDE;
  static constexpr int LDS_BYTES = 2 * LDS_BUF;
};

enum S1Out { S1_OUT_FINAL = 0, S1_OUT_PARTIAL = 1, S1_OUT_DIAG = 2 };

template <int P, int TM, int TN, int OUT>
__global__ __launch_bounds__(256, 1) void k_s1_gemm(
    const int8_t* __restrict__ Ap, const int8_t* __restrict__ Bp, int64_t nchunk_total,
    int64_t steps_per_split, int M, int N, const int32_t* __restrict__ e_row,
    const int32_t* __restrict__ f_col, double alpha, double beta, double* __restrict__ C, int64_t ldc,
    int64_t* __restrict__ zpart, int32_t* __restrict__ diag) {
  using T = S1Tile<P, TM, TN>;
  extern __shared__ __attribute__((aligned(16))) int8_t lds[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t m0 = (int64_t)blockIdx.y * T::BM, n0 = (int64_t)blockIdx.x * T::BN;
  const int64_t step0 = (int64_t)blockIdx.z * steps_per_split;
  int64_t nsteps = nchunk_total - step0;
  if (nsteps > steps_per_split) nsteps = steps_per_split;
  const int64_t row_bytes_g = nchunk_total * T::ROW_BYTES;  // bytes per packed row

  // global -> register staging of one K step
  uint4 stage[T::PIECES_PER_THREAD];
  auto load_step = [&](int64_t s) {
#pragma unroll
    for (int q = 0; q < T::PIECES_PER_THREAD; ++q) {
      const int idx = tid + 256 * q;
      if (idx < T::PIECES) {
        const int row = idx / (2 * P), piece = idx % (2 * P);
        const int8_t* src = (row < T::BM) ? Ap + (m0 + row) * row_bytes_g
                                          : Bp + (n0 + row - T::BM) * row_bytes_g;
        stage[q] = *reinterpret_cast<const uint4*>(src + s * T::ROW_BYTES + piece * 16);
      }
    }
  };
  auto store_step = [&](int buf) {
    int8_t* base = lds + buf * T::LDS_BUF;
#pragma unroll
    for (int q = 0; q < T::PIECES_PER_THREAD; ++q) {
      const int idx = tid + 256 * q;
      if (idx < T::PIECES) {
        const int row = idx / (2 * P), piece = idx % (2 * P);
        *reinterpret_cast<uint4*>(base + row * T::LDS_STRIDE + piece * 16) = stage[q];
      }
    }
  };

  v16i acc[P][TM][TN];
#pragma unroll
  for (int d = 0; d < P; ++d)
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b) acc[d][a][b] = v16i{0};

  const int lrow = lane & 31, lk = 16 * (lane >> 5);
  if (nsteps > 0) {
    load_step(step0);
    store_step(0);
  }
  __syncthreads();
  for (int64_t s = 0; s < nsteps; ++s) {
    const int buf = (int)(s & 1);
    if (s + 1 < nsteps) load_step(step0 + s + 1);
    const int8_t* la = lds + buf * T::LDS_BUF;
    const int8_t* lb = la + T::BM * T::LDS_STRIDE;
    // All P A-fragments stay live; B slices are streamed one at a time and
    // slice u meets A slices t <= P-1-u, adding A_t B_u to diagonal t + u.
    v4i fa[P][TM];
#pragma unroll
    for (int t = 0; t < P; ++t)
#pragma unroll
      for (int a = 0; a < TM; ++a)
        fa[t][a] = *reinterpret_cast<const v4i*>(la + (wm * 32 * TM + a * 32 + lrow) * T::LDS_STRIDE +
                                                 t * OZK_K_CHUNK + lk);
#pragma unroll
    for (int u = 0; u < P; ++u) {
      v4i fb[TN];
#pragma unroll
      for (int b = 0; b < TN; ++b)
        fb[b] = *reinterpret_cast<const v4i*>(lb + (wn * 32 * TN + b * 32 + lrow) * T::LDS_STRIDE +
                                              u * OZK_K_CHUNK + lk);
#pragma unroll
      for (int t = 0; t + u < P; ++t)
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
          for (int b = 0; b < TN; ++b) acc[t + u][a][b] = mfma_i8_32x32x32(fa[t][a], fb[b], acc[t + u][a][b]);
    }
    if (s + 1 < nsteps) store_step(buf ^ 1);
    __syncthreads();
  }

  // epilogue
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = m0 + wm * 32 * TM + a * 32 + 8 * (v / 4) + 4 * (lane >> 5) + (v % 4);
        const int64_t col = n0 + wn * 32 * TN + b * 32 + (lane & 31);
        if (row >= M || col >= N) continue;
        if (OUT == S1_OUT_DIAG) {
#pragma unroll
          for (int d = 0; d < P; ++d) diag[((int64_t)d * M + row) * N + col] = acc[d][a][b][v];
          continue;
        }
        i128 Z = 0;
#pragma unroll
        for (int d = 0; d < P; ++d) Z += (i128)acc[d][a][b][v] << (8 * (P - 1 - d));
        if (OUT == S1_OUT_PARTIAL) {
          int64_t* zp = zpart + 2 * (((int64_t)blockIdx.z * M + row) * N + col);
          zp[0] = (int64_t)(uint64_t)(u128)Z;
          zp[1] = (int64_t)(Z >> 64);
          continue;
        }
        const int er = e_row[row], fc = f_col[col];
        double h;
        if (er == OZK_EXP_NONFINITE || fc == OZK_EXP_NONFINITE) h = __builtin_nan("");
        else if (er == OZK_EXP_ZERO || fc == OZK_EXP_ZERO) h = 0.0;
        else h = round_scaled(Z, er + fc - 12 - 8 * (P - 1));
        double* cp = C + row * ldc + col;
        *cp = axpby(alpha, h, beta, cp);
      }
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

template <int P, int TM, int TN, int OUT>
static hipError_t launch_gemm_t(const S1GemmArgs& g, hipStream_t st) {
  using T = S1Tile<P, TM, TN>;
  auto kern = k_s1_gemm<P, TM, TN, OUT>;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, T::LDS_BYTES);
    if (err != hipSuccess) return err;
    attr_set = true;
  }
  const dim3 grid((unsigned)((g.N + T::BN - 1) / T::BN), (unsigned)((g.M + T::BM - 1) / T::BM),
                  (unsigned)g.nsplit);
  hipLaunchKernelGGL(kern, grid, dim3(256), T::LDS_BYTES, st, g.Ap, g.Bp, g.nchunk, g.steps_per_split,
                     (int)g.M, (int)g.N, g.e, g.f, g.alpha, g.beta, g.C, g.ldc, g.zpart, g.diag);
  return hipGetLastError();
}

template <int P, int OUT>
static hipError_t launch_gemm_p(const S1GemmArgs& g, hipStream_t st) {
  if constexpr (P <= 4) return launch_gemm_t<P, 2, 2, OUT>(g, st);
  else return launch_gemm_t<P, 2, 1, OUT>(g, st);
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
