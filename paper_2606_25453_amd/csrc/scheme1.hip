// Ozaki Scheme I on gfx950 INT8 MFMA (paper Sec. II-C.1 and Sec. III).
//
//   k_s1_split_rows4  row exponents + balanced 8-bit slices of a row operand,
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

// Balanced base-256 digits of X = floor(x 2^(8p-2-e) + 1/2) for 4
// consecutive entries of a line with exponent e (finite, non-zero line),
// packed per slice: word t holds digit t of entry j in byte j.  With
// u = X + 128 (256^(p-2) + ... + 256 + 1), byte p-1-t of u is d_t + 128 for
// t >= 1 (the biased low digits never borrow) and byte p-1, read as a signed
// byte, is d_0 (|X| <= 2^(8p-2) keeps it in [-64, 64]).  Entries equal to
// zero give zero words.
template <int P>
__device__ __forceinline__ void s1_words(const double (&x)[4], int e, uint32_t (&word)[P]) {
  constexpr uint64_t BIAS = P > 1 ? 0x8080808080808080ull >> (8 * (9 - P)) : 0;
  uint64_t u[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) u[j] = (uint64_t)round_half_up_scaled(x[j], 8 * P - 2 - e) + BIAS;
#pragma unroll
  for (int t = 0; t < P; ++t) {
    const int b = 8 * (P - 1 - t);
    uint32_t w = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) w |= (uint32_t)((u[j] >> b) & 255) << (8 * j);
    word[t] = t ? w ^ 0x80808080u : w;
  }
}

__device__ __forceinline__ bool live_exponent(int e) { return e != OZK_EXP_ZERO && e != OZK_EXP_NONFINITE; }

// 8 consecutive k of packed row r from k0 (a multiple of 8): two 4-entry
// word groups, stored as one 8-byte piece per slice at packed[k/32][t][r][k%32].
template <int P>
__device__ __forceinline__ void s1_store_row_words(int8_t* __restrict__ packed, int64_t rows_packed, int64_t r,
                                                   int64_t k0, const uint32_t (&lo)[P], const uint32_t (&hi)[P]) {
  const int64_t c = k0 / OZK_K_CHUNK, kk = k0 % OZK_K_CHUNK;
#pragma unroll
  for (int t = 0; t < P; ++t)
    *reinterpret_cast<uint2*>(packed + ((c * P + t) * rows_packed + r) * OZK_K_CHUNK + kk) = make_uint2(lo[t], hi[t]);
}

// Slices of packed row r (16 lanes per row, lane q taking 8 consecutive k
// per 128): the digits of a live row, zeros for rows past `rows`, zero and
// non-finite rows and k past K.  xr points at a row that may be read
// whatever r (row 0 for rows past the end).
template <int P, typename T>
__device__ __forceinline__ void s1_slice_rows4(const T* __restrict__ xr, int64_t r, bool live, int e, int q,
                                               int64_t K, int64_t Kp, int64_t rows_packed,
                                               int8_t* __restrict__ packed) {
  for (int64_t k0 = 8 * q; k0 < Kp; k0 += 128) {
    uint32_t lo[P], hi[P];
    if (live) {
      double a[4], b[4];
      if (k0 + 8 <= K) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          a[j] = xr[k0 + j];
          b[j] = xr[k0 + 4 + j];
        }
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          a[j] = k0 + j < K ? xr[k0 + j] : 0.0;
          b[j] = k0 + 4 + j < K ? xr[k0 + 4 + j] : 0.0;
        }
      }
      s1_words<P>(a, e, lo);
      s1_words<P>(b, e, hi);
    } else {
#pragma unroll
      for (int t = 0; t < P; ++t) lo[t] = hi[t] = 0;
    }
    if (r < rows_packed) s1_store_row_words<P>(packed, rows_packed, r, k0, lo, hi);
  }
}

// Four packed rows per wave (16 lanes per row, 8 consecutive k per lane,
// 128 k per row per iteration): the row exponent by a 16-lane maximum, then
// the slices.  Each store instruction of a wave writes, per slice, the four
// rows' 32-byte pieces of 4 K chunks, and the four rows of one chunk are
// adjacent in the packed layout: whole 128-byte lines instead of scattered
// quarter lines.  Rows past `rows` (whole 16-lane groups) write zeros; the
// loads of every lane are issued whatever its row, so that all lanes take
// the same path through the shuffles.
template <int P, typename T>
__global__ __launch_bounds__(256) void k_s1_split_rows4(const T* __restrict__ X, int64_t ldx,
                                                        int64_t rows, int64_t K, int64_t Kp,
                                                        int64_t rows_packed, int32_t* __restrict__ e_out,
                                                        int8_t* __restrict__ packed) {
  const int lane = threadIdx.x & 63, q = lane & 15;
  const int64_t r = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 4 + (lane >> 4);
  const bool in = r < rows;
  const T* xr = X + (in ? r : 0) * ldx;  // rows past the end load row 0 and discard it
  int e = OZK_EXP_ZERO;
  for (int64_t k0 = 8 * q; k0 < K; k0 += 128) {
    double v[8];
    if (k0 + 8 <= K) {
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = xr[k0 + j];
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = k0 + j < K ? xr[k0 + j] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int ek = expo_of(v[j]);
      e = ek > e ? ek : e;
    }
  }
  e = group16_max(in ? e : OZK_EXP_ZERO);
  if (in && q == 0) e_out[r] = e;
  s1_slice_rows4<P>(xr, r, in && live_exponent(e), e, q, K, Kp, rows_packed, packed);
}

// The slice kernel of the automatic path: the row exponents come from the
// statistics pass (which read A once already) and p from device memory, so
// A is read once more here, four rows per wave as in k_s1_split_rows4.
__global__ __launch_bounds__(256) void k_s1_slice_rows4_auto(const double* __restrict__ X, int64_t ldx, int64_t rows,
                                                             int64_t K, int64_t Kp, int64_t rows_packed,
                                                             const int32_t* __restrict__ e_in,
                                                             const int32_t* __restrict__ p_dev,
                                                             int8_t* __restrict__ packed) {
  const int p = *p_dev;
  if (p < 1) return;  // p = 0: Scheme II was chosen
  const int lane = threadIdx.x & 63, q = lane & 15;
  const int64_t r = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 4 + (lane >> 4);
  const bool in = r < rows;
  const double* xr = X + (in ? r : 0) * ldx;
  const int e = in ? e_in[r] : OZK_EXP_ZERO;
  const bool live = in && live_exponent(e);
  switch (p) {
    case 1: s1_slice_rows4<1>(xr, r, live, e, q, K, Kp, rows_packed, packed); break;
    case 2: s1_slice_rows4<2>(xr, r, live, e, q, K, Kp, rows_packed, packed); break;
    case 3: s1_slice_rows4<3>(xr, r, live, e, q, K, Kp, rows_packed, packed); break;
    case 4: s1_slice_rows4<4>(xr, r, live, e, q, K, Kp, rows_packed, packed); break;
    case 5: s1_slice_rows4<5>(xr, r, live, e, q, K, Kp, rows_packed, packed); break;
    case 6: s1_slice_rows4<6>(xr, r, live, e, q, K, Kp, rows_packed, packed); break;
    case 7: s1_slice_rows4<7>(xr, r, live, e, q, K, Kp, rows_packed, packed); break;
    default: s1_slice_rows4<8>(xr, r, live, e, q, K, Kp, rows_packed, packed); break;
  }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Column exponents: thread j scans a run of 256 rows of column j.
template <typename T>
__global__ __launch_bounds__(256) void k_s1_exp_cols(const T* __restrict__ X, int64_t ldx,
                                                     int64_t K, int64_t cols, int32_t* __restrict__ f) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= cols) return;
  const int64_t k0 = (int64_t)blockIdx.y * 256;
  const int64_t k1 = k0 + 256 < K ? k0 + 256 : K;
  int e = OZK_EXP_ZERO;
#pragma unroll 8
  for (int64_t k = k0; k < k1; ++k) {
    const int ek = expo_of((double)X[k * ldx + j]);
    e = ek > e ? ek : e;
  }
  if (e != OZK_EXP_ZERO) atomicMax(&f[j], e);
}

// Column operand slices: thread (j, c) turns the 32 k of chunk c of column j
// into p x 32 digits and stores 32 bytes per slice at packed[c][t][j][:]
// (consecutive threads write consecutive 32-byte lines).  Columns past
// `cols`, zero or non-finite columns and k past K are zero; only the chunk
// that straddles K takes the guarded path.
template <int P, typename T>
__device__ __forceinline__ void s1_slice_col(const T* __restrict__ X, int64_t ldx, int64_t K, int64_t cols,
                                             int64_t cols_packed, const int32_t* __restrict__ f,
                                             int8_t* __restrict__ packed, int64_t j, int64_t c) {
  const int e = j < cols ? f[j] : OZK_EXP_ZERO;
  const int64_t kb = c * OZK_K_CHUNK;
  uint32_t word[8][P];
  if (live_exponent(e) && kb + OZK_K_CHUNK <= K) {
    const T* x = X + kb * ldx + j;
    double v[8][4];  // all 32 loads first
#pragma unroll
    for (int g = 0; g < 8; ++g)
#pragma unroll
      for (int i = 0; i < 4; ++i) v[g][i] = x[(4 * g + i) * ldx];
#pragma unroll
    for (int g = 0; g < 8; ++g) s1_words<P>(v[g], e, word[g]);
  } else if (live_exponent(e)) {
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      double v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t k = kb + 4 * g + i;
        v[i] = k < K ? X[k * ldx + j] : 0.0;
      }
      s1_words<P>(v, e, word[g]);
    }
  } else {
#pragma unroll
    for (int g = 0; g < 8; ++g)
#pragma unroll
      for (int t = 0; t < P; ++t) word[g][t] = 0;
  }
#pragma unroll
  for (int t = 0; t < P; ++t) {
    uint4* q = reinterpret_cast<uint4*>(packed + ((c * P + t) * cols_packed + j) * OZK_K_CHUNK);
    q[0] = make_uint4(word[0][t], word[1][t], word[2][t], word[3][t]);
    q[1] = make_uint4(word[4][t], word[5][t], word[6][t], word[7][t]);
  }
}

template <int P, typename T>
__global__ __launch_bounds__(256) void k_s1_split_cols(const T* __restrict__ X, int64_t ldx,
                                                       int64_t K, int64_t cols, int64_t Kp,
                                                       int64_t cols_packed, const int32_t* __restrict__ f,
                                                       int8_t* __restrict__ packed) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= cols_packed) return;
  s1_slice_col<P, T>(X, ldx, K, cols, cols_packed, f, packed, j, blockIdx.y);
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

// ------------------------------------------- 4M complex column operand

// Entry (k2, c) of the real embedding that turns a complex product into one
// real product (the four real products of 4M, Sec. IV-B, with their
// subtraction and addition inside the exact integer sums): for the complex
// column operand B (K x N, interleaved, ldx in complex elements) the 2K x 2N
// matrix whose row 2k holds (Re b_kj, Im b_kj) at columns (2j, 2j+1) and row
// 2k+1 holds (-Im b_kj, Re b_kj).  The complex row operand A needs no such
// step: its row i viewed as 2K reals, (Re a_i0, Im a_i0, Re a_i1, ...), is
// the embedded row, so column 2j of the product is Re (AB)_ij and column
// 2j+1 is Im (AB)_ij -- the interleaved complex result.  Columns 2j and 2j+1
// hold the same magnitudes, so they share one exponent; a row of A shares
// one exponent between its parts.
template <typename T>
__device__ __forceinline__ double embed4m(const T* __restrict__ X, int64_t ldx, int64_t k2, int64_t c) {
  const bool odd_k = (k2 & 1) != 0, odd_c = (c & 1) != 0;
  const T* z = X + 2 * ((k2 >> 1) * ldx + (c >> 1));
  const double v = (double)z[odd_k != odd_c ? 1 : 0];  // Re on the diagonal of the 2 x 2 block, else Im
  return odd_k && !odd_c ? -v : v;
}

// Column exponents of the embedding: thread c scans 256 rows k2 of column c.
template <typename T>
__global__ __launch_bounds__(256) void k_s1_exp_cols_4m(const T* __restrict__ X, int64_t ldx, int64_t K2,
                                                        int64_t cols2, int32_t* __restrict__ f) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= cols2) return;
  const int64_t k0 = (int64_t)blockIdx.y * 256;
  const int64_t k1 = k0 + 256 < K2 ? k0 + 256 : K2;
  int e = OZK_EXP_ZERO;
  for (int64_t k = k0; k < k1; ++k) {
    const int ek = expo_of(embed4m(X, ldx, k, c));
    e = ek > e ? ek : e;
  }
  if (e != OZK_EXP_ZERO) atomicMax(&f[c], e);
}

// Slices of the embedding, thread (c, chunk) as in k_s1_split_cols.
template <int P, typename T>
__global__ __launch_bounds__(256) void k_s1_split_cols_4m(const T* __restrict__ X, int64_t ldx, int64_t K2,
                                                          int64_t cols2, int64_t cols_packed,
                                                          const int32_t* __restrict__ f,
                                                          int8_t* __restrict__ packed) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= cols_packed) return;
  const int64_t ch = blockIdx.y, kb = ch * OZK_K_CHUNK;
  const int e = c < cols2 ? f[c] : OZK_EXP_ZERO;
  uint32_t word[8][P];
  if (live_exponent(e)) {
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      double v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t k = kb + 4 * g + i;
        v[i] = k < K2 ? embed4m(X, ldx, k, c) : 0.0;
      }
      s1_words<P>(v, e, word[g]);
    }
  } else {
#pragma unroll
    for (int g = 0; g < 8; ++g)
#pragma unroll
      for (int t = 0; t < P; ++t) word[g][t] = 0;
  }
#pragma unroll
  for (int t = 0; t < P; ++t) {
    uint4* q = reinterpret_cast<uint4*>(packed + ((ch * P + t) * cols_packed + c) * OZK_K_CHUNK);
    q[0] = make_uint4(word[0][t], word[1][t], word[2][t], word[3][t]);
    q[1] = make_uint4(word[4][t], word[5][t], word[6][t], word[7][t]);
  }
}

// C = alpha H + beta C for a complex result whose parts H (M x 2N reals,
// row stride ldh) hold (Re, Im) pairs: the fixed FMA sequence of the
// complex calls (beta == 0: C is not read), in the output's precision.
template <typename TO>
__global__ __launch_bounds__(256) void k_zaxpby(const TO* __restrict__ H, int64_t ldh, int64_t M, int64_t N,
                                                TO a_re, TO a_im, TO b_re, TO b_im, TO* __restrict__ C,
                                                int64_t ldc) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= M * N) return;
  const int64_t i = idx / N, j = idx % N;
  const TO hre = H[i * ldh + 2 * j], him = H[i * ldh + 2 * j + 1];
  TO* cp = C + 2 * (i * ldc + j);
  TO bre = 0, bim = 0;
  if (!(b_re == 0 && b_im == 0)) {
    const TO cre = cp[0], cim = cp[1];
    bre = fma_any(b_re, cre, -(b_im * cim));
    bim = fma_any(b_re, cim, b_im * cre);
  }
  cp[0] = fma_any(a_re, hre, fma_any(-a_im, him, bre));
  cp[1] = fma_any(a_re, him, fma_any(a_im, hre, bim));
}

// Exact fold of the K-run partials followed by the single rounding.
// TO = float: the binary32 rounding and update (alpha, beta hold binary32 values).
template <typename TO>
__global__ __launch_bounds__(256) void k_s1_fold(const int64_t* __restrict__ zpart, int nsplit, int M, int N,
                                                 int p, const int32_t* __restrict__ p_dev,
                                                 const int32_t* __restrict__ e_row,
                                                 const int32_t* __restrict__ f_col, double alpha,
                                                 double beta, TO* __restrict__ C, int64_t ldc) {
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
  const bool bad = er == OZK_EXP_NONFINITE || fc == OZK_EXP_NONFINITE;
  const bool zero = er == OZK_EXP_ZERO || fc == OZK_EXP_ZERO;
  const int E = er + fc - 12 - 8 * (p - 1);
  TO* cp = C + row * ldc + col;
  if constexpr (sizeof(TO) == 4) {
    const float h = bad ? __builtin_nanf("") : zero ? 0.0f : round_scaled_f32(Z, E);
    *cp = axpby_f32((float)alpha, h, (float)beta, cp);
  } else {
    const double h = bad ? __builtin_nan("") : zero ? 0.0 : round_scaled(Z, E);
    *cp = axpby(alpha, h, beta, cp);
  }
}

// ------------------------------------------------------------- launchers

template <int P, typename T>
static hipError_t launch_split_rows(const T* X, int64_t ldx, int64_t rows, int64_t K, int32_t* e,
                                    int8_t* packed, hipStream_t st) {
  const int64_t rp = round_up(rows, OZK_ROW_ALIGN), kp = round_up(K, OZK_K_CHUNK);
  if (rp == 0) return hipSuccess;  // with K == 0 the launch still writes the exponents
  hipLaunchKernelGGL((k_s1_split_rows4<P, T>), dim3((unsigned)(rp / 16)), dim3(256), 0, st, X, ldx, rows, K, kp,
                     rp, e, packed);
  return hipGetLastError();
}

template <int P, typename T>
static hipError_t launch_split_cols(const T* X, int64_t ldx, int64_t K, int64_t cols, int32_t* f,
                                    int8_t* packed, hipStream_t st) {
  const int64_t cp = round_up(cols, OZK_ROW_ALIGN), kp = round_up(K, OZK_K_CHUNK);
  if (cols > 0) {
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((cols + 255) / 256)), dim3(256), 0, st, f, cols,
                       (int32_t)OZK_EXP_ZERO);
    if (K > 0)
      hipLaunchKernelGGL(k_s1_exp_cols<T>, dim3((unsigned)((cols + 255) / 256), (unsigned)((K + 255) / 256)),
                         dim3(256), 0, st, X, ldx, K, cols, f);
  }
  if (cp > 0 && kp > 0)
    hipLaunchKernelGGL((k_s1_split_cols<P, T>), dim3((unsigned)(cp / 256), (unsigned)(kp / OZK_K_CHUNK)),
                       dim3(256), 0, st, X, ldx, K, cols, kp, cp, f, packed);
  return hipGetLastError();
}

template <typename T>
static hipError_t split_rows_any(int p, const T* X, int64_t ldx, int64_t rows, int64_t K, int32_t* e,
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

template <typename T>
static hipError_t split_cols_any(int p, const T* X, int64_t ldx, int64_t K, int64_t cols, int32_t* f,
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

template <int P, typename T>
static hipError_t launch_split_cols_4m(const T* X, int64_t ldx, int64_t K, int64_t N, int32_t* f, int8_t* packed,
                                       hipStream_t st) {
  const int64_t K2 = 2 * K, cols2 = 2 * N;
  const int64_t cp = round_up(cols2, OZK_ROW_ALIGN), kp = round_up(K2, OZK_K_CHUNK);
  if (cols2 > 0) {
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((cols2 + 255) / 256)), dim3(256), 0, st, f, cols2,
                       (int32_t)OZK_EXP_ZERO);
    if (K2 > 0)
      hipLaunchKernelGGL(k_s1_exp_cols_4m<T>, dim3((unsigned)((cols2 + 255) / 256), (unsigned)((K2 + 255) / 256)),
                         dim3(256), 0, st, X, ldx, K2, cols2, f);
  }
  if (cp > 0 && kp > 0)
    hipLaunchKernelGGL((k_s1_split_cols_4m<P, T>), dim3((unsigned)(cp / 256), (unsigned)(kp / OZK_K_CHUNK)),
                       dim3(256), 0, st, X, ldx, K2, cols2, cp, f, packed);
  return hipGetLastError();
}

template <typename T>
static hipError_t split_cols_4m_any(int p, const T* X, int64_t ldx, int64_t K, int64_t N, int32_t* f,
                                    int8_t* packed, hipStream_t st) {
  switch (p) {
    case 1: return launch_split_cols_4m<1>(X, ldx, K, N, f, packed, st);
    case 2: return launch_split_cols_4m<2>(X, ldx, K, N, f, packed, st);
    case 3: return launch_split_cols_4m<3>(X, ldx, K, N, f, packed, st);
    case 4: return launch_split_cols_4m<4>(X, ldx, K, N, f, packed, st);
    case 5: return launch_split_cols_4m<5>(X, ldx, K, N, f, packed, st);
    case 6: return launch_split_cols_4m<6>(X, ldx, K, N, f, packed, st);
    case 7: return launch_split_cols_4m<7>(X, ldx, K, N, f, packed, st);
    case 8: return launch_split_cols_4m<8>(X, ldx, K, N, f, packed, st);
  }
  return hipErrorInvalidValue;
}

hipError_t s1_split_cols_4m(int p, const double* X, int64_t ldx, int64_t K, int64_t N, int32_t* f, int8_t* packed,
                            hipStream_t st) {
  return split_cols_4m_any(p, X, ldx, K, N, f, packed, st);
}

hipError_t s1_split_cols_4m(int p, const float* X, int64_t ldx, int64_t K, int64_t N, int32_t* f, int8_t* packed,
                            hipStream_t st) {
  return split_cols_4m_any(p, X, ldx, K, N, f, packed, st);
}

template <typename TO>
static hipError_t launch_zaxpby(const TO* H, int64_t ldh, int64_t M, int64_t N, const TO* alpha, const TO* beta,
                                TO* C, int64_t ldc, hipStream_t st) {
  const int64_t n = M * N;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zaxpby<TO>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, H, ldh, M, N, alpha[0],
                     alpha[1], beta[0], beta[1], C, ldc);
  return hipGetLastError();
}

hipError_t zaxpby(const double* H, int64_t ldh, int64_t M, int64_t N, const double* alpha, const double* beta,
                  double* C, int64_t ldc, hipStream_t st) {
  return launch_zaxpby(H, ldh, M, N, alpha, beta, C, ldc, st);
}

hipError_t zaxpby(const float* H, int64_t ldh, int64_t M, int64_t N, const float* alpha, const float* beta,
                  float* C, int64_t ldc, hipStream_t st) {
  return launch_zaxpby(H, ldh, M, N, alpha, beta, C, ldc, st);
}

hipError_t s1_split_rows(int p, const double* X, int64_t ldx, int64_t rows, int64_t K, int32_t* e,
                         int8_t* packed, hipStream_t st) {
  return split_rows_any(p, X, ldx, rows, K, e, packed, st);
}

hipError_t s1_split_rows(int p, const float* X, int64_t ldx, int64_t rows, int64_t K, int32_t* e,
                         int8_t* packed, hipStream_t st) {
  return split_rows_any(p, X, ldx, rows, K, e, packed, st);
}

hipError_t s1_split_cols(int p, const double* X, int64_t ldx, int64_t K, int64_t cols, int32_t* f,
                         int8_t* packed, hipStream_t st) {
  return split_cols_any(p, X, ldx, K, cols, f, packed, st);
}

hipError_t s1_split_cols(int p, const float* X, int64_t ldx, int64_t K, int64_t cols, int32_t* f,
                         int8_t* packed, hipStream_t st) {
  return split_cols_any(p, X, ldx, K, cols, f, packed, st);
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
  if (g.C32)
    hipLaunchKernelGGL(k_s1_fold<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g.zpart,
                       (int)g.nsplit, (int)g.M, (int)g.N, p, p_dev, g.e, g.f, g.alpha, g.beta, g.C32, g.ldc);
  else
    hipLaunchKernelGGL(k_s1_fold<double>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g.zpart,
                       (int)g.nsplit, (int)g.M, (int)g.N, p, p_dev, g.e, g.f, g.alpha, g.beta, g.C, g.ldc);
  return hipGetLastError();
}

hipError_t s1_gemm(int p, const S1GemmArgs& g, hipStream_t st) {
  if (g.M == 0 || g.N == 0) return hipSuccess;
  if (g.diag) return gemm_launch(p, S1_OUT_DIAG, g, nullptr, st);
  if (g.nsplit > 1) {
    hipError_t err = gemm_launch(p, S1_OUT_PARTIAL, g, nullptr, st);
    return err == hipSuccess ? launch_fold(p, nullptr, g, st) : err;
  }
  return gemm_launch(p, g.C32 ? S1_OUT_FINAL_F32 : S1_OUT_FINAL, g, nullptr, st);
}

// ---------------------------------------------------- slice count on device

hipError_t s1_slice_auto(const int32_t* p_dev, const double* A, int64_t lda, int64_t M, const double* B, int64_t ldb,
                         int64_t N, int64_t K, const int32_t* e, const int32_t* f, int8_t* Ap, int8_t* Bp,
                         hipStream_t st) {
  const int64_t ra = round_up(M, OZK_ROW_ALIGN), rb = round_up(N, OZK_ROW_ALIGN), kp = round_up(K, OZK_K_CHUNK);
  if (ra > 0 && kp > 0)
    hipLaunchKernelGGL(k_s1_slice_rows4_auto, dim3((unsigned)(ra / 16)), dim3(256), 0, st, A, lda, M, K, kp, ra, e,
                       p_dev, Ap);
  if (rb > 0 && kp > 0)
    hipLaunchKernelGGL(k_s1_split_cols_auto, dim3((unsigned)(rb / 256), (unsigned)(kp / OZK_K_CHUNK)), dim3(256), 0,
                       st, B, ldb, K, N, kp, rb, f, p_dev, Bp);
  return hipGetLastError();
}

// Every fixed-p kernel is launched, each with the tile variant and raster of
// its own size class; each returns at once unless p_dev holds its slice
// count, so the chosen p runs with its own tiling and no host round trip.
static hipError_t launch_gemm_all(int out, const int32_t* p_dev, const S1GemmArgs& g, const int (*cfg)[3],
                                  hipStream_t st) {
  hipError_t err = hipSuccess;
  for (int p = 1; p <= OZK_MAX_P && err == hipSuccess; ++p) {
    S1GemmArgs gp = g;
    gp.variant = cfg[p - 1][0];
    gp.raster = cfg[p - 1][1];
    gp.group = cfg[p - 1][2];
    err = gemm_launch(p, out, gp, p_dev, st);
  }
  return err;
}

hipError_t s1_gemm_auto(const int32_t* p_dev, const S1GemmArgs& g, const int (*cfg)[3], hipStream_t st) {
  if (g.M == 0 || g.N == 0) return hipSuccess;
  if (g.nsplit <= 1) return launch_gemm_all(S1_OUT_FINAL, p_dev, g, cfg, st);
  hipError_t err = launch_gemm_all(S1_OUT_PARTIAL, p_dev, g, cfg, st);
  return err == hipSuccess ? launch_fold(OZK_MAX_P, p_dev, g, st) : err;
}

}  // namespace ozk
