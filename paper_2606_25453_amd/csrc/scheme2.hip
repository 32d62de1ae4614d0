// Ozaki Scheme II on gfx950 INT8 MFMA (paper Sec. II-C.2 and Sec. IV), real
// and 3M complex.
//
//   k_s2_split_rows     row scale sigma_i from an exact bound on the row's
//                       2-norm, then the s symmetric residue planes (Eq. 5)
//   k_s2_col_scales     the same for the columns of B (LDS reductions of
//                       integers, so the result does not depend on the order)
//   k_s2_gemm_mod       one INT8 GEMM per modulus with smod in the epilogue
//                       (Eqs. 6-7); 3M: three products per modulus and the
//                       combination T1-T2, T3-T1-T2 before the reduction
//   k_s2_crt            CRT recombination in multiword integers (Eq. 8) with
//                       the symmetric lift, then one rounding of Z 2^-(sigma+tau)
#include "mfma_gemm.hpp"
#include "ozk_device.hpp"
#include "ozk_internal.hpp"

namespace ozk {

// ------------------------------------------------------------- moduli table

struct S2Tables {
  int m[OZK_MAX_S];
  double inv_m[OZK_MAX_S];
  uint8_t pow2[OZK_MAX_S][128];  // 2^k mod m_l
};

constexpr int gcd_c(int a, int b) { return b == 0 ? a : gcd_c(b, a % b); }

// Greedy descending pairwise-coprime moduli from 256 (256, 255, 253, ...).
constexpr S2Tables make_s2_tables() {
  S2Tables t{};
  int n = 0;
  for (int c = 256; n < OZK_MAX_S; --c) {
    bool ok = true;
    for (int i = 0; i < n; ++i)
      if (gcd_c(c, t.m[i]) != 1) ok = false;
    if (ok) t.m[n++] = c;
  }
  for (int i = 0; i < OZK_MAX_S; ++i) {
    t.inv_m[i] = 1.0 / t.m[i];
    int r = 1 % t.m[i];
    for (int k = 0; k < 128; ++k) {
      t.pow2[i][k] = (uint8_t)r;
      r = (2 * r) % t.m[i];
    }
  }
  return t;
}

constexpr S2Tables kS2 = make_s2_tables();
__constant__ S2Tables c_s2 = kS2;

int s2_modulus(int l) { return kS2.m[l]; }

// x mod m in [0, m) for |x| < 2^53 given as an exact double.
__device__ __forceinline__ int mod_small(double x, int m, double inv_m) {
  const double q = floor(x * inv_m);
  int r = (int)__fma_rn(-q, (double)m, x);
  if (r < 0) r += m;
  if (r >= m) r -= m;
  return r;
}

// smod: the representative of r (0 <= r < m) in [-floor(m/2), ceil(m/2)-1].
__device__ __forceinline__ int sym(int r, int m) { return r >= (m + 1) / 2 ? r - m : r; }

// smod of an INT32 accumulator.
__device__ __forceinline__ int smod_i32(int x, int l) {
  const int m = c_s2.m[l];
  return sym(mod_small((double)x, m, c_s2.inv_m[l]), m);
}

// a' = trunc(a 2^sigma) as sign * u * 2^k with u < 2^53 an integer (as an
// exact double) and k >= 0.
struct ScaledInt {
  double u;
  int k;
  bool neg;
};

__device__ __forceinline__ ScaledInt scaled_int(double a, int sigma) {
  int64_t m;
  int q;
  split_fp64(a, m, q);
  ScaledInt s;
  s.neg = m < 0;
  uint64_t am = s.neg ? (uint64_t)(-m) : (uint64_t)m;
  const int sh = q + sigma;
  if (am == 0) {
    s.u = 0.0;
    s.k = 0;
  } else if (sh >= 0) {
    s.u = (double)am;
    s.k = sh;
  } else {
    s.u = (-sh >= 64) ? 0.0 : (double)(am >> (-sh));
    s.k = 0;
  }
  return s;
}

__device__ __forceinline__ int residue_of(const ScaledInt& v, int l) {
  const int m = c_s2.m[l];
  int r = mod_small(v.u, m, c_s2.inv_m[l]);
  if (v.k > 0) r = mod_small((double)(r * (int)c_s2.pow2[l][v.k < 128 ? v.k : 127]), m, c_s2.inv_m[l]);
  if (v.neg && r) r = m - r;
  return sym(r, m);
}

// Per-entry exponent for the scale bound: |entry| < 2^ex.  Complex entries
// bound |re| + |im| < 2^(max(expo re, expo im) + 1).
template <bool CPLX>
__device__ __forceinline__ int entry_expo(const double* x) {
  if (!CPLX) return expo_of(x[0]);
  const int a = expo_of(x[0]), b = expo_of(x[1]);
  if (a == OZK_EXP_NONFINITE || b == OZK_EXP_NONFINITE) return OZK_EXP_NONFINITE;
  const int e = a > b ? a : b;
  return e == OZK_EXP_ZERO ? OZK_EXP_ZERO : e + 1;
}

// ceil(2^40 4^(ex - emax)) for an entry with exponent ex <= emax; 0 for zero.
__device__ __forceinline__ int64_t norm_term(int ex, int emax) {
  if (ex == OZK_EXP_ZERO) return 0;
  const int d = ex - emax;
  return d >= -20 ? ((int64_t)1 << (40 + 2 * d)) : 1;
}

// sigma = T - nb with nb = emax + ceil((ceil(log2 S) - 40) / 2).
__device__ __forceinline__ int scale_from(int emax, int64_t S, int T) {
  if (emax == OZK_EXP_NONFINITE) return OZK_EXP_NONFINITE;
  if (emax == OZK_EXP_ZERO || S <= 0) return 0;
  const int clog = S == 1 ? 0 : 64 - __clzll((uint64_t)(S - 1));
  const int c = clog - 40;
  const int half = c >= 0 ? (c + 1) / 2 : -((-c) / 2);
  return T - (emax + half);
}

__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

struct S2Args {
  int s;
  int T;  // T_A for rows, T_B for columns
};

// One wave per packed row: exponent max, norm-bound sum, then residues of 4
// consecutive k per lane (one dword per plane).  Every modulus plane is a
// packed operand of the shared GEMM core: real packed[l][c][r][32], complex
// packed[l][c][q][r][32] (q = re, im, sum).
template <bool CPLX>
__device__ __forceinline__ void s2_split_rows_block(const double* __restrict__ X, int64_t ldx, int64_t rows,
                                                    int64_t K, int64_t Kp, int64_t rows_packed, S2Args sa,
                                                    int32_t* __restrict__ sigma_out, int8_t* __restrict__ packed,
                                                    int64_t blk) {
  constexpr int W = CPLX ? 2 : 1;
  const int lane = threadIdx.x & 63;
  const int64_t r = blk * 4 + (threadIdx.x >> 6);
  if (r >= rows_packed) return;
  const double* xr = X + r * ldx * W;
  int sigma = 0;
  if (r < rows) {
    int e = OZK_EXP_ZERO;
#pragma unroll 8
    for (int64_t k = lane; k < K; k += 64) {
      const int ek = entry_expo<CPLX>(xr + k * W);
      e = ek > e ? ek : e;
    }
    e = wave_max(e);
    int64_t S = 0;
    if (e != OZK_EXP_NONFINITE && e != OZK_EXP_ZERO)
#pragma unroll 8
      for (int64_t k = lane; k < K; k += 64) S += norm_term(entry_expo<CPLX>(xr + k * W), e);
    S = wave_sum64(S);
    sigma = scale_from(e, S, sa.T);
    if (lane == 0) sigma_out[r] = sigma;
  }
  const bool live = r < rows && sigma != OZK_EXP_NONFINITE;
  const int64_t plane = rows_packed * Kp * (CPLX ? 3 : 1);
#pragma unroll 4
  for (int64_t k0 = (int64_t)lane * 4; k0 < Kp; k0 += 256) {
    ScaledInt vr[4], vi[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t k = k0 + j;
      const bool in = live && k < K;
      vr[j] = scaled_int(in ? xr[k * W] : 0.0, sigma);
      if (CPLX) vi[j] = scaled_int(in ? xr[k * W + 1] : 0.0, sigma);
    }
    for (int l = 0; l < sa.s; ++l) {
      const int m = c_s2.m[l];
      uint32_t w0 = 0, w1 = 0, w2 = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int a = residue_of(vr[j], l);
        w0 |= (uint32_t)(uint8_t)a << (8 * j);
        if (CPLX) {
          const int b = residue_of(vi[j], l);
          w1 |= (uint32_t)(uint8_t)b << (8 * j);
          w2 |= (uint32_t)(uint8_t)sym(((a + b) % m + m) % m, m) << (8 * j);
        }
      }
      int8_t* base = packed + l * plane;
      const int64_t c = k0 / OZK_K_CHUNK, kk = k0 % OZK_K_CHUNK;
      constexpr int NP = CPLX ? 3 : 1;
      const int64_t slab = rows_packed * OZK_K_CHUNK;
      int8_t* dst = base + c * NP * slab + r * OZK_K_CHUNK + kk;
      *reinterpret_cast<uint32_t*>(dst) = w0;
      if (CPLX) {
        *reinterpret_cast<uint32_t*>(dst + slab) = w1;
        *reinterpret_cast<uint32_t*>(dst + 2 * slab) = w2;
      }
    }
  }
}

template <bool CPLX>
__global__ __launch_bounds__(256) void k_s2_split_rows(const double* __restrict__ X, int64_t ldx, int64_t rows,
                                                       int64_t K, int64_t Kp, int64_t rows_packed, S2Args sa,
                                                       int32_t* __restrict__ sigma_out,
                                                       int8_t* __restrict__ packed) {
  s2_split_rows_block<CPLX>(X, ldx, rows, K, Kp, rows_packed, sa, sigma_out, packed, blockIdx.x);
}

// Column scales: a block of 256 threads covers 32 consecutive columns with 8
// k-groups per column (coalesced 32-column row segments); the max exponent
// and then the norm-bound sum are reduced through LDS, so no atomics and no
// scratch memory are needed and the result does not depend on the order.
template <bool CPLX>
__device__ __forceinline__ void s2_col_scales_block(const double* __restrict__ X, int64_t ldx, int64_t K,
                                                    int64_t cols, int T, int32_t* __restrict__ tau, int64_t blk) {
  constexpr int W = CPLX ? 2 : 1;
  __shared__ int red_e[8][32];
  __shared__ int64_t red_s[8][32];
  const int cl = threadIdx.x & 31, g = threadIdx.x >> 5;
  const int64_t j = blk * 32 + cl;
  const bool in = j < cols;
  int e = OZK_EXP_ZERO;
  if (in)
#pragma unroll 8
    for (int64_t k = g; k < K; k += 8) {
      const int ek = entry_expo<CPLX>(X + (k * ldx + j) * W);
      e = ek > e ? ek : e;
    }
  red_e[g][cl] = e;
  __syncthreads();
  int emax = red_e[0][cl];
#pragma unroll
  for (int i = 1; i < 8; ++i) emax = red_e[i][cl] > emax ? red_e[i][cl] : emax;
  int64_t S = 0;
  if (in && emax != OZK_EXP_ZERO && emax != OZK_EXP_NONFINITE)
#pragma unroll 8
    for (int64_t k = g; k < K; k += 8) S += norm_term(entry_expo<CPLX>(X + (k * ldx + j) * W), emax);
  red_s[g][cl] = S;
  __syncthreads();
  if (g == 0 && in) {
    int64_t tot = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) tot += red_s[i][cl];
    tau[j] = scale_from(emax, tot, T);
  }
}

template <bool CPLX>
__global__ __launch_bounds__(256) void k_s2_col_scales(const double* __restrict__ X, int64_t ldx, int64_t K,
                                                       int64_t cols, int T, int32_t* __restrict__ tau) {
  s2_col_scales_block<CPLX>(X, ldx, K, cols, T, tau, blockIdx.x);
}

// Thread (j, hc): the 16 k of half-chunk hc (chunk hc / 2, half hc % 2) of
// column j, residues for every modulus, written as one 16-byte piece per
// plane (half a 32-byte packed row; 16 k keep the per-thread state small
// enough for several waves per SIMD).
constexpr int S2_COL_K = OZK_K_CHUNK / 2;

template <bool CPLX>
__device__ __forceinline__ void s2_split_cols_block(const double* __restrict__ X, int64_t ldx, int64_t K,
                                                    int64_t cols, int64_t Kp, int64_t cols_packed, int s,
                                                    const int32_t* __restrict__ tau, int8_t* __restrict__ packed,
                                                    int64_t jb, int64_t hc) {
  constexpr int W = CPLX ? 2 : 1;
  const int64_t j = jb * 256 + threadIdx.x;
  if (j >= cols_packed) return;
  const int64_t c = hc >> 1, k0 = hc * S2_COL_K;
  const int t = j < cols ? tau[j] : 0;
  const bool live = j < cols && t != OZK_EXP_NONFINITE;
  ScaledInt vr[S2_COL_K], vi[CPLX ? S2_COL_K : 1];
#pragma unroll
  for (int kk = 0; kk < S2_COL_K; ++kk) {
    const int64_t k = k0 + kk;
    const bool in = live && k < K;
    vr[kk] = scaled_int(in ? X[(k * ldx + j) * W] : 0.0, t);
    if (CPLX) vi[CPLX ? kk : 0] = scaled_int(in ? X[(k * ldx + j) * W + 1] : 0.0, t);
  }
  const int64_t plane = cols_packed * Kp * (CPLX ? 3 : 1);
  for (int l = 0; l < s; ++l) {
    const int m = c_s2.m[l];
    uint32_t w0[4] = {0, 0, 0, 0}, w1[4] = {0, 0, 0, 0}, w2[4] = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < S2_COL_K; ++kk) {
      const int a = residue_of(vr[kk], l);
      w0[kk / 4] |= (uint32_t)(uint8_t)a << (8 * (kk % 4));
      if (CPLX) {
        const int b = residue_of(vi[CPLX ? kk : 0], l);
        w1[kk / 4] |= (uint32_t)(uint8_t)b << (8 * (kk % 4));
        w2[kk / 4] |= (uint32_t)(uint8_t)sym(((a + b) % m + m) % m, m) << (8 * (kk % 4));
      }
    }
    constexpr int NP = CPLX ? 3 : 1;
    const int64_t slab = cols_packed * OZK_K_CHUNK;
    int8_t* dst = packed + l * plane + c * NP * slab + j * OZK_K_CHUNK + (hc & 1) * S2_COL_K;
    *reinterpret_cast<uint4*>(dst) = make_uint4(w0[0], w0[1], w0[2], w0[3]);
    if (CPLX) {
      *reinterpret_cast<uint4*>(dst + slab) = make_uint4(w1[0], w1[1], w1[2], w1[3]);
      *reinterpret_cast<uint4*>(dst + 2 * slab) = make_uint4(w2[0], w2[1], w2[2], w2[3]);
    }
  }
}

template <bool CPLX>
__global__ __launch_bounds__(256) void k_s2_split_cols(const double* __restrict__ X, int64_t ldx, int64_t K,
                                                       int64_t cols, int64_t Kp, int64_t cols_packed, int s,
                                                       const int32_t* __restrict__ tau,
                                                       int8_t* __restrict__ packed) {
  s2_split_cols_block<CPLX>(X, ldx, K, cols, Kp, cols_packed, s, tau, packed, blockIdx.x, blockIdx.y);
}

// ----------------------------------------------------------- modular GEMM

// Steps per INT32-safe run: |acc| <= 32 * steps * 128^2 must stay below 2^31,
// so the accumulators are reduced mod m every 4095 steps (K = 131040); the
// reduction is exact because only the residue is kept.
constexpr int64_t S2_RUN_STEPS = 4095;

// Tiling of the per-modulus GEMM; variant V = 1 uses one LDS stage fewer.
template <bool CPLX, int V = 0>
struct S2Cfg {
  static constexpr int P = CPLX ? 3 : 1;
  static constexpr int TM = 2, TN = CPLX ? 1 : 2;
  static constexpr int NS = 4 - V;
};

// One output tile of one modulus: the per-modulus products, then smod (3M:
// the combination first) and the int8 output residues.
template <bool CPLX, int V>
__device__ __forceinline__ void s2_gemm_tile(const int8_t* __restrict__ Ap, const int8_t* __restrict__ Bp,
                                             int64_t plane_a, int64_t plane_b, int64_t rows_a, int64_t rows_b,
                                             int64_t nsteps, int64_t M, int64_t N, int8_t* __restrict__ out,
                                             int64_t tile, int l, int raster, int group, int8_t* lds) {
  using Cfg = S2Cfg<CPLX, V>;
  constexpr int P = Cfg::P, TM = Cfg::TM, TN = Cfg::TN, NS = Cfg::NS;
  using T = GemmTile<P, TM, TN, NS>;
  const int64_t tiles_m = (M + T::BM - 1) / T::BM, tiles_n = (N + T::BN - 1) / T::BN;
  int64_t tm, tn;
  tile_of(tile, tiles_m, tiles_n, raster, group, tm, tn);
  const int64_t m0 = tm * T::BM, n0 = tn * T::BN;
  v16i acc[P][TM][TN];
  zero_acc<P, TM, TN>(acc);
  for (int64_t s0 = 0; s0 < nsteps || s0 == 0; s0 += S2_RUN_STEPS) {
    const int64_t n = nsteps - s0 < S2_RUN_STEPS ? nsteps - s0 : S2_RUN_STEPS;
    gemm_tile_accumulate<P, TM, TN, NS, DIAGONAL>(Ap + l * plane_a, Bp + l * plane_b, rows_a, rows_b, m0, n0, s0,
                                                  n, lds, acc);
    if (s0 + S2_RUN_STEPS >= nsteps) break;
    // keep the accumulators small by subtracting a multiple of m (exact mod m)
    const int m = c_s2.m[l];
    const float inv = 1.0f / (float)m;
#pragma unroll
    for (int d = 0; d < P; ++d)
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int x = acc[d][a][b][v];
            acc[d][a][b][v] = x - m * (int)rintf((float)x * inv);
          }
  }
  const int64_t mn = (int64_t)M * N;
  for_each_output<P, TM, TN>(acc, m0, n0, M, N, [&](int64_t row, int64_t col, const int* vals) {
    if (!CPLX) {
      out[l * mn + row * N + col] = (int8_t)smod_i32(vals[0], l);
    } else {
      const int t1 = smod_i32(vals[0], l), t2 = smod_i32(vals[CPLX ? 1 : 0], l),
                t3 = smod_i32(vals[CPLX ? 2 : 0], l);
      out[(2 * l) * mn + row * N + col] = (int8_t)smod_i32(t1 - t2, l);
      out[(2 * l + 1) * mn + row * N + col] = (int8_t)smod_i32(t3 - t1 - t2, l);
    }
  });
}

template <bool CPLX, int V>
__global__ __launch_bounds__(256, 1) void k_s2_gemm_mod(const int8_t* __restrict__ Ap,
                                                       const int8_t* __restrict__ Bp, int64_t plane_a,
                                                       int64_t plane_b, int64_t rows_a, int64_t rows_b,
                                                       int64_t nsteps, int M, int N, int raster, int group,
                                                       int8_t* __restrict__ out) {
  extern __shared__ __attribute__((aligned(1024))) int8_t lds[];
  s2_gemm_tile<CPLX, V>(Ap, Bp, plane_a, plane_b, rows_a, rows_b, nsteps, M, N, out, blockIdx.x, (int)blockIdx.z,
                        raster, group, lds);
}

// ------------------------------------------------------------------- CRT

constexpr int NL = 6;  // 32-bit limbs: P < 2^156 for s <= 20, sums < 2^170

struct CrtArgs {
  int s;
  uint32_t W[OZK_MAX_S][NL];  // (P/m_l) q_l
  uint32_t P[NL];
  double Pf;
};

// Z = smod(sum_l W_l c_l, P) as a sign and magnitude limbs.
__device__ __forceinline__ void crt_combine(const CrtArgs& ca, const int8_t* res, int64_t stride, uint32_t (&mag)[NL],
                                            bool& neg) {
  // all residues first (independent loads in flight together), then the sum
  int cv[OZK_MAX_S];
#pragma unroll
  for (int l = 0; l < OZK_MAX_S; ++l) cv[l] = l < ca.s ? (int)res[l * stride] : 0;
  uint64_t acc[NL] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int l = 0; l < OZK_MAX_S; ++l) {
    if (l >= ca.s) break;
    int c = cv[l];
    if (c < 0) c += c_s2.m[l];
#pragma unroll
    for (int i = 0; i < NL; ++i) acc[i] += (uint64_t)ca.W[l][i] * (uint32_t)c;
  }
  uint32_t v[NL + 1];
  uint64_t carry = 0;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const uint64_t t = acc[i] + carry;
    v[i] = (uint32_t)t;
    carry = t >> 32;
  }
  v[NL] = (uint32_t)carry;
  // quotient estimate by floating point, then exact correction
  double vf = 0.0;
#pragma unroll
  for (int i = NL; i >= 0; --i) vf = vf * 4294967296.0 + (double)v[i];
  int64_t q = (int64_t)floor(vf / ca.Pf);
  if (q < 0) q = 0;
  // r = v - q P (signed, NL+1 limbs, two's complement)
  int64_t borrow = 0;
  uint32_t r[NL + 1];
  uint64_t mc = 0;
#pragma unroll
  for (int i = 0; i <= NL; ++i) {
    const uint64_t pi = i < NL ? ca.P[i] : 0;
    const uint64_t prod = pi * (uint64_t)q + mc;
    mc = prod >> 32;
    const int64_t d = (int64_t)v[i] - (int64_t)(uint32_t)prod + borrow;
    r[i] = (uint32_t)d;
    borrow = d >> 32;  // 0 or -1
  }
  auto negative = [&]() { return (int32_t)r[NL] < 0; };
  auto add_p = [&](int sign) {  // r += sign * P
    int64_t cy = 0;
#pragma unroll
    for (int i = 0; i <= NL; ++i) {
      const int64_t pi = i < NL ? (int64_t)ca.P[i] : 0;
      const int64_t d = (int64_t)r[i] + sign * pi + cy;
      r[i] = (uint32_t)d;
      cy = d >> 32;
    }
  };
  auto ge_p = [&]() {  // r >= P (r non-negative)
    if (r[NL]) return true;
    for (int i = NL - 1; i >= 0; --i) {
      if (r[i] != ca.P[i]) return r[i] > ca.P[i];
    }
    return true;
  };
  while (negative()) add_p(1);
  while (ge_p()) add_p(-1);
  // symmetric lift: r >= P/2  <=>  2r >= P
  uint32_t tw[NL + 1];
  uint32_t cy2 = 0;
#pragma unroll
  for (int i = 0; i <= NL; ++i) {
    tw[i] = (r[i] << 1) | cy2;
    cy2 = r[i] >> 31;
  }
  bool ge = false;
  {
    bool decided = false;
    if (tw[NL]) {
      ge = true;
      decided = true;
    }
    for (int i = NL - 1; i >= 0 && !decided; --i) {
      if (tw[i] != ca.P[i]) {
        ge = tw[i] > ca.P[i];
        decided = true;
      }
    }
    if (!decided) ge = true;
  }
  if (ge) {
    // magnitude = P - r
    int64_t b = 0;
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int64_t d = (int64_t)ca.P[i] - (int64_t)r[i] + b;
      mag[i] = (uint32_t)d;
      b = d >> 32;
    }
    neg = true;
  } else {
#pragma unroll
    for (int i = 0; i < NL; ++i) mag[i] = r[i];
    neg = false;
  }
}

// RN-even of +-mag 2^E (one rounding, gradual underflow included).
__device__ __forceinline__ double round_limbs(const uint32_t (&mag)[NL], bool neg, int E) {
  int top = -1;
#pragma unroll
  for (int i = NL - 1; i >= 0; --i)
    if (top < 0 && mag[i]) top = i;
  if (top < 0) return 0.0;
  const int n = 32 * top + (32 - __clz(mag[top]));
  int drop = n - 53;
  if (-1074 - E > drop) drop = -1074 - E;
  auto bit = [&](int pos) -> uint32_t { return (pos < 0 || pos >= 32 * NL) ? 0u : (mag[pos >> 5] >> (pos & 31)) & 1u; };
  uint64_t q = 0;
  if (drop <= 0) {
    for (int i = n - 1; i >= 0; --i) q = (q << 1) | bit(i);
    drop = 0;
  } else {
    for (int i = n - 1; i >= drop; --i) q = (q << 1) | bit(i);
    const uint32_t rb = bit(drop - 1);
    bool sticky = false;
    for (int i = 0; i < drop - 1 && i < n; ++i) sticky |= bit(i) != 0;
    if (rb && (sticky || (q & 1))) q += 1;
  }
  const double r = ldexp((double)q, E + drop);
  return neg ? -r : r;
}

template <bool CPLX>
__device__ __forceinline__ void s2_crt_block(const CrtArgs& ca, int64_t M, int64_t N, const int8_t* __restrict__ res,
                                             const int32_t* __restrict__ sigma, const int32_t* __restrict__ tau,
                                             double a_re, double a_im, double b_re, double b_im,
                                             double* __restrict__ C, int64_t ldc, int64_t blk) {
  const int64_t idx = blk * 256 + threadIdx.x;
  const int64_t mn = (int64_t)M * N;
  if (idx >= mn) return;
  const int64_t row = idx / N, col = idx % N;
  const int si = sigma[row], tj = tau[col];
  const bool bad = si == OZK_EXP_NONFINITE || tj == OZK_EXP_NONFINITE;
  const int E = -si - tj;
  double h[2];
#pragma unroll
  for (int q = 0; q < (CPLX ? 2 : 1); ++q) {
    if (bad) {
      h[q] = __builtin_nan("");
      continue;
    }
    uint32_t mag[NL];
    bool neg;
    crt_combine(ca, res + (CPLX ? q * mn : 0) + idx, CPLX ? 2 * mn : mn, mag, neg);
    h[q] = round_limbs(mag, neg, E);
  }
  if (!CPLX) {
    double* cp = C + row * ldc + col;
    *cp = axpby(a_re, h[0], b_re, cp);
  } else {
    double* cp = C + 2 * (row * ldc + col);
    double bre = 0.0, bim = 0.0;
    if (!(b_re == 0.0 && b_im == 0.0)) {
      const double cre = cp[0], cim = cp[1];
      bre = __fma_rn(b_re, cre, -(b_im * cim));
      bim = __fma_rn(b_re, cim, b_im * cre);
    }
    const double ore = __fma_rn(a_re, h[0], __fma_rn(-a_im, h[1], bre));
    const double oim = __fma_rn(a_re, h[1], __fma_rn(a_im, h[0], bim));
    cp[0] = ore;
    cp[1] = oim;
  }
}

template <bool CPLX>
__global__ __launch_bounds__(256) void k_s2_crt(CrtArgs ca, int M, int N, const int8_t* __restrict__ res,
                                                const int32_t* __restrict__ sigma, const int32_t* __restrict__ tau,
                                                double a_re, double a_im, double b_re, double b_im,
                                                double* __restrict__ C, int64_t ldc) {
  s2_crt_block<CPLX>(ca, M, N, res, sigma, tau, a_re, a_im, b_re, b_im, C, ldc, blockIdx.x);
}

// ------------------------------------------------------------ host side

// Little host bignum in 32-bit limbs for the CRT constants.
static void big_mul_small(uint32_t* x, int n, uint32_t f) {
  uint64_t c = 0;
  for (int i = 0; i < n; ++i) {
    const uint64_t t = (uint64_t)x[i] * f + c;
    x[i] = (uint32_t)t;
    c = t >> 32;
  }
}
static uint32_t big_div_small(uint32_t* x, int n, uint32_t d) {
  uint64_t r = 0;
  for (int i = n - 1; i >= 0; --i) {
    const uint64_t cur = (r << 32) | x[i];
    x[i] = (uint32_t)(cur / d);
    r = cur % d;
  }
  return (uint32_t)r;
}
static int inv_mod(int a, int m) {
  int t = 0, nt = 1, r = m, nr = a % m;
  while (nr) {
    const int q = r / nr, tt = t - q * nt, rr = r - q * nr;
    t = nt;
    nt = tt;
    r = nr;
    nr = rr;
  }
  return t < 0 ? t + m : t;
}

static void crt_args(int s, CrtArgs& ca, int& ta, int& tb) {
  ca.s = s;
  uint32_t P[NL] = {1, 0, 0, 0, 0, 0};
  for (int l = 0; l < s; ++l) big_mul_small(P, NL, (uint32_t)kS2.m[l]);
  for (int i = 0; i < NL; ++i) ca.P[i] = P[i];
  double pf = 0.0;
  for (int i = NL - 1; i >= 0; --i) pf = pf * 4294967296.0 + (double)P[i];
  ca.Pf = pf;
  for (int l = 0; l < OZK_MAX_S; ++l)
    for (int i = 0; i < NL; ++i) ca.W[l][i] = 0;
  for (int l = 0; l < s; ++l) {
    uint32_t Q[NL];
    for (int i = 0; i < NL; ++i) Q[i] = P[i];
    big_div_small(Q, NL, (uint32_t)kS2.m[l]);  // P / m_l
    uint32_t R[NL];
    for (int i = 0; i < NL; ++i) R[i] = Q[i];
    const int rem = (int)big_div_small(R, NL, (uint32_t)kS2.m[l]);  // (P/m_l) mod m_l
    const int q = kS2.m[l] == 1 ? 0 : inv_mod(rem, kS2.m[l]);
    big_mul_small(Q, NL, (uint32_t)q);
    for (int i = 0; i < NL; ++i) ca.W[l][i] = Q[i];
  }
  // ceil(log2 P) = bit length of P - 1
  uint32_t Pm1[NL];
  for (int i = 0; i < NL; ++i) Pm1[i] = P[i];
  for (int i = 0; i < NL; ++i) {
    if (Pm1[i]--) break;
  }
  int bl = 0;
  for (int i = NL - 1; i >= 0; --i)
    if (Pm1[i]) {
      bl = 32 * i + (32 - __builtin_clz(Pm1[i]));
      break;
    }
  const int L = bl - 2;
  ta = L / 2;
  tb = L - ta;
}

void s2_targets(int s, int& ta, int& tb) {
  CrtArgs ca;
  crt_args(s, ca, ta, tb);
}

hipError_t s2_split_rows(int s, bool cplx, const double* X, int64_t ldx, int64_t rows, int64_t K, int32_t* sigma,
                         int8_t* packed, hipStream_t st) {
  int ta, tb;
  s2_targets(s, ta, tb);
  const int64_t rp = round_up(rows, OZK_ROW_ALIGN), kp = round_up(K, OZK_K_CHUNK);
  if (rp == 0) return hipSuccess;
  S2Args sa{s, ta};
  if (cplx)
    hipLaunchKernelGGL(k_s2_split_rows<true>, dim3((unsigned)(rp / 4)), dim3(256), 0, st, X, ldx, rows, K, kp, rp,
                       sa, sigma, packed);
  else
    hipLaunchKernelGGL(k_s2_split_rows<false>, dim3((unsigned)(rp / 4)), dim3(256), 0, st, X, ldx, rows, K, kp,
                       rp, sa, sigma, packed);
  return hipGetLastError();
}

hipError_t s2_split_cols(int s, bool cplx, const double* X, int64_t ldx, int64_t K, int64_t cols, int32_t* tau,
                         int8_t* packed, hipStream_t st) {
  int ta, tb;
  s2_targets(s, ta, tb);
  const int64_t cp = round_up(cols, OZK_ROW_ALIGN), kp = round_up(K, OZK_K_CHUNK);
  if (cols > 0) {
    const unsigned gx = (unsigned)((cols + 31) / 32);
    if (cplx)
      hipLaunchKernelGGL(k_s2_col_scales<true>, dim3(gx), dim3(256), 0, st, X, ldx, K, cols, tb, tau);
    else
      hipLaunchKernelGGL(k_s2_col_scales<false>, dim3(gx), dim3(256), 0, st, X, ldx, K, cols, tb, tau);
  }
  if (cp > 0 && kp > 0) {
    if (cplx)
      hipLaunchKernelGGL(k_s2_split_cols<true>, dim3((unsigned)(cp / 256), (unsigned)(kp / S2_COL_K)),
                         dim3(256), 0, st, X, ldx, K, cols, kp, cp, s, tau, packed);
    else
      hipLaunchKernelGGL(k_s2_split_cols<false>, dim3((unsigned)(cp / 256), (unsigned)(kp / S2_COL_K)),
                         dim3(256), 0, st, X, ldx, K, cols, kp, cp, s, tau, packed);
  }
  return hipGetLastError();
}

template <bool CPLX, int V>
static hipError_t launch_gemm_mod(int s, int64_t M, int64_t N, int64_t K, const int8_t* Ap, const int8_t* Bp,
                                  int8_t* out, int raster, int group, hipStream_t st) {
  using Cfg = S2Cfg<CPLX, V>;
  constexpr int P = Cfg::P;
  using T = GemmTile<P, Cfg::TM, Cfg::TN, Cfg::NS>;
  auto kern = k_s2_gemm_mod<CPLX, V>;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, T::LDS_BYTES);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int64_t kp = round_up(K, OZK_K_CHUNK);
  const int64_t ra = round_up(M, OZK_ROW_ALIGN), rb = round_up(N, OZK_ROW_ALIGN);
  const int64_t plane_a = ra * kp * P, plane_b = rb * kp * P;
  const int64_t tiles = ((M + T::BM - 1) / T::BM) * ((N + T::BN - 1) / T::BN);
  const dim3 grid((unsigned)tiles, 1, (unsigned)s);
  hipLaunchKernelGGL(kern, grid, dim3(256), T::LDS_BYTES, st, Ap, Bp, plane_a, plane_b, ra, rb, kp / OZK_K_CHUNK,
                     (int)M, (int)N, raster, group, out);
  return hipGetLastError();
}

hipError_t s2_gemm_mod(int s, bool cplx, int64_t M, int64_t N, int64_t K, const int8_t* Ap, const int8_t* Bp,
                       int8_t* out, hipStream_t st, int variant, int raster, int group) {
  if (M == 0 || N == 0) return hipSuccess;
  if (variant == 1)
    return cplx ? launch_gemm_mod<true, 1>(s, M, N, K, Ap, Bp, out, raster, group, st)
                : launch_gemm_mod<false, 1>(s, M, N, K, Ap, Bp, out, raster, group, st);
  return cplx ? launch_gemm_mod<true, 0>(s, M, N, K, Ap, Bp, out, raster, group, st)
              : launch_gemm_mod<false, 0>(s, M, N, K, Ap, Bp, out, raster, group, st);
}

hipError_t s2_crt(int s, bool cplx, int64_t M, int64_t N, const int8_t* res, const int32_t* sigma,
                  const int32_t* tau, const double* alpha, const double* beta, double* C, int64_t ldc,
                  hipStream_t st) {
  if (M == 0 || N == 0) return hipSuccess;
  CrtArgs ca;
  int ta, tb;
  crt_args(s, ca, ta, tb);
  const int64_t n = M * N;
  const double ai = cplx ? alpha[1] : 0.0, bi = cplx ? beta[1] : 0.0;
  if (cplx)
    hipLaunchKernelGGL(k_s2_crt<true>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ca, (int)M, (int)N,
                       res, sigma, tau, alpha[0], ai, beta[0], bi, C, ldc);
  else
    hipLaunchKernelGGL(k_s2_crt<false>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ca, (int)M, (int)N,
                       res, sigma, tau, alpha[0], ai, beta[0], bi, C, ldc);
  return hipGetLastError();
}

// --------------------------------- modulus count chosen on the device

__constant__ CrtArgs c_crt_all[OZK_MAX_S];  // CRT constants of s = 1 .. OZK_MAX_S (index s - 1)

__device__ __forceinline__ bool s2_chosen(const int32_t* __restrict__ info, int& s) {
  if (info[4] != 2) return false;
  s = info[5];
  return s >= 1 && s <= OZK_MAX_S;
}

__global__ __launch_bounds__(256) void k_s2_split_rows_auto(const double* __restrict__ X, int64_t ldx, int64_t rows,
                                                            int64_t K, int64_t Kp, int64_t rows_packed,
                                                            const int32_t* __restrict__ info, S2Budgets bud,
                                                            int32_t* __restrict__ sigma_out,
                                                            int8_t* __restrict__ packed) {
  int s;
  if (!s2_chosen(info, s)) return;
  s2_split_rows_block<false>(X, ldx, rows, K, Kp, rows_packed, S2Args{s, bud.ta[s]}, sigma_out, packed,
                             blockIdx.x);
}

__global__ __launch_bounds__(256) void k_s2_col_scales_auto(const double* __restrict__ X, int64_t ldx, int64_t K,
                                                            int64_t cols, const int32_t* __restrict__ info,
                                                            S2Budgets bud, int32_t* __restrict__ tau) {
  int s;
  if (!s2_chosen(info, s)) return;
  s2_col_scales_block<false>(X, ldx, K, cols, bud.tb[s], tau, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_s2_split_cols_auto(const double* __restrict__ X, int64_t ldx, int64_t K,
                                                            int64_t cols, int64_t Kp, int64_t cols_packed,
                                                            const int32_t* __restrict__ info,
                                                            const int32_t* __restrict__ tau,
                                                            int8_t* __restrict__ packed) {
  int s;
  if (!s2_chosen(info, s)) return;
  s2_split_cols_block<false>(X, ldx, K, cols, Kp, cols_packed, s, tau, packed, blockIdx.x, blockIdx.y);
}

// grid z covers OZK_MAX_S moduli; the planes past the chosen s return
__global__ __launch_bounds__(256, 1) void k_s2_gemm_mod_auto(const int8_t* __restrict__ Ap,
                                                            const int8_t* __restrict__ Bp, int64_t plane_a,
                                                            int64_t plane_b, int64_t rows_a, int64_t rows_b,
                                                            int64_t nsteps, int M, int N,
                                                            const int32_t* __restrict__ info,
                                                            int8_t* __restrict__ out) {
  extern __shared__ __attribute__((aligned(1024))) int8_t lds[];
  int s;
  if (!s2_chosen(info, s) || (int)blockIdx.z >= s) return;
  s2_gemm_tile<false, 0>(Ap, Bp, plane_a, plane_b, rows_a, rows_b, nsteps, M, N, out, blockIdx.x, (int)blockIdx.z,
                         0, 4, lds);
}

__global__ __launch_bounds__(256) void k_s2_crt_auto(int M, int N, const int8_t* __restrict__ res,
                                                     const int32_t* __restrict__ sigma,
                                                     const int32_t* __restrict__ tau,
                                                     const int32_t* __restrict__ info, double alpha, double beta,
                                                     double* __restrict__ C, int64_t ldc) {
  int s;
  if (!s2_chosen(info, s)) return;
  s2_crt_block<false>(c_crt_all[s - 1], M, N, res, sigma, tau, alpha, 0.0, beta, 0.0, C, ldc, blockIdx.x);
}

S2Budgets s2_budgets() {
  S2Budgets b;
  b.ta[0] = b.tb[0] = 0;
  for (int s = 1; s <= OZK_MAX_S; ++s) s2_targets(s, b.ta[s], b.tb[s]);
  return b;
}

hipError_t s2_upload_crt_tables() {
  static CrtArgs all[OZK_MAX_S];
  int ta, tb;
  for (int s = 1; s <= OZK_MAX_S; ++s) crt_args(s, all[s - 1], ta, tb);
  return hipMemcpyToSymbol(HIP_SYMBOL(c_crt_all), all, sizeof(all));
}

hipError_t s2_split_rows_auto(const int32_t* info, const double* X, int64_t ldx, int64_t rows, int64_t K,
                              int32_t* sigma, int8_t* packed, hipStream_t st) {
  const int64_t rp = round_up(rows, OZK_ROW_ALIGN), kp = round_up(K, OZK_K_CHUNK);
  if (rp > 0)
    hipLaunchKernelGGL(k_s2_split_rows_auto, dim3((unsigned)(rp / 4)), dim3(256), 0, st, X, ldx, rows, K, kp, rp,
                       info, s2_budgets(), sigma, packed);
  return hipGetLastError();
}

hipError_t s2_split_cols_auto(const int32_t* info, const double* X, int64_t ldx, int64_t K, int64_t cols,
                              int32_t* tau, int8_t* packed, hipStream_t st) {
  const int64_t cp = round_up(cols, OZK_ROW_ALIGN), kp = round_up(K, OZK_K_CHUNK);
  if (cols > 0)
    hipLaunchKernelGGL(k_s2_col_scales_auto, dim3((unsigned)((cols + 31) / 32)), dim3(256), 0, st, X, ldx, K, cols,
                       info, s2_budgets(), tau);
  if (cp > 0 && kp > 0)
    hipLaunchKernelGGL(k_s2_split_cols_auto, dim3((unsigned)(cp / 256), (unsigned)(kp / S2_COL_K)), dim3(256),
                       0, st, X, ldx, K, cols, kp, cp, info, tau, packed);
  return hipGetLastError();
}

hipError_t s2_gemm_mod_auto(const int32_t* info, int64_t M, int64_t N, int64_t K, const int8_t* Ap,
                            const int8_t* Bp, int8_t* out, hipStream_t st) {
  if (M == 0 || N == 0) return hipSuccess;
  using Cfg = S2Cfg<false, 0>;
  using T = GemmTile<Cfg::P, Cfg::TM, Cfg::TN, Cfg::NS>;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_s2_gemm_mod_auto),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, T::LDS_BYTES);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int64_t kp = round_up(K, OZK_K_CHUNK);
  const int64_t ra = round_up(M, OZK_ROW_ALIGN), rb = round_up(N, OZK_ROW_ALIGN);
  const int64_t tiles = ((M + T::BM - 1) / T::BM) * ((N + T::BN - 1) / T::BN);
  const dim3 grid((unsigned)tiles, 1, (unsigned)OZK_MAX_S);
  hipLaunchKernelGGL(k_s2_gemm_mod_auto, grid, dim3(256), T::LDS_BYTES, st, Ap, Bp, ra * kp, rb * kp, ra, rb,
                     kp / OZK_K_CHUNK, (int)M, (int)N, info, out);
  return hipGetLastError();
}

hipError_t s2_crt_auto(const int32_t* info, int64_t M, int64_t N, const int8_t* res, const int32_t* sigma,
                       const int32_t* tau, double alpha, double beta, double* C, int64_t ldc, hipStream_t st) {
  const int64_t n = M * N;
  if (n > 0)
    hipLaunchKernelGGL(k_s2_crt_auto, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (int)M, (int)N, res,
                       sigma, tau, info, alpha, beta, C, ldc);
  return hipGetLastError();
}

// ------------------------------------------------------- batched problems
//
// Many uneven problems in one launch per step.  The plan uploads a problem
// table and, per step, the prefix sums of the work units of each problem;
// a workgroup finds its problem by binary search.  The GEMM step is one
// persistent launch: the (problem, modulus, tile) items are enumerated with
// the problems in decreasing K (longest items first) and workgroup w takes
// items w, w + G, w + 2G, ... so that the load is balanced without atomics.

namespace {

__device__ __forceinline__ int find_problem(const int64_t* __restrict__ start, int count, int64_t x) {
  int lo = 0, hi = count - 1;  // largest i with start[i] <= x
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace

template <bool CPLX>
__global__ __launch_bounds__(256) void k_b_split_rows(BatchDev bd, int8_t* __restrict__ ws, S2Args sa) {
  const int p = find_problem(bd.rows_start, bd.count, blockIdx.x);
  const BatchProb& q = bd.prob[p];
  s2_split_rows_block<CPLX>(q.A, q.lda, q.M, q.K, q.Kp, q.ra, sa, reinterpret_cast<int32_t*>(ws + q.off_sig),
                            ws + q.off_a, blockIdx.x - bd.rows_start[p]);
}

template <bool CPLX>
__global__ __launch_bounds__(256) void k_b_col_scales(BatchDev bd, int8_t* __restrict__ ws, int T) {
  const int p = find_problem(bd.cols_start, bd.count, blockIdx.x);
  const BatchProb& q = bd.prob[p];
  s2_col_scales_block<CPLX>(q.B, q.ldb, q.K, q.N, T, reinterpret_cast<int32_t*>(ws + q.off_tau),
                            blockIdx.x - bd.cols_start[p]);
}

template <bool CPLX>
__global__ __launch_bounds__(256) void k_b_split_cols(BatchDev bd, int8_t* __restrict__ ws, int s) {
  const int p = find_problem(bd.split_start, bd.count, blockIdx.x);
  const BatchProb& q = bd.prob[p];
  const int64_t local = blockIdx.x - bd.split_start[p];
  const int64_t jblocks = q.rb / 256;
  s2_split_cols_block<CPLX>(q.B, q.ldb, q.K, q.N, q.Kp, q.rb, s, reinterpret_cast<const int32_t*>(ws + q.off_tau),
                            ws + q.off_b, local % jblocks, local / jblocks);
}

template <bool CPLX>
__global__ __launch_bounds__(256, 1) void k_b_gemm_mod(BatchDev bd, int8_t* __restrict__ ws, int s) {
  extern __shared__ __attribute__((aligned(1024))) int8_t lds[];
  constexpr int NP = CPLX ? 3 : 1;
  const int64_t total = bd.item_start[bd.count];
  for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
    const int i = find_problem(bd.item_start, bd.count, it);
    const BatchProb& q = bd.prob[bd.order[i]];
    const int64_t local = it - bd.item_start[i];
    const int l = (int)(local / q.tiles);
    const int64_t tile = local % q.tiles;
    s2_gemm_tile<CPLX, 0>(ws + q.off_a, ws + q.off_b, q.ra * q.Kp * NP, q.rb * q.Kp * NP, q.ra, q.rb,
                          q.Kp / OZK_K_CHUNK, q.M, q.N, ws + q.off_res, tile, l, 0, 4, lds);
  }
  (void)s;
}

template <bool CPLX>
__global__ __launch_bounds__(256) void k_b_crt(CrtArgs ca, BatchDev bd, int8_t* __restrict__ ws) {
  const int p = find_problem(bd.crt_start, bd.count, blockIdx.x);
  const BatchProb& q = bd.prob[p];
  s2_crt_block<CPLX>(ca, q.M, q.N, ws + q.off_res, reinterpret_cast<const int32_t*>(ws + q.off_sig),
                     reinterpret_cast<const int32_t*>(ws + q.off_tau), q.a_re, q.a_im, q.b_re, q.b_im, q.C, q.ldc,
                     blockIdx.x - bd.crt_start[p]);
}

int64_t s2_tile_count(bool cplx, int64_t M, int64_t N) {
  const int bm = cplx ? GemmTile<3, 2, 1, 4>::BM : GemmTile<1, 2, 2, 4>::BM;
  const int bn = cplx ? GemmTile<3, 2, 1, 4>::BN : GemmTile<1, 2, 2, 4>::BN;
  return ((M + bm - 1) / bm) * ((N + bn - 1) / bn);
}

int s2_batch_gemm_blocks_per_cu(bool cplx) {
  int n = 0;
  const int lds = cplx ? GemmTile<3, 2, 1, 4>::LDS_BYTES : GemmTile<1, 2, 2, 4>::LDS_BYTES;
  hipError_t e = cplx ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_b_gemm_mod<true>, 256, lds)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_b_gemm_mod<false>, 256, lds);
  return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t s2_batched(int s, bool cplx, const BatchDev& bd, const BatchTotals& tot, int8_t* ws, int gemm_grid,
                      hipStream_t st) {
  int ta, tb;
  CrtArgs ca;
  crt_args(s, ca, ta, tb);
  if (tot.rows == 0 || tot.crt == 0) return hipSuccess;
  S2Args sa{s, ta};
  const int lds = cplx ? GemmTile<3, 2, 1, 4>::LDS_BYTES : GemmTile<1, 2, 2, 4>::LDS_BYTES;
  static bool attr[2] = {false, false};
  if (!attr[cplx]) {
    hipError_t e = cplx ? hipFuncSetAttribute(reinterpret_cast<const void*>(k_b_gemm_mod<true>),
                                              hipFuncAttributeMaxDynamicSharedMemorySize, lds)
                        : hipFuncSetAttribute(reinterpret_cast<const void*>(k_b_gemm_mod<false>),
                                              hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    attr[cplx] = true;
  }
  if (cplx) {
    hipLaunchKernelGGL(k_b_split_rows<true>, dim3((unsigned)tot.rows), dim3(256), 0, st, bd, ws, sa);
    hipLaunchKernelGGL(k_b_col_scales<true>, dim3((unsigned)tot.cols), dim3(256), 0, st, bd, ws, tb);
    if (tot.split) hipLaunchKernelGGL(k_b_split_cols<true>, dim3((unsigned)tot.split), dim3(256), 0, st, bd, ws, s);
    if (tot.items) hipLaunchKernelGGL(k_b_gemm_mod<true>, dim3((unsigned)gemm_grid), dim3(256), lds, st, bd, ws, s);
    hipLaunchKernelGGL(k_b_crt<true>, dim3((unsigned)tot.crt), dim3(256), 0, st, ca, bd, ws);
  } else {
    hipLaunchKernelGGL(k_b_split_rows<false>, dim3((unsigned)tot.rows), dim3(256), 0, st, bd, ws, sa);
    hipLaunchKernelGGL(k_b_col_scales<false>, dim3((unsigned)tot.cols), dim3(256), 0, st, bd, ws, tb);
    if (tot.split) hipLaunchKernelGGL(k_b_split_cols<false>, dim3((unsigned)tot.split), dim3(256), 0, st, bd, ws, s);
    if (tot.items)
      hipLaunchKernelGGL(k_b_gemm_mod<false>, dim3((unsigned)gemm_grid), dim3(256), lds, st, bd, ws, s);
    hipLaunchKernelGGL(k_b_crt<false>, dim3((unsigned)tot.crt), dim3(256), 0, st, ca, bd, ws);
  }
  return hipGetLastError();
}

}  // namespace ozk
