// Fused Scheme I GEMM (paper Alg. 1, Eqs. 2-3): for every output tile the
// triangular slice-pair MFMAs into p INT32 diagonals held in registers for
// the whole K run, then the exact integer shift-reduce and one rounding per
// output.  Tile variants (for the autotuner) differ only in the wave tile
// shape and the number of LDS stages; every variant, raster order and K
// split computes the same integers, so all give bit-identical results.
#pragma once
#include "mfma_gemm.hpp"
#include "ozk_device.hpp"
#include "ozk_internal.hpp"

namespace ozk {

// Variant V of the tiling for p = P.  Base: p <= 4 takes 2 x 2 MFMA tiles per
// wave (128 x 128 workgroup tile, 16p * 4 accumulator registers), p >= 5
// takes 2 x 1 (128 x 64); stages: as many as fit 160 KB.  V bit 1 flips the
// wave tile (2 x 2 -> 2 x 1, 2 x 1 -> 1 x 2); V bit 0 uses one stage fewer.
template <int P, int V>
struct S1Cfg {
  static constexpr int TN_BASE = P <= 4 ? 2 : 1;
  static constexpr bool FLIP = (V & 2) != 0;
  static constexpr int TM = FLIP && TN_BASE == 1 ? 1 : 2;
  static constexpr int TN = FLIP ? (TN_BASE == 2 ? 1 : 2) : TN_BASE;
  static constexpr int NS = (P <= 2 ? 4 : 3) - (V & 1);
};

enum S1Out { S1_OUT_FINAL = 0, S1_OUT_PARTIAL = 1, S1_OUT_DIAG = 2, S1_OUT_FINAL_F32 = 3 };

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
  float* C32;
  const int32_t* p_dev;  // slice count chosen on the device; the kernel runs only if it equals P (null: always)
  int raster, group;     // workgroup -> tile order
  int64_t ntiles;        // output tiles; workgroup w takes tiles w, w + G, ... (G = grid size)
};

// One output tile (workgroup tile index `tile`, K run z): the triangular
// MFMA accumulation, then the epilogue selected by OUT.
template <int P, int OUT, int TM, int TN, int NS>
__device__ __forceinline__ void s1_gemm_tile(const S1KArgs& g, int64_t tile, int64_t z, int8_t* lds) {
  using T = GemmTile<P, TM, TN, NS>;
  const int64_t M = g.M, N = g.N;
  const int64_t tiles_m = (M + T::BM - 1) / T::BM, tiles_n = (N + T::BN - 1) / T::BN;
  int64_t tm, tn;
  tile_of(tile, tiles_m, tiles_n, g.raster, g.group, tm, tn);
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
    // Zero and non-finite lines have all-zero digits, so Z = 0 there: one
    // rounding for every element, then the NaN of a non-finite line.
    const int er = g.e_row[row], fc = g.f_col[col];
    const bool bad = er == OZK_EXP_NONFINITE || fc == OZK_EXP_NONFINITE;
    const bool live = !bad && er != OZK_EXP_ZERO && fc != OZK_EXP_ZERO;
    if (OUT == S1_OUT_FINAL_F32) {
      float h = round_scaled_f32(Z, live ? er + fc - 12 - 8 * (P - 1) : 0);
      h = bad ? __builtin_nanf("") : h;
      float* cp = g.C32 + row * g.ldc + col;
      *cp = axpby_f32((float)g.alpha, h, (float)g.beta, cp);
      return;
    }
    double h = round_scaled(Z, live ? er + fc - 12 - 8 * (P - 1) : 0);
    h = bad ? __builtin_nan("") : h;
    double* cp = g.C + row * g.ldc + col;
    *cp = axpby(g.alpha, h, g.beta, cp);
  });
}

template <int P, int OUT, int V>
__global__ __launch_bounds__(256, 1) void k_s1_gemm(S1KArgs g) {
  using Cfg = S1Cfg<P, V>;
  extern __shared__ __attribute__((aligned(1024))) int8_t lds[];
  if (g.p_dev && *g.p_dev != P) return;  // another slice count was chosen
  // One tile per workgroup, except on the automatic path, whose grid is
  // capped so that the kernels of the slice counts not chosen dispatch few
  // workgroups; a stride that is a multiple of 8 keeps each tile on the XCD
  // the raster order meant it for.
  for (int64_t tile = blockIdx.x; tile < g.ntiles; tile += gridDim.x)
    s1_gemm_tile<P, OUT, Cfg::TM, Cfg::TN, Cfg::NS>(g, tile, blockIdx.z, lds);
}

// Tiles of the workgroup grid for variant v at p (host side).
template <int P, int V>
inline int64_t s1_tiles_v(int64_t M, int64_t N) {
  using Cfg = S1Cfg<P, V>;
  using T = GemmTile<P, Cfg::TM, Cfg::TN, Cfg::NS>;
  return ((M + T::BM - 1) / T::BM) * ((N + T::BN - 1) / T::BN);
}

template <int P, int OUT, int V>
hipError_t s1_launch_pov(const S1GemmArgs& g, const int32_t* p_dev, hipStream_t st) {
  using Cfg = S1Cfg<P, V>;
  using T = GemmTile<P, Cfg::TM, Cfg::TN, Cfg::NS>;
  static_assert(T::LDS_BYTES <= 160 * 1024, "LDS budget");
  auto kern = k_s1_gemm<P, OUT, V>;
  static std::atomic<uint64_t> lds_done{0};
  const hipError_t e_lds = lds_limit(reinterpret_cast<const void*>(kern), T::LDS_BYTES, lds_done);
  if (e_lds != hipSuccess) return e_lds;
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
  k.C32 = g.C32;
  k.p_dev = p_dev;
  k.raster = g.raster;
  k.group = g.group;
  k.ntiles = s1_tiles_v<P, V>(g.M, g.N);
  // the automatic path: at most 512 workgroups (two per CU, a multiple of 8)
  const int64_t gx = p_dev && k.ntiles > 512 ? 512 : k.ntiles;
  const dim3 grid((unsigned)gx, 1, (unsigned)g.nsplit);
  hipLaunchKernelGGL(kern, grid, dim3(256), T::LDS_BYTES, st, k);
  return hipGetLastError();
}

// The GEMM of slice count P with the output mode and tile variant of g.
static_assert(OZK_S1_VARIANTS == 4, "the variant switch below covers four variants");

template <int P>
hipError_t s1_gemm_launch(int out, const S1GemmArgs& g, const int32_t* p_dev, hipStream_t st) {
  if (out == S1_OUT_DIAG) return s1_launch_pov<P, S1_OUT_DIAG, 0>(g, p_dev, st);
#define OZK_S1_VARIANT_CASES(OUT)                                 \
  switch (g.variant) {                                       \
    case 0: return s1_launch_pov<P, OUT, 0>(g, p_dev, st);   \
    case 1: return s1_launch_pov<P, OUT, 1>(g, p_dev, st);   \
    case 2: return s1_launch_pov<P, OUT, 2>(g, p_dev, st);   \
    case 3: return s1_launch_pov<P, OUT, 3>(g, p_dev, st);   \
  }
  if (out == S1_OUT_PARTIAL) {
    OZK_S1_VARIANT_CASES(S1_OUT_PARTIAL)
  } else if (out == S1_OUT_FINAL_F32) {
    OZK_S1_VARIANT_CASES(S1_OUT_FINAL_F32)
  } else {
    OZK_S1_VARIANT_CASES(S1_OUT_FINAL)
  }
#undef OZK_S1_VARIANT_CASES
  return hipErrorInvalidValue;
}

extern template hipError_t s1_gemm_launch<1>(int, const S1GemmArgs&, const int32_t*, hipStream_t);
extern template hipError_t s1_gemm_launch<2>(int, const S1GemmArgs&, const int32_t*, hipStream_t);
extern template hipError_t s1_gemm_launch<3>(int, const S1GemmArgs&, const int32_t*, hipStream_t);
extern template hipError_t s1_gemm_launch<4>(int, const S1GemmArgs&, const int32_t*, hipStream_t);
extern template hipError_t s1_gemm_launch<5>(int, const S1GemmArgs&, const int32_t*, hipStream_t);
extern template hipError_t s1_gemm_launch<6>(int, const S1GemmArgs&, const int32_t*, hipStream_t);
extern template hipError_t s1_gemm_launch<7>(int, const S1GemmArgs&, const int32_t*, hipStream_t);
extern template hipError_t s1_gemm_launch<8>(int, const S1GemmArgs&, const int32_t*, hipStream_t);

}  // namespace ozk
