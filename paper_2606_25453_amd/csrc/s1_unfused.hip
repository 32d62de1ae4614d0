// The unfused Scheme I baseline of the paper's traffic model (Sec. III,
// Eq. 9), kept as an ablation of the fused kernel: every slice pair (t, u)
// with t + u < p is its own INT8 GEMM whose INT32 result goes to HBM, and a
// reconstruction pass reads the p(p+1)/2 planes back, forms
// Z = sum 2^(8(p-1-t-u)) C_tu exactly and rounds once.  Same operands and
// same result as the fused path; only the INT32 round trip differs.
//
//   k_s1_pair_gemm     C_tu = A_t B_u for one pair per grid z index (the
//                      shared MFMA core with one plane per step: slice t of
//                      the packed operand is every p-th slab)
//   k_s1_pairs_reduce  the exact weighted sum of the planes, one rounding
#include "mfma_gemm.hpp"
#include "ozk_device.hpp"
#include "ozk_internal.hpp"

namespace ozk {

namespace {

constexpr int PAIR_TM = 2, PAIR_TN = 2, PAIR_NS = 4;  // 128 x 128 tiles, four stages
using PairTile = GemmTile<1, PAIR_TM, PAIR_TN, PAIR_NS>;

struct PairArgs {
  int t[36], u[36];  // slice indices of pair z (p(p+1)/2 <= 36 pairs)
};

__global__ __launch_bounds__(256, 1) void k_s1_pair_gemm(const int8_t* __restrict__ Ap, const int8_t* __restrict__ Bp,
                                                        int64_t rows_a, int64_t rows_b, int p, int64_t nchunk, int M,
                                                        int N, PairArgs pa, int32_t* __restrict__ planes) {
  extern __shared__ __attribute__((aligned(1024))) int8_t lds[];
  const int z = blockIdx.z;
  const int64_t tiles_m = (M + PairTile::BM - 1) / PairTile::BM, tiles_n = (N + PairTile::BN - 1) / PairTile::BN;
  int64_t tm, tn;
  tile_of(blockIdx.x, tiles_m, tiles_n, 0, 4, tm, tn);
  const int64_t m0 = tm * PairTile::BM, n0 = tn * PairTile::BN;
  v16i acc[1][PAIR_TM][PAIR_TN];
  zero_acc<1, PAIR_TM, PAIR_TN>(acc);
  // slice t of K chunk c is the slab (c p + t): base t, one chunk step = p slabs
  gemm_tile_accumulate<1, PAIR_TM, PAIR_TN, PAIR_NS, DIAGONAL, 1>(
      Ap + (int64_t)pa.t[z] * rows_a * OZK_K_CHUNK, Bp + (int64_t)pa.u[z] * rows_b * OZK_K_CHUNK, p * rows_a,
      p * rows_b, m0, n0, 0, nchunk, lds, acc);
  int32_t* out = planes + (int64_t)z * M * N;
  for_each_output<1, PAIR_TM, PAIR_TN>(acc, m0, n0, M, N,
                                       [&](int64_t row, int64_t col, const int* vals) { out[row * N + col] = vals[0]; });
}

__global__ __launch_bounds__(256) void k_s1_pairs_reduce(const int32_t* __restrict__ planes, int npairs, PairArgs pa,
                                                         int M, int N, int p, const int32_t* __restrict__ e_row,
                                                         const int32_t* __restrict__ f_col, double alpha, double beta,
                                                         double* __restrict__ C, int64_t ldc) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t mn = (int64_t)M * N;
  if (idx >= mn) return;
  const int64_t row = idx / N, col = idx % N;
  i128 Z = 0;
  for (int z = 0; z < npairs; ++z) Z += (i128)planes[z * mn + idx] * ((i128)1 << (8 * (p - 1 - pa.t[z] - pa.u[z])));
  const int er = e_row[row], fc = f_col[col];
  const bool bad = er == OZK_EXP_NONFINITE || fc == OZK_EXP_NONFINITE;
  const bool zero = er == OZK_EXP_ZERO || fc == OZK_EXP_ZERO;
  const double h = bad ? __builtin_nan("") : zero ? 0.0 : round_scaled(Z, er + fc - 12 - 8 * (p - 1));
  double* cp = C + row * ldc + col;
  *cp = axpby(alpha, h, beta, cp);
}

}  // namespace

int64_t s1_unfused_planes_bytes(int p, int64_t M, int64_t N) { return (int64_t)p * (p + 1) / 2 * M * N * 4; }

hipError_t s1_gemm_unfused(int p, int64_t M, int64_t N, int64_t K, const int8_t* Ap, const int32_t* e,
                           const int8_t* Bp, const int32_t* f, double alpha, double beta, double* C, int64_t ldc,
                           int32_t* planes, hipStream_t st) {
  if (M == 0 || N == 0) return hipSuccess;
  PairArgs pa;
  int n = 0;
  for (int d = 0; d < p; ++d)
    for (int t = 0; t <= d; ++t, ++n) {
      pa.t[n] = t;
      pa.u[n] = d - t;
    }
  static std::atomic<uint64_t> lds_done{0};
  const hipError_t e_lds = lds_limit(reinterpret_cast<const void*>(k_s1_pair_gemm), PairTile::LDS_BYTES, lds_done);
  if (e_lds != hipSuccess) return e_lds;
  const int64_t ra = round_up(M, OZK_ROW_ALIGN), rb = round_up(N, OZK_ROW_ALIGN);
  const int64_t nchunk = round_up(K, OZK_K_CHUNK) / OZK_K_CHUNK;
  const int64_t tiles = ((M + PairTile::BM - 1) / PairTile::BM) * ((N + PairTile::BN - 1) / PairTile::BN);
  hipLaunchKernelGGL(k_s1_pair_gemm, dim3((unsigned)tiles, 1, (unsigned)n), dim3(256), PairTile::LDS_BYTES, st, Ap,
                     Bp, ra, rb, p, nchunk, (int)M, (int)N, pa, planes);
  const int64_t mn = M * N;
  hipLaunchKernelGGL(k_s1_pairs_reduce, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, st, planes, n, pa, (int)M,
                     (int)N, p, e, f, alpha, beta, C, ldc);
  return hipGetLastError();
}

}  // namespace ozk
