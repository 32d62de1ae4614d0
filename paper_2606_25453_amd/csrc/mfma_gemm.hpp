// The INT8 MFMA GEMM core shared by both schemes (gfx950, 32x32x32 i8 MFMA).
//
// Operands are "packed": row r of an operand (a row of A, a column of B)
// holds, K step after K step of 32, the P slices (planes) of that step side
// by side -- the interleaved layout of the paper's Eq. 11 with t_K = 32:
//   packed[r][c][t][kk],  r < rows (padded), c < K/32, t < P, kk < 32.
// The row stride is (K/32) * P * 32 bytes.
//
// Pairing of the P planes:
//   TRIANGULAR (Scheme I, Eq. 2):  acc[t + u] += A_t B_u  for t + u < P,
//                                  i.e. P(P+1)/2 products into P diagonals;
//   DIAGONAL   (3M, Eq. 16):       acc[q] += A_q B_q, P independent products.
//
// Workgroup: 4 waves in a 2 x 2 grid, wave tile (32 TM) x (32 TN), P INT32
// accumulators per 32 x 32 MFMA tile kept in registers for the whole K loop.
// Per K step the workgroup stages BM x (P x 32) bytes of A and BN x (P x 32)
// of B through LDS (two buffers, one barrier per step; rows padded by 16 B
// so that the 16-byte fragment reads of 8 consecutive rows hit distinct
// banks).  Every wave reads its P A-fragments once per step and streams the
// B-fragments one plane at a time.  The epilogue functor receives, for each
// output element it owns, the P accumulator values.
#pragma once
#include "ozk_device.hpp"

namespace ozk {

enum Pairing { TRIANGULAR = 0, DIAGONAL = 1 };

template <int P, int TM, int TN>
struct GemmTile {
  static constexpr int BM = 64 * TM;
  static constexpr int BN = 64 * TN;
  static constexpr int ROW_BYTES = P * OZK_K_CHUNK;
  static constexpr int LDS_STRIDE = ROW_BYTES + 16;
  static constexpr int PIECES = (BM + BN) * ROW_BYTES / 16;
  static constexpr int PIECES_PER_THREAD = (PIECES + 255) / 256;
  static constexpr int LDS_BUF = (BM + BN) * LDS_STRIDE;
  static constexpr int LDS_BYTES = 2 * LDS_BUF;
};

// Accumulate the K steps [step0, step0 + nsteps) of the output tile at
// (m0, n0) into acc.  Ap, Bp point at row 0 of the packed operands; the
// packed row stride is row_bytes.
template <int P, int TM, int TN, int PAIR>
__device__ __forceinline__ void gemm_tile_accumulate(const int8_t* __restrict__ Ap, const int8_t* __restrict__ Bp,
                                                     int64_t row_bytes, int64_t m0, int64_t n0, int64_t step0,
                                                     int64_t nsteps, int8_t* lds, v16i (&acc)[P][TM][TN]) {
  using T = GemmTile<P, TM, TN>;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  uint4 stage[T::PIECES_PER_THREAD];
  auto load_step = [&](int64_t s) {
#pragma unroll
    for (int q = 0; q < T::PIECES_PER_THREAD; ++q) {
      const int idx = tid + 256 * q;
      if (idx < T::PIECES) {
        const int row = idx / (2 * P), piece = idx % (2 * P);
        const int8_t* src = (row < T::BM) ? Ap + (m0 + row) * row_bytes : Bp + (n0 + row - T::BM) * row_bytes;
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
      if (PAIR == TRIANGULAR) {
        // plane u of B meets planes t <= P-1-u of A: A_t B_u adds to diagonal t + u
#pragma unroll
        for (int t = 0; t + u < P; ++t)
#pragma unroll
          for (int a = 0; a < TM; ++a)
#pragma unroll
            for (int b = 0; b < TN; ++b) acc[t + u][a][b] = mfma_i8_32x32x32(fa[t][a], fb[b], acc[t + u][a][b]);
      } else {
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
          for (int b = 0; b < TN; ++b) acc[u][a][b] = mfma_i8_32x32x32(fa[u][a], fb[b], acc[u][a][b]);
      }
    }
    if (s + 1 < nsteps) store_step(buf ^ 1);
    __syncthreads();
  }
}

template <int P, int TM, int TN>
__device__ __forceinline__ void zero_acc(v16i (&acc)[P][TM][TN]) {
#pragma unroll
  for (int d = 0; d < P; ++d)
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b) acc[d][a][b] = v16i{0};
}

// Visit every output element of the wave's tile: f(row, col, vals) with
// vals[d] the accumulator d of that element.  Rows/columns outside
// [0, M) x [0, N) are skipped.
template <int P, int TM, int TN, class F>
__device__ __forceinline__ void for_each_output(const v16i (&acc)[P][TM][TN], int64_t m0, int64_t n0, int64_t M,
                                                int64_t N, F&& f) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = m0 + wm * 32 * TM + a * 32 + 8 * (v / 4) + 4 * (lane >> 5) + (v % 4);
        const int64_t col = n0 + wn * 32 * TN + b * 32 + (lane & 31);
        if (row >= M || col >= N) continue;
        int vals[P];
#pragma unroll
        for (int d = 0; d < P; ++d) vals[d] = acc[d][a][b][v];
        f(row, col, vals);
      }
}

}  // namespace ozk
