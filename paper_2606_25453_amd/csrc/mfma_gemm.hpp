// The INT8 MFMA GEMM core shared by both schemes (gfx950, 32x32x32 i8 MFMA).
//
// Packed operands.  The paper's interleaved matrix (Eq. 11) is M x (P K):
// 32-wide column blocks j = c P + t hold slice t of K step c.  It is stored
// block-column by block-column: block j is one contiguous slab of Rp rows x
// 32 bytes,
//   packed[c][t][r][kk]  (byte ((c P + t) Rp + r) 32 + kk),
// so that the rows a workgroup needs from one block form one contiguous run
// and every 1 KB chunk (32 rows) is one direct-to-LDS wave load.
//
// Pairing of the P planes:
//   TRIANGULAR (Scheme I, Eq. 2):  acc[t + u] += A_t B_u  for t + u < P;
//   DIAGONAL   (3M, Eq. 16):       acc[q] += A_q B_q.
//
// Workgroup: 4 waves in a 2 x 2 grid, wave tile (32 TM) x (32 TN), P INT32
// accumulators per 32 x 32 MFMA tile for the whole K loop.  NS LDS stages of
// [P][BM][32] (A) + [P][BN][32] (B) bytes are filled with 16-byte
// global-to-LDS loads (no staging registers) NS - 1 steps ahead of use; one
// barrier per K step.  In LDS, 8 consecutive rows of one slab are 8 distinct
// 32-byte lines, so the 16-byte fragment reads are bank-conflict free.
#pragma once
#include "ozk_device.hpp"

namespace ozk {

enum Pairing { TRIANGULAR = 0, DIAGONAL = 1 };

template <int P, int TM, int TN, int NS>
struct GemmTile {
  static constexpr int BM = 64 * TM;
  static constexpr int BN = 64 * TN;
  static constexpr int A_BYTES = P * BM * OZK_K_CHUNK;
  static constexpr int B_BYTES = P * BN * OZK_K_CHUNK;
  static constexpr int STAGE = A_BYTES + B_BYTES;
  static constexpr int LDS_BYTES = NS * STAGE;
  static constexpr int CHUNKS = STAGE / 1024;    // 1 KB wave loads per stage
  static constexpr int CHUNKS_MIN = CHUNKS / 4;  // loads every wave issues at least
  static_assert(STAGE % 1024 == 0, "stage must be whole 1 KB chunks");
  static_assert(NS >= 2, "at least two stages");
};

// Workgroup barrier for LDS hand-over only: waits for this wave's LDS
// operations, then s_barrier.  Unlike __syncthreads() it does not drain the
// global loads in flight (the direct-to-LDS loads of later stages).  The
// memory clobber keeps the compiler from moving LDS accesses across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// s_waitcnt with only the vector-memory counter constrained (vmcnt <= n).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// This wave's share of the direct-to-LDS loads of one stage: chunk j of the
// wave is chunk q = 4 j + wave of the stage (A slabs first, then B).  The
// wave index is made wave-uniform (readfirstlane) so that every address is
// scalar except the 16-byte lane offset, and each chunk's source advances by
// a fixed stride per K step.
template <int P, int TM, int TN, int NS>
struct StageLoads {
  using T = GemmTile<P, TM, TN, NS>;
  static constexpr int NQ = (T::CHUNKS + 3) / 4;
  const int8_t* src[NQ];  // chunk source at step 0 (wave-uniform)
  int64_t stride[NQ];     // bytes per K step
  int dst[NQ];            // byte offset inside a stage
  int count;              // chunks this wave issues (NQ or NQ - 1)

  __device__ __forceinline__ StageLoads(const int8_t* Ap, const int8_t* Bp, int64_t rows_a, int64_t rows_b,
                                        int64_t m0, int64_t n0, int wave) {
    constexpr int A_CH = T::A_BYTES / 1024;
    count = 0;
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
      const int q = 4 * j + wave;
      if (q < T::CHUNKS) count = j + 1;
      if (q < A_CH) {
        const int t = q / (T::BM / 32), blk = q % (T::BM / 32);
        src[j] = Ap + ((int64_t)t * rows_a + m0 + 32 * blk) * OZK_K_CHUNK;
        stride[j] = (int64_t)P * rows_a * OZK_K_CHUNK;
        dst[j] = t * T::BM * OZK_K_CHUNK + blk * 1024;
      } else {
        const int qb = q < T::CHUNKS ? q - A_CH : 0;
        const int t = qb / (T::BN / 32), blk = qb % (T::BN / 32);
        src[j] = Bp + ((int64_t)t * rows_b + n0 + 32 * blk) * OZK_K_CHUNK;
        stride[j] = (int64_t)P * rows_b * OZK_K_CHUNK;
        dst[j] = T::A_BYTES + t * T::BN * OZK_K_CHUNK + blk * 1024;
      }
    }
  }

  __device__ __forceinline__ void issue(int64_t step, int8_t* stage_lds, int lane16) const {
#pragma unroll
    for (int j = 0; j < NQ; ++j)
      if (j < count)
        __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(src[j] + step * stride[j] + lane16),
                                         reinterpret_cast<void*>(stage_lds + dst[j]), 16, 0, 0);
  }
};

// Accumulate K steps [step0, step0 + nsteps) of the output tile at (m0, n0)
// into acc.  rows_a / rows_b: padded row counts of the packed operands.
template <int P, int TM, int TN, int NS, int PAIR>
__device__ __forceinline__ void gemm_tile_accumulate(const int8_t* __restrict__ Ap, const int8_t* __restrict__ Bp,
                                                     int64_t rows_a, int64_t rows_b, int64_t m0, int64_t n0,
                                                     int64_t step0, int64_t nsteps, int8_t* lds,
                                                     v16i (&acc)[P][TM][TN]) {
  using T = GemmTile<P, TM, TN, NS>;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  const int lrow = lane & 31, lk = 16 * (lane >> 5);
  const StageLoads<P, TM, TN, NS> ld(Ap, Bp, rows_a, rows_b, m0, n0, wave);
  // prologue: stages 0 .. NS-2
#pragma unroll
  for (int s = 0; s < NS - 1; ++s)
    if (s < nsteps) ld.issue(step0 + s, lds + s * T::STAGE, 16 * lane);
  int cur = 0;           // stage holding K step s
  int nxt = NS - 1;      // stage receiving K step s + NS - 1
  for (int64_t s = 0; s < nsteps; ++s) {
    // stage s complete for this wave: at most NS-2 later stages outstanding
    if (s + NS - 2 < nsteps) wait_vmcnt<(NS - 2) * T::CHUNKS_MIN>();
    else wait_vmcnt<0>();
    lds_barrier();  // every wave's part of stage s is in LDS; stage s-1 is free
    if (s + NS - 1 < nsteps) ld.issue(step0 + s + NS - 1, lds + nxt * T::STAGE, 16 * lane);
    const int8_t* la = lds + cur * T::STAGE;
    const int8_t* lb = la + T::A_BYTES;
    cur = cur + 1 == NS ? 0 : cur + 1;
    nxt = nxt + 1 == NS ? 0 : nxt + 1;
    v4i fa[P][TM];
#pragma unroll
    for (int t = 0; t < P; ++t)
#pragma unroll
      for (int a = 0; a < TM; ++a)
        fa[t][a] = *reinterpret_cast<const v4i*>(la + (t * T::BM + wm * 32 * TM + a * 32 + lrow) * OZK_K_CHUNK + lk);
#pragma unroll
    for (int u = 0; u < P; ++u) {
      v4i fb[TN];
#pragma unroll
      for (int b = 0; b < TN; ++b)
        fb[b] = *reinterpret_cast<const v4i*>(lb + (u * T::BN + wn * 32 * TN + b * 32 + lrow) * OZK_K_CHUNK + lk);
      if (PAIR == TRIANGULAR) {
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
  }
  lds_barrier();  // LDS free for the caller's next use
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

// Workgroup -> output tile.  Workgroups are dispatched round-robin over the
// 8 XCDs (each with its own L2): when the tile count divides by 8, XCD x
// takes a contiguous eighth of the tiles, walked in groups of G tile rows,
// so the ~32 tiles an XCD runs at once form a compact block whose A rows and
// B columns its L2 can keep.
__device__ __forceinline__ void tile_of(int64_t id, int64_t tiles_m, int64_t tiles_n, int64_t& tm, int64_t& tn) {
  const int64_t T = tiles_m * tiles_n;
  int64_t lin = id;
  if (T % 8 == 0) lin = (id % 8) * (T / 8) + id / 8;
  const int64_t G = 4;
  const int64_t per_group = G * tiles_n;
  const int64_t group = lin / per_group;
  const int64_t first = group * G;
  const int64_t gm = tiles_m - first < G ? tiles_m - first : G;
  const int64_t r = lin % per_group;
  tm = first + r % gm;
  tn = r / gm;
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
