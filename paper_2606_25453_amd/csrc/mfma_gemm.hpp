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
//   DIAGONAL   (3M, Eq. 16):       acc[q mod PACC] += A_q B_q.
// With PACC < P the P planes of one K step are G = P / PACC consecutive K
// chunks of a PACC-plane operand (in the block-column layout those are
// consecutive slabs), summed into the same PACC accumulators: a stage then
// carries G chunks and one barrier serves G times the MFMAs.
//
// Workgroup: 4 waves in a 2 x 2 grid, wave tile (32 TM) x (32 TN), P INT32
// accumulators per 32 x 32 MFMA tile for the whole K loop.  NS LDS stages of
// [P][BM][32] (A) + [P][BN][32] (B) bytes are filled with 16-byte
// global-to-LDS loads (no staging registers) up to NS - 1 steps ahead of
// use; one barrier per K step; the fragments of the next step are read from
// LDS while the MFMAs of the current one run.
//
// LDS swizzle.  A fragment read has lane l take row r = l % 32, 16-byte half
// h = l / 32 of a slab; stored plainly, rows r and r + 4 (r + 8) of one
// 8-lane (16-lane) group hit the same banks.  Each 32-byte row therefore
// stores its halves in the order h ^ f(r), f(r) = bit 2 of r ^ bit 3 of r,
// which spreads every group over all banks.  The direct-to-LDS load writes
// lane i's 16 bytes to chunk offset 16 i, so the permutation is applied on
// the global side: lane i loads the piece 16 (i ^ f(i / 2)) of its 1 KB chunk.
#pragma once
#include <utility>

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
  static constexpr int CHUNKS = STAGE / 1024;       // 1 KB wave loads per stage
  static constexpr int WAVE_LOADS = (CHUNKS + 3) / 4;  // loads each wave issues per stage
  static_assert(STAGE % 1024 == 0, "stage must be whole 1 KB chunks");
  static_assert(NS >= 2, "at least two stages");
};

// Workgroup barrier for LDS hand-over only: waits for this wave's LDS
// operations (lgkmcnt(0), through the builtin so that the compiler's own
// wait insertion knows those reads have landed), then s_barrier.  Unlike
// __syncthreads() it does not drain the global loads in flight (the
// direct-to-LDS loads of later stages).  The memory clobber keeps the
// compiler from moving LDS accesses across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // vmcnt 63, expcnt 7, lgkmcnt 0
  asm volatile("s_barrier" ::: "memory");
}

// s_waitcnt with only the vector-memory counter constrained (vmcnt <= n).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// One 16-byte-per-lane direct-to-LDS load: lane i's 16 bytes at gsrc land at
// lds_dst + 16 i.  Issued as inline assembly so that the compiler does not
// track it as an LDS write: its own tracking cannot tell LDS stages apart and
// would wait for every load in flight before each fragment read, which
// defeats staging more than one step ahead.  Completion is therefore the
// caller's business: an explicit vmcnt wait, then a barrier, before any wave
// reads the stage (vmcnt counts these loads like any other).  M0 holds the
// LDS base; one wait state separates its write from the load.
__device__ __forceinline__ void lds_dma16(const int8_t* gsrc, int8_t* lds_dst) {
  const uint32_t m0 = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) int8_t*)lds_dst;
  asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, off" ::"s"(m0), "v"(gsrc) : "memory", "m0");
}

// This wave's share of the direct-to-LDS loads of one stage: chunk j of the
// wave is chunk q = 4 j + wave of the stage (A slabs first, then B).  When
// the stage's chunk count is not a multiple of 4, the waves without a chunk
// of their own reload the last one (the same bytes to the same LDS address),
// so that every wave issues exactly NQ loads and the vmcnt thresholds below
// are exact.  Addresses: a wave-uniform 64-bit base per operand that advances
// by one K step per stage, a wave-uniform 32-bit offset per chunk, and the
// lane's 16-byte offset as the only per-lane value.
template <int P, int TM, int TN, int NS>
struct StageLoads {
  using T = GemmTile<P, TM, TN, NS>;
  static constexpr int NQ = (T::CHUNKS + 3) / 4;
  static constexpr int A_CH = T::A_BYTES / 1024;
  const int8_t* a_next;  // A tile rows at the next K step to issue
  const int8_t* b_next;
  int64_t a_step, b_step;  // bytes per K step
  uint32_t off[NQ];        // chunk offset from its operand's base
  uint32_t dst[NQ];        // byte offset inside a stage

  __device__ __forceinline__ StageLoads(const int8_t* Ap, const int8_t* Bp, int64_t rows_a, int64_t rows_b,
                                        int64_t m0, int64_t n0, int64_t step0, int wave) {
    a_step = (int64_t)P * rows_a * OZK_K_CHUNK;
    b_step = (int64_t)P * rows_b * OZK_K_CHUNK;
    a_next = Ap + m0 * OZK_K_CHUNK + step0 * a_step;
    b_next = Bp + n0 * OZK_K_CHUNK + step0 * b_step;
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
      int q = 4 * j + wave;
      q = q < T::CHUNKS ? q : T::CHUNKS - 1;
      if (q < A_CH) {
        const int t = q / (T::BM / 32), blk = q % (T::BM / 32);
        off[j] = (uint32_t)(t * rows_a * OZK_K_CHUNK + blk * 1024);
        dst[j] = (uint32_t)(t * T::BM * OZK_K_CHUNK + blk * 1024);
      } else {
        const int qb = q - A_CH;
        const int t = qb / (T::BN / 32), blk = qb % (T::BN / 32);
        off[j] = (uint32_t)(t * rows_b * OZK_K_CHUNK + blk * 1024);
        dst[j] = (uint32_t)(T::A_BYTES + t * T::BN * OZK_K_CHUNK + blk * 1024);
      }
    }
  }

  // Bases of the next stage to issue.  A real stage (valid) advances the
  // cursor; past the last real stage the last one is loaded again, into a
  // slot that is never read, so that every step issues the same loads and
  // the vmcnt thresholds stay fixed.
  __device__ __forceinline__ void next(bool valid, const int8_t*& a_base, const int8_t*& b_base) {
    a_base = valid ? a_next : a_next - a_step;
    b_base = valid ? b_next : b_next - b_step;
    if (valid) {
      a_next += a_step;
      b_next += b_step;
    }
  }

  // Chunk j of the stage with bases a_base / b_base into the stage at stage_lds.
  __device__ __forceinline__ void issue_one(int j, const int8_t* a_base, const int8_t* b_base, int8_t* stage_lds,
                                            uint32_t lane16, int wave) {
    // A or B chunk: decided at compile time unless j's group of 4 chunks
    // straddles the end of the A slabs
    const bool is_a = (4 * j + 3 < A_CH) || (4 * j < A_CH && 4 * j + wave < A_CH);
    lds_dma16((is_a ? a_base : b_base) + off[j] + lane16, stage_lds + dst[j]);
  }

  // All loads of the next stage.
  __device__ __forceinline__ void issue(int8_t* stage_lds, uint32_t lane16, int wave, bool valid) {
    const int8_t *a_base, *b_base;
    next(valid, a_base, b_base);
#pragma unroll
    for (int j = 0; j < NQ; ++j) issue_one(j, a_base, b_base, stage_lds, lane16, wave);
  }
};

// The MFMA operands of one K step for one wave: P planes of TM A fragments
// and TN B fragments (16 bytes per lane each).
template <int P, int TM, int TN>
struct StepFrags {
  v4i a[P][TM];
  v4i b[P][TN];
};

// Read a step's fragments from its LDS stage (issued only: the caller's next
// lds_barrier waits for them).  Order of first use: B plane 0, the A planes,
// then B planes 1..P-1.
template <int P, int TM, int TN, int NS>
__device__ __forceinline__ void read_frags(StepFrags<P, TM, TN>& F, const int8_t* la, int wm, int wn, int lrow,
                                           int lk) {
  using T = GemmTile<P, TM, TN, NS>;
  const int8_t* lb = la + T::A_BYTES;
#pragma unroll
  for (int b = 0; b < TN; ++b)
    F.b[0][b] = *reinterpret_cast<const v4i*>(lb + (wn * 32 * TN + b * 32 + lrow) * OZK_K_CHUNK + lk);
#pragma unroll
  for (int t = 0; t < P; ++t)
#pragma unroll
    for (int a = 0; a < TM; ++a)
      F.a[t][a] = *reinterpret_cast<const v4i*>(la + (t * T::BM + wm * 32 * TM + a * 32 + lrow) * OZK_K_CHUNK + lk);
#pragma unroll
  for (int u = 1; u < P; ++u)
#pragma unroll
    for (int b = 0; b < TN; ++b)
      F.b[u][b] = *reinterpret_cast<const v4i*>(lb + (u * T::BN + wn * 32 * TN + b * 32 + lrow) * OZK_K_CHUNK + lk);
}

// Fragment read i of a step, in the order of read_frags (B plane 0, the A
// planes, B planes 1..P-1); i is a compile-time constant after unrolling.
template <int P, int TM, int TN, int NS>
__device__ __forceinline__ void read_frag(StepFrags<P, TM, TN>& F, int i, const int8_t* la, int wm, int wn, int lrow,
                                          int lk) {
  using T = GemmTile<P, TM, TN, NS>;
  const int8_t* lb = la + T::A_BYTES;
  if (i < TN) {
    F.b[0][i] = *reinterpret_cast<const v4i*>(lb + (wn * 32 * TN + i * 32 + lrow) * OZK_K_CHUNK + lk);
  } else if (i < TN + P * TM) {
    const int t = (i - TN) / TM, a = (i - TN) % TM;
    F.a[t][a] = *reinterpret_cast<const v4i*>(la + (t * T::BM + wm * 32 * TM + a * 32 + lrow) * OZK_K_CHUNK + lk);
  } else {
    const int u = 1 + (i - TN - P * TM) / TN, b = (i - TN - P * TM) % TN;
    F.b[u][b] = *reinterpret_cast<const v4i*>(lb + (u * T::BN + wn * 32 * TN + b * 32 + lrow) * OZK_K_CHUNK + lk);
  }
}

// Instruction order of one K step after its barrier: one LDS fragment read,
// then MPR MFMAs, repeated for all NR reads, then the remaining MFMAs.  The
// reads of the next step thus start at once and are spread over most of the
// step instead of being bunched at its end (where the next barrier's wait
// would expose their latency), while never more than one read sits between
// two MFMA issues.  The direct-to-LDS loads of the refill sit in source order
// between the reads (one before each of the first NQ reads; their memory
// clobber pins them there), so they too are spread over the step instead of
// queueing at the texture path before the first MFMA.
template <int MPR, int... I>
__device__ __forceinline__ void sched_reads_mfmas(std::integer_sequence<int, I...>) {
  (((void)I, __builtin_amdgcn_sched_group_barrier(0x100, 1, 0), __builtin_amdgcn_sched_group_barrier(0x008, MPR, 0)),
   ...);
}

template <int NR, int NM>
__device__ __forceinline__ void sched_step() {
  constexpr int MPR = NM / NR >= 2 ? 2 : 1;
  sched_reads_mfmas<MPR>(std::make_integer_sequence<int, NR>{});
  if constexpr (NM > MPR * NR) __builtin_amdgcn_sched_group_barrier(0x008, NM - MPR * NR, 0);
}

template <int P, int TM, int TN>
__device__ __forceinline__ void zero_frags(StepFrags<P, TM, TN>& F) {
#pragma unroll
  for (int t = 0; t < P; ++t) {
#pragma unroll
    for (int a = 0; a < TM; ++a) F.a[t][a] = v4i{0, 0, 0, 0};
#pragma unroll
    for (int b = 0; b < TN; ++b) F.b[t][b] = v4i{0, 0, 0, 0};
  }
}

template <int P, int TM, int TN, int PAIR, int PACC>
__device__ __forceinline__ void step_mfmas(const StepFrags<P, TM, TN>& F, v16i (&acc)[PACC][TM][TN]) {
#pragma unroll
  for (int u = 0; u < P; ++u) {
    if (PAIR == TRIANGULAR) {
#pragma unroll
      for (int t = 0; t + u < P; ++t)
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
          for (int b = 0; b < TN; ++b) acc[t + u][a][b] = mfma_i8_32x32x32(F.a[t][a], F.b[u][b], acc[t + u][a][b]);
    } else {
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
          acc[u % PACC][a][b] = mfma_i8_32x32x32(F.a[u][a], F.b[u][b], acc[u % PACC][a][b]);
    }
  }
}

// Accumulate K steps [step0, step0 + nsteps) of the output tile at (m0, n0)
// into acc.  rows_a / rows_b: padded row counts of the packed operands.
//
// K step r lives in LDS slot r mod NS.  Software pipeline, per step r (its
// fragments already in registers): wait until stage r+1 has landed,
// barrier (every wave is also done reading slot r mod NS), refill that slot
// with stage r+NS, issue the fragment reads of step r+1 into the other
// register set, then the MFMAs of step r, which run while those reads
// complete.  The two register sets alternate, so steps are processed in
// pairs; an odd step count is made even by a leading virtual step r = -1
// with zero fragments (its MFMAs add nothing).  Inside the loop every step
// has a real successor, so no branch there defines a register.
//
// hook(r) runs after the MFMAs of every step r (-1 for the virtual step): a
// caller that walks several independent sums along one K axis (the moduli of
// one output tile) stores and clears the accumulators there, while the loads
// of the following steps are already in flight.
struct NoStepHook {
  __device__ __forceinline__ void operator()(int64_t) const {}
};

template <int P, int TM, int TN, int NS, int PAIR, int PACC = P, class Hook = NoStepHook>
__device__ __forceinline__ void gemm_tile_accumulate(const int8_t* __restrict__ Ap, const int8_t* __restrict__ Bp,
                                                     int64_t rows_a, int64_t rows_b, int64_t m0, int64_t n0,
                                                     int64_t step0, int64_t nsteps, int8_t* lds,
                                                     v16i (&acc)[PACC][TM][TN], Hook hook = Hook()) {
  static_assert(PAIR == DIAGONAL ? P % PACC == 0 : PACC == P, "accumulator planes");
  using T = GemmTile<P, TM, TN, NS>;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  // fragment row and swizzled half (see the LDS swizzle above)
  const int lrow = lane & 31, lk = 16 * ((lane >> 5) ^ (((lane >> 2) ^ (lane >> 3)) & 1));
  StageLoads<P, TM, TN, NS> ld(Ap, Bp, rows_a, rows_b, m0, n0, step0, wave);
  if (nsteps <= 0) return;
  const uint32_t lane16 = 16u * (uint32_t)(lane ^ (((lane >> 3) ^ (lane >> 4)) & 1));  // source piece of lane
  const int lead = (int)(nsteps & 1);  // 1: a virtual step -1 comes first
  // stages issued ahead: 0 .. NS-1 (NS-2 with the virtual step, whose own
  // refill issues stage NS-1); stages past the last one load it again
#pragma unroll
  for (int s = 0; s < NS; ++s)
    if (s < NS - 1 || !lead) ld.issue(lds + s * T::STAGE, lane16, wave, s < nsteps);
  StepFrags<P, TM, TN> F0, F1;
  if (lead) {
    zero_frags<P, TM, TN>(F0);
  } else {
    wait_vmcnt<(NS - 1) * T::WAVE_LOADS>();
    lds_barrier();
    read_frags<P, TM, TN, NS>(F0, lds, wm, wn, lrow, lk);
  }
  int slot = lead ? NS - 1 : 0;  // slot of step r (the virtual step: the slot stage NS-1 goes to)
  // Step r = v - lead with a real successor q = r + 1: MFMAs from Fc, the
  // fragments of q into Fn, the refill of slot r mod NS with stage r + NS.
  // Every step issues one stage, so exactly NS - 2 stages follow stage q when
  // it is waited for.
  auto step = [&](int64_t v, const StepFrags<P, TM, TN>& Fc, StepFrags<P, TM, TN>& Fn) {
    const int64_t r = v - lead;
    constexpr int NQ = StageLoads<P, TM, TN, NS>::NQ;
    constexpr int NR = P * (TM + TN);
    constexpr int NM = (PAIR == TRIANGULAR ? P * (P + 1) / 2 : P) * TM * TN;
    wait_vmcnt<(NS - 2) * T::WAVE_LOADS>();
    lds_barrier();
    const int8_t *a_base, *b_base;
    ld.next(r + NS < nsteps, a_base, b_base);
    int8_t* fill = lds + slot * T::STAGE;
    slot = slot + 1 == NS ? 0 : slot + 1;
    const int8_t* rd = lds + slot * T::STAGE;
#pragma unroll
    for (int i = 0; i < (NQ > NR ? NQ : NR); ++i) {
      if (i < NQ) ld.issue_one(i, a_base, b_base, fill, lane16, wave);
      if (i < NR) read_frag<P, TM, TN, NS>(Fn, i, rd, wm, wn, lrow, lk);
    }
    step_mfmas<P, TM, TN, PAIR, PACC>(Fc, acc);
    sched_step<NR, NM>();
    __builtin_amdgcn_sched_barrier(0);  // nothing of this step moves past the next barrier
    hook(r);
  };
  const int64_t total = nsteps + lead;  // even, >= 2
  int64_t v = 0;
  for (; v + 2 < total; v += 2) {
    step(v, F0, F1);
    step(v + 1, F1, F0);
  }
  step(v, F0, F1);  // the last pair: its second step has no successor
  step_mfmas<P, TM, TN, PAIR, PACC>(F1, acc);
  hook(nsteps - 1);
  wait_vmcnt<0>();  // the repeated last stages have landed too
  lds_barrier();    // LDS free for the caller's next use
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
// 8 XCDs (each with its own L2).  raster 0: when the tile count divides by 8,
// XCD x takes a contiguous eighth of the tiles, so the ~32 tiles an XCD runs
// at once form a compact block whose A rows and B columns its L2 can keep;
// raster 1: dispatch order as is.  Either way the linear order is walked in
// groups of `group` tile rows (column-major inside a group).
__device__ __forceinline__ void tile_of(int64_t id, int64_t tiles_m, int64_t tiles_n, int raster, int group,
                                        int64_t& tm, int64_t& tn) {
  const int64_t T = tiles_m * tiles_n;
  int64_t lin = id;
  if (raster == 0 && T % 8 == 0) lin = (id % 8) * (T / 8) + id / 8;
  const int64_t G = group > 0 ? group : 1;
  const int64_t per_group = G * tiles_n;
  const int64_t grp = lin / per_group;
  const int64_t first = grp * G;
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
