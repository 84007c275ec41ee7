// The two contractions of the method and the modal-current epilogue:
//   Xdot_n(t)   = sum_j E[j][n] u_j(t)        (Eq. 13)
//   A_n^mu(t)   = sum_j E[j][n] w^mu_j(t)     (bracket of Eq. 16)
//   J_n^mu(t)   = Xdot_n(t) A_n^mu(t)         (Eq. 16)
// done as one product of E^T (slots x dofs) with the four stacked channels
// (u, w^x, w^y, w^z) of the B operand, so Xdot and the three A^mu of a
// (mode, step) pair land in the same lane and register of four accumulators.
//
// Two paths:
//   * per-step FP32 matrix-vector product (t_block = 1): E is streamed from
//     HBM once per step;
//   * T-batched matrix-core GEMM (FP32 or split-BF16): E tiles are staged
//     through LDS and reused across the 4 channels and all steps of a tile.
#include <algorithm>

#include "mhc.h"
#include "mhc_common.h"

namespace mhc {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

// Two 16-byte units -> the 32-byte e4m3 operand of one lane.
__device__ __forceinline__ i32x8 cat8(u32x4 a, u32x4 b) {
  return __builtin_bit_cast(i32x8, __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7));
}

// D += A*B for e4m3 x e4m3 (scale exponents 127 = 2^0: no block scaling).
__device__ __forceinline__ f32x16 mfma_fp8(i32x8 a, i32x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
}

// acc += E x activations in the orientation TR (see acc_row below); e is the
// E fragment, b the activation fragment.
template <bool TR>
__device__ __forceinline__ f32x16 mm_bf16(bf16x8 e, bf16x8 b, f32x16 c) {
  return TR ? __builtin_amdgcn_mfma_f32_32x32x16_bf16(b, e, c, 0, 0, 0)
            : __builtin_amdgcn_mfma_f32_32x32x16_bf16(e, b, c, 0, 0, 0);
}
template <bool TR>
__device__ __forceinline__ f32x16 mm_fp8(i32x8 e, i32x8 b, f32x16 c) {
  return TR ? mfma_fp8(b, e, c) : mfma_fp8(e, b, c);
}
template <bool TR>
__device__ __forceinline__ f32x16 mm_f32(float e, float b, f32x16 c) {
  return TR ? __builtin_amdgcn_mfma_f32_32x32x2f32(b, e, c, 0, 0, 0)
            : __builtin_amdgcn_mfma_f32_32x32x2f32(e, b, c, 0, 0, 0);
}

// Row of the 32x32 accumulator held in register j of lane l (column = l % 32).
// The A and B operand layouts of the MFMAs are the same, so the order of the
// arguments chooses the orientation of the accumulators:
//   TR = false (GKMA): E fragment as A, activations as B: rows are slots,
//     columns are steps, so a half-wave's store of one register is 32
//     consecutive steps of one slot;
//   TR = true (HNEMA): activations as A, E as B: rows are steps, columns are
//     slots, so the sum over steps is a sum over the lane's own registers
//     plus one exchange between the two half-waves.
__device__ __forceinline__ int acc_row(int j, int half) { return 8 * (j >> 2) + 4 * half + (j & 3); }

// ----------------------------------------------------------- per-step FP32
// One wave = 8 consecutive slots x one step.  E is stored row-major for this
// path (slot-major, dofs contiguous), so a wave's load of one row is 64 lanes
// x 4 dofs = 1 KiB contiguous; the lane's 4 dofs of the four activation
// channels are loaded once and used for all 8 rows.  Both operands are
// double-buffered in registers (the loads of the next 256 dofs are in flight
// while the current ones are consumed).  Per (row, channel) each lane keeps
// one partial sum; the 64 lanes are combined by a fixed butterfly.  Waves are
// ordered row group fastest, so the chip streams E once per step, step after
// step.
typedef __attribute__((address_space(1))) const f32x4 gf32x4;
constexpr int GEMV_ROWS = 8;

__global__ void __launch_bounds__(256)
k_gemv_f32(const f32x4* __restrict__ E, const float* __restrict__ B, int n_steps, int64_t M_pad,
           int64_t K_pad, float* __restrict__ out, int layout_g, int64_t ld) {
  constexpr int R = GEMV_ROWS;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t n_rg = M_pad / R;
  const int64_t unit = (int64_t)blockIdx.x * 4 + wave;
  if (unit >= n_rg * n_steps) return;
  const int t = (int)(unit / n_rg);
  const int64_t rg = unit - (int64_t)t * n_rg;
  const int64_t KC = K_pad >> 2;                       // 16-byte units per row
  const gf32x4* Er = (const gf32x4*)E + rg * R * KC;
  const gf32x4* Bt = (const gf32x4*)B + (int64_t)t * 4 * KC;
  const int64_t n_it = KC / 64;                         // even: K_pad is a multiple of 512
  float acc[R][4];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.f;
  f32x4 ea[R], eb[R], ba[4], bb[4];
  auto load = [&](f32x4 (&e)[R], f32x4 (&bv)[4], int64_t it) {
    const int64_t u = it * 64 + lane;
#pragma unroll
    for (int r = 0; r < R; ++r) e[r] = __builtin_nontemporal_load(Er + r * KC + u);
#pragma unroll
    for (int c = 0; c < 4; ++c) bv[c] = Bt[c * KC + u];
  };
  auto consume = [&](const f32x4 (&e)[R], const f32x4 (&bv)[4]) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        float a = acc[r][c];
        a = fmaf(e[r].x, bv[c].x, a);
        a = fmaf(e[r].y, bv[c].y, a);
        a = fmaf(e[r].z, bv[c].z, a);
        a = fmaf(e[r].w, bv[c].w, a);
        acc[r][c] = a;
      }
  };
  // iterations in pairs; the prefetch after the last pair re-reads the last
  // iteration and is not consumed
  load(ea, ba, 0);
  for (int64_t it = 0; it < n_it; it += 2) {
    load(eb, bb, it + 1);
    __builtin_amdgcn_sched_barrier(0);   // keep each load batch ahead of the other set's FMAs
    consume(ea, ba);
    __builtin_amdgcn_sched_barrier(0);
    load(ea, ba, min(it + 2, n_it - 1));
    __builtin_amdgcn_sched_barrier(0);
    consume(eb, bb);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      float a = acc[r][c];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
      acc[r][c] = a;
    }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (lane != r) continue;
    const int64_t slot = rg * R + r;
    const float x = acc[r][0];
    if (!layout_g) {
      float* o = out + ((int64_t)t * M_pad + slot) * 3;
      o[0] = x * acc[r][1]; o[1] = x * acc[r][2]; o[2] = x * acc[r][3];
    } else {
      out[(0 * M_pad + slot) * ld + t] = x * acc[r][1];
      out[(1 * M_pad + slot) * ld + t] = x * acc[r][2];
      out[(2 * M_pad + slot) * ld + t] = x * acc[r][3];
    }
  }
}

hipError_t launch_gemv_f32(hipStream_t s, const float* E, const float* B, int n_steps, int64_t M_pad,
                           int64_t K_pad, float* out, int layout_g, int64_t ld) {
  if (n_steps <= 0) return hipSuccess;
  if (M_pad % GEMV_ROWS != 0 || K_pad % K_ALIGN_GEMV != 0) return hipErrorInvalidValue;
  const int64_t units = (M_pad / GEMV_ROWS) * n_steps;
  hipLaunchKernelGGL(k_gemv_f32, dim3((unsigned)((units + 3) / 4)), dim3(256), 0, s,
                     reinterpret_cast<const f32x4*>(E), B, n_steps, M_pad, K_pad, out, layout_g, ld);
  return hipGetLastError();
}

// ------------------------------------------------------------ matrix cores
// Work-group = 4 waves arranged WM x WT; each wave owns MB row blocks (32 slots
// each) and one t-block of 32 steps, for all four channels: 4*MB accumulators
// of 32x32 floats.  A tile is WM*MB row blocks x WT t-blocks.
//
// Both operands are laid out per row/column block as [stage][SU] u32x4
// (SU = 256 units of 16 bytes = 4 KiB per row block per stage):
//   FP32:  stage of 32 dofs,  unit chunk*64 + lane             (chunk = 8 dofs)
//   BF16:  stage of 32 dofs,  unit (chunk*2 + hi/lo)*64 + lane  (chunk = 16 dofs)
//   FP8X3: stage of 64 dofs,  unit (hi/lo*2 + q)*64 + lane      (one 64-dof chunk)
//   FP8:   stage of 128 dofs, unit (chunk*2 + q)*64 + lane      (chunk = 64 dofs)
// (q selects the lower or upper 16 bytes of a lane's 32-byte e4m3 operand).
// e4m3 operands carry a per-slot scale (E) and a per-(channel, step) scale
// (activations) that the epilogue applies.
//
// Pipeline (branch-free, unrolled by two stages so the two A staging sets are
// static).  At the top of stage s a wave issues its share of the A fragments
// of stage s+2 (E streamed from HBM) into staging registers; it then runs the
// MFMAs of stage s chunk by chunk (A from LDS, B from registers), refilling
// each chunk's B registers with the same chunk of stage s+1 as soon as they
// are consumed; finally it stores the A fragments of stage s+1 (issued one
// stage earlier) into the other LDS buffer and synchronizes.  Loads retire in
// issue order, so every wait the compiler inserts leaves the newer loads in
// flight: B (L2-resident activations) has one stage of MFMAs to arrive, A
// (HBM) two.
//
// Scheduling (stream-K): the tiles x stages iteration space is cut into G
// equal contiguous ranges, one per work-group, so every CU gets the same
// number of MFMAs whatever the tile count.  A work-group walks its range tile
// segment by tile segment; a segment that covers a whole tile goes straight
// to the epilogue, a partial one is written (in accumulator register order)
// to a workspace slot.  k_gemm_fixup then adds the partials of each split
// tile in work-group order and runs the same epilogue, so no work-group ever
// waits on another and the result is deterministic.  With ipw = n_stages and
// G = n_tiles this is the plain one-tile-per-work-group schedule.
constexpr int SU = 256;

typedef __attribute__((address_space(1))) const u32x4 gu32x4;

constexpr bool is_fp8(int prec) { return prec == PREC_FP8 || prec == PREC_FP8X3; }
// dofs per k-stage: 32 (FP32, BF16), 64 (FP8X3), 128 (FP8)
constexpr int stage_dofs(int prec) { return prec == PREC_FP8 ? 128 : (prec == PREC_FP8X3 ? 64 : 32); }

// Epilogue of one finished tile (accumulators complete); TR = !layout_g.
// TR: lane l holds slot (row block, l % 32) and, in register j, step
// acc_row(j, l / 32) of the wave's t-block; otherwise the reverse.
// c0: the first channel whose activation scales are still to be undone (e4m3;
// 1 when channel 0 already carries them, as in the later directions of the
// one-contraction split).
template <int PREC, int WM, int WT, int MB, bool TR>
__device__ __forceinline__ void gemm_epilogue(f32x16 (&acc)[MB][4], float* __restrict__ out, const GemmGeom& g,
                                              int64_t rb0, int ntile, float* red, int c0 = 0) {
  constexpr int RBW = WM * MB;
  const int tid = threadIdx.x, lane = tid & 63, half = lane >> 5, wave = tid >> 6;
  const int wm = wave / WT, wt = wave % WT;
  const int64_t t0 = (int64_t)(ntile * WT + wt) * 32;          // first step of the wave's t-block
  const int64_t ld = (int64_t)g.ntb * 32;
  if constexpr (is_fp8(PREC)) {
    // undo the activation scales of each step; the E scale of each slot is
    // applied after the products
    if constexpr (TR) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int64_t t = t0 + acc_row(j, half);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (c < c0) continue;
          const float cs = g.col_scale[c * ld + t];
#pragma unroll
          for (int rb = 0; rb < MB; ++rb) acc[rb][c][j] *= cs;
        }
      }
    } else {
      const int64_t t = t0 + (lane & 31);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (c < c0) continue;
        const float cs = g.col_scale[c * ld + t];
#pragma unroll
        for (int rb = 0; rb < MB; ++rb)
#pragma unroll
          for (int j = 0; j < 16; ++j) acc[rb][c][j] *= cs;
      }
    }
  }
  auto row_factor = [&](int64_t slot) -> float {
    if constexpr (is_fp8(PREC)) {
      const float rs = g.row_scale[slot];
      return rs * rs;                     // J = (s_n Xdot') (s_n A')
    } else {
      return 1.f;
    }
  };
  if constexpr (TR) {
    // HNEMA: sum J_n^mu over the tile's steps -> out[ntile][slot][mu]: the
    // lane's 16 steps in register order, plus the other half-wave's 16, then
    // the WT t-blocks in wave order through LDS
#pragma unroll
    for (int rb = 0; rb < MB; ++rb) {
      float p0 = 0.f, p1 = 0.f, p2 = 0.f;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        p0 += acc[rb][0][j] * acc[rb][1][j];
        p1 += acc[rb][0][j] * acc[rb][2][j];
        p2 += acc[rb][0][j] * acc[rb][3][j];
      }
      p0 += __shfl_xor(p0, 32);
      p1 += __shfl_xor(p1, 32);
      p2 += __shfl_xor(p2, 32);
      if (half == 0) {
        const int row = (wm * MB + rb) * 32 + lane;
        const float f = row_factor(rb0 * 32 + row);
        float* rp = red + ((int64_t)wt * RBW * 32 + row) * 3;
        rp[0] = p0 * f; rp[1] = p1 * f; rp[2] = p2 * f;
      }
    }
    __syncthreads();
    for (int idx = tid; idx < RBW * 32 * 3; idx += 256) {
      float sacc = 0.f;
#pragma unroll
      for (int w = 0; w < WT; ++w) sacc += red[w * RBW * 32 * 3 + idx];
      out[((int64_t)ntile * g.M_pad + rb0 * 32) * 3 + idx] = sacc;
    }
    __syncthreads();
  } else {
    // GKMA: per-step J_n^mu(t) -> out[mu][slot][t]
    const int64_t t = t0 + (lane & 31);
#pragma unroll
    for (int rb = 0; rb < MB; ++rb) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int64_t slot = (rb0 + wm * MB + rb) * 32 + acc_row(j, half);
        const float f = row_factor(slot);
#pragma unroll
        for (int mu = 0; mu < 3; ++mu)
          out[((int64_t)mu * g.M_pad + slot) * ld + t] = acc[rb][0][j] * acc[rb][1 + mu][j] * f;
      }
    }
  }
}

// Work-group id -> position in the iteration space.  Consecutive ids go to
// different XCDs (round-robin dispatch); give each XCD a contiguous range.
__device__ __forceinline__ int64_t wg_linear(int id, int G) {
  return (G % 8 == 0) ? (int64_t)(id % 8) * (G / 8) + id / 8 : id;
}

template <int PREC>
struct GemmCfg {
  static constexpr bool BF = (PREC == PREC_BF16X3);
  static constexpr bool F8 = (PREC == PREC_FP8), F8X3 = (PREC == PREC_FP8X3);
  // units per chunk: FP32 64, BF16 128 (hi, lo), FP8 128 (two q halves), FP8X3 256
  static constexpr int UPC = (PREC == PREC_FP32) ? 64 : (F8X3 ? 256 : 128);
  static constexpr int CPS = SU / UPC;                           // chunks per stage
  static constexpr int NBF = 4 * UPC / 64;                       // B units per chunk per lane
  static constexpr int NBS = NBF * CPS;                          // B units per stage per lane
  // 16-byte units per row block per dof: 4 B per element for FP32 and BF16
  // hi+lo, 2 B for FP8X3, 1 B for FP8 (times 32 rows / 16 bytes)
  static constexpr int UNITS_PER_DOF2 = F8 ? 2 : (F8X3 ? 4 : 8);
};

// Accumulate stages [s0, s1) of the tile with row blocks rb0.. and t-block
// column tb (per wave) into acc, in the orientation TR; channels below c0
// keep their values and add to them.  All 256 threads take part; lds is the
// double-buffered A stage.  Leaves the work-group synchronized.
template <int PREC, int WM, int WT, int MB, bool TR>
__device__ __forceinline__ void gemm_segment(const GemmGeom& g, int64_t rb0, int ntile, int s0, int s1,
                                             f32x16 (&acc)[MB][4], u32x4 (*lds)[WM * MB][SU], int c0 = 0) {
  using C = GemmCfg<PREC>;
  constexpr int RBW = WM * MB;
  constexpr int UPC = C::UPC, CPS = C::CPS, NBF = C::NBF, NBS = C::NBS;
  constexpr int A_PER_THR = RBW * SU / 256;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);     // wave-uniform
  const int lane = tid & 63;
  const int wm = wave / WT;
  const int wt = wave % WT;
  const int tb = ntile * WT + wt;
  const int64_t per_blk = C::UNITS_PER_DOF2 * g.K_pad;          // 16-byte units per row/column block

  u32x4 ast0[A_PER_THR], ast1[A_PER_THR];
  i32x8 bq[NBS / 2];
  // Global-address-space views: the grouped kernel reads g from memory, and
  // through generic pointers the loads would become flat loads, which count
  // against the LDS wait counter too (every LDS wait would drain them).
  // Bases are wave-uniform (scalar registers); the lane offset is added per
  // load, so the loads use the scalar-base form and cost no 64-bit vector
  // address registers.
  static_assert(SU == 256 && A_PER_THR == RBW, "one A unit per thread per row block and stage");
  const gu32x4* Ebase = (const gu32x4*)g.E + rb0 * per_blk;
  // E is streamed once (non-temporal) unless sibling t-tiles of the same
  // rows run alongside and re-read it: then it is kept in L2 for them.
  const bool e_keep = g.n_ntiles > 1;
  auto load_A = [&](int s, u32x4* dst) {
    if (e_keep) {
#pragma unroll
      for (int q = 0; q < A_PER_THR; ++q) dst[q] = Ebase[((int64_t)q * per_blk + (int64_t)s * SU) + tid];
    } else {
#pragma unroll
      for (int q = 0; q < A_PER_THR; ++q)
        dst[q] = __builtin_nontemporal_load(Ebase + ((int64_t)q * per_blk + (int64_t)s * SU) + tid);
    }
  };
  auto store_A = [&](int buf, const u32x4* src) {
#pragma unroll
    for (int q = 0; q < A_PER_THR; ++q) lds[buf][q][tid] = src[q];
  };
  const gu32x4* Bw[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) Bw[c] = (const gu32x4*)g.B + ((int64_t)c * g.ntb + tb) * per_blk;
  // Chunk kk of stage s into NBF/2 eight-dword registers, units paired in
  // (channel, unit) order: FP32 (c0,c1)(c2,c3); BF16 (hi,lo) per channel;
  // FP8 (q0,q1) per channel; FP8X3 (hi q0,q1)(lo q0,q1) per channel.
  auto load_B = [&](int s, int kk, i32x8* dst) {
    constexpr int UPCH = UPC / 64;                      // units per channel per chunk
    const int64_t u = (int64_t)s * SU + kk * UPC;
#pragma unroll
    for (int p = 0; p < NBF / 2; ++p) {
      const int i0 = 2 * p, i1 = 2 * p + 1;
      dst[p] = cat8((Bw[i0 / UPCH] + (u + (i0 % UPCH) * 64))[lane], (Bw[i1 / UPCH] + (u + (i1 % UPCH) * 64))[lane]);
    }
  };
  auto lo4 = [](i32x8 v) { return __builtin_shufflevector(v, v, 0, 1, 2, 3); };
  auto hi4 = [](i32x8 v) { return __builtin_shufflevector(v, v, 4, 5, 6, 7); };
  // MFMAs of one stage (A from LDS buffer `buf`, B from `bs`); after chunk
  // kk is consumed its registers are refilled with chunk kk of `s_next`.
  auto compute = [&](int buf, i32x8* bs, int s_next) {
#pragma unroll
    for (int kk = 0; kk < CPS; ++kk) {
      i32x8* bc = bs + kk * (NBF / 2);
      if constexpr (C::BF) {
        bf16x8 ah[MB], al[MB];
#pragma unroll
        for (int rb = 0; rb < MB; ++rb) {
          ah[rb] = __builtin_bit_cast(bf16x8, lds[buf][wm * MB + rb][(kk * 2 + 0) * 64 + lane]);
          al[rb] = __builtin_bit_cast(bf16x8, lds[buf][wm * MB + rb][(kk * 2 + 1) * 64 + lane]);
        }
        __builtin_amdgcn_sched_barrier(0);     // all fragment reads in flight before the first MFMA
        // hi*hi, hi*lo, lo*hi, interleaved over the 4*MB independent accumulators
        // (lo4 of a channel's register is its hi part, hi4 its lo part)
#pragma unroll
        for (int rb = 0; rb < MB; ++rb)
#pragma unroll
          for (int c = 0; c < 4; ++c)
            acc[rb][c] = mm_bf16<TR>(ah[rb], __builtin_bit_cast(bf16x8, lo4(bc[c])), acc[rb][c]);
#pragma unroll
        for (int rb = 0; rb < MB; ++rb)
#pragma unroll
          for (int c = 0; c < 4; ++c)
            acc[rb][c] = mm_bf16<TR>(ah[rb], __builtin_bit_cast(bf16x8, hi4(bc[c])), acc[rb][c]);
#pragma unroll
        for (int rb = 0; rb < MB; ++rb)
#pragma unroll
          for (int c = 0; c < 4; ++c)
            acc[rb][c] = mm_bf16<TR>(al[rb], __builtin_bit_cast(bf16x8, lo4(bc[c])), acc[rb][c]);
      } else if constexpr (C::F8X3) {
#pragma unroll
        for (int rb = 0; rb < MB; ++rb) {
          const u32x4* ar = &lds[buf][wm * MB + rb][lane];
          const i32x8 ah = cat8(ar[0], ar[64]);
          const i32x8 al = cat8(ar[128], ar[192]);
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[rb][c] = mm_fp8<TR>(ah, bc[2 * c + 0], acc[rb][c]);
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[rb][c] = mm_fp8<TR>(ah, bc[2 * c + 1], acc[rb][c]);
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[rb][c] = mm_fp8<TR>(al, bc[2 * c + 0], acc[rb][c]);
        }
      } else if constexpr (C::F8) {
#pragma unroll
        for (int rb = 0; rb < MB; ++rb) {
          const u32x4* ar = &lds[buf][wm * MB + rb][kk * 128 + lane];
          const i32x8 a = cat8(ar[0], ar[64]);
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[rb][c] = mm_fp8<TR>(a, bc[c], acc[rb][c]);
        }
      } else {
        f32x4 a[MB];
#pragma unroll
        for (int rb = 0; rb < MB; ++rb)
          a[rb] = __builtin_bit_cast(f32x4, lds[buf][wm * MB + rb][kk * 64 + lane]);
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int rb = 0; rb < MB; ++rb)
#pragma unroll
            for (int c = 0; c < 4; ++c)
              acc[rb][c] = mm_f32<TR>(
                  a[rb][e], __builtin_bit_cast(f32x4, (c & 1) ? hi4(bc[c >> 1]) : lo4(bc[c >> 1]))[e], acc[rb][c]);
      }
      // keep the issue order: this chunk's MFMAs, then its refill loads
      __builtin_amdgcn_sched_barrier(0);
      load_B(s_next, kk, bc);
      __builtin_amdgcn_sched_barrier(0);
    }
  };

  // channels c0 .. 3 start from zero (c0 = 1 keeps the running Xdot)
#pragma unroll
  for (int rb = 0; rb < MB; ++rb)
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c >= c0) {
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[rb][c][j] = 0.f;
      }

  // prologue: A(s0) -> LDS buffer 0, A(s0+1) in staging set 1, B(s0) in registers
  const int last = s1 - 1;
  load_A(s0, ast0);
#pragma unroll
  for (int kk = 0; kk < CPS; ++kk) load_B(s0, kk, bq + kk * (NBF / 2));
  load_A(min(s0 + 1, last), ast1);
  store_A(0, ast0);
  __syncthreads();

  int s = s0;
  for (; s + 1 < s1; s += 2) {
    // even stage s: B(s) in bq, A(s+1) in ast1, A(s) in LDS buffer 0
    load_A(min(s + 2, last), ast0);
    __builtin_amdgcn_sched_barrier(0);
    compute(0, bq, min(s + 1, last));
    store_A(1, ast1);
    __syncthreads();
    // odd stage s+1: B(s+1) in bq, A(s+2) in ast0, A(s+1) in LDS buffer 1
    load_A(min(s + 3, last), ast1);
    __builtin_amdgcn_sched_barrier(0);
    compute(1, bq, min(s + 2, last));
    store_A(0, ast0);
    __syncthreads();
  }
  if (s < s1) {
    // odd stage count: the last stage sits in LDS buffer 0, its B in bq
    compute(0, bq, last);
    __syncthreads();
  }
}

// Partial accumulators of one tile in a workspace slot, laid out so that
// every store and load of the 256 threads is one contiguous 1 KiB row.
template <int MB>
__device__ __forceinline__ void acc_store(float* __restrict__ w, const f32x16 (&acc)[MB][4]) {
#pragma unroll
  for (int rb = 0; rb < MB; ++rb)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int j = 0; j < 16; ++j) w[((rb * 4 + c) * 16 + j) * 256] = acc[rb][c][j];
}

template <int MB, bool ADD>
__device__ __forceinline__ void acc_load(const float* __restrict__ w, f32x16 (&acc)[MB][4]) {
#pragma unroll
  for (int rb = 0; rb < MB; ++rb)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const float x = w[((rb * 4 + c) * 16 + j) * 256];
        acc[rb][c][j] = ADD ? acc[rb][c][j] + x : x;
      }
}

template <int PREC, int WM, int WT, int MB, bool TR>
__global__ void __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(1, 1)))
k_gemm(float* __restrict__ ws, GemmGeom g) {
  constexpr int RBW = WM * MB;
  constexpr int NREG = MB * 4 * 16;                              // accumulator floats per lane
  __shared__ u32x4 lds[2][RBW][SU];
  const int tid = threadIdx.x;
  const int n_stages = g.n_stages;
  const int64_t gl = wg_linear(blockIdx.x, gridDim.x);
  const int64_t it_begin = gl * g.ipw;
  const int64_t it_end = min(g.total_iters, it_begin + g.ipw);
  f32x16 acc[MB][4];
  for (int64_t it = it_begin; it < it_end;) {
    const int64_t tile = it / n_stages;
    const int s0 = (int)(it - tile * n_stages);
    const int s1 = (int)min((int64_t)n_stages, s0 + (it_end - it));
    const int mtile = (int)(tile / g.n_ntiles);
    const int ntile = (int)(tile % g.n_ntiles);
    const int64_t rb0 = (int64_t)mtile * RBW;
    gemm_segment<PREC, WM, WT, MB, TR>(g, rb0, ntile, s0, s1, acc, lds);
    if (s0 == 0 && s1 == n_stages) {
      gemm_epilogue<PREC, WM, WT, MB, TR>(acc, g.out, g, rb0, ntile, reinterpret_cast<float*>(&lds[0][0][0]));
    } else {
      // partial tile: slot 0 = this work-group's first segment, 1 = its last
      acc_store<MB>(ws + ((gl * 2 + (it == it_begin ? 0 : 1)) * NREG) * 256 + tid, acc);
    }
    it += s1 - s0;
    __syncthreads();
  }
}

// Lockstep split schedule: one persistent work-group per CU.  The first
// q x G tiles go round by round, one whole tile per work-group.  The R < G
// remaining tiles are cut along k into m pieces so that the idle CUs of the
// last round take part, while every group of work-groups that runs
// concurrently walks the same k-stages (so the activation slices they read
// stay shared in L2):
//   Q > 0 (many remainder tiles): piece 0 = stages [0, c) of tile i on
//     work-group i, piece 1 = [c, S) on work-group R + i % Q, which takes
//     the tails of tiles i, i + Q, ... one after the other (m = 2);
//   Q = 0 (few remainder tiles): piece p = [p S / m, (p + 1) S / m) of tile
//     i on work-group p R + i.
// Each piece is stored to its workspace slot p R + i, and the work-group
// whose piece arrives last (a per-tile counter) adds the m pieces in piece
// order and runs the epilogue, so the result does not depend on the arrival
// order.  That work-group resets the counter, which is zero between
// launches.  No work-group waits for another.
struct SplitPlan {
  int q;      // rounds of whole tiles
  int R;      // remainder tiles q G .. q G + R - 1
  int m;      // pieces per remainder tile (1: whole tiles)
  int Q;      // tail work-groups (Q > 0: main + tail pieces)
  int c;      // Q > 0: first stage of the tail piece
  int* cnt;   // R arrival counters
};

__device__ __forceinline__ int split_stage(const SplitPlan& sp, int S, int p) {
  if (sp.Q > 0) return p == 0 ? 0 : (p == 1 ? sp.c : S);
  return (int)(((int64_t)p * S) / sp.m);
}

template <int PREC, int WM, int WT, int MB, bool TR>
__global__ void __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(1, 1)))
k_gemm_split(float* __restrict__ ws, GemmGeom g, SplitPlan sp) {
  constexpr int RBW = WM * MB;
  constexpr int NREG = MB * 4 * 16;
  __shared__ u32x4 lds[2][RBW][SU];
  __shared__ int arrived;
  const int tid = threadIdx.x;
  const int G = gridDim.x;
  const int gl = (int)wg_linear(blockIdx.x, G);
  const int S = g.n_stages;
  // this work-group's remainder pieces: piece p of tiles i0, i0 + stride, ...
  int p = 0, i0 = sp.R, stride = 1;
  if (sp.R > 0) {
    if (sp.Q > 0) {
      p = gl < sp.R ? 0 : 1;
      i0 = p == 0 ? gl : gl - sp.R;
      stride = p == 0 ? sp.R : sp.Q;
    } else if (gl / sp.R < sp.m) {
      p = gl / sp.R;
      i0 = gl % sp.R;
      stride = sp.R;
    }
  }
  const int64_t per_slot = (int64_t)NREG * 256;
  f32x16 acc[MB][4];
  // jobs 0 .. q-1: whole tiles gl + w G; then the remainder pieces
  for (int job = 0;; ++job) {
    int64_t tile;
    int s0 = 0, s1 = S, i = 0;
    bool piece = false;
    if (job < sp.q) {
      tile = (int64_t)job * G + gl;
    } else {
      i = i0 + (job - sp.q) * stride;
      if (i >= sp.R) break;
      tile = (int64_t)sp.q * G + i;
      s0 = split_stage(sp, S, p);
      s1 = split_stage(sp, S, p + 1);
      piece = sp.m > 1;
    }
    const int64_t rb0 = (tile / g.n_ntiles) * RBW;
    const int ntile = (int)(tile % g.n_ntiles);
    gemm_segment<PREC, WM, WT, MB, TR>(g, rb0, ntile, s0, s1, acc, lds);
    bool finish = true;
    if (piece) {
      float* base = ws + tid;
      acc_store<MB>(base + (int64_t)(p * sp.R + i) * per_slot, acc);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // write this piece back from L2
      __syncthreads();
      if (tid == 0) arrived = atomicAdd(&sp.cnt[i], 1);
      __syncthreads();
      finish = arrived == sp.m - 1;
      if (finish) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // drop stale lines before reading the others
        // pieces 0 + 1 (commutative, so this one may come from registers),
        // then 2 .. m-1 in order
        if (p <= 1) {
          acc_load<MB, true>(base + (int64_t)((1 - p) * sp.R + i) * per_slot, acc);
        } else {
          acc_load<MB, false>(base + (int64_t)i * per_slot, acc);
          acc_load<MB, true>(base + (int64_t)(sp.R + i) * per_slot, acc);
        }
        for (int r = 2; r < sp.m; ++r) acc_load<MB, true>(base + (int64_t)(r * sp.R + i) * per_slot, acc);
        if (tid == 0) sp.cnt[i] = 0;
      }
    }
    if (finish) gemm_epilogue<PREC, WM, WT, MB, TR>(acc, g.out, g, rb0, ntile, reinterpret_cast<float*>(&lds[0][0][0]));
    __syncthreads();
  }
}

// The bracket channels (1 .. 3) of the accumulators in a workspace slot,
// one contiguous 1 KiB row per store or load of the 256 threads.
template <int MB>
__device__ __forceinline__ void bracket_store(float* __restrict__ w, const f32x16 (&acc)[MB][4]) {
#pragma unroll
  for (int rb = 0; rb < MB; ++rb)
#pragma unroll
    for (int c = 1; c < 4; ++c)
#pragma unroll
      for (int j = 0; j < 16; ++j) w[((rb * 3 + c - 1) * 16 + j) * 256] = acc[rb][c][j];
}

template <int MB>
__device__ __forceinline__ void bracket_load(const float* __restrict__ w, f32x16 (&acc)[MB][4]) {
#pragma unroll
  for (int rb = 0; rb < MB; ++rb)
#pragma unroll
    for (int c = 1; c < 4; ++c)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[rb][c][j] = w[((rb * 3 + c - 1) * 16 + j) * 256];
}

// Motion-direction split in one contraction (Sec. II, remark after Eq. 10).
// K is ordered direction-major (dof (i, nu) at k = nu n3 + i, each third a
// whole number s3 of stages), so the bracket of Eq. 16 restricted to
// direction nu, A_n^{mu nu} = sum_i W_i^{mu nu} e_{i,n}^nu / sqrt(m_i), is
// the contraction over third nu alone, while Xdot_n needs all of K.  Channel
// 0 therefore runs on across the thirds and channels 1 .. 3 restart at each;
// the brackets of thirds 0 and 1 wait in the work-group's two workspace slots
// until Xdot is complete, then the epilogue runs once per direction into
// out + nu * region.  The MFMA work is that of one plain contraction.
// Persistent: work-group b takes tiles b, b + G, ...
// One tile of the one-contraction direction split: the three thirds, the
// brackets of thirds 0 and 1 through the work-group's slots (slot = this
// thread's position in them), then the three epilogues.  Leaves the
// work-group synchronized.
template <int PREC, int WM, int WT, int MB, bool TR>
__device__ __forceinline__ void dir_tile(const GemmGeom& g, int64_t rb0, int ntile, float* slot, f32x16 (&acc)[MB][4],
                                         u32x4 (*lds)[WM * MB][SU]) {
  constexpr int NBR = MB * 3 * 16;                               // bracket floats per lane
  float* red = reinterpret_cast<float*>(&lds[0][0][0]);
  for (int nu = 0; nu < 3; ++nu) {
    gemm_segment<PREC, WM, WT, MB, TR>(g, rb0, ntile, nu * g.s3, (nu + 1) * g.s3, acc, lds, nu == 0 ? 0 : 1);
    if (nu < 2) bracket_store<MB>(slot + (int64_t)nu * NBR * 256, acc);
  }
  // e4m3: every third of a channel was quantised with the whole column's
  // scale, so the scales are undone once on Xdot and once per bracket
  gemm_epilogue<PREC, WM, WT, MB, TR>(acc, g.out + 2 * g.region, g, rb0, ntile, red);
  for (int nu = 0; nu < 2; ++nu) {
    bracket_load<MB>(slot + (int64_t)nu * NBR * 256, acc);
    gemm_epilogue<PREC, WM, WT, MB, TR>(acc, g.out + nu * g.region, g, rb0, ntile, red, 1);
  }
  __syncthreads();
}

// Persistent: work-group b takes tiles b, b + G, ... of one system.
template <int PREC, int WM, int WT, int MB, bool TR>
__global__ void __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(1, 1)))
k_gemm_dir(GemmGeom g) {
  constexpr int RBW = WM * MB;
  constexpr int NBR = MB * 3 * 16;
  __shared__ u32x4 lds[2][RBW][SU];
  static_assert(2 * RBW * SU * 4 >= WT * RBW * 32 * 3, "the epilogue reuses the A stages' LDS");
  const int64_t n_tiles = (g.M_pad / (RBW * 32)) * g.n_ntiles;
  float* slot = g.ws + (int64_t)blockIdx.x * 2 * NBR * 256 + threadIdx.x;
  f32x16 acc[MB][4];
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x)
    dir_tile<PREC, WM, WT, MB, TR>(g, (tile / g.n_ntiles) * RBW, (int)(tile % g.n_ntiles), slot, acc, lds);
}

// Several systems in one persistent launch: work-groups pull whole tiles
// (system, m-tile, n-tile) from a queue ordered largest-first; every tile is
// computed entirely by one work-group, so the results do not depend on which
// work-group took it.  The queue ends for every wave at the same counter
// value, so all work-groups exit.

// DIRG: the group holds systems with the one-contraction direction split
// (their tiles take the three-third procedure).  A separate instantiation,
// because the extra path raises the register pressure of the e4m3 kernels
// into spills inside their product loops.
template <int PREC, int WM, int WT, int MB, bool DIRG>
__global__ void __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(1, 1)))
k_gemm_group(const GemmGeom* __restrict__ sys, const GroupTile* __restrict__ tiles, int n_tiles,
             int* __restrict__ counter) {
  constexpr int RBW = WM * MB;
  __shared__ u32x4 lds[2][RBW][SU];
  __shared__ int next;
  f32x16 acc[MB][4];
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    __syncthreads();
    const int idx = next;
    __syncthreads();
    if (idx >= n_tiles) break;
    const GroupTile gt = tiles[idx];
    const GemmGeom g = sys[gt.sys];
    const int mtile = gt.tile / g.n_ntiles;
    const int ntile = gt.tile % g.n_ntiles;
    const int64_t rb0 = (int64_t)mtile * RBW;
    // the orientation follows the system's method (uniform per work-group)
    if constexpr (DIRG) {
      if (g.s3 > 0) {
        float* slot = g.ws + (int64_t)blockIdx.x * 2 * (MB * 3 * 16) * 256 + threadIdx.x;
        if (g.layout_g)
          dir_tile<PREC, WM, WT, MB, false>(g, rb0, ntile, slot, acc, lds);
        else
          dir_tile<PREC, WM, WT, MB, true>(g, rb0, ntile, slot, acc, lds);
        continue;
      }
    }
    if (g.layout_g) {
      gemm_segment<PREC, WM, WT, MB, false>(g, rb0, ntile, 0, g.n_stages, acc, lds);
      gemm_epilogue<PREC, WM, WT, MB, false>(acc, g.out, g, rb0, ntile, reinterpret_cast<float*>(&lds[0][0][0]));
    } else {
      gemm_segment<PREC, WM, WT, MB, true>(g, rb0, ntile, 0, g.n_stages, acc, lds);
      gemm_epilogue<PREC, WM, WT, MB, true>(acc, g.out, g, rb0, ntile, reinterpret_cast<float*>(&lds[0][0][0]));
    }
    __syncthreads();
  }
}

// Sum the workspace partials of every split tile in work-group order and run
// the epilogue.  Tiles finished inside k_gemm are skipped.
template <int PREC, int WM, int WT, int MB, bool TR>
__global__ void __launch_bounds__(256) k_gemm_fixup(const float* __restrict__ ws, GemmGeom g) {
  constexpr int RBW = WM * MB;
  constexpr int NREG = MB * 4 * 16;
  __shared__ float red[4 * RBW * 32 * 3];
  const int64_t tile = blockIdx.x;
  const int64_t first_it = tile * g.n_stages, last_it = first_it + g.n_stages - 1;
  const int64_t g0 = first_it / g.ipw, g1 = last_it / g.ipw;
  if (g0 == g1) return;
  const int tid = threadIdx.x;
  f32x16 acc[MB][4];
#pragma unroll
  for (int rb = 0; rb < MB; ++rb)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[rb][c][j] = 0.f;
  for (int64_t gl = g0; gl <= g1; ++gl) {
    const int slot = (gl * g.ipw >= first_it) ? 0 : 1;
    const float* w = ws + ((gl * 2 + slot) * NREG) * 256 + tid;
#pragma unroll
    for (int rb = 0; rb < MB; ++rb)
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[rb][c][j] += w[((rb * 4 + c) * 16 + j) * 256];
  }
  const int mtile = (int)(tile / g.n_ntiles), ntile = (int)(tile % g.n_ntiles);
  gemm_epilogue<PREC, WM, WT, MB, TR>(acc, g.out, g, (int64_t)mtile * RBW, ntile, red);
}

// Plan of the lockstep split for n_tiles tiles of S stages on G = n_cu
// work-groups; false if it would not shorten the launch (estimated in
// stage-times of one CU) by at least min_gain, or the workspace is short.
static bool plan_split(int64_t n_tiles, int S, int G, int64_t slot_floats, int64_t ws_floats, double min_gain,
                       SplitPlan* sp) {
  constexpr int MIN_PIECE = 8;                                   // stages per piece
  if (G < 2 || n_tiles < 1) return false;
  const int64_t q = n_tiles / G;
  const int R = (int)(n_tiles % G);
  if (R == 0 || q > (1 << 20)) return false;
  SplitPlan p{};
  p.q = (int)q;
  p.R = R;
  double span;                                                   // stages on the busiest CU
  const int Q = G - R;
  if (R >= Q) {
    // main pieces [0, c), tails [c, S) k per tail work-group; a tail
    // work-group runs its stages about 8 % slower (several short pieces,
    // each with a pipeline start and a partial store)
    constexpr double TAIL_COST = 1.08;
    const int k = (R + Q - 1) / Q;
    int best = -1;
    double best_span = 1e300;
    const int r0 = (int)(S / (1.0 + TAIL_COST * k));
    for (int r = r0; r <= r0 + 1; ++r) {
      if (r < MIN_PIECE || S - r < MIN_PIECE) continue;
      const double sp_r = std::max<double>(S - r, TAIL_COST * k * r);
      if (sp_r < best_span) { best_span = sp_r; best = r; }
    }
    if (best < 0) return false;
    p.m = 2;
    p.Q = Q;
    p.c = S - best;
    span = best_span;
  } else {
    const int m = std::min(G / R, S / MIN_PIECE);
    if (m < 2) return false;
    p.m = m;
    p.Q = 0;
    span = (double)((S + m - 1) / m);
  }
  if ((int64_t)p.m * R * slot_floats > ws_floats) return false;
  const double plain = (double)(q + 1) * S, split = (double)q * S + span;
  if (split > (1.0 - min_gain) * plain) return false;
  *sp = p;
  return true;
}

template <int PREC, int WM, int WT, int MB, bool TR>
static hipError_t launch_gemm_shape(hipStream_t s, const void* E, const void* B, float* out, float* ws,
                                    int64_t ws_floats, int* tile_cnt, GemmGeom g, int n_mtiles, int n_cu,
                                    int sched, int* used) {
  constexpr int NREG = MB * 4 * 16;
  const int64_t n_tiles = (int64_t)n_mtiles * g.n_ntiles;
  g.total_iters = n_tiles * g.n_stages;
  g.E = E;
  g.B = B;
  g.out = out;
  // Lockstep split when the last round of tiles would leave CUs idle
  // (AUTO: only when it saves at least 5 %).
  if ((sched == MHC_SCHED_SPLIT || sched == MHC_SCHED_AUTO) && tile_cnt) {
    SplitPlan sp{};
    if (plan_split(n_tiles, g.n_stages, n_cu, (int64_t)NREG * 256, ws_floats,
                   sched == MHC_SCHED_AUTO ? 0.05 : 0.0, &sp)) {
      sp.cnt = tile_cnt;
      hipLaunchKernelGGL((k_gemm_split<PREC, WM, WT, MB, TR>), dim3((unsigned)n_cu), dim3(256), 0, s, ws, g, sp);
      *used = MHC_SCHED_SPLIT;
      return hipGetLastError();
    }
  }
  int64_t G = n_tiles;
  g.ipw = g.n_stages;
  // Stream-K only on request: work-groups that start at different k-stages no
  // longer share the activation k-slices in L2 (the tiled schedule marches
  // all work-groups of an XCD through k together), and on the 27648-mode
  // slab that extra MALL traffic costs more than the idle CUs it recovers.
  bool sk = (sched == MHC_SCHED_STREAMK);
  if (sk) {
    G = std::min<int64_t>(n_cu, std::max<int64_t>(1, g.total_iters / 4));
    g.ipw = (g.total_iters + G - 1) / G;
    G = (g.total_iters + g.ipw - 1) / g.ipw;
    if (G * 2 * NREG * 256 > ws_floats || G == n_tiles) {
      sk = false;
      G = n_tiles;
      g.ipw = g.n_stages;
    }
  }
  hipLaunchKernelGGL((k_gemm<PREC, WM, WT, MB, TR>), dim3((unsigned)G), dim3(256), 0, s, ws, g);
  *used = sk ? MHC_SCHED_STREAMK : MHC_SCHED_TILES;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !sk) return e;
  hipLaunchKernelGGL((k_gemm_fixup<PREC, WM, WT, MB, TR>), dim3((unsigned)n_tiles), dim3(256), 0, s, ws, g);
  return hipGetLastError();
}

template <int PREC>
static hipError_t launch_gemm_prec(hipStream_t s, const void* E, const void* B, int64_t M_pad, int64_t K_pad, int ntb,
                                   float* out, int layout_g, int* n_parts, float* ws, int64_t ws_floats,
                                   int* tile_cnt, int n_cu, int sched, const float* row_scale,
                                   const float* col_scale, int* used) {
  GemmGeom g{};
  g.K_pad = K_pad;
  g.M_pad = M_pad;
  g.ntb = ntb;
  // dofs per stage: 32 (FP32, BF16), 64 (FP8X3), 128 (FP8)
  g.n_stages = (int)(K_pad / (PREC == PREC_FP8 ? 128 : (PREC == PREC_FP8X3 ? 64 : 32)));
  g.layout_g = layout_g;
  g.row_scale = row_scale;
  g.col_scale = col_scale;
  // HNEMA (layout 0) in the step-major accumulator orientation, GKMA in the
  // slot-major one
#define MHC_SHAPE(WM, WT, MB, ROWS)                                                                              \
  (layout_g ? launch_gemm_shape<PREC, WM, WT, MB, false>(s, E, B, out, ws, ws_floats, tile_cnt, g,               \
                                                         (int)(M_pad / (ROWS)), n_cu, sched, used)              \
            : launch_gemm_shape<PREC, WM, WT, MB, true>(s, E, B, out, ws, ws_floats, tile_cnt, g,                \
                                                        (int)(M_pad / (ROWS)), n_cu, sched, used))
  if (ntb % 4 == 0) {
    // 128 slots x 4 t-blocks per tile
    g.n_ntiles = ntb / 4;
    *n_parts = g.n_ntiles;
    return MHC_SHAPE(1, 4, 4, 128);
  } else if (ntb % 2 == 0) {
    g.n_ntiles = ntb / 2;
    *n_parts = g.n_ntiles;
    return MHC_SHAPE(2, 2, 4, 256);
  }
  g.n_ntiles = ntb;
  *n_parts = g.n_ntiles;
  return MHC_SHAPE(4, 1, 2, 256);
#undef MHC_SHAPE
}

hipError_t launch_gemm(hipStream_t s, int prec, const void* E, const void* B, int64_t M_pad, int64_t K_pad,
                       int ntb, float* out, int layout_g, int* n_parts, float* ws, int64_t ws_floats,
                       int* tile_cnt, int n_cu, int sched, const float* row_scale, const float* col_scale,
                       int* used) {
#define MHC_GEMM(P) \
  launch_gemm_prec<P>(s, E, B, M_pad, K_pad, ntb, out, layout_g, n_parts, ws, ws_floats, tile_cnt, n_cu, sched, \
                      row_scale, col_scale, used)
  switch (prec) {
    case PREC_BF16X3: return MHC_GEMM(PREC_BF16X3);
    case PREC_FP8: return MHC_GEMM(PREC_FP8);
    case PREC_FP8X3: return MHC_GEMM(PREC_FP8X3);
    default: return MHC_GEMM(PREC_FP32);
  }
#undef MHC_GEMM
}

template <int PREC, int WM, int WT, int MB, bool TR>
static hipError_t launch_dir_shape(hipStream_t s, GemmGeom g, int s3, int64_t region, float* ws, int64_t ws_floats,
                                   int n_cu) {
  constexpr int NBR = MB * 3 * 16;
  const int64_t n_tiles = (g.M_pad / (WM * MB * 32)) * g.n_ntiles;
  const int64_t G = std::min<int64_t>({n_tiles, (int64_t)n_cu, ws_floats / ((int64_t)2 * NBR * 256)});
  if (G < 1) return hipErrorInvalidValue;
  g.s3 = s3;
  g.region = region;
  g.ws = ws;
  hipLaunchKernelGGL((k_gemm_dir<PREC, WM, WT, MB, TR>), dim3((unsigned)G), dim3(256), 0, s, g);
  return hipGetLastError();
}

template <int PREC>
static hipError_t launch_gemm_dir_prec(hipStream_t s, const void* E, const void* B, int64_t M_pad, int64_t n3, int ntb,
                                       float* out, int64_t region, int layout_g, int* n_parts, float* ws,
                                       int64_t ws_floats, int n_cu, const float* row_scale, const float* col_scale) {
  constexpr int SD = stage_dofs(PREC);
  if (n3 % SD != 0) return hipErrorInvalidValue;
  GemmGeom g{};
  g.K_pad = 3 * n3;
  g.M_pad = M_pad;
  g.ntb = ntb;
  g.n_stages = (int)(g.K_pad / SD);
  g.layout_g = layout_g;
  g.E = E;
  g.B = B;
  g.out = out;
  g.row_scale = row_scale;
  g.col_scale = col_scale;
  const int s3 = (int)(n3 / SD);
#define MHC_DSHAPE(WM, WT, MB)                                                                           \
  (layout_g ? launch_dir_shape<PREC, WM, WT, MB, false>(s, g, s3, region, ws, ws_floats, n_cu)            \
            : launch_dir_shape<PREC, WM, WT, MB, true>(s, g, s3, region, ws, ws_floats, n_cu))
  if (ntb % 4 == 0) {
    g.n_ntiles = ntb / 4;
    *n_parts = g.n_ntiles;
    return MHC_DSHAPE(1, 4, 4);
  } else if (ntb % 2 == 0) {
    g.n_ntiles = ntb / 2;
    *n_parts = g.n_ntiles;
    return MHC_DSHAPE(2, 2, 4);
  }
  g.n_ntiles = ntb;
  *n_parts = g.n_ntiles;
  return MHC_DSHAPE(4, 1, 2);
#undef MHC_DSHAPE
}

hipError_t launch_gemm_dir(hipStream_t s, int prec, const void* E, const void* B, int64_t M_pad, int64_t n3, int ntb,
                           float* out, int64_t region, int layout_g, int* n_parts, float* ws, int64_t ws_floats,
                           int n_cu, const float* row_scale, const float* col_scale) {
  if (n3 <= 0) return hipErrorInvalidValue;
#define MHC_DIRP(P) \
  launch_gemm_dir_prec<P>(s, E, B, M_pad, n3, ntb, out, region, layout_g, n_parts, ws, ws_floats, n_cu, row_scale, \
                          col_scale)
  switch (prec) {
    case PREC_BF16X3: return MHC_DIRP(PREC_BF16X3);
    case PREC_FP8: return MHC_DIRP(PREC_FP8);
    case PREC_FP8X3: return MHC_DIRP(PREC_FP8X3);
    case PREC_FP32: return MHC_DIRP(PREC_FP32);
    default: return hipErrorInvalidValue;
  }
#undef MHC_DIRP
}

int stage_dofs_of(int prec) {
  return prec == PREC_FP8 ? stage_dofs(PREC_FP8) : (prec == PREC_FP8X3 ? stage_dofs(PREC_FP8X3) : stage_dofs(PREC_FP32));
}

// ----------------------------------------------------------- tile shapes
// shape 0: 128 slots x 4 t-blocks (waves 1 x 4, 4 row blocks each)
// shape 1: 256 slots x 2 t-blocks (waves 2 x 2, 4 row blocks each)
// shape 2: 256 slots x 1 t-block  (waves 4 x 1, 2 row blocks each)
int gemm_shape_rows(int shape) { return shape == 0 ? 128 : 256; }
int gemm_shape_tbs(int shape) { return shape == 0 ? 4 : (shape == 1 ? 2 : 1); }
bool gemm_shape_valid(int shape, int ntb) { return shape >= 0 && shape <= 2 && ntb % gemm_shape_tbs(shape) == 0; }

void gemm_geom(int prec, int shape, const void* E, const void* B, float* out, int64_t M_pad, int64_t K_pad, int ntb,
               int layout_g, const float* row_scale, const float* col_scale, GemmGeom* g, int* n_mtiles) {
  *g = GemmGeom{};
  g->E = E;
  g->B = B;
  g->out = out;
  g->K_pad = K_pad;
  g->M_pad = M_pad;
  g->ntb = ntb;
  g->n_ntiles = ntb / gemm_shape_tbs(shape);
  g->n_stages = (int)(K_pad / (prec == PREC_FP8 ? 128 : (prec == PREC_FP8X3 ? 64 : 32)));
  g->layout_g = layout_g;
  g->row_scale = row_scale;
  g->col_scale = col_scale;
  *n_mtiles = (int)(M_pad / gemm_shape_rows(shape));
  g->total_iters = (int64_t)(*n_mtiles) * g->n_ntiles * g->n_stages;
  g->ipw = g->n_stages;
}

template <int PREC, bool DIRG>
static hipError_t launch_group_prec(hipStream_t s, int shape, const GemmGeom* d_sys, const GroupTile* d_tiles,
                                    int n_tiles, int* counter, int n_wg) {
  dim3 grid((unsigned)n_wg), block(256);
  if (shape == 0)
    hipLaunchKernelGGL((k_gemm_group<PREC, 1, 4, 4, DIRG>), grid, block, 0, s, d_sys, d_tiles, n_tiles, counter);
  else if (shape == 1)
    hipLaunchKernelGGL((k_gemm_group<PREC, 2, 2, 4, DIRG>), grid, block, 0, s, d_sys, d_tiles, n_tiles, counter);
  else
    hipLaunchKernelGGL((k_gemm_group<PREC, 4, 1, 2, DIRG>), grid, block, 0, s, d_sys, d_tiles, n_tiles, counter);
  return hipGetLastError();
}

hipError_t launch_gemm_group(hipStream_t s, int prec, int shape, const GemmGeom* d_sys, const GroupTile* d_tiles,
                             int n_tiles, int* counter, int n_wg, bool with_dir) {
#define MHC_GRP(P)                                                                                   \
  (with_dir ? launch_group_prec<P, true>(s, shape, d_sys, d_tiles, n_tiles, counter, n_wg)          \
            : launch_group_prec<P, false>(s, shape, d_sys, d_tiles, n_tiles, counter, n_wg))
  switch (prec) {
    case PREC_BF16X3: return MHC_GRP(PREC_BF16X3);
    case PREC_FP8: return MHC_GRP(PREC_FP8);
    case PREC_FP8X3: return MHC_GRP(PREC_FP8X3);
    default: return MHC_GRP(PREC_FP32);
  }
#undef MHC_GRP
}

__global__ void k_fill_i32(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(hipStream_t s, int* p, int n, int v) {
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace mhc
