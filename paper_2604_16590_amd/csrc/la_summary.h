// la_summary.h -- the summary's per-step machinery (internal), shared by
// the summary kernel of the forward and backward passes (la_forward.hip)
// and by the tile summaries of the fused tiled attention (la_tiled.hip).
//
// A wave holds R tokens per lane group per step; lane (g, m) owns the
// key/value features [F*m, F*m + F) (F = d/16) of each.  summary_step
// applies phi to the keys, transposes token pairs into the matrix cores'
// feature-major operands (for bf16 the two tokens of a pair go into one
// word, which costs nothing beyond the pack that rounds phi), and
// accumulates S += phi(K)^T V and z += phi(K)^T 1 on the matrix cores.
#pragma once
#include "la_kernels.h"

namespace la {

template <int DT, int D, int MODE = MODE_FWD>
struct SummaryCfg {
  static constexpr int F = D / 16;                 // features per lane (S tile grid is F x F)
  // waves sharing one token range; each owns F/SPLIT rows of S tiles and
  // loads F/SPLIT of the value features, whose matrix-core operands it
  // shares with the others through LDS, so K and V are each read once.
  // bf16 at d = 128 keeps the whole S (256 accumulator registers) in one
  // wave, in the accumulation registers, at one wave per SIMD; fp32 there
  // needs more registers for its operands and splits in two.
  static constexpr int SPLIT = D >= 128 && DT == DT_FP32 ? 2 : 1;
  static constexpr int WAVES_PER_SIMD = D >= 128 && DT == DT_BF16 ? 1 : 2;
  static constexpr int FR = F / SPLIT;             // S tile rows (key features) per wave
  static constexpr int FC = F / SPLIT;             // value features loaded per wave
  static constexpr int ES = DT == DT_BF16 ? 2 : 4;
  static constexpr int KB = FR * ES;               // key bytes per lane per token
  static constexpr int VB = FC * ES;               // value bytes per lane per token
  static constexpr int KW = KB >= 4 ? KB / 4 : 1;
  static constexpr int VW = VB >= 4 ? VB / 4 : 1;
  static constexpr int R = DT == DT_BF16 ? 8 : 4;  // tokens per lane group per step
  static constexpr int STEP = 4 * R;               // tokens per wave per step
  static constexpr int THREADS = SPLIT > 1 ? 64 * SPLIT : 256;
  static constexpr int PPB = SPLIT > 1 ? 1 : 4;    // partials per workgroup
  // LDS words exchanged per buffer: bf16 -> F operands x 4 words x 64 lanes;
  // fp32 -> R tokens x F values x 64 lanes
  static constexpr int XW = SPLIT > 1 ? (DT == DT_BF16 ? F * 4 * 64 : R * F * 64) : 1;
};

template <int DT, int D, int MODE>
struct SummaryRegs {
  using C = SummaryCfg<DT, D, MODE>;
  uint32_t kw[C::R][C::KW];
  uint32_t vw[C::R][C::VW];
  // backward mode: lane (g, m), m < R, holds the pair of token R*g + m;
  // the step broadcasts it across the lane group when it is needed
  float2 tok;
};

// The pair of token R*g + r of this lane's group (lane 16g + r holds it):
// a DPP row broadcast (rows of the DPP unit are the 16-lane groups), a
// plain VALU move with no LDS round trip.  r is a constant after
// unrolling, so the switch folds to one case.
template <int L>
__device__ __forceinline__ float row_bcast(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x150 + L,
                                                               0xf, 0xf, false));
}
__device__ __forceinline__ float2 group_bcast(float2 v, int r) {
  switch (r) {
#define LA_BC(L) case L: return float2{row_bcast<L>(v.x), row_bcast<L>(v.y)};
    LA_BC(0) LA_BC(1) LA_BC(2) LA_BC(3) LA_BC(4) LA_BC(5) LA_BC(6) LA_BC(7)
#undef LA_BC
    default: return float2{0.f, 0.f};
  }
}

// One step of the summary: phi on the keys, register transpose, MFMAs.
// MODE_FWD: rows = phi(k), columns = v, z += phi(k).
// MODE_BWD: rows = phi(q) / den, columns = dO, z += -(dO . O) phi(q) / den,
// which accumulates dS = sum phi(q) (dO / den)^T and dz = sum dden phi(q)
// (dden = -(dO . O) / den) of the backward pass; the per-token pair
// (1/den, -(dO . O)) comes from the query kernel.
// `xch` is this step's LDS exchange buffer (SPLIT > 1).
template <int DT, int D, int MODE>
__device__ __forceinline__ void summary_step(const SummaryRegs<DT, D, MODE>& x, int part, int lane,
                                             uint32_t* xch,
                                             f32x4 (&acc)[SummaryCfg<DT, D, MODE>::FR][SummaryCfg<DT, D, MODE>::F],
                                             float (&zacc)[SummaryCfg<DT, D, MODE>::FR]) {
  using C = SummaryCfg<DT, D, MODE>;
  constexpr int F = C::F, FR = C::FR, FC = C::FC;
  if constexpr (DT == DT_BF16) {
    // value operands of this wave's features: token pairs of one feature
    // packed into words
    uint32_t own[FC][4];
#pragma unroll
    for (int jj = 0; jj < FC; ++jj)
#pragma unroll
      for (int pp = 0; pp < 4; ++pp) {
        const uint32_t lo = word_bits16<DT>(x.vw[2 * pp], jj);
        const uint32_t hi = word_bits16<DT>(x.vw[2 * pp + 1], jj);
        own[jj][pp] = lo | (hi << 16);
      }
    if constexpr (C::SPLIT > 1) {
#pragma unroll
      for (int jj = 0; jj < FC; ++jj)
#pragma unroll
        for (int pp = 0; pp < 4; ++pp) xch[((part * FC + jj) * 4 + pp) * 64 + lane] = own[jj][pp];
      __syncthreads();
    }
    // key operands of this wave's rows (token pair outermost, so only
    // one pair of per-token scalars is live in the backward mode)
    uint32_t pk[FR][4];
#pragma unroll
    for (int pp = 0; pp < 4; ++pp) {
      float2 t0 = float2{1.f, 0.f}, t1 = float2{1.f, 0.f};
      if constexpr (MODE == MODE_BWD) {
        t0 = group_bcast(x.tok, 2 * pp);
        t1 = group_bcast(x.tok, 2 * pp + 1);
      }
#pragma unroll
      for (int i = 0; i < FR; ++i) {
        float p0 = phi<DT>(word_elem<DT>(x.kw[2 * pp], i));
        float p1 = phi<DT>(word_elem<DT>(x.kw[2 * pp + 1], i));
        if constexpr (MODE == MODE_BWD) {
          p0 *= t0.x;
          p1 *= t1.x;
        }
        pk[i][pp] = pack_bf16(p0, p1);
        if constexpr (MODE == MODE_FWD) {
          // normaliser from the same rounded phi values that feed S
          zacc[i] = add_bf16_pair(zacc[i], pk[i][pp]);
        } else {
          zacc[i] = fmaf(t0.y, bf16lo(pk[i][pp]), zacc[i]);
          zacc[i] = fmaf(t1.y, bf16hi(pk[i][pp]), zacc[i]);
        }
      }
    }
    bf16x8 ak[FR];
#pragma unroll
    for (int i = 0; i < FR; ++i) ak[i] = as_bf16x8(u32x4{pk[i][0], pk[i][1], pk[i][2], pk[i][3]});
#pragma unroll
    for (int j = 0; j < F; ++j) {
      bf16x8 bv;
      if constexpr (C::SPLIT > 1) {
        bv = as_bf16x8(u32x4{xch[(j * 4 + 0) * 64 + lane], xch[(j * 4 + 1) * 64 + lane],
                             xch[(j * 4 + 2) * 64 + lane], xch[(j * 4 + 3) * 64 + lane]});
      } else {
        bv = as_bf16x8(u32x4{own[j][0], own[j][1], own[j][2], own[j][3]});
      }
#pragma unroll
      for (int i = 0; i < FR; ++i) acc[i][j] = mfma_bf16(ak[i], bv, acc[i][j]);
    }
  } else {
    if constexpr (C::SPLIT > 1) {
#pragma unroll
      for (int r = 0; r < C::R; ++r)
#pragma unroll
        for (int jj = 0; jj < FC; ++jj) xch[(r * F + part * FC + jj) * 64 + lane] = x.vw[r][jj];
      __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < C::R; ++r) {
      float pk[FR];
      float2 tr = float2{1.f, 0.f};
      if constexpr (MODE == MODE_BWD) tr = group_bcast(x.tok, r);
#pragma unroll
      for (int i = 0; i < FR; ++i) {
        pk[i] = phi<DT>(word_elem<DT>(x.kw[r], i));
        if constexpr (MODE == MODE_FWD) {
          zacc[i] += pk[i];
        } else {
          pk[i] *= tr.x;
          zacc[i] = fmaf(tr.y, pk[i], zacc[i]);
        }
      }
#pragma unroll
      for (int j = 0; j < F; ++j) {
        const float vj = C::SPLIT > 1 ? __uint_as_float(xch[(r * F + j) * 64 + lane])
                                      : word_elem<DT>(x.vw[r], j);
#pragma unroll
        for (int i = 0; i < FR; ++i) acc[i][j] = mfma_f32(pk[i], vj, acc[i][j]);
      }
    }
  }
}

}  // namespace la
