// la_backward.hip -- gfx950 kernels of the backward pass.
//
// Gradients of L = <O, G> (G = dL/dO) for O_i = phi(q_i)^T S / den_i,
// den_i = phi(q_i) . z:
//   X_i    = S G_i                      (d-vector per query)
//   G_i.O_i = phi(q_i) . X_i / den_i     (so O itself is never formed)
//   dden_i = -(G_i . O_i) / den_i
//   dQ_i   = (X_i / den_i + dden_i z) * phi'(q_i)
//   dS     = sum_i phi(q_i) (G_i / den_i)^T,   dz = sum_i dden_i phi(q_i)
//   dV_j   = dS^T phi(k_j),   dK_j = (dS v_j + dz) * phi'(k_j)
// phi(Q) and phi(K) are recomputed from the inputs here, never stored by
// the forward (the paper trains with activation recomputation, Sec. III-D).
//
// Passes: (1) images of S; (2) the query pass: dQ and each wave's partial
// sums of dS, dz in one kernel for bf16 at d >= 32 (bwd_qds_kernel,
// bwd_qds4_kernel), otherwise the query kernel (dQ and per-token
// (1/den, dden)) followed by the token reduction for dS, dz (the forward's
// summary kernel in its backward mode); (3) FP64 combine of dS, dz;
// (4) key kernel: dK, dV.
#include <type_traits>

#include "la_kernels.h"
#include "la_profile.h"

namespace la {

// Layout shared by the query and key kernels: lane (g, n) holds token n of
// a 16-token tile and a run of Q4 = d/4 features (Run: 16-byte chunks
// interleaved over the lane groups); the matrix-core results of A x (that
// run) land in the same lane and run positions.
template <int DT, int D>
struct RowCfg {
  static constexpr int Q4 = D / 4;
  static constexpr int NT = D / 16;
  static constexpr int NS = ImageCfg<D>::NS;
  static constexpr int ES = DT == DT_BF16 ? 2 : 4;
  static constexpr int RB = Q4 * ES;
  static constexpr int RWD = RB >= 4 ? RB / 4 : 1;
  // 16-token tiles per step sharing each LDS operand read (bf16); the fp32
  // path is matrix-core bound and keeps one tile to stay within registers
  static constexpr int TT = DT == DT_BF16 ? 2 : 1;
  // per-lane run held as: bf16 -> packed words (NS*4, zero padded past Q4),
  // fp32 -> one float per feature
  static constexpr int PW = DT == DT_BF16 ? NS * 4 : Q4;
  // prefetch one step ahead, except where it would not fit the registers
  // of two waves per SIMD (d = 128, and fp32 from d = 64)
  static constexpr bool PF = D < 128 && !(DT == DT_FP32 && D >= 64);
};

// phi over the lane's run: bf16 packs phi rounded to bf16 (the values the
// matrix cores use); fp32 keeps fp32 phi.  phi' is recovered as
// min(phi, 1): it is 1 where x > 0 (phi >= 1 there) and phi(x) elsewhere.
template <int DT, int D>
__device__ __forceinline__ void phi_words(const uint32_t* w, uint32_t* pw) {
  using C = RowCfg<DT, D>;
  constexpr int Q4 = C::Q4;
  if constexpr (DT == DT_BF16) {
#pragma unroll
    for (int k = 0; k < C::PW; ++k) {
      const int c0 = 2 * k;
      pw[k] = c0 < Q4 ? pack_bf16(phi<DT>(word_elem<DT>(w, c0)), phi<DT>(word_elem<DT>(w, c0 + 1)))
                      : 0u;
    }
  } else {
#pragma unroll
    for (int c = 0; c < Q4; ++c) pw[c] = __float_as_uint(phi<DT>(word_elem<DT>(w, c)));
  }
}

// Raw bf16 words of a lane's run, zero padded to whole k-steps.
template <int DT, int D>
__device__ __forceinline__ void raw_words(const uint32_t* w, uint32_t* pw) {
  using C = RowCfg<DT, D>;
#pragma unroll
  for (int k = 0; k < C::PW; ++k) {
    if constexpr (DT == DT_BF16) pw[k] = 2 * k < C::Q4 ? w[k] : 0u;
    else pw[k] = w[k];
  }
}

// Value of feature c of a run held as words.
template <int DT>
__device__ __forceinline__ float run_val(const uint32_t* pw, int c) {
  if constexpr (DT == DT_BF16) return (c & 1) ? bf16hi(pw[c >> 1]) : bf16lo(pw[c >> 1]);
  else return __uint_as_float(pw[c]);
}

// acc[t][i] += A_image[i] x B_t (the run of tile t) for the TT tiles of a
// step: every LDS operand read feeds TT matrix-core ops.  bf16 images hold
// hi then lo words per (tile, k-step); with USE_LO both parts are applied,
// otherwise the staged image holds hi words only.
template <int DT, int D, bool USE_LO>
__device__ __forceinline__ void image_times_runs(
    const u32x4* simg, int lane,
    const uint32_t (&pw)[RowCfg<DT, D>::TT][RowCfg<DT, D>::PW],
    f32x4 (&acc)[RowCfg<DT, D>::TT][D / 16]) {
  using C = RowCfg<DT, D>;
  constexpr int TT = C::TT;
  if constexpr (DT == DT_BF16) {
#pragma unroll
    for (int i = 0; i < C::NT; ++i) {
#pragma unroll
      for (int s = 0; s < C::NS; ++s) {
        bf16x8 b[TT];
#pragma unroll
        for (int t = 0; t < TT; ++t)
          b[t] = as_bf16x8(u32x4{pw[t][4 * s], pw[t][4 * s + 1], pw[t][4 * s + 2], pw[t][4 * s + 3]});
        if constexpr (USE_LO) {
          const bf16x8 hi = as_bf16x8(simg[((i * C::NS + s) * 2 + 0) * 64 + lane]);
          const bf16x8 lo = as_bf16x8(simg[((i * C::NS + s) * 2 + 1) * 64 + lane]);
#pragma unroll
          for (int t = 0; t < TT; ++t) {
            // the chain's first product starts from zero (no separate clear)
            acc[t][i] = mfma_bf16(hi, b[t], s == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[t][i]);
            acc[t][i] = mfma_bf16(lo, b[t], acc[t][i]);
          }
        } else {
          const bf16x8 hi = as_bf16x8(simg[(i * C::NS + s) * 64 + lane]);
#pragma unroll
          for (int t = 0; t < TT; ++t)
            acc[t][i] = mfma_bf16(hi, b[t], s == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[t][i]);
        }
      }
      if constexpr (D >= 128) __builtin_amdgcn_sched_barrier(0);
    }
  } else {
    constexpr int Q4 = C::Q4;
#pragma unroll
    for (int i = 0; i < C::NT; ++i) {
#pragma unroll
      for (int s4 = 0; s4 < Q4 / 4; ++s4) {
        const u32x4 a = simg[(i * (Q4 / 4) + s4) * 64 + lane];
#pragma unroll
        for (int t4 = 0; t4 < 4; ++t4)
#pragma unroll
          for (int t = 0; t < TT; ++t)
            acc[t][i] = mfma_f32(__uint_as_float(a[t4]), __uint_as_float(pw[t][4 * s4 + t4]),
                                 s4 == 0 && t4 == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[t][i]);
      }
      if constexpr (D >= 128) __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// acc[t][0] += (one 16-row tile, e.g. the z tile) x B_t for the TT tiles of
// a step; bf16 tiles hold hi then lo words per k-step.
template <int DT, int D>
__device__ __forceinline__ void tile_times_runs(
    const u32x4* tile, int lane,
    const uint32_t (&pw)[RowCfg<DT, D>::TT][RowCfg<DT, D>::PW],
    f32x4 (&acc)[RowCfg<DT, D>::TT][1]) {
  using C = RowCfg<DT, D>;
  constexpr int TT = C::TT;
  if constexpr (DT == DT_BF16) {
#pragma unroll
    for (int s = 0; s < C::NS; ++s) {
      const bf16x8 hi = as_bf16x8(tile[(s * 2 + 0) * 64 + lane]);
      const bf16x8 lo = as_bf16x8(tile[(s * 2 + 1) * 64 + lane]);
#pragma unroll
      for (int t = 0; t < TT; ++t) {
        const bf16x8 bt = as_bf16x8(u32x4{pw[t][4 * s], pw[t][4 * s + 1], pw[t][4 * s + 2], pw[t][4 * s + 3]});
        acc[t][0] = mfma_bf16(hi, bt, s == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[t][0]);
        acc[t][0] = mfma_bf16(lo, bt, acc[t][0]);
      }
    }
  } else {
    constexpr int Q4 = C::Q4;
#pragma unroll
    for (int s4 = 0; s4 < Q4 / 4; ++s4) {
      const u32x4 a = tile[s4 * 64 + lane];
#pragma unroll
      for (int t4 = 0; t4 < 4; ++t4)
#pragma unroll
        for (int t = 0; t < TT; ++t)
          acc[t][0] = mfma_f32(__uint_as_float(a[t4]), __uint_as_float(pw[t][4 * s4 + t4]),
                               s4 == 0 && t4 == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[t][0]);
    }
  }
}

// Copy `words` 16-byte words of an image into LDS; with `hi_only` only the
// hi half of each (tile, k-step) pair of a bf16 image is kept.
__device__ __forceinline__ void stage_image(u32x4* dst, const u32x4* src, int words, bool hi_only) {
  for (int w = threadIdx.x; w < words; w += blockDim.x) {
    if (hi_only) {
      const int pair = w >> 6, lane = w & 63;
      dst[w] = src[pair * 128 + lane];
    } else {
      dst[w] = src[w];
    }
  }
}

// ---------------------------------------------------------------------------
// Query kernel: dQ, plus (1/den, -(G . O)) per token for the dS/dz reduction.
// LDS holds the N image of S (A[row = q feature c][k = value feature e])
// and the T image's z tile, whose product with phi(q) is den for every
// output row.  bf16 inputs: the per-token dot product G . O and the dQ
// combination run in fp32 (the terms come from bf16 data and fp32
// matrix-core sums); fp32 inputs keep them in FP64.
// ---------------------------------------------------------------------------
template <int DT, int OT, int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void bwd_query_kernel(
    const void* __restrict__ q, const void* __restrict__ dout, int64_t sb, int64_t sh,
    int64_t sn, void* __restrict__ dq, int64_t osb, int64_t osh, int64_t osn, int H,
    int64_t N, int Ta, const void* __restrict__ img, const double* __restrict__ z64,
    float2* __restrict__ stash) {
  using C = RowCfg<DT, D>;
  using IC = ImageCfg<D>;
  using real = typename std::conditional<DT == DT_BF16, float, double>::type;
  constexpr int Q4 = C::Q4, NT = C::NT, TT = C::TT;
  constexpr int OES = OT == DT_BF16 ? 2 : 4;
  constexpr int IMG_WORDS = IC::mat_bytes(DT) / 16;  // the N image
  constexpr int Z_WORDS = IC::tile_bytes(DT) / 16;   // the T image's z tile
  __shared__ u32x4 simg[IMG_WORDS + Z_WORDS];
  const u32x4* zimg = simg + IMG_WORDS;

  const int bh = blockIdx.y;
  const int64_t b = bh / H, h = bh % H;
  {
    const char* head = (const char*)img + (int64_t)bh * IC::head_bytes(DT);
    stage_image(simg, (const u32x4*)(head + IC::img_bytes(DT)), IMG_WORDS, false);
    stage_image(simg + IMG_WORDS, (const u32x4*)(head + IC::mat_bytes(DT)), Z_WORDS, false);
  }
  const int lane = threadIdx.x & 63, wave = wave_index();
  const int g = lane >> 4, n = lane & 15;
  real zr[Q4];
#pragma unroll
  for (int c = 0; c < Q4; ++c) zr[c] = (real)z64[(int64_t)bh * D + Run<D, DT>::feature(g, c)];
  __syncthreads();

  const int64_t wg_begin = (int64_t)blockIdx.x * Ta;
  const int64_t wg_end = min(N, wg_begin + (int64_t)Ta);
  // wave-uniform head pointers plus loop-invariant 32-bit lane offsets
  const int64_t row_bytes = sn * C::ES, orow_bytes = osn * OES;
  const char* qh = (const char*)q + (b * sb + h * sh) * C::ES;
  const char* gh = (const char*)dout + (b * sb + h * sh) * C::ES;
  char* oh = (char*)dq + (b * osb + h * osh) * OES;
  const uint32_t ioff = (uint32_t)n * (uint32_t)row_bytes + (uint32_t)(g * Run<D, DT>::CB);
  const uint32_t ooff =
      (uint32_t)n * (uint32_t)orow_bytes + (uint32_t)(g * Run<D, DT>::CH * OES);

  // one tile's query and gradient runs
  auto load_one = [&](int64_t tb, uint32_t* qw, uint32_t* gw) {
    if (tb + n < wg_end) {
      load_run<D, DT>(qh + tb * row_bytes + ioff, qw);
      load_run<D, DT>(gh + tb * row_bytes + ioff, gw);
    } else {
#pragma unroll
      for (int w = 0; w < C::RWD; ++w) { qw[w] = 0; gw[w] = 0; }
    }
  };
  constexpr int PT = C::PF ? TT : 1;  // tiles held ahead of their step
  typedef uint32_t Regs[PT][2][C::RWD];
  auto load = [&](int64_t t0, Regs& x) {
#pragma unroll
    for (int tt = 0; tt < PT; ++tt) load_one(t0 + 16 * tt, x[tt][0], x[tt][1]);
  };

  auto compute = [&](int64_t t0, const Regs& x) {
    uint32_t pq[TT][C::PW], pg[TT][C::PW];
    if constexpr (C::PF) {
#pragma unroll
      for (int tt = 0; tt < TT; ++tt) {
        phi_words<DT, D>(x[tt][0], pq[tt]);
        raw_words<DT, D>(x[tt][1], pg[tt]);
      }
    } else {
      // load and convert one tile at a time (fewer live registers)
#pragma unroll
      for (int tt = 0; tt < TT; ++tt) {
        uint32_t one[2][C::RWD];
        load_one(t0 + 16 * tt, one[0], one[1]);
        phi_words<DT, D>(one[0], pq[tt]);
        raw_words<DT, D>(one[1], pg[tt]);
      }
    }
    f32x4 acc[TT][NT];
#pragma unroll
    for (int tt = 0; tt < TT; ++tt)
#pragma unroll
      for (int i = 0; i < NT; ++i) acc[tt][i] = f32x4{0.f, 0.f, 0.f, 0.f};
    image_times_runs<DT, D, true>(simg, lane, pg, acc);  // X = S G
    f32x4 dacc[TT][1];
#pragma unroll
    for (int tt = 0; tt < TT; ++tt) dacc[tt][0] = f32x4{0.f, 0.f, 0.f, 0.f};
    tile_times_runs<DT, D>(zimg, lane, pq, dacc);        // den = phi(q) . z
#pragma unroll
    for (int tt = 0; tt < TT; ++tt) {
      real gn = 0;
#pragma unroll
      for (int i = 0; i < NT; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int c = 4 * i + r;
          gn += (real)run_val<DT>(pq[tt], c) * (real)acc[tt][i][r];
        }
      gn = sum_groups(gn);
      const double rden = 1.0 / (double)dacc[tt][0][0];
      const real go = (real)(gn * (real)rden);  // G . O
      const real rd = (real)rden;
      if (t0 + 16 * tt + n < wg_end) {
        float out[Q4];
#pragma unroll
        for (int i = 0; i < NT; ++i)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int c = 4 * i + r;
            const float dphi_c = dphi_of_phi(run_val<DT>(pq[tt], c));
            out[c] = (float)(fma(-go, zr[c], (real)acc[tt][i][r]) * rd) * dphi_c;
          }
        store_run<D, DT, OT>(oh + (t0 + 16 * tt) * orow_bytes + ooff, out);
        if (g == 0) stash[(int64_t)bh * N + t0 + 16 * tt + n] = float2{(float)rden, (float)(-go)};
      }
    }
  };

  // two register sets in turn where the registers allow a step ahead
  constexpr int STRIDE = 16 * TT * 4;
  Regs ra, rb;
  int64_t t0 = wg_begin + 16 * TT * wave;
  if (C::PF && t0 < wg_end) load(t0, ra);
  while (t0 < wg_end) {
    const int64_t t1 = t0 + STRIDE;
    if (C::PF && t1 < wg_end) load(t1, rb);
    compute(t0, ra);
    if (t1 >= wg_end) break;
    const int64_t t2 = t1 + STRIDE;
    if (C::PF && t2 < wg_end) load(t2, ra);
    compute(t1, rb);
    t0 = t2;
  }
}

// ---------------------------------------------------------------------------
// Fused query backward (bf16 inputs, d = 32 or 64): dQ exactly as in the
// query kernel, and in the same pass each wave's partial sums over its own
// tokens (32-token blocks p, p + P, ..., at most Tw tokens) of
//   dS = sum_i phi(q_i) (G_i / den_i)^T,   dz = sum_i dden_i phi(q_i),
// so Q and G are read once.  The reduction contracts over tokens, but the
// query pass holds one token per lane; the token-major operands are made
// on the matrix cores themselves: a lane run taken as A[m = token][k =
// feature] times a 0/1 selection matrix B[k][n] = (k == n + 16h) gives
// D[token][n] = run feature 32s + 16h + n, i.e. 16 features x 4 tokens in
// each lane, which is what a contraction over tokens takes.  The whole
// d x d partial dS stays in registers, so the next step's Q and G are
// prefetched straight into LDS (global_load_lds, 16 bytes per lane)
// instead of registers.
// Partial tile (i, j) holds, in lane (g, n) register r, dS[16i + 4g + r][16j + n]
// (the combine's block layout); the partial's dz follows at offset d*d.
// ---------------------------------------------------------------------------
template <int D>
struct FusedCfg {
  using R = Run<D, DT_BF16>;
  static constexpr int NB = D / 16;                   // 16-feature blocks
  static constexpr int NS = D / 32;                   // k-steps of a run
  static constexpr int TT = 2;                        // tiles per step: 32 tokens
  static constexpr int RW = D / 8;                    // words of a lane's run
  static constexpr int NCH = R::NCH;                  // 16-byte chunks per run
  static constexpr int STAGE = TT * 2 * NCH * 1024;   // LDS bytes per wave per step
  static constexpr int WAVES_PER_SIMD = 2;
};

typedef __attribute__((address_space(3))) void* lds_void_ptr;
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) s16x4* lds_s16x4_ptr;

// gfx950 transposing LDS read of 16-bit elements: within each 16-lane
// block, lane i receives as element k (k = 0..3) element i & 3 of the
// 8-byte chunk addressed by lane (i >> 2) + 4k of the block.  When lane L
// of a block addresses token row t0 + (L >> 2), features f0 + 4 (L & 3)
// .. + 3 of a row-major bf16 tile, lane i receives tokens t0 .. t0 + 3 of
// feature f0 + i: a token-major matrix-core operand straight from LDS.
__device__ __forceinline__ u32x2 lds_read_tr16(const void* p) {
  const s16x4 r = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4_ptr)(p));
  return __builtin_bit_cast(u32x2, r);
}

// Wait until at most N vector memory operations of this wave are
// outstanding; also a compiler barrier.
template <int N>
__device__ __forceinline__ void wait_vmem() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

template <int OT, int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FusedCfg<D>::WAVES_PER_SIMD)))
void bwd_qds_kernel(const void* __restrict__ q, const void* __restrict__ dout, int64_t sb,
                    int64_t sh, int64_t sn, void* __restrict__ dq, int64_t osb, int64_t osh,
                    int64_t osn, int H, int64_t N, int P, int Tw, const void* __restrict__ img,
                    const double* __restrict__ z64, float* __restrict__ part) {
  using C = RowCfg<DT_BF16, D>;
  using FC = FusedCfg<D>;
  using IC = ImageCfg<D>;
  using RN = Run<D, DT_BF16>;
  constexpr int Q4 = D / 4, NT = D / 16, TT = FC::TT, NB = FC::NB, NS = FC::NS;
  constexpr int RW = FC::RW, NCH = FC::NCH;
  constexpr int OES = OT == DT_BF16 ? 2 : 4;
  constexpr int IMG_WORDS = IC::mat_bytes(DT_BF16) / 16;  // the N image
  constexpr int Z_WORDS = IC::tile_bytes(DT_BF16) / 16;   // the T image's z tile
  constexpr int E = D * D + D;
  static_assert(TT == C::TT && RW == C::PW, "run layout");
  __shared__ u32x4 simg[IMG_WORDS + Z_WORDS];
  __shared__ float zf[D];
  __shared__ u32x4 stage[4 * FC::STAGE / 16];
  const u32x4* zimg = simg + IMG_WORDS;

  const int bh = blockIdx.y;
  const int64_t b = bh / H, h = bh % H;
  {
    const char* head = (const char*)img + (int64_t)bh * IC::head_bytes(DT_BF16);
    stage_image(simg, (const u32x4*)(head + IC::img_bytes(DT_BF16)), IMG_WORDS, false);
    stage_image(simg + IMG_WORDS, (const u32x4*)(head + IC::mat_bytes(DT_BF16)), Z_WORDS, false);
    for (int c = threadIdx.x; c < D; c += 256) zf[c] = (float)z64[(int64_t)bh * D + c];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = wave_index();
  const int g = lane >> 4, n = lane & 15;
  const int p = blockIdx.x * 4 + wave;
  if (p >= P) return;  // no barriers follow
  // partial p takes the head's 32-token blocks p, p + P, p + 2P, ... (at
  // most Tw tokens), so the grid's waves move through Q, G and dQ together
  const int64_t nb = (N + 16 * TT - 1) / (16 * TT);
  const int nsteps = (int)((nb - 1 - p) / P + 1);  // >= 1: P <= N / 64 < nb
  auto first_token = [&](int k) { return ((int64_t)p + (int64_t)k * P) * (16 * TT); };

  const int64_t row_bytes = sn * 2, orow_bytes = osn * OES;
  const char* qh = (const char*)q + (b * sb + h * sh) * 2;
  const char* gh = (const char*)dout + (b * sb + h * sh) * 2;
  char* oh = (char*)dq + (b * osb + h * osh) * OES;
  const uint32_t ioff = (uint32_t)n * (uint32_t)row_bytes + (uint32_t)(g * RN::CB);
  const uint32_t ooff = (uint32_t)n * (uint32_t)orow_bytes + (uint32_t)(g * RN::CH * OES);
  u32x4* stg = stage + wave * (FC::STAGE / 16);

  // Prefetch a step's Q and G runs into this wave's LDS stage: slot
  // [(tt*2 + tensor)*NCH + chunk][lane].  Rows past the head's end are
  // skipped (their slots keep stale data; the reader zeroes those tokens).
  auto prefetch = [&](int64_t t0) {
#pragma unroll
    for (int tt = 0; tt < TT; ++tt) {
      const bool ok = t0 + 16 * tt + n < N;
#pragma unroll
      for (int ten = 0; ten < 2; ++ten) {
        const char* src = (ten == 0 ? qh : gh) + (t0 + 16 * tt) * row_bytes + ioff;
#pragma unroll
        for (int w = 0; w < NCH; ++w) {
          if (ok)
            __builtin_amdgcn_global_load_lds((const void*)(src + w * 4 * RN::CB),
                                             (lds_void_ptr)(stg + ((tt * 2 + ten) * NCH + w) * 64),
                                             16, 0, 0);
        }
      }
    }
  };

  // 0/1 selection operands: lane (g, n) supplies B[8g + j][n] = (8g + j == n + 16h)
  bf16x8 sel[2];
#pragma unroll
  for (int hh = 0; hh < 2; ++hh) {
    uint32_t w4[4] = {0u, 0u, 0u, 0u};
    const int k = n + 16 * hh;
    if (k / 8 == g) w4[(k % 8) >> 1] = (k & 1) ? 0x3f800000u : 0x00003f80u;
    sel[hh] = as_bf16x8(u32x4{w4[0], w4[1], w4[2], w4[3]});
  }

  f32x4 ds[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) ds[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // dz partial sums: lane (g', n) of block i holds feature 16i + n over the
  // tokens 4g' + r it saw
  float dzb[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) dzb[i] = 0.f;

  prefetch(first_token(0));
  for (int kstep = 0; kstep < nsteps; ++kstep) {
    const int64_t t0 = first_token(kstep);
    // this step's runs: wait for its prefetch, read them, then refill the
    // stage.  The loads into LDS share the vector memory counter with the
    // previous step's dQ stores, and nothing orders a load's retirement
    // before a store issued after it, so only a zero count proves the
    // stage has landed (the compiler emits the same full wait before any
    // LDS read that a load into LDS may have written)
    wait_vmem<0>();
    uint32_t pq[TT][RW], pg[TT][RW];
#pragma unroll
    for (int tt = 0; tt < TT; ++tt) {
      const bool ok = t0 + 16 * tt + n < N;
      uint32_t qw[RW];
#pragma unroll
      for (int w = 0; w < NCH; ++w) {
        const u32x4 a = stg[((tt * 2 + 0) * NCH + w) * 64 + lane];
        const u32x4 c = stg[((tt * 2 + 1) * NCH + w) * 64 + lane];
        qw[4 * w] = ok ? a.x : 0u; qw[4 * w + 1] = ok ? a.y : 0u;
        qw[4 * w + 2] = ok ? a.z : 0u; qw[4 * w + 3] = ok ? a.w : 0u;
        pg[tt][4 * w] = ok ? c.x : 0u; pg[tt][4 * w + 1] = ok ? c.y : 0u;
        pg[tt][4 * w + 2] = ok ? c.z : 0u; pg[tt][4 * w + 3] = ok ? c.w : 0u;
      }
      phi_words<DT_BF16, D>(qw, pq[tt]);
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    if (kstep + 1 < nsteps) prefetch(first_token(kstep + 1));

    // X = S G and den = phi(q) . z on the matrix cores
    f32x4 acc[TT][NT];
#pragma unroll
    for (int tt = 0; tt < TT; ++tt)
#pragma unroll
      for (int i = 0; i < NT; ++i) acc[tt][i] = f32x4{0.f, 0.f, 0.f, 0.f};
    image_times_runs<DT_BF16, D, true>(simg, lane, pg, acc);
    f32x4 dacc[TT][1];
#pragma unroll
    for (int tt = 0; tt < TT; ++tt) dacc[tt][0] = f32x4{0.f, 0.f, 0.f, 0.f};
    tile_times_runs<DT_BF16, D>(zimg, lane, pq, dacc);

    // token-major G operands for dS: bg[j] = G of feature block j, 8 tokens
    bf16x8 bg[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      f32x4 tr[TT];
#pragma unroll
      for (int tt = 0; tt < TT; ++tt) {
        const int s0 = j >> 1;
        const bf16x8 a = as_bf16x8(u32x4{pg[tt][4 * s0], pg[tt][4 * s0 + 1], pg[tt][4 * s0 + 2],
                                         pg[tt][4 * s0 + 3]});
        tr[tt] = mfma_bf16(a, sel[j & 1], f32x4{0.f, 0.f, 0.f, 0.f});
      }
      // exact: the products are bf16 values times 1
      bg[j] = as_bf16x8(u32x4{pack_bf16(tr[0][0], tr[0][1]), pack_bf16(tr[0][2], tr[0][3]),
                              pack_bf16(tr[1][0], tr[1][1]), pack_bf16(tr[1][2], tr[1][3])});
    }

    // per token: den, G . O, dQ, and the scales 1/den and dden = -(G . O)/den
    float rdt[TT], ddt[TT];
#pragma unroll
    for (int tt = 0; tt < TT; ++tt) {
      float gn = 0.f;
#pragma unroll
      for (int i = 0; i < NT; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) gn += run_val<DT_BF16>(pq[tt], 4 * i + r) * acc[tt][i][r];
      gn = sum_groups(gn);
      const double rden = 1.0 / (double)dacc[tt][0][0];
      const float rd = (float)rden;
      const float go = gn * rd;  // G . O
      rdt[tt] = rd;
      ddt[tt] = -go * rd;        // zero for padded tokens (G = 0)
      const int64_t t = t0 + 16 * tt + n;
      const bool ok = t < N;
      // dQ chunk by chunk (few live registers): run positions [CH*w, +CH)
      constexpr int CH = RN::CH;
      constexpr int OCB = CH * OES;
      char* orow = oh + (t0 + 16 * tt) * orow_bytes + ooff;
#pragma unroll
      for (int w = 0; w < NCH; ++w) {
        uint32_t ow[OCB / 4];
#pragma unroll
        for (int j = 0; j < CH; j += 2) {
          float o2[2];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const int c = CH * w + j + u;
            const float ph = run_val<DT_BF16>(pq[tt], c);
            const float zc = zf[RN::feature(g, c)];
            o2[u] = (fmaf(-go, zc, acc[tt][c >> 2][c & 3]) * rd) * dphi_of_phi(ph);
          }
          if constexpr (OT == DT_BF16) {
            ow[j >> 1] = pack_bf16(o2[0], o2[1]);
          } else {
            ow[j] = __float_as_uint(o2[0]);
            ow[j + 1] = __float_as_uint(o2[1]);
          }
        }
        if (ok) store_words<OCB>(orow + w * 4 * OCB, ow);
      }
    }

    // dS[i][j] += (phi(q)/den of block i, token-major) x bg[j], and
    // dz[block i] += token sums of phi(q) dden, both made token-major by
    // the selection product
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int s0 = i >> 1;
      f32x4 tr[TT], tz[TT];
#pragma unroll
      for (int tt = 0; tt < TT; ++tt) {
        uint32_t wa[4], wz[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const uint32_t w = pq[tt][4 * s0 + k];
          wa[k] = pack_bf16(bf16lo(w) * rdt[tt], bf16hi(w) * rdt[tt]);
          wz[k] = pack_bf16(bf16lo(w) * ddt[tt], bf16hi(w) * ddt[tt]);
        }
        tr[tt] = mfma_bf16(as_bf16x8(u32x4{wa[0], wa[1], wa[2], wa[3]}), sel[i & 1],
                           f32x4{0.f, 0.f, 0.f, 0.f});
        tz[tt] = mfma_bf16(as_bf16x8(u32x4{wz[0], wz[1], wz[2], wz[3]}), sel[i & 1],
                           f32x4{0.f, 0.f, 0.f, 0.f});
      }
      dzb[i] += ((tz[0][0] + tz[0][1]) + (tz[0][2] + tz[0][3])) +
                ((tz[1][0] + tz[1][1]) + (tz[1][2] + tz[1][3]));
      const bf16x8 ai = as_bf16x8(u32x4{pack_bf16(tr[0][0], tr[0][1]), pack_bf16(tr[0][2], tr[0][3]),
                                        pack_bf16(tr[1][0], tr[1][1]), pack_bf16(tr[1][2], tr[1][3])});
#pragma unroll
      for (int j = 0; j < NB; ++j) ds[i][j] = mfma_bf16(ai, bg[j], ds[i][j]);
    }
  }

  // the wave's partial: dS tiles in lane order, then dz
  float* out = part + ((int64_t)bh * P + p) * E;
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) *(f32x4*)(out + ((i * NB + j) * 64 + lane) * 4) = ds[i][j];
  // dz: add the four lane groups' token subsets
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const float v = sum_groups(dzb[i]);
    if (g == 0) out[D * D + 16 * i + n] = v;
  }
}

// ---------------------------------------------------------------------------
// Fused query backward at d = 128 (bf16): the four waves of a workgroup
// share one partial (64-token blocks p, p + P, ..., at most Tw tokens),
// taking 16-token tiles in turn (one block per step); two workgroups fit a compute unit, so one
// waiting at a barrier leaves the SIMDs to the other.  Each wave does the
// query pass for its tile and makes its tile's token-major operands (as in
// bwd_qds_kernel, by selection products) into LDS; after a barrier, wave w
// accumulates a 4 x 4 patch of the 8 x 8 grid of dS tiles over the four
// tiles (two 32-token contractions), so its share of the partial is 16
// tiles (64 registers) instead of the whole 128 x 128.  dz = sum_i dden_i
// phi(q_i) rides along as one more column block of the same products (the
// waves of the left column of patches take it).
// ---------------------------------------------------------------------------
template <int OT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void bwd_qds4_kernel(const void* __restrict__ q, const void* __restrict__ dout, int64_t sb,
                     int64_t sh, int64_t sn, void* __restrict__ dq, int64_t osb, int64_t osh,
                     int64_t osn, int H, int64_t N, int P, int Tw, const void* __restrict__ img,
                     const double* __restrict__ z64, float* __restrict__ part) {
  constexpr int D = 128;
  using IC = ImageCfg<D>;
  using RN = Run<D, DT_BF16>;
  constexpr int Q4 = D / 4, NT = D / 16, NB = D / 16, NS = IC::NS;
  constexpr int RW = D / 8, NCH = RN::NCH, CH = RN::CH;
  constexpr int OES = OT == DT_BF16 ? 2 : 4;
  constexpr int OCB = CH * OES;
  constexpr int IMG_WORDS = IC::mat_bytes(DT_BF16) / 32;  // the N image, hi parts
  constexpr int Z_WORDS = IC::tile_bytes(DT_BF16) / 16;   // the T image's z tile
  constexpr int E = D * D + D;
  __shared__ u32x4 simg[IMG_WORDS + Z_WORDS];
  __shared__ float zf[D];
  constexpr int NW = 4;             // waves (tiles per step)
  // each wave's tile as it holds it, row-major (16 token rows of d bf16
  // values: phi(q)/den in rowq, G in rowg); the contraction reads them back
  // token-major with the transposing LDS read.  The 16-byte chunks of a
  // row are XOR-swizzled by the row (tile_slot), so that the four rows one
  // 16-lane block reads lie in distinct banks.  xz: -G.O (hi, lo) of each
  // token in columns 0 and 1, token-major; tiles 2*kap and 2*kap + 1 fill
  // the low and high halves of a lane's 16-byte slot
  constexpr int RC = D * 2 / 16;    // 16-byte chunks per row
  __shared__ u32x4 rowq[NW][16 * RC];
  __shared__ u32x4 rowg[NW][16 * RC];
  __shared__ u32x4 xz[NW / 2][64];
  auto tile_slot = [](int row, int chunk) {
    return row * RC + (chunk ^ (2 * (row & 3) + 8 * ((row >> 2) & 1)));
  };
  const u32x4* zimg = simg + IMG_WORDS;

  const int bh = blockIdx.y;
  const int64_t b = bh / H, h = bh % H;
  {
    const char* head = (const char*)img + (int64_t)bh * IC::head_bytes(DT_BF16);
    stage_image(simg, (const u32x4*)(head + IC::img_bytes(DT_BF16)), IMG_WORDS, true);
    stage_image(simg + IMG_WORDS, (const u32x4*)(head + IC::mat_bytes(DT_BF16)), Z_WORDS, false);
    for (int c = threadIdx.x; c < D; c += 64 * NW) zf[c] = (float)z64[(int64_t)bh * D + c];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = wave_index();
  const int g = lane >> 4, n = lane & 15;
  // partial p (this workgroup) takes the head's 64-token blocks p, p + P,
  // p + 2P, ... (at most Tw tokens), so the grid moves through Q, G and dQ
  // together; the step count is the same for all waves
  const int p = blockIdx.x;
  const int64_t nb = (N + 16 * NW - 1) / (16 * NW);
  const int nsteps = (int)((nb - 1 - p) / P + 1);  // >= 1: P <= N / 64 <= nb
  auto block_token = [&](int k) { return ((int64_t)p + (int64_t)k * P) * (16 * NW); };

  const int64_t row_bytes = sn * 2, orow_bytes = osn * OES;
  const char* qh = (const char*)q + (b * sb + h * sh) * 2;
  const char* gh = (const char*)dout + (b * sb + h * sh) * 2;
  char* oh = (char*)dq + (b * osb + h * osh) * OES;
  const uint32_t ooff = (uint32_t)n * (uint32_t)orow_bytes + (uint32_t)(g * OCB);

  typedef uint32_t Regs[2][RW];  // Q run, G run of this wave's tile
  // Rows past the head's end read its last token again (finite values, no
  // zero fill); the step gives such tokens a zero scale, so they add
  // nothing to dS or dz and their dQ rows are not stored.
  auto load = [&](int k, Regs& x) {
    const int64_t tb = min(block_token(k) + 16 * wave, N - 1);  // wave-uniform
    const int last = (int)min((int64_t)15, N - 1 - tb);
    const uint32_t off = (uint32_t)min(n, last) * (uint32_t)row_bytes + (uint32_t)(g * RN::CB);
    load_run<D, DT_BF16>(qh + tb * row_bytes + off, x[0]);
    load_run<D, DT_BF16>(gh + tb * row_bytes + off, x[1]);
  };

  bf16x8 sel[2];
#pragma unroll
  for (int hh = 0; hh < 2; ++hh) {
    uint32_t w4[4] = {0u, 0u, 0u, 0u};
    const int k = n + 16 * hh;
    if (k / 8 == g) w4[(k % 8) >> 1] = (k & 1) ? 0x3f800000u : 0x00003f80u;
    sel[hh] = as_bf16x8(u32x4{w4[0], w4[1], w4[2], w4[3]});
  }

  // wave w accumulates the 4 x 4 patch of dS tiles at (i0, j0); the waves
  // with j0 = 0 also take the column block NB of their rows, whose columns
  // 0 and 1 sum to dz (see the step)
  constexpr int IW = 4, JW = 4;  // row and column blocks per wave
  const int i0 = IW * (wave >> 1), j0 = JW * (wave & 1);
  const bool has_dz = (wave & 1) == 0;
  f32x4 ds[IW][JW], dzb[IW];
#pragma unroll
  for (int ii = 0; ii < IW; ++ii) {
    dzb[ii] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int jj = 0; jj < JW; ++jj) ds[ii][jj] = f32x4{0.f, 0.f, 0.f, 0.f};
  }

  auto step = [&](int k, const Regs& x) {
    const int64_t tb = block_token(k) + 16 * wave;
    uint32_t pq[RW];
    phi_words<DT_BF16, D>(x[0], pq);
    const uint32_t* pg = x[1];
    // X = S G (S as its bf16 hi part) and den = phi(q) . z (the z tile,
    // hi + lo) for the tile
    f32x4 acc[NT], dacc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < NT; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    // the wave's issue priority is raised over these products, so that the
    // other workgroup's wave on the SIMD fills their latency with its
    // vector work (2.57 -> 2.53 ms; raising it over the dS contraction
    // instead gained nothing)
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int i = 0; i < NT; ++i) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const bf16x8 bt = as_bf16x8(u32x4{pg[4 * s], pg[4 * s + 1], pg[4 * s + 2], pg[4 * s + 3]});
        acc[i] = mfma_bf16(as_bf16x8(simg[(i * NS + s) * 64 + lane]), bt,
                           s == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[i]);
      }
    }
    __builtin_amdgcn_s_setprio(0);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const bf16x8 bt = as_bf16x8(u32x4{pq[4 * s], pq[4 * s + 1], pq[4 * s + 2], pq[4 * s + 3]});
      dacc = mfma_bf16(as_bf16x8(zimg[(s * 2 + 0) * 64 + lane]), bt,
                       s == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : dacc);
      dacc = mfma_bf16(as_bf16x8(zimg[(s * 2 + 1) * 64 + lane]), bt, dacc);
    }
    // this tile's G rows into LDS: chunk w of the lane's run is the row's
    // 16-byte chunk 4w + g
#pragma unroll
    for (int w = 0; w < NCH; ++w)
      rowg[wave][tile_slot(n, 4 * w + g)] = u32x4{pg[4 * w], pg[4 * w + 1], pg[4 * w + 2], pg[4 * w + 3]};
    const bool ok = tb + n < N;
    const double rden = 1.0 / (double)dacc[0];
    const float rd = ok ? (float)rden : 0.f;  // zero past the end: no dS, dz share
    // G . O = phi(q) . X / den per token
    float gn = 0.f;
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) gn += run_val<DT_BF16>(pq, 4 * i + r) * acc[i][r];
    gn = sum_groups(gn);
    const float go = gn * rd;
    // dz = sum_i dden_i phi(q_i) = sum_i (phi(q_i)/den_i)(-G_i . O_i): one
    // more column block of the dS product, whose B operand holds -G.O of
    // each token as a bf16 pair hi + lo in columns 0 and 1 (made
    // token-major by the same selection product)
    {
      const float hi = bf16f(to_bf16(-go));
      const uint32_t w0 = g == 0 ? pack_bf16(hi, -go - hi) : 0u;
      const f32x4 tr = mfma_bf16(as_bf16x8(u32x4{w0, 0u, 0u, 0u}), sel[0], f32x4{0.f, 0.f, 0.f, 0.f});
      ((u32x2*)&xz[wave >> 1][lane])[wave & 1] = u32x2{pack_bf16(tr[0], tr[1]), pack_bf16(tr[2], tr[3])};
    }
    // dQ
    char* orow = oh + tb * orow_bytes + ooff;
#pragma unroll
    for (int w = 0; w < NCH; ++w) {
      uint32_t ow[OCB / 4];
#pragma unroll
      for (int j = 0; j < CH; j += 2) {
        float o2[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int c = CH * w + j + u;
          const float ph = run_val<DT_BF16>(pq, c);
          o2[u] = (fmaf(-go, zf[RN::feature(g, c)], acc[c >> 2][c & 3]) * rd) * dphi_of_phi(ph);
        }
        if constexpr (OT == DT_BF16) {
          ow[j >> 1] = pack_bf16(o2[0], o2[1]);
        } else {
          ow[j] = __float_as_uint(o2[0]);
          ow[j + 1] = __float_as_uint(o2[1]);
        }
      }
      if (ok) store_words<OCB>(orow + w * 4 * OCB, ow);
    }
    // this tile's phi(q)/den rows into LDS (bf16, as the contraction
    // takes them)
#pragma unroll
    for (int w = 0; w < NCH; ++w) {
      uint32_t wa[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const uint32_t x = pq[4 * w + kk];
        wa[kk] = pack_bf16(bf16lo(x) * rd, bf16hi(x) * rd);
      }
      rowq[wave][tile_slot(n, 4 * w + g)] = u32x4{wa[0], wa[1], wa[2], wa[3]};
    }
    __syncthreads();
    // the wave's dS patch (and dz columns) over the step's tiles: tiles
    // (2k, 2k + 1) make one 32-token contraction
    // operand of feature block f of the tile pair: lane (g, m) addresses
    // row 4g + (m >> 2), features 16f + 4 (m & 3) .. + 3 of each tile, and
    // receives tokens 4g .. 4g + 3 of feature 16f + m: of tile 2 kap as
    // elements 0..3, of tile 2 kap + 1 as elements 4..7 (the token order
    // of xz)
    const int rrow = 4 * g + (n >> 2);
    auto operand = [&](const u32x4 (*t)[16 * RC], int kap, int f) {
      const int slot = tile_slot(rrow, 2 * f + ((n & 3) >> 1));
      const int half = (n & 1) * 8;
      const u32x2 lo = lds_read_tr16((const char*)&t[2 * kap][slot] + half);
      const u32x2 hi = lds_read_tr16((const char*)&t[2 * kap + 1][slot] + half);
      return as_bf16x8(u32x4{lo[0], lo[1], hi[0], hi[1]});
    };
#pragma unroll
    for (int kap = 0; kap < NW / 2; ++kap) {
      bf16x8 aa[IW];
#pragma unroll
      for (int ii = 0; ii < IW; ++ii) aa[ii] = operand(rowq, kap, i0 + ii);
#pragma unroll
      for (int jj = 0; jj < JW; ++jj) {
        const bf16x8 bb = operand(rowg, kap, j0 + jj);
#pragma unroll
        for (int ii = 0; ii < IW; ++ii) ds[ii][jj] = mfma_bf16(aa[ii], bb, ds[ii][jj]);
      }
      if (has_dz) {
        const bf16x8 bz = as_bf16x8(xz[kap][lane]);
#pragma unroll
        for (int ii = 0; ii < IW; ++ii) dzb[ii] = mfma_bf16(aa[ii], bz, dzb[ii]);
      }
    }
    __syncthreads();  // before the next step rewrites rowq, rowg, xz
  };

  // two register sets in turn: the next step's inputs are in flight while
  // this step computes.  The loads are unconditional and the loop body has
  // no early exit (a step past the end reads the partial's last row and
  // adds nothing, see load and step), so the compiler's wait counts cover
  // only the set a step is about to use; an odd step count runs one such
  // empty step.  The scheduling barriers keep each load at the start of
  // the step before its use (the scheduler would otherwise sink it).
  Regs ra, rb;
  load(0, ra);
  for (int k = 0; k < nsteps; k += 2) {
    load(k + 1, rb);
    __builtin_amdgcn_sched_barrier(0);
    step(k, ra);
    load(k + 2, ra);
    __builtin_amdgcn_sched_barrier(0);
    step(k + 1, rb);
  }

  // the workgroup's partial: each wave's dS patch, and dz (the sum of
  // columns 0 and 1 of block NB: lanes n = 0 and 1) from the left half
  float* out = part + ((int64_t)bh * P + p) * E;
#pragma unroll
  for (int ii = 0; ii < IW; ++ii)
#pragma unroll
    for (int jj = 0; jj < JW; ++jj)
      *(f32x4*)(out + (((i0 + ii) * NB + j0 + jj) * 64 + lane) * 4) = ds[ii][jj];
  if (has_dz) {
#pragma unroll
    for (int ii = 0; ii < IW; ++ii)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float v = dzb[ii][r] + __shfl_xor(dzb[ii][r], 1);
        if (n == 0) out[D * D + 16 * (i0 + ii) + 4 * g + r] = v;
      }
  }
}

// ---------------------------------------------------------------------------
// Key kernel: dV = phi(K) dS (T image of dS) and dK = (V dS^T + dz) phi'(K)
// (N image of dS).  WHICH: 1 = dV only, 2 = dK only, 3 = both.
// The dS operands are the hi parts of the bf16 images.  As in the apply,
// the G workgroups of a head take its blocks of 4 * 16 * TT tokens in turn
// (blocks g, g + G, ...), so the whole grid moves through the tensors
// together.
// ---------------------------------------------------------------------------
template <int DT, int OT, int D, int WHICH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void bwd_key_kernel(
    const void* __restrict__ k, const void* __restrict__ v, int64_t sb, int64_t sh,
    int64_t sn, void* __restrict__ dk, void* __restrict__ dv, int64_t osb, int64_t osh,
    int64_t osn, int H, int64_t N, int G, const void* __restrict__ dimg,
    const double* __restrict__ dz64) {
  using C = RowCfg<DT, D>;
  using IC = ImageCfg<D>;
  constexpr int Q4 = C::Q4, NT = C::NT, TT = C::TT;
  constexpr int OES = OT == DT_BF16 ? 2 : 4;
  // matrix tiles only (the z tile is not needed here); bf16: hi parts only
  constexpr int ONE = DT == DT_BF16 ? IC::mat_bytes(DT) / 32 : IC::mat_bytes(DT) / 16;
  constexpr bool DO_V = WHICH & 1, DO_K = WHICH & 2;
  __shared__ u32x4 simg[(DO_V ? ONE : 0) + (DO_K ? ONE : 0)];
  u32x4* timg = simg;
  u32x4* nimg = simg + (DO_V ? ONE : 0);

  const int bh = blockIdx.y;
  const int64_t b = bh / H, h = bh % H;
  const u32x4* head = (const u32x4*)((const char*)dimg + (int64_t)bh * IC::head_bytes(DT));
  if (DO_V) stage_image(timg, head, ONE, DT == DT_BF16);
  if (DO_K) stage_image(nimg, head + IC::img_bytes(DT) / 16, ONE, DT == DT_BF16);
  const int lane = threadIdx.x & 63, wave = wave_index();
  const int g = lane >> 4, n = lane & 15;
  // dz is added in FP32 for bf16 inputs (their dS operands are bf16 hi
  // parts, whose rounding is some 2^15 times that of dz to FP32) and in
  // FP64 for fp32 inputs
  using DzT = typename std::conditional<DT == DT_BF16, float, double>::type;
  DzT dzr[DO_K ? Q4 : 1];
  if constexpr (DO_K) {
#pragma unroll
    for (int c = 0; c < Q4; ++c) dzr[c] = (DzT)dz64[(int64_t)bh * D + Run<D, DT>::feature(g, c)];
  }
  __syncthreads();

  const int64_t in_head = (b * sb + h * sh) * C::ES + (int64_t)g * Run<D, DT>::CB;
  const char* kbase = (const char*)k + in_head;
  const char* vbase = (const char*)v + in_head;
  const int64_t out_head = (b * osb + h * osh) * OES + (int64_t)g * Run<D, DT>::CH * OES;

  // (rows past the head's end are zero-filled; reading the last row again
  // instead saves the fill but measured 1.5 % slower at d = 128)
  auto load_one = [&](int64_t t0, uint32_t* kw, uint32_t* vw) {
    const int64_t t = t0 + n;
    if (t < N) {
      load_run<D, DT>(kbase + t * sn * C::ES, kw);
      if (DO_K) load_run<D, DT>(vbase + t * sn * C::ES, vw);
    } else {
#pragma unroll
      for (int w = 0; w < C::RWD; ++w) { kw[w] = 0; vw[w] = 0; }
    }
  };
  auto load = [&](int64_t t0, uint32_t (&kw)[C::PF ? TT : 1][C::RWD],
                  uint32_t (&vw)[C::PF ? TT : 1][C::RWD]) {
#pragma unroll
    for (int tt = 0; tt < (C::PF ? TT : 1); ++tt) load_one(t0 + 16 * tt, kw[tt], vw[tt]);
  };
  constexpr int BLK = 16 * TT * 4;  // tokens per block
  const int64_t nblk = (N + BLK - 1) / BLK;
  const int64_t blk0 = blockIdx.x;
  const int nk = blk0 < nblk ? (int)((nblk - 1 - blk0) / G + 1) : 0;
  // first token of this wave's part of the k-th block it takes
  auto tok = [&](int kk) { return (blk0 + (int64_t)kk * G) * BLK + 16 * TT * wave; };
  uint32_t kcur[C::PF ? TT : 1][C::RWD], vcur[C::PF ? TT : 1][C::RWD];
  if constexpr (C::PF) {
    if (nk > 0) load(tok(0), kcur, vcur);
  }
  for (int kk = 0; kk < nk; ++kk) {
    const int64_t t0 = tok(kk);
    // next step's inputs are in flight while this step computes
    uint32_t knext[C::PF ? TT : 1][C::RWD], vnext[C::PF ? TT : 1][C::RWD];
    const bool more = C::PF && kk + 1 < nk;
    uint32_t pk[TT][C::PW], pv[TT][C::PW];
    if constexpr (C::PF) {
      if (more) load(tok(kk + 1), knext, vnext);
#pragma unroll
      for (int tt = 0; tt < TT; ++tt) {
        phi_words<DT, D>(kcur[tt], pk[tt]);
        if (DO_K) raw_words<DT, D>(vcur[tt], pv[tt]);
      }
    } else {
      // load and convert one tile at a time (fewer live registers)
#pragma unroll
      for (int tt = 0; tt < TT; ++tt) {
        uint32_t one_k[C::RWD], one_v[C::RWD];
        load_one(t0 + 16 * tt, one_k, one_v);
        phi_words<DT, D>(one_k, pk[tt]);
        if (DO_K) raw_words<DT, D>(one_v, pv[tt]);
      }
    }
    if constexpr (DO_V) {
      f32x4 acc[TT][NT];
#pragma unroll
      for (int tt = 0; tt < TT; ++tt)
#pragma unroll
        for (int i = 0; i < NT; ++i) acc[tt][i] = f32x4{0.f, 0.f, 0.f, 0.f};
      image_times_runs<DT, D, false>(timg, lane, pk, acc);
#pragma unroll
      for (int tt = 0; tt < TT; ++tt) {
        const int64_t t = t0 + 16 * tt + n;
        if (t < N) {
          float out[Q4];
#pragma unroll
          for (int i = 0; i < NT; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) out[4 * i + r] = acc[tt][i][r];
          store_run<D, DT, OT>((char*)dv + out_head + t * osn * OES, out);
        }
      }
    }
    if constexpr (DO_K) {
      f32x4 acc[TT][NT];
#pragma unroll
      for (int tt = 0; tt < TT; ++tt)
#pragma unroll
        for (int i = 0; i < NT; ++i) acc[tt][i] = f32x4{0.f, 0.f, 0.f, 0.f};
      image_times_runs<DT, D, false>(nimg, lane, pv, acc);
#pragma unroll
      for (int tt = 0; tt < TT; ++tt) {
        const int64_t t = t0 + 16 * tt + n;
        if (t < N) {
          float out[Q4];
#pragma unroll
          for (int i = 0; i < NT; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int c = 4 * i + r;
              const float dphi_c = dphi_of_phi(run_val<DT>(pk[tt], c));
              out[c] = (float)((DzT)acc[tt][i][r] + dzr[c]) * dphi_c;
            }
          store_run<D, DT, OT>((char*)dk + out_head + t * osn * OES, out);
        }
      }
    }
    if (more) {
#pragma unroll
      for (int tt = 0; tt < (C::PF ? TT : 1); ++tt)
#pragma unroll
        for (int w = 0; w < C::RWD; ++w) { kcur[tt][w] = knext[tt][w]; vcur[tt][w] = vnext[tt][w]; }
    }
  }
}

// ---------------------------------------------------------------------------
// Each step's launch status is taken as soon as it is known: the
// launchers of the combine and the summary read (and so clear) the
// runtime's last error, which would otherwise hide an earlier failure.
template <int DT, int OT, int D>
static hipError_t launch_rows(const BwdArgs& a) {
  hipError_t e = hipSuccess;
  const int BH = (int)(a.B * a.H);
  dim3 grid((unsigned)((a.N + a.Ta - 1) / a.Ta), BH);
  if constexpr (DT == DT_BF16 && D == 128) {
    // one pass, four waves sharing each partial
    ProfScope prof("bwd_query_ds", a.stream);
    dim3 fgrid((unsigned)a.P, BH);
    bwd_qds4_kernel<OT><<<fgrid, 256, 0, a.stream>>>(
        a.q, a.dout, a.sb, a.sh, a.sn, a.dq, a.osb, a.osh, a.osn, (int)a.H, a.N, a.P, a.Tw,
        a.img, a.z64, a.part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = launch_combine(a.part, a.P, a.dS64, a.dz64, a.dimg, DT, BH, D, PART_BLOCKS, a.stream);
  } else if constexpr (DT == DT_BF16 && (D == 32 || D == 64)) {
    // one pass: dQ and the per-wave partials of dS, dz (at d = 128 the
    // whole partial dS plus the query pass's state exceed the registers of
    // one wave, so there four waves share a partial, above)
    ProfScope prof("bwd_query_ds", a.stream);
    dim3 fgrid((unsigned)((a.P + 3) / 4), BH);
    bwd_qds_kernel<OT, D><<<fgrid, 256, 0, a.stream>>>(
        a.q, a.dout, a.sb, a.sh, a.sn, a.dq, a.osb, a.osh, a.osn, (int)a.H, a.N, a.P, a.Tw,
        a.img, a.z64, a.part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = launch_combine(a.part, a.P, a.dS64, a.dz64, a.dimg, DT, BH, D, PART_BLOCKS, a.stream);
  } else {
    {
      ProfScope prof("bwd_query", a.stream);
      bwd_query_kernel<DT, OT, D><<<grid, 256, 0, a.stream>>>(
          a.q, a.dout, a.sb, a.sh, a.sn, a.dq, a.osb, a.osh, a.osn, (int)a.H, a.N, a.Ta, a.img,
          a.z64, a.stash);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = launch_summary(MODE_BWD, DT, D, a.q, a.dout, a.sb, a.sh, a.sn, a.B, a.H, a.N, a.P, a.Tw,
                       a.stash, a.part, a.stream);
    if (e != hipSuccess) return e;
    e = launch_combine(a.part, a.P, a.dS64, a.dz64, a.dimg, DT, BH, D, PART_SUMMARY, a.stream);
  }
  if (e != hipSuccess) return e;
  // both dS images fit in LDS except fp32 at d = 128 (2 x 64 KB): two passes
  ProfScope prof("bwd_key", a.stream);
  const dim3 kgrid((unsigned)a.Gk, BH);
  if constexpr (DT == DT_FP32 && D >= 128) {
    bwd_key_kernel<DT, OT, D, 1><<<kgrid, 256, 0, a.stream>>>(
        a.k, a.v, a.sb, a.sh, a.sn, a.dk, a.dv, a.osb, a.osh, a.osn, (int)a.H, a.N, a.Gk,
        a.dimg, a.dz64);
    bwd_key_kernel<DT, OT, D, 2><<<kgrid, 256, 0, a.stream>>>(
        a.k, a.v, a.sb, a.sh, a.sn, a.dk, a.dv, a.osb, a.osh, a.osn, (int)a.H, a.N, a.Gk,
        a.dimg, a.dz64);
  } else {
    bwd_key_kernel<DT, OT, D, 3><<<kgrid, 256, 0, a.stream>>>(
        a.k, a.v, a.sb, a.sh, a.sn, a.dk, a.dv, a.osb, a.osh, a.osn, (int)a.H, a.N, a.Gk,
        a.dimg, a.dz64);
  }
  return hipGetLastError();
}

template <int D>
static hipError_t launch_backward_d(const BwdArgs& a) {
  hipError_t e = launch_images(a.S64, a.z64, a.img, a.in_dt, a.B * a.H, D, a.stream);
  if (e != hipSuccess) return e;
  if (a.in_dt == DT_BF16 && a.out_dt == DT_BF16) return launch_rows<DT_BF16, DT_BF16, D>(a);
  if (a.in_dt == DT_BF16) return launch_rows<DT_BF16, DT_FP32, D>(a);
  if (a.out_dt == DT_BF16) return launch_rows<DT_FP32, DT_BF16, D>(a);
  return launch_rows<DT_FP32, DT_FP32, D>(a);
}

hipError_t launch_backward(const BwdArgs& a) {
  switch (a.D) {
    case 16: return launch_backward_d<16>(a);
    case 32: return launch_backward_d<32>(a);
    case 64: return launch_backward_d<64>(a);
    case 128: return launch_backward_d<128>(a);
  }
  return hipErrorInvalidValue;
}

}  // namespace la
