// la_forward.hip -- gfx950 kernels of the forward pass and of the FP64
// cross-tile combine.
//
// Forward of kernelised linear attention per (b, h):
//   S = phi(K)^T V, z = phi(K)^T 1 over all N tokens (summary_kernel, then
//   combine_kernel), O_i = phi(q_i)^T S / (phi(q_i) . z) (apply_kernel,
//   which can also blend O with another branch's output by a noise gate).
// Both phases stream HBM once: summary reads K and V, apply reads Q and
// writes O.  The d x d contractions run on the matrix cores.
#include "la_kernels.h"
#include "la_profile.h"
#include "la_summary.h"

namespace la {

// ---------------------------------------------------------------------------
// Summary: per wave, a contiguous token range [p*Tw, p*Tw + Tw) of one head.
// Lane (g, m) owns key/value features [F*m, F*m + F) (F = d/16) of R tokens
// per lane group per step.  Loads are contiguous F-feature runs of a token,
// so one load instruction covers whole token rows.  The feature-major
// operands the matrix core needs (a token run per feature) are assembled in
// registers: for bf16 the two tokens of a pair are packed into one word, so
// the transpose costs nothing beyond the pack that rounds phi(k) anyway.
//
// Tile (i, j) of the accumulator holds rows m <-> key feature F*m + i and
// columns n <-> value feature F*n + j, so lane (g, n) ends with
//   S[F*(4g + r) + i][F*n + j],  r = 0..3.
// These FP32 per-wave sums are written out; combine_kernel adds them in
// FP64 in partial order.
// ---------------------------------------------------------------------------
// Rows past the end of the range load K = -inf (phi = 0) and V = 0, so
// they add exactly nothing to S or z and the step itself needs no masks.
// In the backward mode the per-token pair (1/den, -(dO . O)) is loaded too.
// Addresses split into a wave-uniform part (head + (t0 + r) rows, scalar
// registers) and a loop-invariant 32-bit lane offset (koff, voff: the lane
// group's first row and the lane's feature run), so the loads need no
// per-lane address arithmetic.
template <int DT, int D, int MODE>
__device__ __forceinline__ void summary_load(const char* kh, const char* vh, uint32_t koff,
                                             uint32_t voff, const float2* stash,
                                             int64_t row_bytes, int64_t t0, int g, int m,
                                             int64_t t_end, SummaryRegs<DT, D, MODE>& x) {
  using C = SummaryCfg<DT, D, MODE>;
  const uint32_t neg_inf = DT == DT_BF16 ? 0xff80ff80u : 0xff800000u;
  if (t0 + C::STEP <= t_end) {
#pragma unroll
    for (int r = 0; r < C::R; ++r) {
      const int64_t ur = (t0 + r) * row_bytes;
      load_words_nt<C::KB>(kh + ur + koff, x.kw[r]);
      load_words_nt<C::VB>(vh + ur + voff, x.vw[r]);
    }
  } else {
#pragma unroll
    for (int r = 0; r < C::R; ++r) {
      const int64_t ur = (t0 + r) * row_bytes;
      if (t0 + C::R * g + r < t_end) {
        load_words_nt<C::KB>(kh + ur + koff, x.kw[r]);
        load_words_nt<C::VB>(vh + ur + voff, x.vw[r]);
      } else {
#pragma unroll
        for (int w = 0; w < C::KW; ++w) x.kw[r][w] = neg_inf;
#pragma unroll
        for (int w = 0; w < C::VW; ++w) x.vw[r][w] = 0;
      }
    }
  }
  if constexpr (MODE == MODE_BWD) {
    const int64_t t = t0 + C::R * g + m;
    x.tok = (m < C::R && t < t_end) ? stash[t] : float2{0.f, 0.f};
  }
}

// Grid: with SPLIT = 1, one dimension of waves in (partial, (b, h)) order,
// (b, h) fastest: wave w takes partial w / BH of (b, h) = w % BH, so a
// block's four waves are four heads over the same tokens (with heads
// interleaved in a token row, BNHD, one compute unit then reads adjacent
// slices of the same rows: the summary at d = 64, 16 heads, went from 1.55
// to 1.32 ms; BHND is unaffected).  Otherwise x = partial, y = (b, h), and
// the block's SPLIT waves share partial x, wave w owning S tile rows
// [FR*w, +FR).  Which waves share a block does not change any partial's
// arithmetic.
template <int DT, int D, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SummaryCfg<DT, D, MODE>::WAVES_PER_SIMD))) void summary_kernel(
    const void* __restrict__ k, const void* __restrict__ v, int64_t sb,
    int64_t sh, int64_t sn, int H, int64_t N, int P, int Tw,
    const float2* __restrict__ stash, float* __restrict__ part, int BH) {
  using C = SummaryCfg<DT, D, MODE>;
  constexpr int F = C::F, FR = C::FR;
  constexpr int E = D * D + D;
  const int lane = threadIdx.x & 63, wave = wave_index();
  const int g = lane >> 4, m = lane & 15;
  const int64_t wid = (int64_t)blockIdx.x * 4 + wave;  // SPLIT = 1
  const int p = C::SPLIT > 1 ? (int)blockIdx.x : (int)(wid / BH);
  const int half = C::SPLIT > 1 ? wave : 0;
  if (p >= P) return;  // uniform across a SPLIT group (it shares p)
  const int bh = C::SPLIT > 1 ? (int)blockIdx.y : (int)(wid % BH);
  const int64_t b = bh / H, h = bh % H;
  const int64_t t_begin = (int64_t)p * Tw;
  const int64_t t_end = min(N, t_begin + (int64_t)Tw);
  const int64_t head = (b * sb + h * sh) * C::ES;
  // lane m reads key features [F*m + FR*half, +FR) and value features
  // [F*m + FC*half, +FC) of rows R*g + r (the host bounds 32 rows of the
  // token stride to 2^24 bytes, so the lane offsets fit 32 bits)
  const int64_t row_bytes = sn * C::ES;
  const char* kh = (const char*)k + head;
  const char* vh = (const char*)v + head;
  const uint32_t roff = (uint32_t)(C::R * g) * (uint32_t)row_bytes;
  const uint32_t koff = roff + (uint32_t)((F * m + FR * half) * C::ES);
  const uint32_t voff = roff + (uint32_t)((F * m + C::FC * half) * C::ES);
  const float2* tstash = MODE == MODE_BWD ? stash + (int64_t)bh * N : nullptr;

  f32x4 acc[FR][F];
#pragma unroll
  for (int i = 0; i < FR; ++i)
#pragma unroll
    for (int j = 0; j < F; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  float zacc[FR];
#pragma unroll
  for (int i = 0; i < FR; ++i) zacc[i] = 0.f;

  // double-buffered exchange: one barrier per step suffices, because a
  // buffer is rewritten only after the barrier of the step in between
  __shared__ uint32_t xch[2 * C::XW];
  // two register sets in turn: while one step computes, the next one's
  // loads are in flight in the other set (no copies between them)
  SummaryRegs<DT, D, MODE> ra, rb;
  auto load = [&](int64_t t0, SummaryRegs<DT, D, MODE>& x) {
    summary_load<DT, D, MODE>(kh, vh, koff, voff, tstash, row_bytes, t0, g, m, t_end, x);
  };
  int64_t t0 = t_begin;
  load(t0, ra);
  while (true) {
    const int64_t t1 = t0 + C::STEP;
    if (t1 < t_end) load(t1, rb);
    summary_step<DT, D, MODE>(ra, half, lane, xch, acc, zacc);
    if (t1 >= t_end) break;
    const int64_t t2 = t1 + C::STEP;
    if (t2 < t_end) load(t2, ra);
    summary_step<DT, D, MODE>(rb, half, lane, xch + C::XW, acc, zacc);
    if (t2 >= t_end) break;
    t0 = t2;
  }

  // this wave's share of the partial: S tiles in lane order, then z
  float* out = part + ((int64_t)bh * P + p) * E;
#pragma unroll
  for (int il = 0; il < FR; ++il) {
    const int i = FR * half + il;
#pragma unroll
    for (int j = 0; j < F; ++j)
      *(f32x4*)(out + ((i * F + j) * 64 + lane) * 4) = acc[il][j];
  }
#pragma unroll
  for (int il = 0; il < FR; ++il) {
    const float zs = sum_groups(zacc[il]);
    if (g == 0) out[D * D + F * m + FR * half + il] = zs;
  }
}

// ---------------------------------------------------------------------------
// Combine: FP64 sum of the P per-wave partials in a fixed order (so
// results are bitwise reproducible), writing the dense FP64 matrix M
// (S or dS) and vector (z or dz), plus the matrix-core operand images.
// ---------------------------------------------------------------------------
// Partial layouts: PART_SUMMARY (the summary kernel's tiles: tile (i, j),
// lane (g, n), register r holds M[F(4g + r) + i][F n + j], F = d/16) and
// PART_BLOCKS (the fused query backward's: M[16i + 4g + r][16j + n]).
// Block: 64 elements x 4 quarters of the partials; quarter w sums its
// partials in order, and the four quarter sums are added as
// (w0 + w1) + (w2 + w3) -- a fixed order for a given P, so results are
// bitwise reproducible.
template <int D, int LAYOUT>
__global__ __launch_bounds__(256) void combine_kernel(
    const float* __restrict__ part, int P, double* __restrict__ M64,
    double* __restrict__ v64, void* __restrict__ img, int img_dt) {
  constexpr int F = D / 16;
  constexpr int E = D * D + D;
  __shared__ double qs[4][64];
  const int bh = blockIdx.y;
  const int e64 = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int u = blockIdx.x * 64 + e64;
  const int pq = (P + 3) / 4;
  const int p0 = min(P, w * pq), p1 = min(P, p0 + pq);
  double sq = 0.0;
  if (u < E) {
    // in order (the sum's order is fixed), but eight loads at a time in
    // flight rather than one
    const float* src = part + (int64_t)bh * P * E + u;
    int p = p0;
    for (; p + 8 <= p1; p += 8) {
      float x[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) x[k] = src[(int64_t)(p + k) * E];
#pragma unroll
      for (int k = 0; k < 8; ++k) sq += (double)x[k];
    }
    for (; p < p1; ++p) sq += (double)src[(int64_t)p * E];
  }
  qs[w][e64] = sq;
  __syncthreads();
  if (w != 0 || u >= E) return;
  const double s = (qs[0][e64] + qs[1][e64]) + (qs[2][e64] + qs[3][e64]);
  if (u < D * D) {
    const int r = u & 3, lane = (u >> 2) & 63, ij = u >> 8;
    const int i = ij / F, j = ij % F;
    const int g = lane >> 4, n = lane & 15;
    const int c = LAYOUT == PART_SUMMARY ? F * (4 * g + r) + i : 16 * i + 4 * g + r;
    const int e = LAYOUT == PART_SUMMARY ? F * n + j : 16 * j + n;
    M64[(int64_t)bh * D * D + c * D + e] = s;
    write_images<D>(img, img_dt, bh, c, e, s);
  } else {
    v64[(int64_t)bh * D + (u - D * D)] = s;
    write_z_tile<D>(img, img_dt, bh, u - D * D, s);
  }
}

// Images from a dense FP64 matrix and vector (used when S, z come from the
// caller).
template <int D>
__global__ __launch_bounds__(256) void image_kernel(const double* __restrict__ M64,
                                                    const double* __restrict__ v64,
                                                    void* __restrict__ img, int img_dt) {
  const int bh = blockIdx.y;
  const int u = blockIdx.x * 256 + threadIdx.x;
  if (u < D * D) {
    write_images<D>(img, img_dt, bh, u / D, u % D, M64[(int64_t)bh * D * D + u]);
  } else if (u < D * D + D) {
    write_z_tile<D>(img, img_dt, bh, u - D * D, v64[(int64_t)bh * D + (u - D * D)]);
  }
}

// ---------------------------------------------------------------------------
// Apply: O^T = S^T phi(Q)^T per 16-token tile.  The G workgroups of a head
// take the head's blocks of 4 * 16 * TT tokens in turn (workgroup g: blocks
// g, g + G, g + 2G, ...; each wave 16 * TT tokens of a block), so the waves
// of the whole grid move through every tensor together and the accesses in
// flight at any moment lie in a narrow window of it: a copy stream laid
// out this way reached 5.49 TB/s on MI355X against 5.21 TB/s for the same
// copy with one contiguous range per wave.  Lane (g, n) holds token n
// and a run of Q4 = d/4 query features (Run: 16-byte chunks interleaved
// over the lane groups); the matrix-core result puts the value features of
// the same run positions of the same token in the same lane.  The normaliser den = phi(q) . z comes from
// the same matrix-core pass (the image's z tile: every output row of it is
// den of the lane's token), so the FP64 division and the store stay
// in-lane.  The S^T operands (bf16 hi + lo parts, or fp32) sit in LDS for
// the whole workgroup.
// ---------------------------------------------------------------------------
template <int DT, int D>
struct ApplyCfg {
  // 16-token tiles per step; every LDS operand read feeds TT matrix-core
  // ops (fp32 at d = 128: one, for registers)
  static constexpr int TT = DT == DT_FP32 && D >= 128 ? 1 : 2;
  static constexpr int ES = DT == DT_BF16 ? 2 : 4;
  static constexpr int QB = D / 4 * ES;             // bytes of a lane's query run
  static constexpr int QW = QB / 4;
};

//
// MIX: the noise-gated epilogue.  Batch element b's spatial weight
// g_b = sigma_data / (sigma_data + sigma[b]) (FP64, once per workgroup)
// blends this attention with another branch's stored output (same dtype
// and strides as o): o = g_b A + (1 - g_b) other, in FP32 before the
// store.  The other branch's rows travel in the same register sets as the
// queries, a step ahead, where registers allow (bf16 in and out).  `other`
// may be `o` itself: each lane reads its elements before it writes them.
template <int DT, int OT, int D, bool MIX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void apply_kernel(
    const void* __restrict__ q, int64_t sb, int64_t sh, int64_t sn,
    void* o, int64_t osb, int64_t osh, int64_t osn, int H,
    int64_t N, int G, const void* __restrict__ img, const void* other,
    const double* __restrict__ sigma, double sigma_data) {
  using IC = ImageCfg<D>;
  using AC = ApplyCfg<DT, D>;
  constexpr int Q4 = D / 4;
  constexpr int NT = D / 16;
  constexpr int ES = AC::ES;
  constexpr int OES = OT == DT_BF16 ? 2 : 4;
  constexpr int QW = AC::QW;
  constexpr int IMG_WORDS = IC::img_bytes(DT) / 16;
  constexpr int TT = AC::TT;
  __shared__ u32x4 simg[IMG_WORDS];

  const int bh = blockIdx.y;
  const int64_t b = bh / H, h = bh % H;
  const int lane = threadIdx.x & 63, wave = wave_index();
  const int g = lane >> 4, n = lane & 15;

  // wave-uniform head pointers plus loop-invariant 32-bit lane offsets
  // (token n of the tile, lane group g's feature run)
  const int64_t row_bytes = sn * ES, orow_bytes = osn * OES;
  const char* qh = (const char*)q + (b * sb + h * sh) * ES;
  char* oh = (char*)o + (b * osb + h * osh) * OES;
  using RN = Run<D, DT>;
  const uint32_t ooff = (uint32_t)n * (uint32_t)orow_bytes + (uint32_t)(g * RN::CH * OES);

  // the gate: spatial weight gw, the other branch's weight hw
  float gw = 1.f, hw = 0.f;
  const char* xh = nullptr;
  if constexpr (MIX) {
    const double gg = sigma_data / (sigma_data + sigma[b]);
    gw = (float)gg;
    hw = (float)(1.0 - gg);
    xh = (const char*)other + (b * osb + h * osh) * OES;
  }
  constexpr int XW = MIX ? Q4 * OES / 4 : 1;  // words of a lane's run of `other`
  // bf16 in and out: `other` rides in the query register sets, a step
  // ahead; otherwise (registers) it is loaded as its step starts
  constexpr bool XPF = MIX && DT == DT_BF16 && OT == DT_BF16;

  struct QRegs {
    uint32_t q[TT][QW];
    uint32_t x[TT][XPF ? XW : 1];
  };
  auto load_x = [&](int64_t tb, uint32_t* xw) {
    load_out_run<D, DT, OT>(xh + tb * orow_bytes + ooff, xw);
  };
  // Rows past the head's last token read that token again (no zero fill
  // and no branch around the loads); their results are not stored.
  auto load_q = [&](int64_t t0, QRegs& r) {
#pragma unroll
    for (int tt = 0; tt < TT; ++tt) {
      const int64_t tb = min(t0 + 16 * tt, N - 1);  // wave-uniform
      const uint32_t row = (uint32_t)min(n, (int)min((int64_t)15, N - 1 - tb));
      load_run<D, DT>(qh + tb * row_bytes + (row * (uint32_t)row_bytes + (uint32_t)(g * RN::CB)),
                      r.q[tt]);
      if constexpr (XPF)
        load_out_run<D, DT, OT>(
            xh + tb * orow_bytes + (row * (uint32_t)orow_bytes + (uint32_t)(g * RN::CH * OES)),
            r.x[tt]);
    }
  };

  auto compute = [&](int64_t t0, const QRegs& r) {
    const auto& qw = r.q;
    // `other` when not prefetched: loaded as the step starts (bf16 queries)
    // or just before its use (fp32 queries, whose runs fill the registers)
    uint32_t xs[TT][MIX && !XPF ? XW : 1];
    if constexpr (MIX && !XPF && DT == DT_BF16) {
#pragma unroll
      for (int tt = 0; tt < TT; ++tt)
        if (t0 + 16 * tt + n < N) load_x(t0 + 16 * tt, xs[tt]);
    }
    // phi(q) as matrix-core operands; acc[tt][NT] is the z tile (den)
    f32x4 acc[TT][NT + 1];
#pragma unroll
    for (int tt = 0; tt < TT; ++tt)
#pragma unroll
      for (int i = 0; i <= NT; ++i) acc[tt][i] = f32x4{0.f, 0.f, 0.f, 0.f};
    if constexpr (DT == DT_BF16) {
      constexpr int NS = IC::NS;
      bf16x8 bq[TT][NS];
#pragma unroll
      for (int tt = 0; tt < TT; ++tt)
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          u32x4 w;
#pragma unroll
          for (int pp = 0; pp < 4; ++pp) {
            const int c0 = 8 * s + 2 * pp;
            if (c0 < Q4) {
              const float p0 = phi<DT>(word_elem<DT>(qw[tt], c0));
              const float p1 = phi<DT>(word_elem<DT>(qw[tt], c0 + 1));
              w[pp] = pack_bf16(p0, p1);
            } else {
              w[pp] = 0;
            }
          }
          bq[tt][s] = as_bf16x8(w);
        }
#pragma unroll
      for (int i = 0; i <= NT; ++i)
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const bf16x8 hi = as_bf16x8(simg[((i * NS + s) * 2 + 0) * 64 + lane]);
          const bf16x8 lo = as_bf16x8(simg[((i * NS + s) * 2 + 1) * 64 + lane]);
#pragma unroll
          for (int tt = 0; tt < TT; ++tt) {
            // the chain's first product starts from zero (no separate clear)
            acc[tt][i] = mfma_bf16(hi, bq[tt][s], s == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[tt][i]);
            acc[tt][i] = mfma_bf16(lo, bq[tt][s], acc[tt][i]);
          }
          // keep the operand reads next to their use (bounded registers)
          if constexpr (D >= 128) __builtin_amdgcn_sched_barrier(0);
        }
    } else {
      float pq[TT][Q4];
#pragma unroll
      for (int tt = 0; tt < TT; ++tt)
#pragma unroll
        for (int c = 0; c < Q4; ++c) pq[tt][c] = phi<DT>(word_elem<DT>(qw[tt], c));
#pragma unroll
      for (int i = 0; i <= NT; ++i)
#pragma unroll
        for (int s4 = 0; s4 < Q4 / 4; ++s4) {
          const u32x4 a = simg[(i * (Q4 / 4) + s4) * 64 + lane];
#pragma unroll
          for (int t4 = 0; t4 < 4; ++t4)
#pragma unroll
            for (int tt = 0; tt < TT; ++tt)
              acc[tt][i] = mfma_f32(__uint_as_float(a[t4]), pq[tt][4 * s4 + t4],
                                    s4 == 0 && t4 == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[tt][i]);
          if constexpr (D >= 128) __builtin_amdgcn_sched_barrier(0);
        }
    }
#pragma unroll
    for (int tt = 0; tt < TT; ++tt) {
      // O = num / den: FP64 reciprocal, applied as its two-float expansion
      // rh + rl (num * rh + num * rl with one rounding: within an ulp of
      // the FP64 product rounded to fp32)
      const double rden = 1.0 / (double)acc[tt][NT][0];
      const float rh = (float)rden, rl = (float)(rden - (double)rh);
      if (t0 + 16 * tt + n < N) {
        float out[Q4];
#pragma unroll
        for (int i = 0; i < NT; ++i)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            out[4 * i + r] = fmaf(acc[tt][i][r], rh, acc[tt][i][r] * rl);
        if constexpr (MIX) {
          if constexpr (!XPF && DT != DT_BF16) load_x(t0 + 16 * tt, xs[tt]);
#pragma unroll
          for (int c = 0; c < Q4; ++c)
            out[c] = fmaf(gw, out[c], hw * word_elem<OT>(XPF ? r.x[tt] : xs[tt], c));
        }
        store_run<D, DT, OT>(oh + (t0 + 16 * tt) * orow_bytes + ooff, out);
      }
    }
  };

  // two register sets in turn: the next step's queries are in flight in
  // one while the other's step computes (no copies between them).  The
  // loads are unconditional and the loop body has no early exit, so the
  // compiler's wait counts cover only the set a step is about to use (an
  // odd step count runs one step with nothing to store); the scheduling
  // barriers keep each load ahead of the step that overlaps it.
  constexpr int BLK = 16 * TT * 4;  // tokens per block
  const int64_t nblk = (N + BLK - 1) / BLK;
  const int64_t blk0 = blockIdx.x;
  const int nk = blk0 < nblk ? (int)((nblk - 1 - blk0) / G + 1) : 0;
  // first token of this wave's part of the k-th block it takes
  auto tok = [&](int k) { return (blk0 + (int64_t)k * G) * BLK + 16 * TT * wave; };
  // the first queries are in flight while the workgroup stages the T image
  // (the first of the head's two, S^T operands) into LDS
  QRegs qa, qb;
  if (nk > 0) load_q(tok(0), qa);
  {
    const u32x4* src = (const u32x4*)((const char*)img + (int64_t)bh * IC::head_bytes(DT));
    for (int w = threadIdx.x; w < IMG_WORDS; w += 256) simg[w] = src[w];
  }
  __syncthreads();
  if (nk > 0) {
    for (int k = 0; k < nk; k += 2) {
      load_q(tok(k + 1), qb);
      __builtin_amdgcn_sched_barrier(0);
      compute(tok(k), qa);
      load_q(tok(k + 2), qa);
      __builtin_amdgcn_sched_barrier(0);
      compute(tok(k + 1), qb);
    }
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
template <int DT, int D, int MODE>
static void launch_summary_t(const void* k, const void* v, int64_t sb, int64_t sh, int64_t sn,
                             int64_t BH, int64_t H, int64_t N, int P, int Tw,
                             const float2* stash, float* part, hipStream_t stream) {
  using C = SummaryCfg<DT, D, MODE>;
  // block geometry comes from the kernel's own configuration: SPLIT waves
  // share one partial, or four waves take one partial each
  static_assert(C::THREADS == 64 * (C::SPLIT > 1 ? C::SPLIT : 4), "block shape");
  static_assert(C::SPLIT == 1 || C::PPB == 1, "split blocks hold one partial");
  const dim3 grid = C::SPLIT > 1 ? dim3((unsigned)P, (unsigned)BH)
                                 : dim3((unsigned)((P * BH + 3) / 4));
  summary_kernel<DT, D, MODE><<<grid, C::THREADS, 0, stream>>>(k, v, sb, sh, sn, (int)H, N, P, Tw,
                                                               stash, part, (int)BH);
}

template <int D>
static void launch_summary_d(int mode, int dt, const void* k, const void* v, int64_t sb,
                             int64_t sh, int64_t sn, int64_t B, int64_t H, int64_t N, int P,
                             int Tw, const float2* stash, float* part, hipStream_t stream) {
  ProfScope prof(mode == MODE_FWD ? "summary_fwd" : "summary_bwd", stream);
  const int64_t BH = B * H;
#define LA_SUM(DTI, M) \
  launch_summary_t<DTI, D, M>(k, v, sb, sh, sn, BH, H, N, P, Tw, stash, part, stream)
  if (mode == MODE_FWD) {
    if (dt == DT_BF16) LA_SUM(DT_BF16, MODE_FWD); else LA_SUM(DT_FP32, MODE_FWD);
  } else {
    if (dt == DT_BF16) LA_SUM(DT_BF16, MODE_BWD); else LA_SUM(DT_FP32, MODE_BWD);
  }
#undef LA_SUM
}

hipError_t launch_summary(int mode, int dt, int D, const void* k, const void* v, int64_t sb,
                          int64_t sh, int64_t sn, int64_t B, int64_t H, int64_t N, int P,
                          int Tw, const float2* stash, float* part, hipStream_t stream) {
  switch (D) {
    case 16: launch_summary_d<16>(mode, dt, k, v, sb, sh, sn, B, H, N, P, Tw, stash, part, stream); break;
    case 32: launch_summary_d<32>(mode, dt, k, v, sb, sh, sn, B, H, N, P, Tw, stash, part, stream); break;
    case 64: launch_summary_d<64>(mode, dt, k, v, sb, sh, sn, B, H, N, P, Tw, stash, part, stream); break;
    case 128: launch_summary_d<128>(mode, dt, k, v, sb, sh, sn, B, H, N, P, Tw, stash, part, stream); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int D>
static void launch_combine_d(const float* part, int P, double* M64, double* v64, void* img,
                             int img_dt, int64_t BH, int layout, hipStream_t stream) {
  dim3 grid((D * D + D + 63) / 64, (unsigned)BH);
  if (layout == PART_SUMMARY)
    combine_kernel<D, PART_SUMMARY><<<grid, 256, 0, stream>>>(part, P, M64, v64, img, img_dt);
  else
    combine_kernel<D, PART_BLOCKS><<<grid, 256, 0, stream>>>(part, P, M64, v64, img, img_dt);
}

hipError_t launch_combine(const float* part, int P, double* M64, double* v64, void* img,
                          int img_dt, int64_t BH, int D, int layout, hipStream_t stream) {
  ProfScope prof("combine", stream);
  switch (D) {
    case 16: launch_combine_d<16>(part, P, M64, v64, img, img_dt, BH, layout, stream); break;
    case 32: launch_combine_d<32>(part, P, M64, v64, img, img_dt, BH, layout, stream); break;
    case 64: launch_combine_d<64>(part, P, M64, v64, img, img_dt, BH, layout, stream); break;
    case 128: launch_combine_d<128>(part, P, M64, v64, img, img_dt, BH, layout, stream); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int D>
static hipError_t launch_apply_only(const FwdArgs& a);

template <int D>
static hipError_t launch_forward_d(const FwdArgs& a) {
  const int BH = (int)(a.B * a.H);
  launch_summary_d<D>(MODE_FWD, a.in_dt, a.k, a.v, a.sb, a.sh, a.sn, a.B, a.H, a.N, a.P, a.Tw,
                      nullptr, a.part, a.stream);
  {
    dim3 cgrid((D * D + D + 63) / 64, BH);
    ProfScope prof("combine", a.stream);
    combine_kernel<D, PART_SUMMARY><<<cgrid, 256, 0, a.stream>>>(a.part, a.P, a.S64, a.z64, a.img,
                                                                 a.in_dt);
  }
  return launch_apply_only<D>(a);
}

template <int D>
static hipError_t launch_apply_only(const FwdArgs& a) {
  const int BH = (int)(a.B * a.H);
  dim3 agrid((unsigned)a.Ga, BH);
  ProfScope prof(a.other ? "apply_gated" : "apply", a.stream);
#define LA_APPLY(DTI, DTO, MIX)                                                   \
  apply_kernel<DTI, DTO, D, MIX><<<agrid, 256, 0, a.stream>>>(                     \
      a.q, a.sb, a.sh, a.sn, a.o, a.osb, a.osh, a.osn, (int)a.H, a.N, a.Ga, a.img, a.other, \
      a.sigma, a.sigma_data)
#define LA_APPLY_DT(MIX)                                                \
  if (a.in_dt == DT_BF16 && a.out_dt == DT_BF16) LA_APPLY(DT_BF16, DT_BF16, MIX); \
  else if (a.in_dt == DT_BF16) LA_APPLY(DT_BF16, DT_FP32, MIX);                   \
  else if (a.out_dt == DT_BF16) LA_APPLY(DT_FP32, DT_BF16, MIX);                  \
  else LA_APPLY(DT_FP32, DT_FP32, MIX);
  if (a.other) {
    LA_APPLY_DT(true)
  } else {
    LA_APPLY_DT(false)
  }
#undef LA_APPLY_DT
#undef LA_APPLY
  return hipGetLastError();
}

hipError_t launch_forward(const FwdArgs& a) {
  switch (a.D) {
    case 16: return launch_forward_d<16>(a);
    case 32: return launch_forward_d<32>(a);
    case 64: return launch_forward_d<64>(a);
    case 128: return launch_forward_d<128>(a);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_apply(const FwdArgs& a) {
  hipError_t e = launch_images(a.S64, a.z64, a.img, a.in_dt, a.B * a.H, a.D, a.stream);
  if (e != hipSuccess) return e;
  switch (a.D) {
    case 16: return launch_apply_only<16>(a);
    case 32: return launch_apply_only<32>(a);
    case 64: return launch_apply_only<64>(a);
    case 128: return launch_apply_only<128>(a);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_images(const double* M64, const double* v64, void* img, int img_dt, int64_t BH,
                         int D, hipStream_t stream) {
  dim3 grid((D * D + D + 255) / 256, (unsigned)BH);
  ProfScope prof("images", stream);
  switch (D) {
    case 16: image_kernel<16><<<grid, 256, 0, stream>>>(M64, v64, img, img_dt); break;
    case 32: image_kernel<32><<<grid, 256, 0, stream>>>(M64, v64, img, img_dt); break;
    case 64: image_kernel<64><<<grid, 256, 0, stream>>>(M64, v64, img, img_dt); break;
    case 128: image_kernel<128><<<grid, 256, 0, stream>>>(M64, v64, img, img_dt); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace la
