// la_tiled.hip -- the paper's tiled global-attention step in two passes
// over the token fields (la_tiled_forward in include/la.h).
//
// Sec. III-C: the spatiotemporal token grid is cut into tiles, each
// extended by halos that overlap its neighbours; every tile is processed on
// its own; the outputs are averaged where tiles overlap, each contribution
// weighted by a Hann window.  With kernelised attention inside each tile,
// a tile's attention is its summary (S_t, z_t) over its extended, border-
// clamped token set, applied to the queries of the tile, so
//     out(p) = sum_t w_t(p) O_t(p) / sum_t w_t(p),
//     O_t(p) = phi(q_p)^T S_t / (phi(q_p) . z_t),
// over the tiles t covering grid position p.  Nothing per tile is stored
// but (S_t, z_t):
//  1. tile summaries: each tile's extended token set is read from the K
//     and V fields in place (clamped coordinates, as tile extraction does)
//     by one workgroup per (tile, head), summed by the summary machinery
//     (four FP32 partials of at most 16,384 tokens), the partials added in
//     FP64 in a fixed order, and the result written as the apply's operands
//     (S_t^T hi parts, z_t hi + lo);
//  2. apply and blend: the grid is cut into cells between tile centres,
//     whose positions are covered by at most two tiles per dimension (when
//     every halo is at most half its core), so a workgroup stages the
//     images of the <= 8 covering tiles of its cell once and, for each
//     query of the cell, forms every covering tile's O_t(p) on the matrix
//     cores and the Hann-weighted average in registers: Q is read once and
//     the output written once, with no tile of any tensor in memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "../../include/la.h"
#include "la_kernels.h"
#include "la_profile.h"
#include "la_summary.h"

namespace la {
namespace {

struct TGeo {
  int64_t dims[3], core[3], halo[3], L[3], n[3];
  int64_t cells[3];  // cells per dimension: n + 1
  int64_t C;         // channels: heads * d
  int64_t H, d;
  int64_t tile_tokens, n_tiles, n_cells;
  int P, Tw;         // partials per (tile, head), tokens per partial
};

__device__ __forceinline__ uint32_t clamp32(int32_t v, int32_t hi) {
  return (uint32_t)min(max(v, 0), hi);
}

// Hann weight of coordinate u of a tile extent L (cell centres, strictly
// positive on [0, L)): sin^2(pi (u + 1/2) / L); zero outside the tile.
// w(u) = sin^2(pi (u + 1/2) / L) for 0 <= u < L, else 0; inv2L = 1 / (2L).
// The hardware sine takes its argument in revolutions (sin(2 pi x)); its
// error (about 1e-6) is far below the bf16 rounding of the blended output.
__device__ __forceinline__ float hann_w(int32_t u, int32_t L, float inv2L) {
  const float s = __builtin_amdgcn_sinf(((float)u + 0.5f) * inv2L);
  return (u >= 0 && u < L) ? s * s : 0.f;
}

// Operands of one (tile, head) for the apply pass, in the matrix cores'
// lane order (ImageCfg's T image): S^T as bf16 hi parts (NT output tiles x
// NS k-steps x 64 lanes of 16 bytes), then the z tile as hi and lo parts.
template <int D>
struct TiledCfg {
  using IC = ImageCfg<D>;
  static constexpr int NT = D / 16, NS = IC::NS, Q4 = D / 4;
  static constexpr int S_WORDS = NT * NS * 64;  // S^T hi parts
  // z tile: one operand per k-step whose even rows hold z's bf16 hi parts
  // and odd rows its lo parts, so output rows 4g and 4g + 1 of a product
  // are the hi and lo parts of den in the same lane
  static constexpr int Z_WORDS = NS * 64;
  static constexpr int SLOT = S_WORDS + Z_WORDS;
  // four waves per apply workgroup: two workgroups share a compute unit
  // (the eight slots take 80 KiB of LDS at d = 64), so one's staging
  // overlaps the other's streaming (3.75 -> 3.29 ms against eight waves)
  static constexpr int WAVES = 4, TT = 2;
  static constexpr int QW = Q4 * 2 / 4;         // words of a lane's query run
};

// ---------------------------------------------------------------------------
// Pass 1: per (tile, head), the summary over the tile's extended token set
// [ut][uy][ux] (row-major), coordinates clamped into the grid.  One
// workgroup per (tile, head); wave w sums tokens [w*Tw, w*Tw + Tw) in FP32
// (Tw <= 16,384), the four partials are added in FP64 in a fixed order
// through LDS, and the result is written as the apply's operand slot.
// grid: one workgroup per (tile, head), head fastest: the H workgroups of
// a tile run side by side and together read whole token rows (each reads
// only its head's d features of a row).
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void tile_summary_kernel(TGeo g, const void* __restrict__ k, const void* __restrict__ v,
                         u32x4* __restrict__ slots) {
  using C = SummaryCfg<DT_BF16, D, MODE_FWD>;
  using TC = TiledCfg<D>;
  using RB = Run<D, DT_BF16>;
  static_assert(C::SPLIT == 1, "one wave per partial");
  constexpr int F = C::F, FR = C::FR, R = C::R, STEP = C::STEP;
  constexpr int E = D * D + D;
  __shared__ __align__(16) float red[4][E];
  const int lane = threadIdx.x & 63, wave = wave_index();
  const int gq = lane >> 4, m = lane & 15;
  const int64_t tile = blockIdx.x / g.H;
  const int p = wave;
  const int64_t head = blockIdx.x % g.H;
  const int64_t t_begin = (int64_t)p * g.Tw;
  const int64_t t_end = min(g.tile_tokens, t_begin + (int64_t)g.Tw);
  float* out = red[p];
  // the tile's origin in the grid (core start minus halo)
  const int64_t a = tile / (g.n[1] * g.n[2]), b = (tile / g.n[2]) % g.n[1], c = tile % g.n[2];
  const int64_t o0 = a * g.core[0] - g.halo[0], o1 = b * g.core[1] - g.halo[1],
                o2 = c * g.core[2] - g.halo[2];
  const int64_t rowb = g.C * 2;  // bytes per token of a field
  const char* kb = (const char*)k + head * D * 2 + (int64_t)(F * m) * 2;
  const char* vb = (const char*)v + head * D * 2 + (int64_t)(F * m) * 2;
  f32x4 acc[FR][F];
  float zacc[FR];
#pragma unroll
  for (int i = 0; i < FR; ++i) {
    zacc[i] = 0.f;
#pragma unroll
    for (int j = 0; j < F; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  if (t_begin < t_end) {
    const uint32_t neg_inf = 0xff80ff80u;
    uint32_t* xch = nullptr;
    // the step at t0: lane group gq takes tokens t0 + R*gq + r; decompose
    // the first one, then walk in (ut, uy, ux) order.  32-bit throughout
    // (an extended tile holds at most 65,536 tokens, the field fewer than
    // 2^31), so the walk costs a few instructions per token
    const uint32_t L1 = (uint32_t)g.L[1], L2 = (uint32_t)g.L[2], L12 = L1 * L2;
    const int32_t O0 = (int32_t)o0, O1 = (int32_t)o1, O2 = (int32_t)o2;
    const int32_t M0 = (int32_t)g.dims[0] - 1, M1 = (int32_t)g.dims[1] - 1,
                  M2 = (int32_t)g.dims[2] - 1;
    const uint32_t N1 = (uint32_t)g.dims[1], N2 = (uint32_t)g.dims[2];
    const uint32_t tend = (uint32_t)t_end;
    auto load = [&](int64_t t0, SummaryRegs<DT_BF16, D, MODE_FWD>& x) {
      const uint32_t j = (uint32_t)t0 + R * gq;
      uint32_t ut = j / L12;
      const uint32_t rem = j - ut * L12;
      uint32_t uy = rem / L2;
      uint32_t ux = rem - uy * L2;
      // a whole step in range (all but a partial's last): no row checks
      const bool full = (uint32_t)t0 + STEP <= tend;  // wave-uniform
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (full || j + r < tend) {
          const uint32_t gt = clamp32(O0 + (int32_t)ut, M0);
          const uint32_t gy = clamp32(O1 + (int32_t)uy, M1);
          const uint32_t gx = clamp32(O2 + (int32_t)ux, M2);
          const int64_t off = (int64_t)((gt * N1 + gy) * N2 + gx) * rowb;
          // plain loads: halo tokens are read again by the neighbouring
          // tiles, dispatched at about the same time
          load_words<C::KB>(kb + off, x.kw[r]);
          load_words<C::VB>(vb + off, x.vw[r]);
        } else {
#pragma unroll
          for (int w = 0; w < C::KW; ++w) x.kw[r][w] = neg_inf;
#pragma unroll
          for (int w = 0; w < C::VW; ++w) x.vw[r][w] = 0;
        }
        if (++ux == L2) {
          ux = 0;
          if (++uy == L1) {
            uy = 0;
            ++ut;
          }
        }
      }
    };
    // two register sets in turn: the next step's loads are in flight while
    // the current one computes
    SummaryRegs<DT_BF16, D, MODE_FWD> ra, rb;
    int64_t t0 = t_begin;
    load(t0, ra);
    while (true) {
      const int64_t t1 = t0 + STEP;
      if (t1 < t_end) load(t1, rb);
      summary_step<DT_BF16, D, MODE_FWD>(ra, 0, lane, xch, acc, zacc);
      if (t1 >= t_end) break;
      const int64_t t2 = t1 + STEP;
      if (t2 < t_end) load(t2, ra);
      summary_step<DT_BF16, D, MODE_FWD>(rb, 0, lane, xch, acc, zacc);
      if (t2 >= t_end) break;
      t0 = t2;
    }
  }
#pragma unroll
  for (int i = 0; i < FR; ++i)
#pragma unroll
    for (int j = 0; j < F; ++j) *(f32x4*)(out + ((i * F + j) * 64 + lane) * 4) = acc[i][j];
#pragma unroll
  for (int i = 0; i < FR; ++i) {
    const float zs = sum_groups(zacc[i]);
    if (gq == 0) out[D * D + F * m + i] = zs;
  }
  __syncthreads();
  // FP64 sum of the four partials, (p0 + p1) + (p2 + p3), element u of the
  // partial layout (tile (i, j), lane (g, n), register r: S[F(4g + r) + i][F n + j];
  // then z), into the operand slot: S^T hi parts at (row e, contraction c),
  // z's hi parts in the even rows of the z tile and its lo parts in the odd
  uint16_t* slot = (uint16_t*)(slots + (tile * g.H + head) * TC::SLOT);
  for (int u = threadIdx.x; u < E; u += 256) {
    const double sum = ((double)red[0][u] + (double)red[1][u]) + ((double)red[2][u] + (double)red[3][u]);
    const uint16_t hi = to_bf16((float)sum);
    if (u < D * D) {
      const int r = u & 3, ln = (u >> 2) & 63, ij = u >> 8;
      const int i = ij / F, j = ij % F;
      const int c = F * (4 * (ln >> 4) + r) + i, e = F * (ln & 15) + j;
      // T image: A[row = value feature e][k = key feature c]
      const int rp = RB::pos(e), kp = RB::pos(c);
      const int word = ((rp >> 2) * TC::NS + (kp >> 3)) * 64 + 16 * RB::group(c) + 4 * RB::group(e) + (rp & 3);
      slot[word * 8 + (kp & 7)] = hi;
      if (TC::Q4 < 8) slot[word * 8 + (kp & 7) + 4] = 0;  // d = 16: padding of the k-step
    } else {
      const int c = u - D * D;
      const uint16_t lo = to_bf16((float)(sum - (double)bf16f(hi)));
      const int kp = RB::pos(c);
      for (int mm = 0; mm < 16; ++mm) {
        const int word = TC::S_WORDS + (kp >> 3) * 64 + 16 * RB::group(c) + mm;
        slot[word * 8 + (kp & 7)] = (mm & 1) ? lo : hi;
        if (TC::Q4 < 8) slot[word * 8 + (kp & 7) + 4] = 0;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Pass 2: apply and blend, one workgroup per (cell, head).  Cell j of a
// dimension covers [j*core - a, j*core - a + core) of the grid, a =
// core / 2; its positions are covered only by tiles j - 1 and j of that
// dimension (halo <= core / 2).  Slot s = (st, sy, sx) in {0, 1}^3 holds
// tile (jt - 1 + st, jy - 1 + sy, jx - 1 + sx) if it exists: the S^T hi
// parts (S_t to about 2^-9) and the hi / lo z tile.  Eight waves take the
// cell's 16-token tiles (row-major over the cell) two at a time.  The
// eight slots take 80 KiB of LDS at d = 64, so two workgroups share a
// compute unit and one's staging overlaps the other's streaming.
// ---------------------------------------------------------------------------

template <int D>
__global__ __launch_bounds__(64 * TiledCfg<D>::WAVES) __attribute__((amdgpu_waves_per_eu(2)))
void tile_apply_kernel(TGeo g, const void* __restrict__ q, void* __restrict__ o,
                       const void* __restrict__ img) {
  using TC = TiledCfg<D>;
  using IC = ImageCfg<D>;
  using RN = Run<D, DT_BF16>;
  constexpr int NT = TC::NT, NS = TC::NS, Q4 = TC::Q4, TT = TC::TT, QW = TC::QW;
  __shared__ u32x4 simg[8 * TC::SLOT];

  // one workgroup per (cell, head), head fastest (as the summary pass)
  const int64_t head = blockIdx.x % g.H;
  const int64_t cell = blockIdx.x / g.H;
  const int64_t jc[3] = {cell / (g.cells[1] * g.cells[2]), (cell / g.cells[2]) % g.cells[1],
                         cell % g.cells[2]};
  int64_t lo[3], ext[3];
  for (int k = 0; k < 3; ++k) {
    const int64_t a = g.core[k] / 2;
    const int64_t s0 = jc[k] * g.core[k] - a;
    lo[k] = max(s0, (int64_t)0);
    ext[k] = min(s0 + g.core[k], g.dims[k]) - lo[k];
  }
  if (ext[0] <= 0 || ext[1] <= 0 || ext[2] <= 0) return;  // uniform over the workgroup
  const int64_t vol = ext[0] * ext[1] * ext[2];

  const int lane = threadIdx.x & 63, wave = wave_index();
  const int gl = lane >> 4, n = lane & 15;
  const int64_t rowb = g.C * 2;
  const char* qh = (const char*)q + head * D * 2;
  char* oh = (char*)o + head * D * 2;

  // per lane: token e of the cell -> grid position, field offset and the
  // Hann weights of the (up to) two covering tiles per dimension.  32-bit
  // coordinates (a cell holds fewer than 65,536 tokens, the field fewer
  // than 2^31); the covering tiles' origins are the same for the whole
  // workgroup (origin -1 << 30 marks a tile outside the grid: weight 0)
  struct Tok {
    int64_t off;
    float wt[2], wy[2], wx[2];
    bool ok;
  };
  const uint32_t E1 = (uint32_t)ext[1], E2 = (uint32_t)ext[2], E12 = E1 * E2;
  const uint32_t VOL = (uint32_t)vol;
  const int32_t P0 = (int32_t)lo[0], P1 = (int32_t)lo[1], P2 = (int32_t)lo[2];
  const uint32_t N1 = (uint32_t)g.dims[1], N2 = (uint32_t)g.dims[2];
  int32_t org[3][2], Lk[3];
  float inv2L[3];
  for (int k = 0; k < 3; ++k) {
    Lk[k] = (int32_t)g.L[k];
    inv2L[k] = 0.5f / (float)g.L[k];
    for (int sidx = 0; sidx < 2; ++sidx) {
      const int64_t tix = jc[k] - 1 + sidx;
      org[k][sidx] = (tix >= 0 && tix < g.n[k]) ? (int32_t)(tix * g.core[k] - g.halo[k]) : -(1 << 30);
    }
  }
  auto locate = [&](int64_t e64) {
    Tok t;
    const uint32_t e = (uint32_t)e64;
    t.ok = e64 < (int64_t)VOL;
    const uint32_t ee = t.ok ? e : VOL - 1;
    const uint32_t a0 = ee / E12, r0 = ee - a0 * E12;
    const uint32_t a1 = r0 / E2, a2 = r0 - a1 * E2;
    const int32_t p[3] = {P0 + (int32_t)a0, P1 + (int32_t)a1, P2 + (int32_t)a2};
    t.off = (int64_t)(((uint32_t)p[0] * N1 + (uint32_t)p[1]) * N2 + (uint32_t)p[2]) * rowb;
    float* w[3] = {t.wt, t.wy, t.wx};
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int sidx = 0; sidx < 2; ++sidx) w[k][sidx] = hann_w(p[k] - org[k][sidx], Lk[k], inv2L[k]);
    return t;
  };

  const int64_t ntile = (vol + 15) / 16;
  const int64_t per_step = (int64_t)TC::WAVES * TT;
  // two register sets in turn: a step's queries are loaded while the
  // previous step computes
  struct Step {
    Tok tk[TT];
    uint32_t qw[TT][QW];
  };
  auto fetch = [&](int64_t base, Step& x) {
#pragma unroll
    for (int u = 0; u < TT; ++u) {
      x.tk[u] = locate((base + u) * 16 + n);
      load_run<D, DT_BF16>(qh + x.tk[u].off + gl * RN::CB, x.qw[u]);
    }
  };
  Step sa, sb;
  const int64_t base0 = (int64_t)wave * TT;
  if (base0 < ntile) fetch(base0, sa);

  // stage the covering tiles' operands (the first queries are in flight):
  // every load of a thread is issued before its LDS stores (in two rounds
  // of loads, then stores, to bound the registers held)
  {
    constexpr int NTH = 64 * TC::WAVES;
    constexpr int PER = (8 * TC::SLOT + NTH - 1) / NTH;  // words per thread
    constexpr int HALF = (PER + 1) / 2;
#pragma unroll
    for (int r0 = 0; r0 < PER; r0 += HALF) {
      u32x4 buf[HALF];
#pragma unroll
      for (int i = 0; i < HALF; ++i) {
        const int w = threadIdx.x + NTH * (r0 + i);
        const int s = w / TC::SLOT, ws = w % TC::SLOT;
        const int64_t tt = jc[0] - 1 + (s >> 2), ty = jc[1] - 1 + ((s >> 1) & 1), tx = jc[2] - 1 + (s & 1);
        const bool ok = r0 + i < PER && w < 8 * TC::SLOT && tt >= 0 && tt < g.n[0] && ty >= 0 &&
                        ty < g.n[1] && tx >= 0 && tx < g.n[2];
        if (ok) buf[i] = ((const u32x4*)img)[(((tt * g.n[1] + ty) * g.n[2] + tx) * g.H + head) * TC::SLOT + ws];
      }
#pragma unroll
      for (int i = 0; i < HALF; ++i) {
        const int w = threadIdx.x + NTH * (r0 + i);
        if (r0 + i < PER && w < 8 * TC::SLOT) simg[w] = buf[i];  // slots of missing tiles are never read
      }
    }
  }
  // the slots whose tile exists (the same for every thread)
  int vmask = 0;
  for (int s = 0; s < 8; ++s) {
    const int64_t tt = jc[0] - 1 + (s >> 2), ty = jc[1] - 1 + ((s >> 1) & 1), tx = jc[2] - 1 + (s & 1);
    if (tt >= 0 && tt < g.n[0] && ty >= 0 && ty < g.n[1] && tx >= 0 && tx < g.n[2]) vmask |= 1 << s;
  }
  __syncthreads();

  auto compute = [&](const Step& x) {
    // phi(q) as matrix-core operands
    bf16x8 bq[TT][NS];
#pragma unroll
    for (int u = 0; u < TT; ++u)
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        u32x4 w;
#pragma unroll
        for (int pp = 0; pp < 4; ++pp) {
          const int c0 = 8 * s + 2 * pp;
          w[pp] = c0 < Q4 ? pack_bf16(phi<DT_BF16>(word_elem<DT_BF16>(x.qw[u], c0)),
                                      phi<DT_BF16>(word_elem<DT_BF16>(x.qw[u], c0 + 1)))
                          : 0u;
        }
        bq[u][s] = as_bf16x8(w);
      }
    float oacc[TT][Q4], wacc[TT];
#pragma unroll
    for (int u = 0; u < TT; ++u) {
      wacc[u] = 0.f;
#pragma unroll
      for (int c = 0; c < Q4; ++c) oacc[u][c] = 0.f;
    }
    for (int s = 0; s < 8; ++s) {
      if (!((vmask >> s) & 1)) continue;
      float ws[TT];
      bool any = false;
#pragma unroll
      for (int u = 0; u < TT; ++u) {
        ws[u] = x.tk[u].ok ? x.tk[u].wt[s >> 2] * x.tk[u].wy[(s >> 1) & 1] * x.tk[u].wx[s & 1] : 0.f;
        any |= ws[u] > 0.f;
      }
      if (!__any(any)) continue;  // no token of these tiles in this slot's tile
      const u32x4* sl = simg + s * TC::SLOT;
      const u32x4* zt = sl + TC::S_WORDS;
      f32x4 acc[TT][NT + 1];
#pragma unroll
      for (int i = 0; i < NT; ++i)
#pragma unroll
        for (int ks = 0; ks < NS; ++ks) {
          const bf16x8 a = as_bf16x8(sl[(i * NS + ks) * 64 + lane]);
#pragma unroll
          for (int u = 0; u < TT; ++u)
            acc[u][i] = mfma_bf16(a, bq[u][ks], ks == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[u][i]);
        }
#pragma unroll
      for (int ks = 0; ks < NS; ++ks) {
        const bf16x8 z2 = as_bf16x8(zt[ks * 64 + lane]);
#pragma unroll
        for (int u = 0; u < TT; ++u)
          acc[u][NT] = mfma_bf16(z2, bq[u][ks], ks == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[u][NT]);
      }
#pragma unroll
      for (int u = 0; u < TT; ++u) {
        // this tile's O_t(p) = num / den (den: rows 4g and 4g + 1, the
        // products with z's hi and lo parts), weighted; the hardware
        // reciprocal (1 ulp) is far below the bf16 rounding of the output
        const float r = ws[u] * __builtin_amdgcn_rcpf(acc[u][NT][0] + acc[u][NT][1]);
#pragma unroll
        for (int i = 0; i < NT; ++i)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) oacc[u][4 * i + rr] = fmaf(acc[u][i][rr], r, oacc[u][4 * i + rr]);
        wacc[u] += ws[u];
      }
    }
#pragma unroll
    for (int u = 0; u < TT; ++u) {
      if (!x.tk[u].ok) continue;
      const float rw = __builtin_amdgcn_rcpf(wacc[u]);
      float out[Q4];
#pragma unroll
      for (int c = 0; c < Q4; ++c) out[c] = oacc[u][c] * rw;
      store_run<D, DT_BF16, DT_BF16>(oh + x.tk[u].off + gl * RN::CH * 2, out);
    }
  };

  for (int64_t base = base0; base < ntile; base += 2 * per_step) {
    if (base + per_step < ntile) fetch(base + per_step, sb);
    compute(sa);
    if (base + per_step >= ntile) break;
    if (base + 2 * per_step < ntile) fetch(base + 2 * per_step, sa);
    compute(sb);
  }
}

la_status make_tgeo(const la_tile_desc* td, int64_t heads, TGeo* g) {
  if (!td || heads < 1) return LA_ERR_INVALID_ARG;
  if (td->dtype != LA_BF16 && td->dtype != LA_FP32) return LA_ERR_INVALID_ARG;
  if (td->C < 8 || td->C % 8 || td->C % heads) return LA_ERR_INVALID_ARG;
  g->C = td->C;
  g->H = heads;
  g->d = td->C / heads;
  int64_t tiles = 1, tok = 1, cells = 1;
  for (int k = 0; k < 3; ++k) {
    if (td->dims[k] < 1 || td->core[k] < 1 || td->halo[k] < 0 || td->halo[k] > td->core[k])
      return LA_ERR_INVALID_ARG;
    g->dims[k] = td->dims[k];
    g->core[k] = td->core[k];
    g->halo[k] = td->halo[k];
    g->L[k] = td->core[k] + 2 * td->halo[k];
    g->n[k] = (td->dims[k] + td->core[k] - 1) / td->core[k];
    g->cells[k] = g->n[k] + 1;
    tiles *= g->n[k];
    tok *= g->L[k];
    cells *= g->cells[k];
  }
  if (td->dtype != LA_BF16) return LA_ERR_UNSUPPORTED;
  if (g->d != 16 && g->d != 32 && g->d != 64) return LA_ERR_UNSUPPORTED;
  for (int k = 0; k < 3; ++k)
    if (2 * g->halo[k] > g->core[k]) return LA_ERR_UNSUPPORTED;  // cells need <= 2 tiles per dim
  const int64_t field = td->dims[0] * td->dims[1] * td->dims[2];
  // 32-bit token coordinates in the kernels; flat grids (cells >= tiles)
  if (heads > 65535 || tok > 65536 || field >= (int64_t(1) << 31) ||
      cells * heads >= (int64_t(1) << 31))
    return LA_ERR_UNSUPPORTED;
  g->tile_tokens = tok;
  g->n_tiles = tiles;
  g->n_cells = cells;
  // four FP32 partials per (tile, head), each of at most 16,384 tokens
  const int64_t Tw = ((tok + 3) / 4 + 31) / 32 * 32;
  if (Tw > 16384) return LA_ERR_UNSUPPORTED;
  g->P = 4;
  g->Tw = (int)Tw;
  return LA_OK;
}

struct TLayout {
  size_t img, total;
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

size_t slot_bytes(int64_t D) {
  switch (D) {
    case 16: return TiledCfg<16>::SLOT * 16;
    case 32: return TiledCfg<32>::SLOT * 16;
    default: return TiledCfg<64>::SLOT * 16;
  }
}

// the workspace holds one operand slot per (tile, head)
TLayout tlayout(const TGeo& g) {
  TLayout L{};
  L.img = 0;
  L.total = align256((size_t)g.n_tiles * g.H * slot_bytes(g.d));
  return L;
}

template <int D>
hipError_t launch_tiled(const TGeo& g, const TLayout& L, const void* q, const void* k,
                        const void* v, void* o, char* ws, hipStream_t st) {
  {
    ProfScope prof("tile_summary", st);
    hipLaunchKernelGGL(tile_summary_kernel<D>, dim3((unsigned)(g.n_tiles * g.H)), dim3(256), 0, st,
                       g, k, v, (u32x4*)(ws + L.img));
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  {
    ProfScope prof("tile_apply", st);
    hipLaunchKernelGGL(tile_apply_kernel<D>, dim3((unsigned)(g.n_cells * g.H)),
                       dim3(64 * TiledCfg<D>::WAVES), 0, st,
                       g, q, o, (const void*)(ws + L.img));
  }
  return hipGetLastError();
}

}  // namespace
}  // namespace la

extern "C" {

la_status la_tiled_workspace_size(const la_tile_desc* desc, int64_t heads, size_t* bytes) {
  if (!bytes) return LA_ERR_INVALID_ARG;
  la::TGeo g;
  const la_status st = la::make_tgeo(desc, heads, &g);
  if (st != LA_OK) return st;
  *bytes = la::tlayout(g).total;
  return LA_OK;
}

la_status la_tiled_forward(const la_tile_desc* desc, int64_t heads, const void* q, const void* k,
                           const void* v, void* o, void* ws, size_t ws_bytes, la_stream stream) {
  la::TGeo g;
  la_status st = la::make_tgeo(desc, heads, &g);
  if (st != LA_OK) return st;
  for (const void* p : {q, k, v, (const void*)o})
    if (!p || ((uintptr_t)p & 15u)) return LA_ERR_INVALID_ARG;
  if (!ws || ((uintptr_t)ws & 255u)) return LA_ERR_INVALID_ARG;
  const la::TLayout L = la::tlayout(g);
  if (ws_bytes < L.total) return LA_ERR_OOM;
  const hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  switch (g.d) {
    case 16: e = la::launch_tiled<16>(g, L, q, k, v, o, (char*)ws, s); break;
    case 32: e = la::launch_tiled<32>(g, L, q, k, v, o, (char*)ws, s); break;
    default: e = la::launch_tiled<64>(g, L, q, k, v, o, (char*)ws, s); break;
  }
  if (e != hipSuccess) return (la_status)la::record_hip_error((int32_t)e);
  return LA_OK;
}

}  // extern "C"
