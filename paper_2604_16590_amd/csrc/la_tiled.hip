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
//  1. tile summaries, read from the K and V fields in place (clamped
//     coordinates, as tile extraction does).  Neighbouring tiles share
//     their halo tokens, so the extended token sets are cut into segment
//     pairs in (y, x) and walked along t: each token's phi(k) and operands
//     are formed once per segment pair and added into the FP32 sums of the
//     one or two t-neighbouring tiles that hold it (1a, column partials of
//     at most 16,384 tokens); each tile's column partials are then added
//     in FP64 in a fixed order and written as the apply's operands (1b:
//     S_t^T hi parts, z_t hi + lo);
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
  int64_t ns[3];     // segments per dimension (y, x): 2n + 1
  int Pf;            // parts per segment pair footprint (<= 8)
  int64_t CH, nch;   // tiles per t chunk, chunks
  int64_t n_items;   // column walks: nch * ns[1] * ns[2] * Pf * H
};

__device__ __forceinline__ uint32_t clamp32(int32_t v, int32_t hi) {
  return (uint32_t)min(max(v, 0), hi);
}

// Hann weight of coordinate u of a tile extent L, sampled at cell centres:
// w(u) = sin^2(pi (u + 1/2) / L) for 0 <= u < L (strictly positive), else
// 0; inv2L = 1 / (2L).  The hardware sine takes its argument in
// revolutions (sin(2 pi x)); its error (about 1e-6) is far below the bf16
// rounding of the blended output.
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
// Pass 1: the tile summaries, with phi(k) and the operand packing done once
// per token (and t chunk) instead of once per covering tile.  Along
// y and x, tile j's extended range [jc - h, (j+1)c + h) is the union of
// three segments: Z_j = [jc - h, jc + h) (shared with tile j - 1), I_j =
// [jc + h, (j+1)c - h) (its own) and Z_{j+1}; numbered s = 2j (Z_j) and
// s = 2j + 1 (I_j), tile j covers segments 2j, 2j + 1 and 2j + 2.
//  1a. One wave per (t chunk, y segment, x segment, footprint part, head)
//      walks the t planes of its chunk's tiles over that segment pair,
//      coordinates clamped into the grid.  A plane lies in at most two
//      tiles of the chunk (2 halo <= core): the wave keeps both tiles' FP32
//      sums and adds each step's products into the one or two that hold
//      the plane, from the same rounded operands.  After a tile's last
//      plane its sum is written out as the tile's column partial for this
//      segment pair (an FP32 run of at most 16,384 tokens).
//  1b. One workgroup per (tile, head) adds its column partials (3 x 3
//      segment pairs times the footprint parts) in FP64 in a fixed order
//      and writes the apply's operand slot.
// ---------------------------------------------------------------------------

// segment s of dimension k (1 or 2): first virtual coordinate and width
__device__ __forceinline__ void segment(const TGeo& g, int k, int64_t s, int32_t& start,
                                        int32_t& width) {
  const int32_t j = (int32_t)(s >> 1), c = (int32_t)g.core[k], h = (int32_t)g.halo[k];
  start = (s & 1) ? j * c + h : j * c - h;
  width = (s & 1) ? c - 2 * h : 2 * h;
}

// part f of the (y, x) footprint of segment pair (sy, sx): positions
// [p0, p1) of the footprint, row-major; false when it is empty (a
// zero-width segment, or fewer positions than parts)
__device__ __forceinline__ bool col_part(const TGeo& g, int64_t sy, int64_t sx, int f, int32_t& ys,
                                         int32_t& xs, uint32_t& xw, uint32_t& p0, uint32_t& p1) {
  int32_t yw, w;
  segment(g, 1, sy, ys, yw);
  segment(g, 2, sx, xs, w);
  xw = (uint32_t)w;
  const uint32_t fp = (uint32_t)yw * xw;
  const uint32_t pl = (fp + (uint32_t)g.Pf - 1) / (uint32_t)g.Pf;
  p0 = (uint32_t)f * pl;
  p1 = min(fp, p0 + pl);
  return p0 < p1;
}

// the column partial of tile row a (along t), segment pair (sy, sx), part
// f, head: D*D + D floats (S in the matrix cores' lane order, then z)
__device__ __forceinline__ int64_t col_index(const TGeo& g, int64_t a, int64_t sy, int64_t sx, int f,
                                             int64_t head) {
  return (((a * g.ns[1] + sy) * g.ns[2] + sx) * g.Pf + f) * g.H + head;
}

// One step of a column walk (R tokens per lane group, loaded as the
// summary step takes them): phi on the keys and the token-pair packing
// once, then the products into the current tile's sum and, on a plane
// shared with the next tile, into that one's too.
template <int D>
__device__ __forceinline__ void col_step(const SummaryRegs<DT_BF16, D, MODE_FWD>& x, bool both,
                                         f32x4 (&ac)[D / 16][D / 16], float (&zc)[D / 16],
                                         f32x4 (&an)[D / 16][D / 16], float (&zn)[D / 16]) {
  constexpr int F = D / 16;
  uint32_t own[F][4];
#pragma unroll
  for (int jj = 0; jj < F; ++jj)
#pragma unroll
    for (int pp = 0; pp < 4; ++pp)
      own[jj][pp] = (uint32_t)word_bits16<DT_BF16>(x.vw[2 * pp], jj) |
                    ((uint32_t)word_bits16<DT_BF16>(x.vw[2 * pp + 1], jj) << 16);
  bf16x8 ak[F];
#pragma unroll
  for (int i = 0; i < F; ++i) {
    uint32_t pk[4];
    float zs = 0.f;
#pragma unroll
    for (int pp = 0; pp < 4; ++pp) {
      pk[pp] = pack_bf16(phi<DT_BF16>(word_elem<DT_BF16>(x.kw[2 * pp], i)),
                         phi<DT_BF16>(word_elem<DT_BF16>(x.kw[2 * pp + 1], i)));
      // normaliser from the same rounded phi values that feed S
      zs = add_bf16_pair(zs, pk[pp]);
    }
    zc[i] += zs;
    if (both) zn[i] += zs;
    ak[i] = as_bf16x8(u32x4{pk[0], pk[1], pk[2], pk[3]});
  }
#pragma unroll
  for (int j = 0; j < F; ++j) {
    const bf16x8 bv = as_bf16x8(u32x4{own[j][0], own[j][1], own[j][2], own[j][3]});
#pragma unroll
    for (int i = 0; i < F; ++i) ac[i][j] = mfma_bf16(ak[i], bv, ac[i][j]);
  }
  if (both) {
#pragma unroll
    for (int j = 0; j < F; ++j) {
      const bf16x8 bv = as_bf16x8(u32x4{own[j][0], own[j][1], own[j][2], own[j][3]});
#pragma unroll
      for (int i = 0; i < F; ++i) an[i][j] = mfma_bf16(ak[i], bv, an[i][j]);
    }
  }
}

// 1a. grid: four waves per workgroup, each its own item; items ordered
// head fastest, so the waves reading one token row's head slices run side
// by side.  The bound of one wave per SIMD lets the compiler keep the two
// tiles' sums in the accumulation registers: at d = 64 it takes 242
// registers in all, so two waves per SIMD still run; held to two waves per
// SIMD it kept them in the vector registers and spilled (5 % slower)
template <int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1)))
void tile_cols_kernel(TGeo g, const void* __restrict__ k, const void* __restrict__ v,
                      float* __restrict__ cols) {
  using C = SummaryCfg<DT_BF16, D, MODE_FWD>;
  using Regs = SummaryRegs<DT_BF16, D, MODE_FWD>;
  static_assert(C::SPLIT == 1 && C::FR == C::F, "one wave holds a whole sum");
  constexpr int F = C::F, R = C::R, STEP = C::STEP, E = D * D + D;
  const int lane = threadIdx.x & 63;
  const int gq = lane >> 4, m = lane & 15;
  const int64_t item = (int64_t)blockIdx.x * 4 + wave_index();
  if (item >= g.n_items) return;  // uniform over the wave
  const int64_t head = item % g.H;
  int64_t rest = item / g.H;
  const int f = (int)(rest % g.Pf);
  rest /= g.Pf;
  const int64_t sx = rest % g.ns[2];
  rest /= g.ns[2];
  const int64_t sy = rest % g.ns[1];
  const int64_t q = rest / g.ns[1];
  int32_t ys, xs;
  uint32_t xw, p0, p1;
  if (!col_part(g, sy, sx, f, ys, xs, xw, p0, p1)) return;  // uniform
  const int64_t a0 = q * g.CH, a1 = min(g.n[0], a0 + g.CH);
  const int32_t c0 = (int32_t)g.core[0], h0 = (int32_t)g.halo[0];
  // virtual planes [t_first, t_stop): the chunk's tiles' extended t ranges
  const int32_t t_first = (int32_t)a0 * c0 - h0, t_stop = (int32_t)a1 * c0 + h0;
  const uint32_t spp = (p1 - p0 + STEP - 1) / STEP;  // steps per plane
  const int64_t total = (int64_t)(t_stop - t_first) * spp;

  const int64_t rowb = g.C * 2;  // bytes per token of a field
  const char* kb = (const char*)k + head * D * 2 + (int64_t)(F * m) * 2;
  const char* vb = (const char*)v + head * D * 2 + (int64_t)(F * m) * 2;
  const int32_t M0 = (int32_t)g.dims[0] - 1, M1 = (int32_t)g.dims[1] - 1,
                M2 = (int32_t)g.dims[2] - 1;
  const uint32_t N1 = (uint32_t)g.dims[1], N2 = (uint32_t)g.dims[2];
  const uint32_t neg_inf = 0xff80ff80u;
  // the step js of plane t: lane group gq takes footprint positions
  // p0 + STEP*js + R*gq + r; 32-bit coordinates (a field holds fewer
  // than 2^31 tokens).  Every load is issued: positions past the part's
  // end are clamped into the grid like all others, and the step drops
  // them (bit r of the lane's mask is clear), so no branch stands between
  // a step's loads and the compiler's count of them
  auto load = [&](int32_t t, uint32_t js, Regs& x, uint32_t& mask) {
    const uint32_t j = p0 + STEP * js + R * gq;
    uint32_t uy = j / xw;
    uint32_t ux = j - uy * xw;
    const uint32_t gt = clamp32(t, M0);
    mask = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      mask |= (uint32_t)(j + r < p1) << r;
      const uint32_t gy = clamp32(ys + (int32_t)uy, M1);
      const uint32_t gx = clamp32(xs + (int32_t)ux, M2);
      const int64_t off = (int64_t)((gt * N1 + gy) * N2 + gx) * rowb;
      // plain loads (non-temporal ones ran 1 % slower here, and the slot
      // pass after them 10 % slower)
      load_words<C::KB>(kb + off, x.kw[r]);
      load_words<C::VB>(vb + off, x.vw[r]);
      if (++ux == xw) {
        ux = 0;
        ++uy;
      }
    }
  };

  f32x4 ac[F][F], an[F][F];
  float zc[F], zn[F];
#pragma unroll
  for (int i = 0; i < F; ++i) {
    zc[i] = 0.f;
    zn[i] = 0.f;
#pragma unroll
    for (int j = 0; j < F; ++j) {
      ac[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
      an[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  }
  int64_t a = a0;  // the tile whose sum is ac; an is tile a + 1's
  auto process = [&](Regs& x, uint32_t mask, int32_t t, uint32_t js) {
    if (p0 + STEP * (js + 1) > p1) {  // a part's last, partial step (wave-uniform)
      // dropped positions: phi(-inf) = 0 and v = 0 add nothing
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const bool keep = (mask >> r) & 1u;
#pragma unroll
        for (int w = 0; w < C::KW; ++w) x.kw[r][w] = keep ? x.kw[r][w] : neg_inf;
#pragma unroll
        for (int w = 0; w < C::VW; ++w) x.vw[r][w] = keep ? x.vw[r][w] : 0u;
      }
    }
    const int32_t next_first = (int32_t)(a + 1) * c0 - h0;  // tile a + 1's first plane
    col_step<D>(x, a + 1 < a1 && t >= next_first, ac, zc, an, zn);
    if (js == spp - 1 && t == next_first + 2 * h0 - 1) {  // tile a's last plane done
      float* out = cols + col_index(g, a, sy, sx, f, head) * E;
#pragma unroll
      for (int i = 0; i < F; ++i)
#pragma unroll
        for (int j = 0; j < F; ++j) *(f32x4*)(out + ((i * F + j) * 64 + lane) * 4) = ac[i][j];
#pragma unroll
      for (int i = 0; i < F; ++i) {
        const float zs = sum_groups(zc[i]);
        if (gq == 0) out[D * D + F * m + i] = zs;
      }
#pragma unroll
      for (int i = 0; i < F; ++i) {
        zc[i] = zn[i];
        zn[i] = 0.f;
#pragma unroll
        for (int j = 0; j < F; ++j) {
          ac[i][j] = an[i][j];
          an[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
      }
      ++a;
    }
  };
  auto advance = [&](int32_t& t, uint32_t& js) {
    if (++js == spp) {
      js = 0;
      ++t;
    }
  };
  // two register sets in turn, the next step's loads in flight while the
  // current one computes; every load is issued (past the last step the
  // last one is read again, unused), so a step waits only for its own
  int32_t lt = t_first, ct = t_first;
  uint32_t ljs = 0, cjs = 0;
  auto advance_load = [&]() {
    if (lt != t_stop - 1 || ljs != spp - 1) advance(lt, ljs);
  };
  Regs ra, rb;
  uint32_t ma, mb;
  load(lt, ljs, ra, ma);
  advance_load();
  for (int64_t s = 0; s < total; s += 2) {
    load(lt, ljs, rb, mb);
    advance_load();
    __builtin_amdgcn_sched_barrier(0);
    process(ra, ma, ct, cjs);
    advance(ct, cjs);
    load(lt, ljs, ra, ma);
    advance_load();
    __builtin_amdgcn_sched_barrier(0);
    if (s + 1 < total) {
      process(rb, mb, ct, cjs);
      advance(ct, cjs);
    }
  }
}

// 1b. grid: one workgroup per (tile, head), head fastest
template <int D>
__global__ __launch_bounds__(256)
void tile_slot_kernel(TGeo g, const float* __restrict__ cols, u32x4* __restrict__ slots) {
  using TC = TiledCfg<D>;
  using RB = Run<D, DT_BF16>;
  constexpr int F = D / 16, E = D * D + D;
  static_assert(E % 4 == 0, "whole 16-byte groups of a partial");
  const int64_t tile = blockIdx.x / g.H;
  const int64_t head = blockIdx.x % g.H;
  const int64_t a = tile / (g.n[1] * g.n[2]), b = (tile / g.n[2]) % g.n[1], c = tile % g.n[2];
  // the tile's column partials (at most 9 x 8), in a fixed order
  __shared__ int64_t src[9 * 8];
  __shared__ int nsrc;
  if (threadIdx.x == 0) {
    int n = 0;
    for (int64_t sy = 2 * b; sy <= 2 * b + 2; ++sy)
      for (int64_t sx = 2 * c; sx <= 2 * c + 2; ++sx)
        for (int f = 0; f < g.Pf; ++f) {
          int32_t ys, xs;
          uint32_t xw, p0, p1;
          if (col_part(g, sy, sx, f, ys, xs, xw, p0, p1)) src[n++] = col_index(g, a, sy, sx, f, head) * E;
        }
    nsrc = n;
  }
  __syncthreads();
  const int ns = nsrc;
  // FP64 sum of the column partials, four consecutive elements per thread
  // (16-byte loads of every partial in flight together); element u of the
  // partial layout (tile (i, j), lane (g, n), register r: S[F(4g + r) + i]
  // [F n + j]; then z) goes into the operand slot: S^T hi parts at (row e,
  // contraction c), z's hi parts in the even rows of the z tile and its lo
  // parts in the odd.  The slot is assembled in LDS (every one of its
  // halfwords is written) and stored with whole 16-byte vectors.
  __shared__ u32x4 simg[TC::SLOT];
  uint16_t* slot = (uint16_t*)simg;
  for (int u4 = threadIdx.x; u4 < E / 4; u4 += 256) {
    double sum[4] = {0.0, 0.0, 0.0, 0.0};
    for (int s0 = 0; s0 < ns; s0 += 9) {
      const int cnt = min(9, ns - s0);
      f32x4 x[9];
#pragma unroll
      for (int s = 0; s < 9; ++s)
        if (s < cnt) x[s] = *(const f32x4*)(cols + src[s0 + s] + 4 * u4);
#pragma unroll
      for (int s = 0; s < 9; ++s)
        if (s < cnt)
#pragma unroll
          for (int r = 0; r < 4; ++r) sum[r] += (double)x[s][r];
    }
#pragma unroll
    for (int r4 = 0; r4 < 4; ++r4) {
      const int u = 4 * u4 + r4;
      const uint16_t hi = to_bf16((float)sum[r4]);
      if (u < D * D) {
        const int r = u & 3, ln = (u >> 2) & 63, ij = u >> 8;
        const int i = ij / F, j = ij % F;
        const int cc = F * (4 * (ln >> 4) + r) + i, e = F * (ln & 15) + j;
        // T image: A[row = value feature e][k = key feature cc]
        const int rp = RB::pos(e), kp = RB::pos(cc);
        const int word = ((rp >> 2) * TC::NS + (kp >> 3)) * 64 + 16 * RB::group(cc) + 4 * RB::group(e) + (rp & 3);
        slot[word * 8 + (kp & 7)] = hi;
        if (TC::Q4 < 8) slot[word * 8 + (kp & 7) + 4] = 0;  // d = 16: padding of the k-step
      } else {
        const int cc = u - D * D;
        const uint16_t lo = to_bf16((float)(sum[r4] - (double)bf16f(hi)));
        const int kp = RB::pos(cc);
        for (int mm = 0; mm < 16; ++mm) {
          const int word = TC::S_WORDS + (kp >> 3) * 64 + 16 * RB::group(cc) + mm;
          slot[word * 8 + (kp & 7)] = (mm & 1) ? lo : hi;
          if (TC::Q4 < 8) slot[word * 8 + (kp & 7) + 4] = 0;
        }
      }
    }
  }
  __syncthreads();
  u32x4* dst = slots + (tile * g.H + head) * TC::SLOT;
  for (int w = threadIdx.x; w < TC::SLOT; w += 256) dst[w] = simg[w];
}

// ---------------------------------------------------------------------------
// Pass 2: apply and blend, one workgroup per (cell, head).  Cell j of a
// dimension covers [j*core - a, j*core - a + core) of the grid, a =
// core / 2; its positions are covered only by tiles j - 1 and j of that
// dimension (halo <= core / 2).  Slot s = (st, sy, sx) in {0, 1}^3 holds
// tile (jt - 1 + st, jy - 1 + sy, jx - 1 + sx) if it exists: the S^T hi
// parts (S_t to about 2^-9) and the hi / lo z tile.  The waves take the
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

  // one workgroup per (cell, head), cell fastest: neighbouring cells share
  // covering tiles, whose operand slots they then stage from L2 (head
  // fastest ran 1.5 % slower)
  const int64_t head = blockIdx.x / g.n_cells;
  const int64_t cell = blockIdx.x % g.n_cells;
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
  // fetches past the cell's end locate its last token again (no branch
  // around the loads); such tokens are not ok: no weight, nothing stored
  Step sa, sb;
  const int64_t base0 = (int64_t)wave * TT;
  fetch(base0, sa);

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

  // two register sets in turn.  The fetches are unconditional and the loop
  // body has no early exit (an odd step count runs one step with nothing
  // to weigh or store), so the compiler's wait before a step covers only
  // that step's queries, not the next step's nor the previous outputs'
  // stores; the scheduling barriers keep each fetch ahead of the step it
  // overlaps
  const int64_t nsteps = base0 < ntile ? (ntile - 1 - base0) / per_step + 1 : 0;
  for (int64_t k = 0; k < nsteps; k += 2) {
    fetch(base0 + (k + 1) * per_step, sb);
    __builtin_amdgcn_sched_barrier(0);
    compute(sa);
    fetch(base0 + (k + 2) * per_step, sa);
    __builtin_amdgcn_sched_barrier(0);
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
    if (2 * g->halo[k] > g->core[k]) return LA_ERR_UNSUPPORTED;  // <= 2 tiles per dim at a point
  const int64_t field = td->dims[0] * td->dims[1] * td->dims[2];
  // 32-bit token coordinates in the kernels; flat grids (cells >= tiles);
  // a tile's t extent is one FP32 run of a column partial
  if (heads > 65535 || tok > 65536 || field >= (int64_t(1) << 31) ||
      cells * heads >= (int64_t(1) << 31) || g->L[0] > 16384)
    return LA_ERR_UNSUPPORTED;
  g->tile_tokens = tok;
  g->n_tiles = tiles;
  g->n_cells = cells;
  // footprint parts: a column partial sums the tile's t extent times one
  // part of the widest segment pair's footprint, at most 16,384 tokens
  g->ns[0] = 1;
  int64_t wmax[3] = {0, 0, 0};
  for (int k = 1; k < 3; ++k) {
    g->ns[k] = 2 * g->n[k] + 1;
    wmax[k] = std::max(2 * g->halo[k], g->core[k] - 2 * g->halo[k]);
  }
  const int64_t fpmax = wmax[1] * wmax[2];
  int Pf = 1;
  while (g->L[0] * ((fpmax + Pf - 1) / Pf) > 16384) ++Pf;
  if (Pf > 8) return LA_ERR_UNSUPPORTED;
  g->Pf = Pf;
  // t chunks: enough column walks to fill the machine a few times over;
  // each chunk re-reads the planes its first tile shares with the one
  // before (2 halo of every CH * core)
  const int64_t base = g->ns[1] * g->ns[2] * Pf * heads;
  const int64_t want = std::min(g->n[0], std::max<int64_t>(1, (8192 + base - 1) / base));
  g->CH = (g->n[0] + want - 1) / want;
  g->nch = (g->n[0] + g->CH - 1) / g->CH;
  g->n_items = g->nch * base;
  if ((g->n_items + 3) / 4 >= (int64_t(1) << 31)) return LA_ERR_UNSUPPORTED;
  return LA_OK;
}

struct TLayout {
  size_t img, cols, total;
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

size_t slot_bytes(int64_t D) {
  switch (D) {
    case 16: return TiledCfg<16>::SLOT * 16;
    case 32: return TiledCfg<32>::SLOT * 16;
    default: return TiledCfg<64>::SLOT * 16;
  }
}

// the workspace holds one operand slot per (tile, head), then the column
// partials (per tile row along t, segment pair, part and head)
TLayout tlayout(const TGeo& g) {
  TLayout L{};
  L.img = 0;
  L.cols = align256((size_t)g.n_tiles * g.H * slot_bytes(g.d));
  const size_t E = (size_t)(g.d * g.d + g.d);
  L.total = L.cols + align256((size_t)g.n[0] * g.ns[1] * g.ns[2] * g.Pf * g.H * E * sizeof(float));
  return L;
}

template <int D>
hipError_t launch_tiled(const TGeo& g, const TLayout& L, const void* q, const void* k,
                        const void* v, void* o, char* ws, hipStream_t st) {
  {
    ProfScope prof("tile_cols", st);
    hipLaunchKernelGGL(tile_cols_kernel<D>, dim3((unsigned)((g.n_items + 3) / 4)), dim3(256), 0, st,
                       g, k, v, (float*)(ws + L.cols));
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  {
    ProfScope prof("tile_slots", st);
    hipLaunchKernelGGL(tile_slot_kernel<D>, dim3((unsigned)(g.n_tiles * g.H)), dim3(256), 0, st,
                       g, (const float*)(ws + L.cols), (u32x4*)(ws + L.img));
  }
  e = hipGetLastError();
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
