// la_tiles.hip -- tiles with halos and Hann-weighted overlap averaging
// (la_tile_* in include/la.h).  Both kernels are pure HBM streams: extract
// is a gather with clamped coordinates, blend reads each covering tile's
// value once per output token.  Every lane moves 16-byte runs of channels,
// and per-block row geometry keeps the per-lane index arithmetic in 32 bits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "../../include/la.h"
#include "la_device.h"
#include "la_profile.h"

namespace {

struct Geo {
  int64_t dims[3], core[3], halo[3], L[3], n[3];
  int64_t C, chunks;  // 16-byte chunks per token
  int64_t tile_tokens;
  int es;
};

__device__ __forceinline__ int64_t clampi(int64_t v, int64_t hi) { return v < 0 ? 0 : (v > hi ? hi : v); }

__device__ __forceinline__ float hann(int64_t u, int64_t L) {
  const float s = sinpif(((float)u + 0.5f) / (float)L);
  return s * s;
}

// One block per row of a tile (fixed (ut, uy)): the row's Lx tokens are
// contiguous in the tile array, and its source is one row of the field
// read at clamped x.  Row geometry is uniform per block; a lane only
// splits its 32-bit work index into (token, chunk), and copies four
// 16-byte chunks per pass so that four loads are in flight at once.
// grid: x = row of the tile (ut * Ly + uy), y = tile
__global__ __launch_bounds__(256) void tile_extract_kernel(Geo g, const char* __restrict__ field,
                                                           char* __restrict__ tiles) {
  const int64_t tile = blockIdx.y, r = blockIdx.x;
  const int64_t a = tile / (g.n[1] * g.n[2]), i = (tile / g.n[2]) % g.n[1], j = tile % g.n[2];
  const int64_t ut = r / g.L[1], uy = r % g.L[1];
  const int64_t row = g.C * g.es;
  const int64_t gt = clampi(a * g.core[0] - g.halo[0] + ut, g.dims[0] - 1);
  const int64_t gy = clampi(i * g.core[1] - g.halo[1] + uy, g.dims[1] - 1);
  const char* src = field + (gt * g.dims[1] + gy) * g.dims[2] * row;
  char* dst = tiles + (tile * g.tile_tokens + r * g.L[2]) * row;
  const uint32_t chunks = (uint32_t)g.chunks, work = (uint32_t)(g.L[2] * g.chunks);
  const int32_t x0 = (int32_t)(j * g.core[2] - g.halo[2]), xmax = (int32_t)g.dims[2] - 1;
  const uint32_t urow = (uint32_t)row;
  for (uint32_t w0 = threadIdx.x; w0 < work; w0 += 4 * 256) {
    la::u32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t w = w0 + 256 * u;
      if (w < work) {
        const uint32_t ux = w / chunks, ch = w - ux * chunks;
        const int32_t gx = min(max(x0 + (int32_t)ux, 0), xmax);
        v[u] = *(const la::u32x4*)(src + ((uint64_t)gx * urow + ch * 16));
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t w = w0 + 256 * u;
      if (w < work) *(la::u32x4*)(dst + (uint64_t)w * 16) = v[u];
    }
  }
}

// One block per field row (fixed (t, y)) and span of x: the covering
// tiles in t and y, and their weights, are uniform per block; a lane
// splits its work index into (x, chunk) and visits the (at most 3) tiles
// covering x.  The x weights come from a table of the Hann window over
// the tile's x extent, built in LDS by the block (the same sinpi values
// the per-tap evaluation gave).
// grid: x = span of the row's (x, chunk) pairs, y = (t, y) row of the field
template <int DT>
__global__ __launch_bounds__(256) void tile_blend_kernel(Geo g, const char* __restrict__ tiles,
                                                         char* __restrict__ field) {
  constexpr int PER = DT == la::DT_BF16 ? 8 : 4;  // channels per 16-byte chunk
  extern __shared__ float hx[];                   // Hann weights over x, L[2] entries
  for (int64_t u = threadIdx.x; u < g.L[2]; u += 256) hx[u] = hann(u, g.L[2]);
  const int64_t rowid = blockIdx.y;
  const int64_t pt = rowid / g.dims[1], py = rowid % g.dims[1];
  const int64_t row = g.C * g.es;
  // tiles covering (pt, py) in t and y: tile i covers p iff
  // i*core - halo <= p < (i+1)*core + halo
  int64_t lo[2], hi[2];
  {
    const int64_t p[2] = {pt, py};
    for (int k = 0; k < 2; ++k) {
      lo[k] = p[k] - g.halo[k] - g.core[k] + 1;
      lo[k] = lo[k] <= 0 ? 0 : (lo[k] + g.core[k] - 1) / g.core[k];
      hi[k] = std::min(g.n[k] - 1, (p[k] + g.halo[k]) / g.core[k]);
    }
  }
  __syncthreads();
  const uint32_t chunks = (uint32_t)g.chunks, work = (uint32_t)(g.dims[2] * g.chunks);
  const uint32_t core2 = (uint32_t)g.core[2], halo2 = (uint32_t)g.halo[2], L2 = (uint32_t)g.L[2];
  const uint32_t nx = (uint32_t)g.n[2], urow = (uint32_t)row;
  for (uint32_t w = blockIdx.x * 256 + threadIdx.x; w < work; w += gridDim.x * 256) {
    const uint32_t px = w / chunks, ch = w - px * chunks;
    const uint32_t xlo = px >= halo2 ? (px - halo2) / core2 : 0;
    const uint32_t xhi = min(nx - 1, (px + halo2) / core2);
    float acc[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) acc[e] = 0.f;
    float wsum = 0.f;
    for (int64_t a = lo[0]; a <= hi[0]; ++a) {
      const int64_t ut = pt - (a * g.core[0] - g.halo[0]);
      const float wt = hann(ut, g.L[0]);
      for (int64_t i = lo[1]; i <= hi[1]; ++i) {
        const int64_t uy = py - (i * g.core[1] - g.halo[1]);
        const float wy = wt * hann(uy, g.L[1]);
        // the (a, i) row of tiles: tile (a, i, 0), token (ut, uy, 0)
        const char* trow = tiles + ((a * g.n[1] + i) * g.n[2] * g.tile_tokens +
                                    (ut * g.L[1] + uy) * g.L[2]) * row;
        for (uint32_t j = xlo; j <= xhi; ++j) {
          const uint32_t ux = px + halo2 - j * core2;
          const float wgt = wy * hx[ux];
          const la::u32x4 v = *(const la::u32x4*)(trow + ((uint64_t)j * g.tile_tokens + ux) * urow + ch * 16);
          if constexpr (DT == la::DT_BF16) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              acc[2 * e] = fmaf(wgt, la::bf16lo(v[e]), acc[2 * e]);
              acc[2 * e + 1] = fmaf(wgt, la::bf16hi(v[e]), acc[2 * e + 1]);
            }
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[e] = fmaf(wgt, __uint_as_float(v[e]), acc[e]);
          }
          wsum += wgt;
        }
      }
    }
    const float r = 1.0f / wsum;
    la::u32x4 o;
    if constexpr (DT == la::DT_BF16) {
#pragma unroll
      for (int e = 0; e < 4; ++e) o[e] = la::pack_bf16(acc[2 * e] * r, acc[2 * e + 1] * r);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) o[e] = __float_as_uint(acc[e] * r);
    }
    *(la::u32x4*)(field + (rowid * g.dims[2]) * row + (uint64_t)w * 16) = o;
  }
}

la_status make_geo(const la_tile_desc* d, Geo* g) {
  if (!d) return LA_ERR_INVALID_ARG;
  if (d->dtype != LA_BF16 && d->dtype != LA_FP32) return LA_ERR_INVALID_ARG;
  if (d->C < 8 || d->C % 8) return LA_ERR_INVALID_ARG;
  g->es = d->dtype == LA_BF16 ? 2 : 4;
  g->C = d->C;
  g->chunks = d->C * g->es / 16;
  int64_t tiles = 1, tok = 1;
  for (int k = 0; k < 3; ++k) {
    if (d->dims[k] < 1 || d->core[k] < 1 || d->halo[k] < 0 || d->halo[k] > d->core[k])
      return LA_ERR_INVALID_ARG;
    g->dims[k] = d->dims[k];
    g->core[k] = d->core[k];
    g->halo[k] = d->halo[k];
    g->L[k] = d->core[k] + 2 * d->halo[k];
    g->n[k] = (d->dims[k] + d->core[k] - 1) / d->core[k];
    tiles *= g->n[k];
    tok *= g->L[k];
  }
  g->tile_tokens = tok;
  if (tiles > 65535 || d->dims[0] * d->dims[1] > 65535) return LA_ERR_UNSUPPORTED;
  // 32-bit lane indices within a row; the x window table fits LDS
  if (g->L[2] * g->chunks >= (int64_t(1) << 31) || g->dims[2] * g->chunks >= (int64_t(1) << 31) ||
      g->L[2] * g->C * g->es >= (int64_t(1) << 32) || g->L[2] > 16384)
    return LA_ERR_UNSUPPORTED;
  return LA_OK;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

}  // namespace

extern "C" {

la_status la_tile_geometry(const la_tile_desc* desc, int64_t* n_tiles, int64_t* tile_tokens) {
  if (!n_tiles || !tile_tokens) return LA_ERR_INVALID_ARG;
  Geo g;
  la_status st = make_geo(desc, &g);
  if (st != LA_OK) return st;
  *n_tiles = g.n[0] * g.n[1] * g.n[2];
  *tile_tokens = g.tile_tokens;
  return LA_OK;
}

la_status la_tile_extract(const la_tile_desc* desc, const void* field, void* tiles,
                          la_stream stream) {
  Geo g;
  la_status st = make_geo(desc, &g);
  if (st != LA_OK) return st;
  if (!field || !tiles || !aligned16(field) || !aligned16(tiles)) return LA_ERR_INVALID_ARG;
  const int64_t ntiles = g.n[0] * g.n[1] * g.n[2];
  la::ProfScope prof("tile_extract", (hipStream_t)stream);
  hipLaunchKernelGGL(tile_extract_kernel, dim3((unsigned)(g.L[0] * g.L[1]), (unsigned)ntiles),
                     dim3(256), 0, (hipStream_t)stream, g, (const char*)field, (char*)tiles);
  return hipGetLastError() == hipSuccess ? LA_OK : LA_ERR_HIP;
}

la_status la_tile_blend(const la_tile_desc* desc, const void* tiles, void* field,
                        la_stream stream) {
  Geo g;
  la_status st = make_geo(desc, &g);
  if (st != LA_OK) return st;
  if (!field || !tiles || !aligned16(field) || !aligned16(tiles)) return LA_ERR_INVALID_ARG;
  const int64_t rows = g.dims[0] * g.dims[1];
  const int64_t work = g.dims[2] * g.chunks;
  const unsigned bx = (unsigned)std::min<int64_t>((work + 255) / 256, std::max<int64_t>(1, 65536 / rows));
  const size_t lds = (size_t)g.L[2] * sizeof(float);
  la::ProfScope prof("tile_blend", (hipStream_t)stream);
  if (desc->dtype == LA_BF16)
    hipLaunchKernelGGL(tile_blend_kernel<la::DT_BF16>, dim3(bx, (unsigned)rows), dim3(256), lds,
                       (hipStream_t)stream, g, (const char*)tiles, (char*)field);
  else
    hipLaunchKernelGGL(tile_blend_kernel<la::DT_FP32>, dim3(bx, (unsigned)rows), dim3(256), lds,
                       (hipStream_t)stream, g, (const char*)tiles, (char*)field);
  return hipGetLastError() == hipSuccess ? LA_OK : LA_ERR_HIP;
}

}  // extern "C"
