// la_tiles.hip -- tiles with halos and Hann-weighted overlap averaging
// (la_tile_* in include/la.h).  Both kernels are pure HBM streams: extract
// is a gather with clamped coordinates, blend reads each covering tile's
// value once per output token.  Every lane moves 16-byte runs of channels.
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

// grid: y = tile, x strides over the tile's (token, chunk) pairs
__global__ __launch_bounds__(256) void tile_extract_kernel(Geo g, const char* __restrict__ field,
                                                           char* __restrict__ tiles) {
  const int64_t tile = blockIdx.y;
  const int64_t a = tile / (g.n[1] * g.n[2]), i = (tile / g.n[2]) % g.n[1], j = tile % g.n[2];
  const int64_t work = g.tile_tokens * g.chunks;
  const int64_t row = g.C * g.es;
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < work;
       w += (int64_t)gridDim.x * blockDim.x) {
    const int64_t tok = w / g.chunks, ch = w - tok * g.chunks;
    const int64_t ux = tok % g.L[2], uy = (tok / g.L[2]) % g.L[1], ut = tok / (g.L[2] * g.L[1]);
    const int64_t gt = clampi(a * g.core[0] - g.halo[0] + ut, g.dims[0] - 1);
    const int64_t gy = clampi(i * g.core[1] - g.halo[1] + uy, g.dims[1] - 1);
    const int64_t gx = clampi(j * g.core[2] - g.halo[2] + ux, g.dims[2] - 1);
    const la::u32x4 v = *(const la::u32x4*)(field + ((gt * g.dims[1] + gy) * g.dims[2] + gx) * row + ch * 16);
    *(la::u32x4*)(tiles + (tile * g.tile_tokens + tok) * row + ch * 16) = v;
  }
}

// grid: y = (t, y) row of the field, x strides over the row's (x, chunk)
// pairs; each thread visits the (at most 3 per dim) tiles covering its token
template <int DT>
__global__ __launch_bounds__(256) void tile_blend_kernel(Geo g, const char* __restrict__ tiles,
                                                         char* __restrict__ field) {
  constexpr int PER = DT == la::DT_BF16 ? 8 : 4;  // channels per 16-byte chunk
  const int64_t rowid = blockIdx.y;
  const int64_t pt = rowid / g.dims[1], py = rowid % g.dims[1];
  const int64_t work = g.dims[2] * g.chunks;
  const int64_t row = g.C * g.es;
  int64_t lo[2], hi[2];
  {
    const int64_t p[2] = {pt, py};
    for (int k = 0; k < 2; ++k) {
      // tile i covers p iff i*core - halo <= p < (i+1)*core + halo
      lo[k] = p[k] - g.halo[k] - g.core[k] + 1;
      lo[k] = lo[k] <= 0 ? 0 : (lo[k] + g.core[k] - 1) / g.core[k];
      hi[k] = std::min(g.n[k] - 1, (p[k] + g.halo[k]) / g.core[k]);
    }
  }
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < work;
       w += (int64_t)gridDim.x * blockDim.x) {
    const int64_t px = w / g.chunks, ch = w - px * g.chunks;
    int64_t xlo = px - g.halo[2] - g.core[2] + 1;
    xlo = xlo <= 0 ? 0 : (xlo + g.core[2] - 1) / g.core[2];
    const int64_t xhi = std::min(g.n[2] - 1, (px + g.halo[2]) / g.core[2]);
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
        for (int64_t j = xlo; j <= xhi; ++j) {
          const int64_t ux = px - (j * g.core[2] - g.halo[2]);
          const float wgt = wy * hann(ux, g.L[2]);
          const int64_t tile = (a * g.n[1] + i) * g.n[2] + j;
          const int64_t tok = (ut * g.L[1] + uy) * g.L[2] + ux;
          const la::u32x4 v = *(const la::u32x4*)(tiles + (tile * g.tile_tokens + tok) * row + ch * 16);
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
    *(la::u32x4*)(field + (rowid * g.dims[2] + px) * row + ch * 16) = o;
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
  const int64_t work = g.tile_tokens * g.chunks;
  const unsigned bx = (unsigned)std::min<int64_t>((work + 255) / 256, std::max<int64_t>(1, 16384 / ntiles));
  la::ProfScope prof("tile_extract", (hipStream_t)stream);
  hipLaunchKernelGGL(tile_extract_kernel, dim3(bx, (unsigned)ntiles), dim3(256), 0,
                     (hipStream_t)stream, g, (const char*)field, (char*)tiles);
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
  const unsigned bx = (unsigned)std::min<int64_t>((work + 255) / 256, std::max<int64_t>(1, 16384 / rows));
  la::ProfScope prof("tile_blend", (hipStream_t)stream);
  if (desc->dtype == LA_BF16)
    hipLaunchKernelGGL(tile_blend_kernel<la::DT_BF16>, dim3(bx, (unsigned)rows), dim3(256), 0,
                       (hipStream_t)stream, g, (const char*)tiles, (char*)field);
  else
    hipLaunchKernelGGL(tile_blend_kernel<la::DT_FP32>, dim3(bx, (unsigned)rows), dim3(256), 0,
                       (hipStream_t)stream, g, (const char*)tiles, (char*)field);
  return hipGetLastError() == hipSuccess ? LA_OK : LA_ERR_HIP;
}

}  // extern "C"
