// gen.hip -- liblagen.so: seeded synthetic inputs in device memory.
//
// Holds the input generator only, no attention arithmetic; the definition
// is documented in include/la_gen.h and mirrored on the host by
// paper_2604_16590_amd/inputs.py.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/la_gen.h"

namespace {

// Philox4x32-10 (Salmon et al., SC 2011).
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    const uint32_t lo0 = M0 * c[0], hi0 = __umulhi(M0, c[0]);
    const uint32_t lo1 = M1 * c[2], hi1 = __umulhi(M1, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n1 = lo1, n2 = hi0 ^ c[3] ^ k1, n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
  }
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

struct GenArgs {
  void* dst;
  int dtype;
  int64_t B, H, N, d, sb, sh, sn;
  uint64_t seed;
  uint32_t stream;
  int tensor_id;
  double mean, std;
  int grid_T, grid_lat, grid_lon;
  double amplitude;
  int64_t b_offset;
};

__device__ __forceinline__ double structure(const GenArgs& a, int64_t h, int64_t n, int64_t c) {
  const double kPi = 3.14159265358979323846;
  const int64_t nlon = a.grid_lon, nlat = a.grid_lat;
  const int64_t j = n % nlon, i = (n / nlon) % nlat, t = n / (nlon * nlat);
  const double lat = kPi * (((double)i + 0.5) / (double)nlat - 0.5);
  const double lon = 2.0 * kPi * (double)j / (double)nlon;
  const double m = (double)(1 + c % 4), l = (double)(1 + c % 3);
  const double key = 0.6180339887 * (double)(a.tensor_id * a.H * a.d + h * a.d + c);
  const double psi = 2.0 * kPi * (key - floor(key));
  return a.amplitude * sin(m * lon + l * lat + 2.0 * kPi * (double)t / (double)a.grid_T + psi);
}

__global__ __launch_bounds__(256) void gen_kernel(GenArgs a) {
  const int64_t pairs = a.B * a.H * a.N * a.d / 2;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const double kTwoPi = 6.28318530717958647692;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < pairs; p += stride) {
    // logical pair index in the [b_offset + B, H, N, d] tensor
    const int64_t lp = p + a.b_offset * a.H * a.N * a.d / 2;
    uint32_t c[4] = {(uint32_t)lp, (uint32_t)((uint64_t)lp >> 32), a.stream, 0u};
    philox4x32_10(c, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
    const double u1 = ((double)(c[0] >> 9) + 0.5) * 0x1p-23;
    const double u2 = (double)(c[1] >> 8) * 0x1p-24;
    const double r = sqrt(-2.0 * log(u1));
    const double t = kTwoPi * u2;
    const double z[2] = {r * cos(t), r * sin(t)};
    const int64_t e0 = 2 * p;
    const int64_t cc = e0 % a.d, n = (e0 / a.d) % a.N;
    const int64_t h = (e0 / (a.d * a.N)) % a.H, b = e0 / (a.d * a.N * a.H);
    const int64_t off = b * a.sb + h * a.sh + n * a.sn + cc;
    float f[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      double val = a.mean + a.std * z[s];
      if (a.grid_T > 0) val += structure(a, h, n, cc + s);
      f[s] = (float)val;
    }
    if (a.dtype == 0) {
      const uint32_t w = (uint32_t)f32_to_bf16_rne(f[0]) | ((uint32_t)f32_to_bf16_rne(f[1]) << 16);
      *(uint32_t*)((uint16_t*)a.dst + off) = w;
    } else {
      float2 w = {f[0], f[1]};
      *(float2*)((float*)a.dst + off) = w;
    }
  }
}

}  // namespace

extern "C" int32_t la_gen_fill(void* dst, int32_t dtype, int64_t B, int64_t H, int64_t N,
                               int64_t d, int64_t sb, int64_t sh, int64_t sn,
                               const la_gen_spec* spec, void* stream) {
  if (!dst || !spec || (dtype != 0 && dtype != 1)) return 1;
  if (B < 1 || H < 1 || N < 1 || d < 2 || (d & 1)) return 1;
  if (((uintptr_t)dst & 15u) != 0 || sb < 0 || sh < 0 || sn < d) return 1;
  if ((sb & 1) || (sh & 1) || (sn & 1)) return 1;  // pairs are stored as one word
  if (spec->grid_T < 0) return 1;
  if (spec->grid_T > 0) {
    if (spec->grid_lat < 1 || spec->grid_lon < 1) return 1;
    if ((int64_t)spec->grid_T * spec->grid_lat * spec->grid_lon != N) return 1;
  }
  GenArgs a;
  a.dst = dst; a.dtype = dtype;
  a.B = B; a.H = H; a.N = N; a.d = d; a.sb = sb; a.sh = sh; a.sn = sn;
  a.seed = spec->seed; a.stream = spec->stream; a.tensor_id = spec->tensor_id;
  a.mean = spec->mean; a.std = spec->std;
  a.grid_T = spec->grid_T; a.grid_lat = spec->grid_lat; a.grid_lon = spec->grid_lon;
  a.amplitude = spec->amplitude;
  a.b_offset = spec->b_offset;
  if (a.b_offset < 0) return 1;
  const int64_t pairs = B * H * N * d / 2;
  int64_t blocks = (pairs + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(gen_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, a);
  return hipGetLastError() == hipSuccess ? 0 : 4;
}
