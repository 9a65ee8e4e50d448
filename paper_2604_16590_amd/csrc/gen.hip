// gen.hip -- liblagen.so: seeded synthetic inputs in device memory.
//
// Holds the input generator only, no attention arithmetic; the definition
// is documented in include/la_gen.h and mirrored on the host by
// paper_2604_16590_amd/inputs.py.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/la_gen.h"

namespace {

// Philox4x32-10 (Salmon et al., SC 2011).
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    // one 32 x 32 -> 64-bit product each (both halves from one instruction)
    const uint64_t p0 = (uint64_t)M0 * c[0], p1 = (uint64_t)M1 * c[2];
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n1 = lo1, n2 = hi0 ^ c[3] ^ k1, n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
  }
}

// Two floats -> bfloat16 pair (lo in bits 0..15), round to nearest even:
// one v_cvt_pk_bf16_f32 (the values here are finite, never NaN).
__device__ __forceinline__ uint32_t bf16_pair_rne(float lo, float hi) {
  typedef __bf16 bf16v2 __attribute__((ext_vector_type(2)));
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{lo, hi}, bf16v2));
}

struct GenArgs {
  void* dst;
  int dtype;
  int64_t B, H, N, d, sb, sh, sn;
  uint64_t seed;
  uint32_t stream;
  int tensor_id;
  float mean, std;
  int grid_T, grid_lat, grid_lon;
  float amplitude;
  int64_t b_offset;
  int dshift;   // log2(d) when d is a power of two, else -1
  int wide;     // four consecutive elements may be stored as one vector
};

// Grid term of channel c, head h, token n (FP32).
__device__ __forceinline__ float structure(const GenArgs& a, int h, uint32_t n, uint32_t c) {
  const float kPi = 3.14159265358979f;
  const uint32_t nlon = (uint32_t)a.grid_lon, nlat = (uint32_t)a.grid_lat;
  const uint32_t j = n % nlon, i = (n / nlon) % nlat, t = n / (nlon * nlat);
  const float lat = kPi * (((float)i + 0.5f) / (float)nlat - 0.5f);
  const float lon = 2.0f * kPi * (float)j / (float)nlon;
  const float m = (float)(1 + c % 4), l = (float)(1 + c % 3);
  const float key = 0.6180339887f * (float)(a.tensor_id * (int)a.H * (int)a.d + h * (int)a.d + (int)c);
  const float psi = 2.0f * kPi * (key - floorf(key));
  return a.amplitude * sinf(m * lon + l * lat + 2.0f * kPi * (float)t / (float)a.grid_T + psi);
}

// Box-Muller of one pair of uniform words (FP32, every step rounded on its
// own: the file is built without contraction, like its host mirror).
// FAST (bfloat16 outputs): the hardware's single-instruction log2, square
// root, sine and cosine (v_sin/v_cos take revolutions, so their argument is
// u2 itself) in place of the math library's.  They differ from the library
// in the last bits of the FP32 value, which moves the bf16 rounding of
// about one value in 10^4 by one bf16 ulp; the generator runs about twice
// as fast, its cost being these functions and the Philox multiplies.
template <bool FAST>
__device__ __forceinline__ void box_muller(uint32_t w0, uint32_t w1, float& z0, float& z1) {
  const float u1 = ((float)(w0 >> 9) + 0.5f) * 0x1p-23f;
  if constexpr (FAST) {
    const float u2 = (float)(w1 >> 8) * 0x1p-24f;  // exact
    const float kMinus2Ln2 = -1.38629436111989f;   // -2 ln 2: -2 ln u1 = -2 ln2 log2 u1
    const float r = __builtin_amdgcn_sqrtf(kMinus2Ln2 * __builtin_amdgcn_logf(u1));
    z0 = r * __builtin_amdgcn_cosf(u2);
    z1 = r * __builtin_amdgcn_sinf(u2);
  } else {
    const float t = (float)(w1 >> 8) * 0x1p-23f;  // 2 u2, exact
    const float r = sqrtf(-2.0f * logf(u1));
    float s, c;
    sincospif(t, &s, &c);  // sin, cos of pi t = 2 pi u2 (no range reduction)
    z0 = r * c;
    z1 = r * s;
  }
}

// Element value: mean + std z, plus the grid term.
__device__ __forceinline__ float element(const GenArgs& a, int h, uint32_t n, uint32_t c, float z) {
  float val = a.mean + a.std * z;
  if (a.grid_T > 0) val += structure(a, h, n, c);
  return val;
}

// (token, channel) of element e of a head.
__device__ __forceinline__ void split(const GenArgs& a, uint32_t e, uint32_t& n, uint32_t& cc) {
  if (a.dshift >= 0) {
    n = e >> a.dshift;
    cc = e & ((uint32_t)a.d - 1u);
  } else {
    n = e / (uint32_t)a.d;
    cc = e - n * (uint32_t)a.d;
  }
}

// Store elements (e0, e0 + 1) of a head at token n, channel cc.
__device__ __forceinline__ void store_pair(const GenArgs& a, char* head, int h, uint32_t n,
                                           uint32_t cc, float z0, float z1) {
  const float f0 = element(a, h, n, cc, z0), f1 = element(a, h, n, cc + 1, z1);
  const int64_t off = (int64_t)n * a.sn + cc;
  if (a.dtype == 0) *(uint32_t*)((uint16_t*)head + off) = bf16_pair_rne(f0, f1);
  else *(float2*)((float*)head + off) = float2{f0, f1};
}

// Grid: y = (b, h) of the filled tensor, x strides over the head's element
// pairs.  Pair p of the logical tensor takes Philox block p >> 1 and its
// words (x0, x1) for even p, (x2, x3) for odd p; with d % 4 == 0 a thread
// makes both pairs of a block from one Philox call.  FAST: bf16 outputs.
template <bool FAST>
__global__ __launch_bounds__(256) void gen_kernel(GenArgs a) {
  const int64_t bh = blockIdx.y;
  const int64_t b = bh / a.H, h = bh % a.H;
  const uint32_t d = (uint32_t)a.d;
  const int64_t head_pairs = a.N * a.d / 2;
  const int64_t base = ((a.b_offset + b) * a.H + h) * head_pairs;  // logical pair index
  char* head = (char*)a.dst + (b * a.sb + h * a.sh) * (a.dtype == 0 ? 2 : 4);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if ((d & 3) == 0) {
    // base is even here (head_pairs is even), so blocks never straddle heads
    const int64_t head_quads = head_pairs / 2;
    for (int64_t ql = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ql < head_quads; ql += stride) {
      const uint64_t blk = (uint64_t)(base / 2 + ql);
      uint32_t c[4] = {(uint32_t)blk, (uint32_t)(blk >> 32), a.stream, 0u};
      philox4x32_10(c, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
      float z0, z1, z2, z3;
      box_muller<FAST>(c[0], c[1], z0, z1);
      box_muller<FAST>(c[2], c[3], z2, z3);
      const uint32_t e0 = (uint32_t)(4 * ql);  // element within the head (N * d < 2^32)
      uint32_t n, cc;
      split(a, e0, n, cc);
      if (a.wide) {
        // the four elements are consecutive in one row: one 8- or 16-byte store
        const float f0 = element(a, (int)h, n, cc, z0), f1 = element(a, (int)h, n, cc + 1, z1);
        const float f2 = element(a, (int)h, n, cc + 2, z2), f3 = element(a, (int)h, n, cc + 3, z3);
        const int64_t off = (int64_t)n * a.sn + cc;
        if (a.dtype == 0) {
          typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
          *(u32x2*)((uint16_t*)head + off) = u32x2{bf16_pair_rne(f0, f1), bf16_pair_rne(f2, f3)};
        } else {
          *(float4*)((float*)head + off) = float4{f0, f1, f2, f3};
        }
      } else {
        store_pair(a, head, (int)h, n, cc, z0, z1);
        store_pair(a, head, (int)h, n, cc + 2, z2, z3);
      }
    }
  } else {
    for (int64_t pl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pl < head_pairs; pl += stride) {
      const uint64_t lp = (uint64_t)(base + pl);
      const uint64_t blk = lp >> 1;
      uint32_t c[4] = {(uint32_t)blk, (uint32_t)(blk >> 32), a.stream, 0u};
      philox4x32_10(c, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
      float z0, z1;
      if (lp & 1) box_muller<FAST>(c[2], c[3], z0, z1);
      else box_muller<FAST>(c[0], c[1], z0, z1);
      const uint32_t e0 = (uint32_t)(2 * pl);
      uint32_t n, cc;
      split(a, e0, n, cc);
      store_pair(a, head, (int)h, n, cc, z0, z1);
    }
  }
}

}  // namespace

extern "C" int32_t la_gen_fill(void* dst, int32_t dtype, int64_t B, int64_t H, int64_t N,
                               int64_t d, int64_t sb, int64_t sh, int64_t sn,
                               const la_gen_spec* spec, void* stream) {
  if (!dst || !spec || (dtype != 0 && dtype != 1)) return 1;
  if (B < 1 || H < 1 || N < 1 || d < 2 || (d & 1)) return 1;
  if (B * H > 65535 || N * d >= (int64_t(1) << 32)) return 1;  // grid.y and 32-bit element index
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
  a.mean = (float)spec->mean; a.std = (float)spec->std;
  a.grid_T = spec->grid_T; a.grid_lat = spec->grid_lat; a.grid_lon = spec->grid_lon;
  a.amplitude = (float)spec->amplitude;
  a.b_offset = spec->b_offset;
  if (a.b_offset < 0) return 1;
  a.dshift = -1;
  for (int k = 0; k < 31; ++k)
    if ((int64_t(1) << k) == d) a.dshift = k;
  // four-element vectors stay aligned when every stride is a multiple of 4
  a.wide = (d % 4 == 0) && sb % 4 == 0 && sh % 4 == 0 && sn % 4 == 0;
  const int64_t head_pairs = N * d / 2;
  int64_t bx = (head_pairs + 255) / 256;
  const int64_t cap = std::max<int64_t>(1, 16384 / (B * H));  // ~16K blocks in total
  if (bx > cap) bx = cap;
  if (dtype == 0)
    hipLaunchKernelGGL(gen_kernel<true>, dim3((unsigned)bx, (unsigned)(B * H)), dim3(256), 0,
                       (hipStream_t)stream, a);
  else
    hipLaunchKernelGGL(gen_kernel<false>, dim3((unsigned)bx, (unsigned)(B * H)), dim3(256), 0,
                       (hipStream_t)stream, a);
  return hipGetLastError() == hipSuccess ? 0 : 4;
}
