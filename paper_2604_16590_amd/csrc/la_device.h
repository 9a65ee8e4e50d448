// la_device.h -- device helpers shared by the gfx950 kernels of liblinattn.
//
// Matrix-core conventions used throughout (16x16 MFMA tiles, 64 lanes):
//   lane l = 16*g + m, g = l >> 4 (lane group 0..3), m = l & 15.
//   v_mfma_f32_16x16x32_bf16: lane l supplies A[m][8g .. 8g+7] and
//     B[8g .. 8g+7][m]; the result D[4g + r][m], r = 0..3, lands in lane l.
//   v_mfma_f32_16x16x4_f32:   lane l supplies A[m][g] and B[g][m]; same D.
// The contraction index is only summed over, so any fixed assignment of
// contraction items (tokens or features) to (g, slot) is valid as long as A
// and B use the same one.  The kernels exploit this to keep every global
// load a contiguous run of a token's features.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace la {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

enum { DT_BF16 = 0, DT_FP32 = 1 };

__device__ __forceinline__ float bf16lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
__device__ __forceinline__ float bf16f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

typedef float f32x2 __attribute__((ext_vector_type(2)));

// Two floats -> packed bfloat16 pair (lo in bits 0..15), round to nearest
// even: one gfx950 v_cvt_pk_bf16_f32.
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  typedef __bf16 bf16v2 __attribute__((ext_vector_type(2)));
  const bf16v2 r = __builtin_convertvector(f32x2{lo, hi}, bf16v2);
  return __builtin_bit_cast(uint32_t, r);
}

// x + (sum of the two bfloat16 halves of w), exact products, FP32 sums.
__device__ __forceinline__ float add_bf16_pair(float x, uint32_t w) {
  return x + (bf16lo(w) + bf16hi(w));
}
__device__ __forceinline__ uint16_t to_bf16(float x) {
  return __builtin_bit_cast(uint16_t, (__bf16)x);
}

// Feature map phi(x) = elu(x) + 1 and its derivative, in FP32, with the
// hardware exp2 of x log2(e) for x <= 0: its error is the exp2's (about an
// ulp) plus the rounding of the product, |x| log2(e) 2^-24 relative (3e-7
// at x = -4), far below both the bf16 rounding and the fp32 path's 1e-5
// bound.  (The library expf cost the fp32 kernels 8 %: its range
// reduction is some 20 instructions per element.)
template <int DT>
__device__ __forceinline__ float phi(float x) {
  return x > 0.0f ? x + 1.0f : __expf(x);
}
template <int DT>
__device__ __forceinline__ float dphi(float x) {
  return x > 0.0f ? 1.0f : __expf(x);
}

// phi'(x) from phi(x): min(phi, 1) (phi = x + 1 > 1 for x > 0, and
// phi = exp(x) <= 1 = phi' otherwise).  phi >= 0, and non-negative floats
// order as their bit patterns do as unsigned integers, so one integer min
// gives it (fminf would canonicalise its operand first: two instructions).
__device__ __forceinline__ float dphi_of_phi(float ph) {
  return __uint_as_float(min(__float_as_uint(ph), 0x3f800000u));
}

__device__ __forceinline__ f32x4 mfma_bf16(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_f32(float a, float b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 as_bf16x8(const u32x4& w) {
  return __builtin_bit_cast(bf16x8, w);
}

// Index of the calling wave within its workgroup, as a wave-uniform value
// (scalar register), so that everything derived from it stays scalar.
__device__ __forceinline__ int wave_index() {
  return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

// Butterfly sum over the four lane groups (lanes m, m+16, m+32, m+48).
__device__ __forceinline__ double sum_groups(double x) {
  x += __shfl_xor(x, 16);
  x += __shfl_xor(x, 32);
  return x;
}
__device__ __forceinline__ float sum_groups(float x) {
  x += __shfl_xor(x, 16);
  x += __shfl_xor(x, 32);
  return x;
}

// Load `BYTES` contiguous bytes (2, 4, 8 or a multiple of 16) into 32-bit
// words, 16 bytes per load instruction where possible.
template <int BYTES>
__device__ __forceinline__ void load_words(const void* p, uint32_t* w) {
  if constexpr (BYTES >= 16) {
    static_assert(BYTES % 16 == 0, "unsupported width");
#pragma unroll
    for (int i = 0; i < BYTES / 16; ++i) {
      const u32x4 a = ((const u32x4*)p)[i];
      w[4 * i] = a.x; w[4 * i + 1] = a.y; w[4 * i + 2] = a.z; w[4 * i + 3] = a.w;
    }
  } else if constexpr (BYTES == 8) {
    u32x2 a = *(const u32x2*)p;
    w[0] = a.x; w[1] = a.y;
  } else if constexpr (BYTES == 4) {
    w[0] = *(const uint32_t*)p;
  } else {
    static_assert(BYTES == 2, "unsupported width");
    w[0] = *(const uint16_t*)p;
  }
}

// The same with the non-temporal hint: for data streamed exactly once (the
// summary's token ranges), which then does not displace reused lines in
// the caches; on gfx950 such read-only streams run measurably closer to
// the HBM peak.
template <int BYTES>
__device__ __forceinline__ void load_words_nt(const void* p, uint32_t* w) {
  if constexpr (BYTES >= 16) {
    static_assert(BYTES % 16 == 0, "unsupported width");
#pragma unroll
    for (int i = 0; i < BYTES / 16; ++i) {
      const u32x4 a = __builtin_nontemporal_load((const u32x4*)p + i);
      w[4 * i] = a.x; w[4 * i + 1] = a.y; w[4 * i + 2] = a.z; w[4 * i + 3] = a.w;
    }
  } else if constexpr (BYTES == 8) {
    const u32x2 a = __builtin_nontemporal_load((const u32x2*)p);
    w[0] = a.x; w[1] = a.y;
  } else if constexpr (BYTES == 4) {
    w[0] = __builtin_nontemporal_load((const uint32_t*)p);
  } else {
    static_assert(BYTES == 2, "unsupported width");
    w[0] = __builtin_nontemporal_load((const uint16_t*)p);
  }
}

template <int BYTES>
__device__ __forceinline__ void store_words(void* p, const uint32_t* w) {
  if constexpr (BYTES >= 16) {
#pragma unroll
    for (int i = 0; i < BYTES / 16; ++i)
      ((u32x4*)p)[i] = u32x4{w[4 * i], w[4 * i + 1], w[4 * i + 2], w[4 * i + 3]};
  } else if constexpr (BYTES == 8) {
    *(u32x2*)p = u32x2{w[0], w[1]};
  } else if constexpr (BYTES == 4) {
    *(uint32_t*)p = w[0];
  } else {
    static_assert(BYTES == 2, "unsupported width");
    *(uint16_t*)p = (uint16_t)w[0];
  }
}

// Element `f` of a run of words holding elements of type DT.
template <int DT>
__device__ __forceinline__ float word_elem(const uint32_t* w, int f) {
  if constexpr (DT == DT_BF16) return (f & 1) ? bf16hi(w[f >> 1]) : bf16lo(w[f >> 1]);
  else return __uint_as_float(w[f]);
}
template <int DT>
__device__ __forceinline__ uint16_t word_bits16(const uint32_t* w, int f) {
  return (uint16_t)((f & 1) ? (w[f >> 1] >> 16) : (w[f >> 1] & 0xffffu));
}

}  // namespace la
