/*
 * la_gen.h -- C ABI of liblagen.so, the seeded synthetic-input generator.
 *
 * This library holds no attention arithmetic.  It materialises the inputs
 * that stand in for the paper's ERA5/HRRR token tensors (Sec. IV) directly
 * in device memory, so that benchmarks and the serving loop can make
 * multi-gigabyte inputs without a host round trip.  The host module
 * paper_2604_16590_amd/inputs.py implements the same definition:
 *
 *  - Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011).  Element e of the
 *    logical [b_offset + B, H, N, d] tensor (row-major flat index; the
 *    filled tensor is its batches b_offset .. b_offset + B - 1) is in pair
 *    p = e >> 1, which uses Philox block c = p >> 1: counter
 *    (lo32(c), hi32(c), stream, 0), key (lo32(seed), hi32(seed)), and of the
 *    block's output words (w0, w1) = (x0, x1) for even p, (x2, x3) for odd p.
 *  - u1 = ((w0 >> 9) + 0.5) * 2^-23, u2 = (w1 >> 8) * 2^-24 (exact in
 *    FP32); Box-Muller in FP32: r = sqrt(-2 ln u1); with t = 2 pi u2 even e
 *    takes r cos t, odd e takes r sin t, cos t and sin t rounded to FP32
 *    (evaluated as cospi/sinpi of 2 u2, exact in FP32).
 *  - value = mean + std * normal (+ grid structure when grid_T > 0):
 *    token n = (t*n_lat + i)*n_lon + j; channel c of tensor `tensor_id`
 *    and head h adds amplitude * sin(m_c lon_j + l_c lat_i + 2 pi t/T + psi)
 *    with lat_i = pi((i + 1/2)/n_lat - 1/2), lon_j = 2 pi j/n_lon,
 *    m_c = 1 + c mod 4, l_c = 1 + c mod 3,
 *    psi = 2 pi frac(0.6180339887 (tensor_id*H*d + h*d + c)).
 *    The paper's temporal-scaling runs use 32 x 64 patch grids per frame
 *    (Sec. IV, Table of maximal sequence lengths).
 *  - All of it in FP32 (mean + std * normal + grid term), then (for
 *    bfloat16) float32 -> bfloat16 round to nearest even.
 * Transcendentals may differ from the host's in the last bits, so the two
 * generators agree to within a few FP32 ulps (one bf16 rounding).  For
 * bfloat16 outputs the device takes the hardware's single-instruction
 * log2, sqrt, sin and cos (a few FP32 ulps from the library functions), so
 * about one value in 10^4 lands one bf16 ulp from the host's.
 * Limits: B*H <= 65535, N*d < 2^32.
 */
#ifndef LA_GEN_H
#define LA_GEN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  uint64_t seed;
  uint32_t stream;   /* 0 = Q, 1 = K, 2 = V, 3 = upstream gradient, ... */
  int32_t tensor_id; /* index in the structure phase */
  double mean, std;
  int32_t grid_T, grid_lat, grid_lon; /* grid_T = 0: no structure */
  double amplitude;
  int64_t b_offset;  /* first logical batch index of the filled tensor */
} la_gen_spec;

/*
 * Fill dst (device pointer, 16-byte aligned) with the logical [B,H,N,d]
 * tensor, dtype 0 = bfloat16 or 1 = float32, element strides (sb, sh, sn)
 * with the feature axis contiguous.  Asynchronous on `stream` (hipStream_t,
 * NULL = null stream).  Returns 0 on success, 1 on a bad argument, 4 when
 * the launch fails.  When grid_T > 0, N must equal grid_T*grid_lat*grid_lon.
 */
int32_t la_gen_fill(void* dst, int32_t dtype, int64_t B, int64_t H, int64_t N,
                    int64_t d, int64_t sb, int64_t sh, int64_t sn,
                    const la_gen_spec* spec, void* stream);

#ifdef __cplusplus
}
#endif
#endif
