/*
 * la.h -- C ABI of liblinattn.so: kernelised linear global attention on one
 * MI355X (gfx950).
 *
 * The operation.  The paper's denoiser runs global, non-causal attention
 * over a K-frame x N-patch spatiotemporal token sequence at every layer
 * (Sec. II-C for the token layout; Sec. III-B for spatial self-attention
 * and temporal cross-attention), and asks that global attention cost grow
 * linearly with the token count (Sec. III-C).  This library computes that
 * attention in kernelised form.  Per batch b and head h, with
 * phi(x) = elu(x) + 1 (x + 1 for x > 0, exp(x) otherwise):
 *     S   = sum_j phi(k_j) v_j^T      d x d summary
 *     z   = sum_j phi(k_j)            normaliser
 *     O_i = phi(q_i)^T S / (phi(q_i) . z)
 * so the cost is O(N d^2) per head instead of O(N^2 d).  The paper fixes
 * bfloat16 mixed precision (Sec. III-D); here bfloat16 inputs feed the
 * matrix cores with FP32 accumulation, per-tile sums are combined across
 * tiles in FP64, and the final division by the normaliser is FP64.
 *
 * Conventions shared by every entry point:
 *  - Every function returns la_status; none throws, aborts or exits.
 *    Output parameters are written only when LA_OK is returned.
 *  - Tensor pointers are DEVICE pointers owned by the caller.  The library
 *    never frees them and keeps no reference after the call returns.
 *  - Compute calls are asynchronous: arguments are checked synchronously
 *    (errors returned at once, nothing enqueued), then kernels are enqueued
 *    on `stream` and the call returns.  Faults inside kernels surface at
 *    the caller's next synchronisation with that stream.
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *  - Apart from the opt-in kernel timer (la_profile_*), the library holds no
 *    mutable global state; calls may come from several host threads.
 *  - Results are bitwise reproducible: tile sizes and the number of
 *    partial sums depend only on (N, d, dtype), and every cross-tile sum
 *    runs in a fixed order (no floating-point atomics).
 */
#ifndef LA_H
#define LA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LA_OK = 0,
  LA_ERR_INVALID_ARG = 1, /* null/misaligned pointer, bad size or stride   */
  LA_ERR_UNSUPPORTED = 2, /* valid request this build does not implement    */
  LA_ERR_OOM = 3,         /* workspace too small, or HBM budget exceeded    */
  LA_ERR_HIP = 4,         /* a HIP runtime call failed; see la_last_hip_error */
  LA_ERR_NOT_FOUND = 5,   /* unknown request id                             */
  LA_ERR_SHUTDOWN = 6,    /* server is shutting down                        */
  LA_ERR_BUSY = 7         /* resource temporarily unavailable               */
} la_status;

/* Element types. */
enum { LA_BF16 = 0, LA_FP32 = 1 };
/* Feature maps. */
enum { LA_PHI_ELU1 = 0 };

/*
 * Problem descriptor.
 *  B, H   batch (ensemble members) and heads, >= 1.
 *  N      tokens per (b, h), >= 1 (all keys are visible to all queries).
 *  d      head dimension: 16, 32, 64 or 128 (others: LA_ERR_UNSUPPORTED).
 *  in_dtype   type of Q, K, V and the upstream gradient dO.
 *  out_dtype  type of O and of the gradients dQ, dK, dV.
 *  in_s*  element strides (batch, head, token) of Q, K, V and dO; the
 *         feature axis is contiguous.  [B,H,N,d] contiguous is
 *         (H*N*d, N*d, d); a fused-projection [B,N,H,d] view is
 *         (N*H*d, d, H*d).
 *  out_s* element strides of O, dQ, dK and dV.
 *  Strides must be >= 0, in_sn/out_sn >= d, and every stride times the
 *  element size a multiple of 16 bytes; base pointers 16-byte aligned.
 */
typedef struct {
  int64_t B, H, N, d;
  int32_t in_dtype, out_dtype;
  int64_t in_sb, in_sh, in_sn;
  int64_t out_sb, out_sh, out_sn;
  int32_t feature_map; /* LA_PHI_ELU1 */
  uint32_t flags;      /* reserved, must be 0 */
} la_attn_desc;

typedef void* la_stream; /* hipStream_t */

/* Human-readable name of a status code (static string, never NULL). */
const char* la_status_string(la_status s);

/* The hipError_t of the most recent failed HIP call on this host thread
 * (0 if none). */
int32_t la_last_hip_error(void);

/* Library version. */
la_status la_version(int32_t* major, int32_t* minor);

/*
 * Device workspace the caller must provide for a pass (0 = forward,
 * 1 = backward), in bytes, 256-byte aligned.  The forward's size depends on
 * (B, H, d, dtype) and on N only through the number of per-tile partial
 * sums, which is capped, so it is bounded independently of N: the state of
 * linear attention per head is O(d^2), whatever the token count.  The
 * backward adds 8 bytes per (b, h, token) for the per-query pair
 * (1/den, dden) passed from its query pass to its dS reduction.
 */
la_status la_workspace_size(const la_attn_desc* desc, int32_t pass, size_t* bytes);

/*
 * Forward pass.  q, k, v: inputs (in_dtype, in strides); o: output
 * (out_dtype, out strides).  s_out [B][H][d][d] (row = key feature,
 * column = value feature) and z_out [B][H][d], both FP64 and dense, receive
 * the summary and normaliser when non-NULL; a backward pass needs them.
 * ws: device workspace of ws_bytes >= la_workspace_size(desc, 0).
 * The output must not overlap any input.
 */
la_status la_forward(const la_attn_desc* desc, const void* q, const void* k,
                     const void* v, void* o, double* s_out, double* z_out,
                     void* ws, size_t ws_bytes, la_stream stream);

/*
 * Backward pass of L = <O, dO>: writes (does not accumulate) dq, dk, dv in
 * out_dtype with the out strides.  s and z are the forward's s_out and
 * z_out for the same q, k, v.  phi(Q) and phi(K) are recomputed from the
 * inputs, never stored.  ws: ws_bytes >= la_workspace_size(desc, 1).
 * Gradients must not overlap any input.
 */
la_status la_backward(const la_attn_desc* desc, const void* q, const void* k,
                      const void* v, const double* s, const double* z,
                      const void* dout, void* dq, void* dk, void* dv, void* ws,
                      size_t ws_bytes, la_stream stream);

/*
 * Opt-in kernel timing.  la_profile_enable(1) clears earlier records and
 * makes every subsequent kernel launch of this library record a pair of
 * hipEvents around itself on its own stream; la_profile_enable(0) clears
 * and stops.  This is the one piece of process-wide mutable state of the
 * library (guarded by a mutex); it costs nothing while disabled.
 * la_profile_read() waits for the recorded events and returns, per kernel
 * name in first-launch order, the launch count and summed duration.  At most
 * `capacity` entries are written; *count receives the number available.
 */
typedef struct {
  char name[32];
  int64_t launches;
  double total_ms;
} la_kernel_stat;

la_status la_profile_enable(int32_t on);
la_status la_profile_read(la_kernel_stat* out, int32_t capacity, int32_t* count);

#ifdef __cplusplus
}
#endif
#endif /* LA_H */
