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
  LA_ERR_UNSUPPORTED = 2, /* valid request the library does not implement   */
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
 *  A token stride above 16 MiB (in_sn or out_sn times the element size),
 *  N above 2^36 or B*H above 65535 is LA_ERR_UNSUPPORTED.
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
 * 1 = backward, 2 = apply), in bytes, 256-byte aligned.  It holds O(d^2)
 * per head (the FP64 summary and its matrix-core operand images) plus the
 * per-tile partial sums of the token reduction.  Each partial sums at most
 * 16,384 tokens (bf16 inputs; 4,096 for fp32) in FP32 before the partials
 * are added in FP64, so the FP32 part of every sum over tokens is bounded
 * whatever N is; the partial count is 128 (d = 128) or 64 (d < 128) until
 * that bound is reached (2,097,152 or 1,048,576 bf16 tokens per head) and
 * grows with N beyond it, by (d*d + d) * 4 bytes per 16,384 tokens per
 * head (0.8 % of the bytes of K and V at d = 128).  Where the backward runs
 * its query pass and its dS reduction separately (fp32 inputs, and
 * d = 16) it adds 8 bytes per (b, h, token) for the per-query pair
 * (1/den, dden) passed between them; bf16 at d >= 32 runs them as one pass
 * and needs no such buffer.
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
 * The forward pass for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): la_forward with its workspace taken from a fixed array of
 * LA_NOALLOC_SCRATCH_BYTES bytes that the library holds on each device
 * until the process ends, so the call itself allocates nothing.  Arguments
 * and results are those of la_forward (same kernels, so the same bits);
 * the array of the CURRENT device is used, and `stream` must belong to that
 * device.  LA_ERR_OOM when la_workspace_size(desc, 0) exceeds the array
 * (bf16 inputs: 8 heads at d = 128 fit up to 4,079,616 tokens each,
 * 64 heads at d = 64 up to 1,982,464; fp32 inputs, 8 heads at d = 128: up
 * to 1,019,904).  All calls on one device share its
 * array: calls whose work overlaps on the device (different streams, or
 * other host threads, without ordering between them) race on it and must
 * be serialised by the caller.
 */
#define LA_NOALLOC_SCRATCH_BYTES (128u << 20)
la_status la_forward_noalloc(const la_attn_desc* desc, const void* q, const void* k,
                             const void* v, void* o, double* s_out, double* z_out,
                             la_stream stream);

/*
 * Apply a given summary: O_i = phi(q_i)^T S / (phi(q_i) . z) for every query,
 * with S [B][H][d][d] and z [B][H][d] FP64 (dense) from an earlier
 * la_forward (s_out, z_out).  This is the per-step work when the keys and
 * values stay fixed while the queries change, as in the paper's temporal
 * cross-attention against a compressed history (Sec. III-B) evaluated at
 * every diffusion step (Sec. V, 80 steps per ensemble sample): the summary
 * is computed once and only Q is streamed.  Same conventions as
 * la_forward; ws_bytes >= la_workspace_size(desc, 2).
 */
la_status la_apply(const la_attn_desc* desc, const void* q, const double* s,
                   const double* z, void* o, void* ws, size_t ws_bytes, la_stream stream);

/*
 * Noise-gated mixing of two attention branches (Sec. III-B: each denoiser
 * layer weighs its spatial self-attention against its temporal
 * cross-attention by the diffusion noise level, leaning on the temporal
 * branch when the noise is high and on the spatial one when it is low).
 * The paper does not give the gate; this library reads it as a logistic
 * function of log noise centred on the EDM data scale sigma_data (the
 * paper's diffusion follows Karras et al., Sec. III-A):
 *     g_b   = sigma_data / (sigma_data + sigma[b])
 *           = 1 / (1 + exp(ln sigma[b] - ln sigma_data))     spatial weight
 *     out_i = g_b * A_i + (1 - g_b) * other_i
 * where A is the attention these calls compute (la_forward_gated: of
 * q, k, v; la_apply_gated: of q against a given S, z) and other is the
 * other branch's stored output.  g_b is 1 at sigma = 0 (out = A), 1/2 at
 * sigma = sigma_data and 0 at sigma = +inf (out = other).  The blend is
 * fused into the attention's output pass: other is read once, A is never
 * stored, and the cost over la_forward / la_apply is one more read of a
 * tensor of o's size.
 *
 * other: device, out_dtype with the out strides (the layout of o); it may
 * be o itself (in place), and must not otherwise overlap o.  sigma: device,
 * B FP64 noise levels, each >= 0 (+inf allowed); other values give
 * unspecified weights (never a fault).  sigma_data: host, finite, > 0
 * (EDM uses 0.5).  The remaining arguments and the workspace (pass 0 for
 * la_forward_gated, 2 for la_apply_gated) are those of la_forward and
 * la_apply.  Errors: LA_ERR_INVALID_ARG for a NULL or misaligned other or
 * sigma (16 and 8 bytes) or a bad sigma_data, then as la_forward/la_apply.
 */
la_status la_forward_gated(const la_attn_desc* desc, const void* q, const void* k,
                           const void* v, const void* other, const double* sigma,
                           double sigma_data, void* o, double* s_out, double* z_out,
                           void* ws, size_t ws_bytes, la_stream stream);
la_status la_apply_gated(const la_attn_desc* desc, const void* q, const double* s,
                         const double* z, const void* other, const double* sigma,
                         double sigma_data, void* o, void* ws, size_t ws_bytes,
                         la_stream stream);

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

/* ------------------------------------------------------------------------
 * Tiles with halos and window-weighted overlap averaging.
 *
 * The paper's own route to global context at linear cost (Sec. III-C):
 * the spatiotemporal token grid is cut into tiles, each extended by halos
 * that overlap its neighbours; every tile is processed on its own (here:
 * la_forward with the tiles as the batch); the outputs are averaged where
 * tiles overlap, each contribution weighted by a Hann window that trusts a
 * tile's centre more than its border.  Repeated at every diffusion step,
 * this lets context cross tile boundaries without all-to-all attention.
 *
 * Geometry: the field is [T][Y][X][C] (channels contiguous).  Tile cores of
 * (ct, cy, cx) tokens lie on a regular grid (ceil(T/ct) x ceil(Y/cy) x
 * ceil(X/cx) tiles, row-major), each extended by halos (ht, hy, hx) with
 * 0 <= halo <= core on every side, so a tile holds
 * L = (ct+2ht) x (cy+2hy) x (cx+2hx) tokens, stored [tile][Lt][Ly][Lx][C].
 *  - extract: tile values are the field at the covered positions, with
 *    coordinates clamped into the grid at its borders.
 *  - blend: out(p) = sum_tiles w(p) D_tile(p) / sum_tiles w(p) over the
 *    tiles covering p, w = prod over the three dims of sin^2(pi (u+1/2)/L)
 *    (u = coordinate within the tile); positions a tile covers outside the
 *    grid are ignored.  Consistent tiles blend back to the field exactly.
 * C must be a multiple of 8; the grid's y dimension limits (tiles, and
 * T*Y rows) to 65535 each.
 * ------------------------------------------------------------------------ */
typedef struct {
  int64_t dims[3];  /* T, Y, X */
  int64_t core[3];
  int64_t halo[3];
  int64_t C;
  int32_t dtype;    /* LA_BF16 or LA_FP32, field and tiles alike */
} la_tile_desc;

la_status la_tile_geometry(const la_tile_desc* desc, int64_t* n_tiles, int64_t* tile_tokens);
la_status la_tile_extract(const la_tile_desc* desc, const void* field, void* tiles,
                          la_stream stream);
la_status la_tile_blend(const la_tile_desc* desc, const void* tiles, void* field,
                        la_stream stream);

/*
 * The whole tiled attention step in two passes over the fields, with no
 * tile materialised: q, k, v, o are [T][Y][X][C] fields (C = heads * d
 * channels, head h in channels [h*d, h*d + d)), bf16, 16-byte aligned,
 * device, caller-owned.  The result is that of extracting the q, k, v
 * tiles, running la_forward with the tiles as the batch and blending the
 * tile outputs with la_tile_blend:
 *     o(p) = sum_t w_t(p) O_t(p) / sum_t w_t(p),
 *     O_t(p) = phi(q_p)^T S_t / (phi(q_p) . z_t),
 * S_t, z_t the summary over tile t's extended, border-clamped token set,
 * w_t the tile's Hann weight at p -- except that the tile outputs O_t are
 * kept in FP32 instead of being rounded to bf16, and S_t enters as its bf16
 * hi part (about 2^-9 relative; z_t as hi + lo).  Pass 1 reads K and V in
 * place, walking each (y, x) segment pair of the tiles' extended ranges
 * along t so that a token shared by neighbouring tiles is mapped once per
 * segment pair; it sums in FP32 runs of at most 16,384 tokens, adds a
 * tile's runs in FP64 in a fixed order (results are bitwise reproducible)
 * and keeps per (tile, head) only S_t, z_t as matrix-core operands; pass 2
 * reads Q once and writes O once.  Requirements beyond la_tile_desc's:
 * dtype LA_BF16, d = C / heads in {16, 32, 64}, 2 * halo <= core in every
 * dimension (then each position lies in at most two tiles per dimension),
 * at most 65,536 tokens per extended tile and 16,384 along t (core[0] +
 * 2 * halo[0]), fewer than 2^31 tokens per field; otherwise
 * LA_ERR_UNSUPPORTED.  The
 * Hann weights use the hardware sine and the divisions by den and by the
 * weight sum the hardware reciprocal (about 1e-6 relative, far below the
 * bf16 rounding of o).
 * ws: ws_bytes >= la_tiled_workspace_size(desc, heads), 256-byte aligned
 * (per head: one operand slot per tile, and n_t (2 n_y + 1)(2 n_x + 1)
 * FP32 column sums of d^2 + d floats, times the footprint parts when a
 * segment pair's run would exceed 16,384 tokens; n_* tiles per dimension).
 */
la_status la_tiled_workspace_size(const la_tile_desc* desc, int64_t heads, size_t* bytes);
la_status la_tiled_forward(const la_tile_desc* desc, int64_t heads, const void* q, const void* k,
                           const void* v, void* o, void* ws, size_t ws_bytes, la_stream stream);

/* ------------------------------------------------------------------------
 * Serving: a continuous-batching request loop for ensemble members.
 *
 * The paper generates large posterior ensembles, one member per sampler,
 * each running the denoiser (and its attention) at every diffusion step
 * (Sec. V, large-scale ensemble generation, 80 diffusion steps).  Requests
 * here are attention calls of one ensemble batch (B members sharing N, H,
 * d).  The server:
 *  - queues requests FIFO and splits each into member slices;
 *  - admits the next slice of the oldest request when a slot is free and
 *    the slice's device memory fits the free HBM budget; by default a
 *    request never overtakes an older one, while with
 *    max_slices_per_request a request holding that many slots leaves the
 *    free ones to the next requests in arrival order;
 *  - runs each slice (optional input generation, summary, combine, apply)
 *    on one of its HIP streams, so slices of different requests overlap on
 *    the GPU;
 *  - keeps each request's FP64 summary S and normaliser z (and, for
 *    generated inputs, the output O) in device memory until the client
 *    releases the request.
 * Member results do not depend on how a request is sliced or what else
 * runs: tiling depends only on (N, d, dtype), so a request computes the
 * same bits alone and in a mix.
 * ------------------------------------------------------------------------ */
typedef struct la_server la_server;

typedef struct {
  int32_t device;                 /* HIP device ordinal */
  uint64_t hbm_budget_bytes;      /* device memory the server may hold at once */
  int32_t max_slots;              /* slices in flight at once, >= 1 */
  int32_t n_streams;              /* HIP streams the slices rotate over, >= 1 */
  int32_t max_members_per_slice;  /* 0 = as many as fit */
  int32_t fake_executor;          /* test hook: 1 = no GPU work, slices finish
                                     fake_slice_ns after launch (budget, FIFO
                                     and slicing logic only) */
  int64_t fake_slice_ns;
  int32_t max_slices_per_request; /* 0 = strict FIFO: the oldest request takes
                                     every slot and as much budget as it can;
                                     k > 0 = a request holds at most k slots and
                                     each of its slices at most budget/max_slots
                                     bytes (one member at least), and when it
                                     holds k the next requests in arrival order
                                     are served, so a long request does not
                                     hold back the short ones behind it */
} la_server_config;

typedef struct {
  la_attn_desc desc;     /* B = members; H, N, d, dtypes; strides as for la_forward */
  const void* q;         /* caller-owned device inputs and output, kept alive by */
  const void* k;         /* the caller until the request is DONE or FAILED;      */
  const void* v;         /* all NULL when generate = 1                           */
  void* o;
  int32_t generate;      /* 1: the server allocates Q, K, V, O in its budget and
                            fills Q, K, V with the seeded generator (streams 0, 1,
                            2 of gen_seed, N(0, gen_std^2)); desc strides are then
                            ignored ([B,H,N,d] contiguous) */
  uint64_t gen_seed;
  double gen_std;
  uint64_t t_arrival_ns; /* scheduled arrival on CLOCK_MONOTONIC; 0 = at submit */
  uint64_t reuse_summary_of; /* 0: compute S, z of this request's keys and
                            values (the forward).  Otherwise the id of an
                            earlier, not yet released request of this server
                            with the same B, H, d and in_dtype (N may differ):
                            this request applies its own queries against that
                            request's S and z (la_apply) -- the per-step work
                            of temporal cross-attention against a fixed
                            history (Sec. III-B) over an ensemble member's
                            diffusion steps (Sec. V).  k and v must be NULL;
                            with generate = 1 only Q is generated (stream 0 of
                            gen_seed).  It starts once that request is DONE
                            and FAILs with its error if it FAILED; while it is
                            pending, releasing that request returns
                            LA_ERR_BUSY.  Errors at submit: LA_ERR_NOT_FOUND
                            (unknown id), LA_ERR_INVALID_ARG (a request that
                            itself reuses, one that FAILED, or a mismatch). */
} la_request;

enum { LA_REQ_QUEUED = 0, LA_REQ_RUNNING = 1, LA_REQ_DONE = 2, LA_REQ_FAILED = 3 };

typedef struct {
  int32_t state;          /* LA_REQ_* */
  la_status error;        /* why it FAILED */
  uint64_t t_arrival_ns, t_admit_ns, t_done_ns;  /* CLOCK_MONOTONIC */
  int32_t slices;         /* member slices the request was split into */
  void* o;                /* output (server-owned for generated requests) */
  double* s;              /* [B][H][d][d] FP64 summary, server-owned (NULL
                             for a request that reuses another's) */
  double* z;              /* [B][H][d]    FP64 normaliser, server-owned (idem) */
  double gen_ms;          /* device time generating inputs, summed over slices */
  double attn_ms;         /* device time of the attention, summed over slices */
} la_result;

typedef struct {
  uint64_t submitted, completed, failed, rejected;
  int64_t queued, in_flight_slices;
  uint64_t bytes_in_use, peak_bytes_in_use, budget_bytes;
} la_serve_counters;

/* Create a server (allocates its budget on `device` and starts its
 * scheduler thread).  Errors: LA_ERR_INVALID_ARG, LA_ERR_OOM, LA_ERR_HIP. */
la_status la_serve_create(const la_server_config* cfg, la_server** out);
/* Stop accepting work, cancel queued requests (FAILED, LA_ERR_SHUTDOWN),
 * wait for slices in flight, free everything. */
la_status la_serve_destroy(la_server* srv);
/* Non-blocking.  LA_ERR_OOM when even a one-member slice cannot fit the
 * budget; LA_ERR_SHUTDOWN during destroy; argument errors as la_forward. */
la_status la_serve_submit(la_server* srv, const la_request* req, uint64_t* id);
/* Non-blocking snapshot.  LA_ERR_NOT_FOUND for unknown or released ids. */
la_status la_serve_poll(la_server* srv, uint64_t id, la_result* out);
/* Free a finished request's device memory (S, z, generated O).
 * LA_ERR_BUSY while it is queued or running, or while requests reusing its
 * summary are pending. */
la_status la_serve_release(la_server* srv, uint64_t id);
la_status la_serve_stats(la_server* srv, la_serve_counters* out);
/* Test hook: slice `slice` (0-based) of request `id` fails instead of
 * running, as a device-side failure would. */
la_status la_serve_debug_fail_slice(la_server* srv, uint64_t id, int32_t slice);
/* Test hook: slice `slice` of request `id` fails after its inputs are on
 * its stream (generated, or its start recorded), before the attention, as
 * a launch failing midway would; its memory stays held until the work
 * already enqueued has drained. */
la_status la_serve_debug_fail_slice_late(la_server* srv, uint64_t id, int32_t slice);
/* Test hook: while paused (1) the scheduler admits nothing; slices already
 * in flight still finish.  0 resumes. */
la_status la_serve_debug_pause(la_server* srv, int32_t paused);

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

/*
 * Plain HBM streams, the ceilings the attention kernels' rates are read
 * against: each kernel of the method is bound by HBM traffic with a fixed
 * mix of reads and writes, and these measure what a kernel of the same mix
 * reaches on the device (grid-stride loops over 16-byte words).
 *  kind   LA_STREAM_READ: reads `bytes` of src; dst receives at most 16
 *         bytes of unspecified content (a sink that keeps the loads live).
 *         LA_STREAM_WRITE: fills `bytes` of dst with the 32-bit `pattern`
 *         (src unused, may be NULL).
 *         LA_STREAM_COPY: copies `bytes` from src to dst (no overlap).
 *  bytes  > 0, a multiple of 16; device pointers 16-byte aligned, owned by
 *         the caller.  Violations are LA_ERR_INVALID_ARG, checked before
 *         anything is enqueued; the call is asynchronous on `stream` and is
 *         timed by the kernel timer as stream_read / stream_write /
 *         stream_copy.
 */
enum { LA_STREAM_READ = 0, LA_STREAM_WRITE = 1, LA_STREAM_COPY = 2 };
la_status la_stream_probe(int32_t kind, const void* src, void* dst, size_t bytes,
                          uint32_t pattern, la_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* LA_H */
