// la_api.cpp -- the C ABI of liblinattn (include/la.h): argument checks,
// tiling choices, workspace layout and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>

#include "../../include/la.h"
#include "la_kernels.h"

namespace {

thread_local int32_t g_last_hip_error = 0;

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

la_status hip_fail(hipError_t e) {
  g_last_hip_error = (int32_t)e;
  return LA_ERR_HIP;
}

int elem_size(int32_t dt) { return dt == LA_BF16 ? 2 : 4; }

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

la_status check_desc(const la_attn_desc* d) {
  if (!d) return LA_ERR_INVALID_ARG;
  if (d->B < 1 || d->H < 1 || d->N < 1 || d->d < 1) return LA_ERR_INVALID_ARG;
  if (d->in_dtype != LA_BF16 && d->in_dtype != LA_FP32) return LA_ERR_INVALID_ARG;
  if (d->out_dtype != LA_BF16 && d->out_dtype != LA_FP32) return LA_ERR_INVALID_ARG;
  if (d->feature_map != LA_PHI_ELU1) return LA_ERR_UNSUPPORTED;
  if (d->flags != 0) return LA_ERR_INVALID_ARG;
  if (d->d != 16 && d->d != 32 && d->d != 64 && d->d != 128) return LA_ERR_UNSUPPORTED;
  // the grid's y dimension carries (b, h); token indices are 64-bit, while
  // partials (N / 4096 at most) and workgroups along x (N / 2048 at most)
  // are counted in 32 bits
  if (d->B * d->H > 65535 || d->N > (int64_t(1) << 36)) return LA_ERR_UNSUPPORTED;
  const int64_t s[2][3] = {{d->in_sb, d->in_sh, d->in_sn}, {d->out_sb, d->out_sh, d->out_sn}};
  const int es[2] = {elem_size(d->in_dtype), elem_size(d->out_dtype)};
  for (int t = 0; t < 2; ++t) {
    for (int i = 0; i < 3; ++i) {
      if (s[t][i] < 0) return LA_ERR_INVALID_ARG;
      if ((s[t][i] * es[t]) % 16 != 0) return LA_ERR_INVALID_ARG;
    }
    if (s[t][2] < d->d) return LA_ERR_INVALID_ARG;
    // kernels address 32 consecutive token rows with 32-bit lane offsets
    if (s[t][2] * es[t] > (int64_t(1) << 24)) return LA_ERR_UNSUPPORTED;
  }
  return LA_OK;
}

// Tiling.  Depends only on (N, d, dtype) so that the same (b, h) problem
// gives bitwise the same result whatever batch it is part of.
struct Tiling {
  int P;   // partial sums per (b, h)
  int Tw;  // tokens per partial (a multiple of 64, at most max_fp32_run)
  int Tk;  // tokens per workgroup of the key (and two-pass query) backward
};

// The longest token range any kernel sums in FP32: each partial sum covers
// at most this many tokens, and partials are added in FP64 (the combine),
// so the FP32 part of every sum over tokens is bounded whatever N is.
// The fp32 path, which is held to a tighter tolerance, takes shorter runs.
int64_t max_fp32_run(int dt) { return dt == LA_BF16 ? 16384 : 4096; }

Tiling choose_tiling(int64_t N, int d, int dt) {
  // at least 2048 (d = 128) or 512 tokens per partial: the 16,384-token
  // grid shape (64 heads, d = 64) gave 0.151 / 0.146 / 0.159 ms for its
  // cache-flushed forward at 1024 / 512 / 256
  const int64_t tw_min = d >= 128 ? 2048 : 512;
  // at most 128 partials at d = 128 and 64 below while that keeps each
  // FP32 run within max_fp32_run: longer ranges per wave paid off at d = 64
  // (summary of 32 heads x 262,144 tokens 0.38 -> 0.33 ms), while 8 heads
  // at d = 128 need the 128 to give each SIMD a wave.  Beyond that the
  // partial count grows with N (about (d^2 + d) * 4 bytes of workspace per
  // max_fp32_run tokens per head: 0.8 % of the inputs' bytes at d = 128).
  const int64_t p_max = d >= 128 ? 128 : 64;
  int64_t P = std::min<int64_t>(p_max, ceil_div(N, tw_min));
  P = std::max<int64_t>(P, ceil_div(N, max_fp32_run(dt)));
  // a multiple of 64: the summary steps over 32 tokens, the fused
  // backward over 64 (four waves x 16); max_fp32_run is one too, so
  // rounding up keeps Tw <= max_fp32_run
  int64_t Tw = ceil_div(ceil_div(N, P), 64) * 64;
  P = ceil_div(N, Tw);
  Tiling t;
  t.P = (int)P;
  t.Tw = (int)Tw;
  // per-token kernels: no cross-token sums, so these ranges change no bits
  // (measured: the key backward is fastest at 2048 tokens per workgroup)
  t.Tk = (int)std::min<int64_t>(2048, ceil_div(N, 64) * 64);
  return t;
}

// Apply workgroups per head: about kApplyGrid in the whole grid (a few per
// compute unit), at most one per token block.  Per-token work, so this
// changes no bits and may depend on the batch size.
int apply_groups(int64_t N, int64_t BH, int dt, int d) {
  const int64_t blk = dt == LA_FP32 && d >= 128 ? 64 : 128;  // tokens per block
  const int64_t grid = 4096;
  int64_t ga = std::min(ceil_div(N, blk), ceil_div(grid, BH));
  // while the grid keeps 2048 workgroups or more, at least four blocks per
  // workgroup: each workgroup stages the operand images first, and at
  // 16,384 tokens x 64 heads (d = 64) 32 workgroups per head took 58 us
  // against 60 us for 64 (16: 60 us)
  ga = std::min(ga, std::max(ceil_div(N, 4 * blk), ceil_div(2048, BH)));
  return (int)std::max<int64_t>(1, ga);
}

// Bytes of the two matrix-core operand images of one head.
size_t head_image_bytes(int D, int dt) {
  const int idt = dt == LA_BF16 ? la::DT_BF16 : la::DT_FP32;
  switch (D) {
    case 16: return la::ImageCfg<16>::head_bytes(idt);
    case 32: return la::ImageCfg<32>::head_bytes(idt);
    case 64: return la::ImageCfg<64>::head_bytes(idt);
    default: return la::ImageCfg<128>::head_bytes(idt);
  }
}

struct Layout {
  size_t part, S64, z64, img, stash, dS64, dz64, dimg, total;
};

// Forward: [part][S64][z64][img].  Apply: [img].
// Backward: [img][part][stash][dS64][dz64][dimg]; the stash holds two floats
// per query token (1/den, -(dO . O)) between the query kernel and the dS
// reduction, the only part of any workspace that grows with N.  bf16 at
// d >= 32 fuses the two passes and needs no stash.
bool fused_backward(const la_attn_desc* d) { return d->in_dtype == LA_BF16 && d->d >= 32; }

Layout layout_for(const la_attn_desc* d, int pass) {
  const int64_t BH = d->B * d->H, D = d->d;
  const Tiling t = choose_tiling(d->N, (int)D, d->in_dtype);
  const size_t part = align_up((size_t)BH * t.P * (D * D + D) * sizeof(float));
  const size_t mat = align_up((size_t)BH * D * D * sizeof(double));
  const size_t vec = align_up((size_t)BH * D * sizeof(double));
  const size_t img = align_up((size_t)BH * head_image_bytes((int)D, d->in_dtype));
  Layout L{};
  size_t off = 0;
  if (pass == 2) {
    L.img = off; off += img;
  } else if (pass == 0) {
    L.part = off; off += part;
    L.S64 = off; off += mat;
    L.z64 = off; off += vec;
    L.img = off; off += img;
  } else {
    L.img = off; off += img;
    L.part = off; off += part;
    L.stash = off;
    if (!fused_backward(d)) off += align_up((size_t)BH * d->N * 2 * sizeof(float));
    L.dS64 = off; off += mat;
    L.dz64 = off; off += vec;
    L.dimg = off; off += img;
  }
  L.total = off;
  return L;
}

// The gate's arguments (the attention's own are checked by the caller).
// Key-backward workgroups per head, as apply_groups (the fp32 path at
// d = 128 takes one tile per wave step, like the apply).
int key_groups(int64_t N, int64_t BH, int dt, int d) {
  const int64_t blk = dt == LA_FP32 ? 64 : 128;  // tokens per block (4 waves x 16 x TT)
  int64_t grid = 8192;
  return (int)std::max<int64_t>(1, std::min(ceil_div(N, blk), ceil_div(grid, BH)));
}

la_status check_gate(const void* other, const double* sigma, double sigma_data) {
  if (!other || !sigma) return LA_ERR_INVALID_ARG;
  if (!aligned16(other) || ((uintptr_t)sigma & 7u)) return LA_ERR_INVALID_ARG;
  if (!(sigma_data > 0.0) || !std::isfinite(sigma_data)) return LA_ERR_INVALID_ARG;
  return LA_OK;
}

la_status forward_impl(const la_attn_desc* desc, const void* q, const void* k, const void* v,
                       void* o, double* s_out, double* z_out, void* ws, size_t ws_bytes,
                       la_stream stream, const void* other, const double* sigma,
                       double sigma_data) {
  la_status st = check_desc(desc);
  if (st != LA_OK) return st;
  if (!q || !k || !v || !o || !ws) return LA_ERR_INVALID_ARG;
  if (!aligned16(q) || !aligned16(k) || !aligned16(v) || !aligned16(o)) return LA_ERR_INVALID_ARG;
  if (((uintptr_t)ws % kAlign) != 0) return LA_ERR_INVALID_ARG;
  if (((uintptr_t)s_out & 7u) || ((uintptr_t)z_out & 7u)) return LA_ERR_INVALID_ARG;
  const Layout L = layout_for(desc, 0);
  if (ws_bytes < L.total) return LA_ERR_OOM;
  const Tiling t = choose_tiling(desc->N, (int)desc->d, desc->in_dtype);
  char* w = (char*)ws;
  la::FwdArgs a{};
  a.B = desc->B; a.H = desc->H; a.N = desc->N; a.D = (int)desc->d;
  a.in_dt = desc->in_dtype; a.out_dt = desc->out_dtype;
  a.sb = desc->in_sb; a.sh = desc->in_sh; a.sn = desc->in_sn;
  a.osb = desc->out_sb; a.osh = desc->out_sh; a.osn = desc->out_sn;
  a.q = q; a.k = k; a.v = v; a.o = o;
  a.P = t.P; a.Tw = t.Tw;
  a.Ga = apply_groups(desc->N, desc->B * desc->H, desc->in_dtype, (int)desc->d);
  a.part = (float*)(w + L.part);
  a.S64 = s_out ? s_out : (double*)(w + L.S64);
  a.z64 = z_out ? z_out : (double*)(w + L.z64);
  a.img = w + L.img;
  a.other = other; a.sigma = sigma; a.sigma_data = sigma_data;
  a.stream = (hipStream_t)stream;
  hipError_t e = la::launch_forward(a);
  if (e != hipSuccess) return hip_fail(e);
  return LA_OK;
}

la_status apply_impl(const la_attn_desc* desc, const void* q, const double* s, const double* z,
                     void* o, void* ws, size_t ws_bytes, la_stream stream, const void* other,
                     const double* sigma, double sigma_data) {
  la_status st = check_desc(desc);
  if (st != LA_OK) return st;
  if (!q || !s || !z || !o || !ws) return LA_ERR_INVALID_ARG;
  if (!aligned16(q) || !aligned16(o)) return LA_ERR_INVALID_ARG;
  if (((uintptr_t)s & 7u) || ((uintptr_t)z & 7u)) return LA_ERR_INVALID_ARG;
  if (((uintptr_t)ws % kAlign) != 0) return LA_ERR_INVALID_ARG;
  const Layout L = layout_for(desc, 2);
  if (ws_bytes < L.total) return LA_ERR_OOM;
  const Tiling t = choose_tiling(desc->N, (int)desc->d, desc->in_dtype);
  la::FwdArgs a{};
  a.B = desc->B; a.H = desc->H; a.N = desc->N; a.D = (int)desc->d;
  a.in_dt = desc->in_dtype; a.out_dt = desc->out_dtype;
  a.sb = desc->in_sb; a.sh = desc->in_sh; a.sn = desc->in_sn;
  a.osb = desc->out_sb; a.osh = desc->out_sh; a.osn = desc->out_sn;
  a.q = q; a.o = o;
  a.Ga = apply_groups(desc->N, desc->B * desc->H, desc->in_dtype, (int)desc->d);
  a.S64 = const_cast<double*>(s);
  a.z64 = const_cast<double*>(z);
  a.img = (char*)ws + L.img;
  a.other = other; a.sigma = sigma; a.sigma_data = sigma_data;
  a.stream = (hipStream_t)stream;
  hipError_t e = la::launch_apply(a);
  if (e != hipSuccess) return hip_fail(e);
  return LA_OK;
}

}  // namespace

namespace la {
// A failed HIP call seen outside this file: kept for la_last_hip_error().
int32_t record_hip_error(int32_t e) {
  g_last_hip_error = e;
  return LA_ERR_HIP;
}
}  // namespace la

extern "C" {

const char* la_status_string(la_status s) {
  switch (s) {
    case LA_OK: return "LA_OK";
    case LA_ERR_INVALID_ARG: return "LA_ERR_INVALID_ARG";
    case LA_ERR_UNSUPPORTED: return "LA_ERR_UNSUPPORTED";
    case LA_ERR_OOM: return "LA_ERR_OOM";
    case LA_ERR_HIP: return "LA_ERR_HIP";
    case LA_ERR_NOT_FOUND: return "LA_ERR_NOT_FOUND";
    case LA_ERR_SHUTDOWN: return "LA_ERR_SHUTDOWN";
    case LA_ERR_BUSY: return "LA_ERR_BUSY";
  }
  return "LA_ERR_UNKNOWN";
}

int32_t la_last_hip_error(void) { return g_last_hip_error; }

la_status la_version(int32_t* major, int32_t* minor) {
  if (!major || !minor) return LA_ERR_INVALID_ARG;
  *major = 1;
  *minor = 0;
  return LA_OK;
}

la_status la_workspace_size(const la_attn_desc* desc, int32_t pass, size_t* bytes) {
  if (!bytes || pass < 0 || pass > 2) return LA_ERR_INVALID_ARG;
  la_status st = check_desc(desc);
  if (st != LA_OK) return st;
  *bytes = layout_for(desc, pass).total;
  return LA_OK;
}

la_status la_forward(const la_attn_desc* desc, const void* q, const void* k,
                     const void* v, void* o, double* s_out, double* z_out,
                     void* ws, size_t ws_bytes, la_stream stream) {
  return forward_impl(desc, q, k, v, o, s_out, z_out, ws, ws_bytes, stream, nullptr, nullptr, 0.0);
}

la_status la_forward_gated(const la_attn_desc* desc, const void* q, const void* k,
                           const void* v, const void* other, const double* sigma,
                           double sigma_data, void* o, double* s_out, double* z_out,
                           void* ws, size_t ws_bytes, la_stream stream) {
  const la_status st = check_gate(other, sigma, sigma_data);
  if (st != LA_OK) return st;
  return forward_impl(desc, q, k, v, o, s_out, z_out, ws, ws_bytes, stream, other, sigma,
                      sigma_data);
}

la_status la_apply(const la_attn_desc* desc, const void* q, const double* s,
                   const double* z, void* o, void* ws, size_t ws_bytes, la_stream stream) {
  return apply_impl(desc, q, s, z, o, ws, ws_bytes, stream, nullptr, nullptr, 0.0);
}

la_status la_apply_gated(const la_attn_desc* desc, const void* q, const double* s,
                         const double* z, const void* other, const double* sigma,
                         double sigma_data, void* o, void* ws, size_t ws_bytes,
                         la_stream stream) {
  const la_status st = check_gate(other, sigma, sigma_data);
  if (st != LA_OK) return st;
  return apply_impl(desc, q, s, z, o, ws, ws_bytes, stream, other, sigma, sigma_data);
}

la_status la_backward(const la_attn_desc* desc, const void* q, const void* k,
                      const void* v, const double* s, const double* z,
                      const void* dout, void* dq, void* dk, void* dv, void* ws,
                      size_t ws_bytes, la_stream stream) {
  la_status st = check_desc(desc);
  if (st != LA_OK) return st;
  if (!q || !k || !v || !s || !z || !dout || !dq || !dk || !dv || !ws) return LA_ERR_INVALID_ARG;
  for (const void* p : {q, k, v, dout, (const void*)dq, (const void*)dk, (const void*)dv})
    if (!aligned16(p)) return LA_ERR_INVALID_ARG;
  if (((uintptr_t)s & 7u) || ((uintptr_t)z & 7u)) return LA_ERR_INVALID_ARG;
  if (((uintptr_t)ws % kAlign) != 0) return LA_ERR_INVALID_ARG;
  const Layout L = layout_for(desc, 1);
  if (ws_bytes < L.total) return LA_ERR_OOM;
  const Tiling t = choose_tiling(desc->N, (int)desc->d, desc->in_dtype);
  char* w = (char*)ws;
  la::BwdArgs a{};
  a.B = desc->B; a.H = desc->H; a.N = desc->N; a.D = (int)desc->d;
  a.in_dt = desc->in_dtype; a.out_dt = desc->out_dtype;
  a.sb = desc->in_sb; a.sh = desc->in_sh; a.sn = desc->in_sn;
  a.osb = desc->out_sb; a.osh = desc->out_sh; a.osn = desc->out_sn;
  a.q = q; a.k = k; a.v = v; a.dout = dout;
  a.dq = dq; a.dk = dk; a.dv = dv;
  a.S64 = s; a.z64 = z;
  a.P = t.P; a.Tw = t.Tw; a.Ta = t.Tk;
  a.Gk = key_groups(desc->N, desc->B * desc->H, desc->in_dtype, (int)desc->d);
  a.img = w + L.img;
  a.part = (float*)(w + L.part);
  a.stash = (float2*)(w + L.stash);
  a.dS64 = (double*)(w + L.dS64);
  a.dz64 = (double*)(w + L.dz64);
  a.dimg = w + L.dimg;
  a.stream = (hipStream_t)stream;
  hipError_t e = la::launch_backward(a);
  if (e != hipSuccess) return hip_fail(e);
  return LA_OK;
}

}  // extern "C"
