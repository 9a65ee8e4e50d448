// la_kernels.h -- launch arguments, operand-image layout and launcher
// declarations of the gfx950 kernels (internal to liblinattn).
#pragma once
#include "la_device.h"

namespace la {

// Lane runs of the row kernels (apply, query and key backward).  Lane
// (g, n) holds Q4 = d/4 features of token n: chunk w (CH features, 16 bytes
// of the input type) of lane group g is features [4*CH*w + CH*g, +CH), so
// one load or store instruction of the wave covers 4*CH contiguous features
// of each of its 16 tokens.  Run position c = CH*w + j <-> feature
// 4*CH*w + CH*g + j.
template <int D, int DT>
struct Run {
  static constexpr int ES = DT == DT_BF16 ? 2 : 4;
  static constexpr int Q4 = D / 4;
  static constexpr int CH = 16 / ES < Q4 ? 16 / ES : Q4;  // features per chunk
  static constexpr int NCH = Q4 / CH;                      // chunks per run
  static constexpr int CB = CH * ES;                       // bytes per chunk
  static __host__ __device__ constexpr int feature(int g, int c) {
    return (c / CH) * 4 * CH + g * CH + c % CH;
  }
  static __host__ __device__ constexpr int group(int f) { return (f % (4 * CH)) / CH; }
  static __host__ __device__ constexpr int pos(int f) { return (f / (4 * CH)) * CH + f % CH; }
};

// Load a lane's run (p = row start + CB * g) into words, chunk by chunk.
template <int D, int DT>
__device__ __forceinline__ void load_run(const char* p, uint32_t* w) {
  using R = Run<D, DT>;
  constexpr int CW = R::CB / 4;
#pragma unroll
  for (int c = 0; c < R::NCH; ++c) load_words<R::CB>(p + c * 4 * R::CB, w + c * CW);
}

// Store a lane's run of output values x[0..Q4) as type OT (p = row start +
// CH * sizeof(OT) * g), chunk by chunk; bf16 rounds to nearest even.
template <int D, int DT, int OT>
__device__ __forceinline__ void store_run(char* p, const float* x) {
  using R = Run<D, DT>;
  constexpr int OES = OT == DT_BF16 ? 2 : 4;
  constexpr int OCB = R::CH * OES;  // output bytes per chunk
  constexpr int OW = OCB / 4;
#pragma unroll
  for (int c = 0; c < R::NCH; ++c) {
    uint32_t ow[OW];
#pragma unroll
    for (int j = 0; j < R::CH; j += 2) {
      const float a = x[c * R::CH + j], b = x[c * R::CH + j + 1];
      if constexpr (OT == DT_BF16) {
        ow[j >> 1] = pack_bf16(a, b);
      } else {
        ow[j] = __float_as_uint(a);
        ow[j + 1] = __float_as_uint(b);
      }
    }
    store_words<OCB>(p + c * 4 * OCB, ow);
  }
}

// Load a lane's run of stored output values (type OT, the layout store_run
// writes; p = row start + CH * sizeof(OT) * g) as words; element c of the
// run is word_elem<OT>(w, c).
template <int D, int DT, int OT>
__device__ __forceinline__ void load_out_run(const char* p, uint32_t* w) {
  using R = Run<D, DT>;
  constexpr int OES = OT == DT_BF16 ? 2 : 4;
  constexpr int OCB = R::CH * OES;
  constexpr int OW = OCB / 4;
#pragma unroll
  for (int c = 0; c < R::NCH; ++c) load_words<OCB>(p + c * 4 * OCB, w + c * OW);
}

// Matrix-core operand images of a d x d matrix M (S or dS), per head:
//   T image: A[row = value feature e][k = key/query feature c] = M[c][e],
//            followed by a z tile: A[row = any of 16][k = c] = v[c] (the
//            normaliser z, or dz), whose product with phi(q) gives the
//            normaliser of every token in every output row
//   N image: A[row = key/query feature c][k = value feature e] = M[c][e]
// A 16-row output tile i maps row m = 4g + r to the feature at run
// position 4i + r of lane group g (Run above), so a lane's four result rows
// over all tiles are its run of output features.  The contraction index k
// maps to lane group Run::group(k) and run position Run::pos(k), matching
// how the B operand (one token per lane, a feature run per lane group) is
// loaded.  bf16 images store a hi part bf16(M) and a lo part bf16(M - hi);
// fp32 images store float(M).
template <int D>
struct ImageCfg {
  static constexpr int Q4 = D / 4;
  static constexpr int NT = D / 16;                  // output tiles
  static constexpr int NS = D >= 32 ? D / 32 : 1;    // bf16 k-steps of 32
  static constexpr int TILE_BF16 = NS * 2 * 64 * 16;  // one 16-row tile, hi + lo
  static constexpr int TILE_F32 = (Q4 / 4) * 64 * 16;
  static constexpr int tile_bytes(int dt) { return dt == DT_BF16 ? TILE_BF16 : TILE_F32; }
  // the NT matrix tiles of one image
  static constexpr int mat_bytes(int dt) { return NT * tile_bytes(dt); }
  // the T image: matrix tiles + z tile (the N image starts right after it)
  static constexpr int img_bytes(int dt) { return (NT + 1) * tile_bytes(dt); }
  static constexpr int head_bytes(int dt) { return img_bytes(dt) + mat_bytes(dt); }
};

// (word, slot) of element (tile i, row m, contraction index k).
template <int D>
__device__ __forceinline__ void tile_slot(int i, int m, int k, int& word, int& slot, int dt) {
  using IC = ImageCfg<D>;
  constexpr int Q4 = IC::Q4;
  if (dt == DT_BF16) {
    using R = Run<D, DT_BF16>;
    const int krem = R::pos(k);
    const int lane = 16 * R::group(k) + m;
    const int s = krem >> 3;
    slot = krem & 7;
    word = ((i * IC::NS + s) * 2) * 64 + lane;  // hi part; lo part is +64
  } else {
    using R = Run<D, DT_FP32>;
    const int krem = R::pos(k);
    const int lane = 16 * R::group(k) + m;
    slot = krem & 3;
    word = (i * (Q4 / 4) + (krem >> 2)) * 64 + lane;
  }
}

template <int D>
__device__ __forceinline__ void image_slot(int row, int k, int& word, int& slot, int dt) {
  int gq, rrem;
  if (dt == DT_BF16) {
    gq = Run<D, DT_BF16>::group(row);
    rrem = Run<D, DT_BF16>::pos(row);
  } else {
    gq = Run<D, DT_FP32>::group(row);
    rrem = Run<D, DT_FP32>::pos(row);
  }
  tile_slot<D>(rrem >> 2, 4 * gq + (rrem & 3), k, word, slot, dt);
}

// Store val (FP64) at (word, slot) of an image: hi/lo bf16 parts or fp32.
template <int D>
__device__ __forceinline__ void put_image(char* base, int word, int slot, int dt, double val) {
  if (dt == DT_BF16) {
    const uint16_t hi = to_bf16((float)val);
    const uint16_t lo = to_bf16((float)(val - (double)bf16f(hi)));
    uint16_t* wh = (uint16_t*)(base + (int64_t)word * 16);
    uint16_t* wl = (uint16_t*)(base + (int64_t)(word + 64) * 16);
    wh[slot] = hi;
    wl[slot] = lo;
    if (ImageCfg<D>::Q4 < 8) {  // d = 16: slots 4..7 of each k-step are padding
      wh[slot + 4] = 0;
      wl[slot + 4] = 0;
    }
  } else {
    ((float*)(base + (int64_t)word * 16))[slot] = (float)val;
  }
}

// Store M[c][e] = val into both images of head bh.
template <int D>
__device__ __forceinline__ void write_images(void* img, int dt, int bh, int c, int e, double val) {
  using IC = ImageCfg<D>;
  char* head = (char*)img + (int64_t)bh * IC::head_bytes(dt);
  for (int which = 0; which < 2; ++which) {
    const int row = which == 0 ? e : c;
    const int k = which == 0 ? c : e;
    int word, slot;
    image_slot<D>(row, k, word, slot, dt);
    put_image<D>(head + which * IC::img_bytes(dt), word, slot, dt, val);
  }
}

// Store v[c] = val into all 16 rows of the T image's z tile of head bh.
template <int D>
__device__ __forceinline__ void write_z_tile(void* img, int dt, int bh, int c, double val) {
  using IC = ImageCfg<D>;
  char* head = (char*)img + (int64_t)bh * IC::head_bytes(dt);
  for (int m = 0; m < 16; ++m) {
    int word, slot;
    tile_slot<D>(IC::NT, m, c, word, slot, dt);
    put_image<D>(head, word, slot, dt, val);
  }
}

struct FwdArgs {
  int64_t B, H, N;
  int D, in_dt, out_dt;
  int64_t sb, sh, sn, osb, osh, osn;
  const void *q, *k, *v;
  void* o;
  int P, Tw;           // partials per head, tokens per partial
  int Ga;              // apply workgroups per head (they take its token blocks in turn)
  float* part;         // [BH][P][D*D + D]
  double* S64;         // [BH][D][D]
  double* z64;         // [BH][D]
  void* img;           // [BH][2 images]
  // noise-gated mix (null `other`: plain output): o = g_b A + (1 - g_b) other,
  // g_b = sigma_data / (sigma_data + sigma[b])
  const void* other;   // output dtype and strides
  const double* sigma; // [B]
  double sigma_data;
  hipStream_t stream;
};

struct BwdArgs {
  int64_t B, H, N;
  int D, in_dt, out_dt;
  int64_t sb, sh, sn, osb, osh, osn;
  const void *q, *k, *v, *dout;
  void *dq, *dk, *dv;
  const double *S64, *z64;
  int P, Tw, Ta;       // Ta: tokens per workgroup of the two-pass query kernel
  int Gk;              // key-backward workgroups per head (they take its token blocks in turn)
  void* img;           // images of S
  float* part;         // partials of dS, dz
  float2* stash;       // [BH][N] per query token: (1/den, -(dO . O))
  double* dS64;
  double* dz64;
  void* dimg;          // images of dS
  hipStream_t stream;
};

enum { MODE_FWD = 0, MODE_BWD = 1 };
enum { PART_SUMMARY = 0, PART_BLOCKS = 1 };  // layouts of per-wave partial sums

// Keeps a failed hipError_t for la_last_hip_error(); returns LA_ERR_HIP.
int32_t record_hip_error(int32_t e);

hipError_t launch_forward(const FwdArgs& a);
// Apply only: images of a given S (into a.img), then the apply kernel.
hipError_t launch_apply(const FwdArgs& a);
// Token-reduction kernel: forward summary (MODE_FWD) or the dS/dz sums of
// the backward (MODE_BWD, k = Q, v = dO, stash = per-token (1/den, -(dO . O))).
hipError_t launch_summary(int mode, int dt, int D, const void* k, const void* v, int64_t sb,
                          int64_t sh, int64_t sn, int64_t B, int64_t H, int64_t N, int P,
                          int Tw, const float2* stash, float* part, hipStream_t stream);
hipError_t launch_combine(const float* part, int P, double* M64, double* v64, void* img,
                          int img_dt, int64_t BH, int D, int layout, hipStream_t stream);
hipError_t launch_backward(const BwdArgs& a);
// Images (both, with the z tile) of a given M and v.
hipError_t launch_images(const double* M64, const double* v64, void* img, int img_dt, int64_t BH,
                         int D, hipStream_t stream);

}  // namespace la
