/*
 * oracle.h -- plain FP64 CPU reference of kernelised linear global attention.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this code; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code with the HIP library.
 *
 * What it computes (per batch b and head h, with phi applied elementwise):
 *   phi(x)  = x + 1     for x > 0
 *           = exp(x)    for x <= 0         (elu(x) + 1)
 *   S       = sum_j phi(k_j) v_j^T          (d x d summary)
 *   z       = sum_j phi(k_j)                (normaliser, d-vector)
 *   O_i     = phi(q_i)^T S / (phi(q_i) . z)
 * and the exact gradients of L = <O, G> with respect to Q, K, V.
 *
 * The paper places a global, non-causal attention over the K x N
 * spatiotemporal tokens at every denoiser layer (Sec. III-B, spatial
 * self-attention and temporal cross-attention), and says that its
 * global attention must be linear in the token count (Sec. III-C).  It
 * prints no feature map; elu+1 is the reading adopted here (Katharopoulos
 * et al., 2020), which keeps the summary exactly d x d and the normaliser
 * strictly positive.
 *
 * Inputs are read exactly as the GPU sees them: bfloat16 bit patterns
 * (uint16), float32 or float64, upcast to FP64 without rounding.  Every
 * floating-point operation below is FP64.  All sums over tokens run in
 * increasing token order, so results do not depend on the thread count.
 *
 * Tensor addressing: element (b, h, n, c) of an input lives at
 *   base[b*sb + h*sh + n*sn + c]                       (element strides)
 * Outputs are dense FP64: O/dQ/dK/dV as [B][H][N][d], S as [B][H][d][d]
 * (row = key feature c, column = value feature e), z as [B][H][d].
 */
#ifndef LA_ORACLE_H
#define LA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_BF16 = 0, ORACLE_FP32 = 1, ORACLE_FP64 = 2 };

typedef struct {
  const void* ptr;
  int32_t dtype;       /* ORACLE_BF16 / ORACLE_FP32 / ORACLE_FP64 */
  int64_t sb, sh, sn;  /* element strides; the feature stride is 1 */
} oracle_tensor;

/* Feature map and its derivative. */
double oracle_phi(double x);
double oracle_dphi(double x);

/* S and z per (b, h).  Returns 0, or -1 on a bad argument. */
int oracle_summary(int64_t B, int64_t H, int64_t N, int64_t d,
                   oracle_tensor k, oracle_tensor v, double* S, double* z);

/* O from Q and a given (S, z) per (b, h). */
int oracle_apply(int64_t B, int64_t H, int64_t N, int64_t d,
                 oracle_tensor q, const double* S, const double* z, double* o);

/* summary followed by apply; S and z may be NULL when not wanted. */
int oracle_forward(int64_t B, int64_t H, int64_t N, int64_t d,
                   oracle_tensor q, oracle_tensor k, oracle_tensor v,
                   double* o, double* S, double* z);

/* Gradients of L = <O, G>.  dq, dk, dv are dense [B][H][N][d]; dS and dz
 * ([B][H][d][d], [B][H][d]) may be NULL. */
int oracle_backward(int64_t B, int64_t H, int64_t N, int64_t d,
                    oracle_tensor q, oracle_tensor k, oracle_tensor v,
                    oracle_tensor g, double* dq, double* dk, double* dv,
                    double* dS, double* dz);

/* The two halves of oracle_backward.  Query side: from Q, G and the
 * forward's S, z, the sums dS, dz over the given queries and (dq non-NULL)
 * dQ of those queries.  Key side: dK, dV of the given keys from dS, dz.
 * dQ rows depend only on (S, z, q_i, g_i) and dK/dV rows only on
 * (dS, dz, k_j, v_j), so both may be evaluated on a subset of rows. */
int oracle_backward_query(int64_t B, int64_t H, int64_t N, int64_t d,
                          oracle_tensor q, oracle_tensor g, const double* S,
                          const double* z, double* dq, double* dS, double* dz);
int oracle_backward_key(int64_t B, int64_t H, int64_t N, int64_t d,
                        oracle_tensor k, oracle_tensor v, const double* dS,
                        const double* dz, double* dk, double* dv);

/*
 * Tiles with halos and window-weighted overlap averaging (the paper's
 * global propagation step, Sec. III-C).  A global field X [T][Y][X][C]
 * (channels contiguous, FP64) is covered by tiles whose cores (ct, cy, cx)
 * lie on a regular grid and which extend by halos (ht, hy, hx) <= the core
 * on every side.  Tile (a, i, j) in row-major order covers positions
 * [a ct - ht, (a+1) ct + ht) x [i cy - hy, ...) x [j cx - hx, ...); its
 * array is [Lt][Ly][Lx][C] with L = core + 2 halo.
 *  extract: tile value at a local position = X at the global position,
 *           with coordinates clamped into the domain.
 *  blend:   out(p) = sum_tiles w(p) D(p) / sum_tiles w(p) over the tiles
 *           covering p, w = product over dims of sin^2(pi (u + 1/2) / L)
 *           (Hann window at cell centres, u the local coordinate).
 * Dimensions: dims[0..2] = (T, Y, X), core[0..2], halo[0..2], C.
 */
int oracle_tile_extract(const int64_t* dims, const int64_t* core, const int64_t* halo,
                        int64_t C, const double* x, double* tiles);
int oracle_tile_blend(const int64_t* dims, const int64_t* core, const int64_t* halo,
                      int64_t C, const double* tiles, double* out);
double oracle_hann(int64_t u, int64_t L);

/*
 * Noise-gated mixing of two attention branches (Sec. III-B: the denoiser
 * weighs spatial self-attention against temporal cross-attention by the
 * diffusion noise level sigma, more temporal at high noise, more spatial at
 * low noise).  The paper gives no formula; the reading adopted is a
 * logistic function of log noise centred on the EDM data scale sigma_data
 * (the diffusion follows Karras et al., Sec. III-A):
 *   g(sigma) = 1 / (1 + exp(ln sigma - ln sigma_data))
 *            = sigma_data / (sigma_data + sigma)        (spatial weight)
 *   out     = g(sigma_b) * A + (1 - g(sigma_b)) * other  per batch element b
 * oracle_gated_mix: a is dense FP64 [B][H][N][d] (this branch's attention,
 * e.g. from oracle_forward), other is read like an input (its stored
 * dtype and strides), sigma has B entries; out is dense FP64.
 */
double oracle_noise_gate(double sigma, double sigma_data);
int oracle_gated_mix(int64_t B, int64_t H, int64_t N, int64_t d, const double* a,
                     oracle_tensor other, const double* sigma, double sigma_data, double* out);

/* Number of OpenMP threads the oracle will use. */
int oracle_threads(void);

#ifdef __cplusplus
}
#endif
#endif
