/*
 * oracle.c -- plain FP64 CPU reference of kernelised linear global attention.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Written for a reader to check
 * against the definition by eye: every token sum is a plain loop in
 * increasing token order, in FP64.  Parallel loops only split work whose
 * results are independent (different heads, rows of S, tokens), so the
 * order of every individual sum is fixed.
 *
 * Definition followed (per batch b, head h):
 *   phi(x) = x + 1 (x > 0), exp(x) (x <= 0); phi'(x) = 1 (x > 0), exp(x).
 *   S = sum_j phi(k_j) v_j^T,  z = sum_j phi(k_j)
 *   den_i = phi(q_i) . z,  num_i = S^T phi(q_i),  O_i = num_i / den_i
 * Backward of L = sum_i G_i . O_i:
 *   dnum_i = G_i / den_i,  dden_i = -(G_i . O_i) / den_i
 *   dS = sum_i phi(q_i) dnum_i^T,  dz = sum_i dden_i phi(q_i)
 *   dQ_i = (S dnum_i + dden_i z) * phi'(q_i)
 *   dV_j = dS^T phi(k_j),  dK_j = (dS v_j + dz) * phi'(k_j)
 * The attention is global and non-causal: every query sees every key, as
 * the paper's spatial self-attention over all tokens of a frame sequence
 * requires (Sec. III-B).
 *
 * Pins: the paper prints no value of this computation, so every function
 * here is pinned to mathematics instead (tests/test_oracle*.py): the
 * brute-force quadratic form, a hand-derived example with exact rational
 * values, closed forms for degenerate inputs, invariances, central finite
 * differences and autograd of the quadratic form, and planted mistakes
 * that must each fail one of those pins.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Exact upcast of one stored element to FP64. */
static double elem(const oracle_tensor* t, int64_t b, int64_t h, int64_t n,
                   int64_t c) {
  int64_t idx = b * t->sb + h * t->sh + n * t->sn + c;
  if (t->dtype == ORACLE_BF16) {
    uint32_t u = (uint32_t)((const uint16_t*)t->ptr)[idx] << 16;
    float f;
    memcpy(&f, &u, sizeof f);
    return (double)f;
  }
  if (t->dtype == ORACLE_FP32) return (double)((const float*)t->ptr)[idx];
  return ((const double*)t->ptr)[idx];
}

double oracle_phi(double x) { return x > 0.0 ? x + 1.0 : exp(x); }
double oracle_dphi(double x) { return x > 0.0 ? 1.0 : exp(x); }

int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static int bad_args(int64_t B, int64_t H, int64_t N, int64_t d) {
  return B < 1 || H < 1 || N < 1 || d < 1;
}

/* Rows of S handled by one parallel task: a task owns rows [c0, c1) of one
 * head and walks all N keys in order, so each S[c][e] is one ordered sum. */
#define ROWS_PER_TASK 16

int oracle_summary(int64_t B, int64_t H, int64_t N, int64_t d,
                   oracle_tensor k, oracle_tensor v, double* S, double* z) {
  if (bad_args(B, H, N, d) || !S || !z) return -1;
  const int64_t nblk = (d + ROWS_PER_TASK - 1) / ROWS_PER_TASK;
  const int64_t ntask = B * H * nblk;
#pragma omp parallel
  {
    double* vrow = (double*)malloc(sizeof(double) * (size_t)d);
    double* phik = (double*)malloc(sizeof(double) * (size_t)d);
#pragma omp for schedule(dynamic, 1)
    for (int64_t task = 0; task < ntask; ++task) {
      const int64_t bh = task / nblk, blk = task % nblk;
      const int64_t b = bh / H, h = bh % H;
      const int64_t c0 = blk * ROWS_PER_TASK;
      const int64_t c1 = c0 + ROWS_PER_TASK < d ? c0 + ROWS_PER_TASK : d;
      double* Sh = S + bh * d * d;
      double* zh = z + bh * d;
      for (int64_t c = c0; c < c1; ++c) {
        zh[c] = 0.0;
        for (int64_t e = 0; e < d; ++e) Sh[c * d + e] = 0.0;
      }
      for (int64_t j = 0; j < N; ++j) {
        for (int64_t e = 0; e < d; ++e) vrow[e] = elem(&v, b, h, j, e);
        for (int64_t c = c0; c < c1; ++c) phik[c] = oracle_phi(elem(&k, b, h, j, c));
        for (int64_t c = c0; c < c1; ++c) {
          const double p = phik[c];
          double* Srow = Sh + c * d;
          for (int64_t e = 0; e < d; ++e) Srow[e] += p * vrow[e];
          zh[c] += p;
        }
      }
    }
    free(vrow);
    free(phik);
  }
  return 0;
}

int oracle_apply(int64_t B, int64_t H, int64_t N, int64_t d,
                 oracle_tensor q, const double* S, const double* z, double* o) {
  if (bad_args(B, H, N, d) || !S || !z || !o) return -1;
  const int64_t rows = B * H * N;
#pragma omp parallel
  {
    double* phiq = (double*)malloc(sizeof(double) * (size_t)d);
#pragma omp for schedule(static)
    for (int64_t r = 0; r < rows; ++r) {
      const int64_t bh = r / N, i = r % N;
      const int64_t b = bh / H, h = bh % H;
      const double* Sh = S + bh * d * d;
      const double* zh = z + bh * d;
      double* orow = o + r * d;
      double den = 0.0;
      for (int64_t c = 0; c < d; ++c) {
        phiq[c] = oracle_phi(elem(&q, b, h, i, c));
        den += phiq[c] * zh[c];
      }
      for (int64_t e = 0; e < d; ++e) {
        double num = 0.0;
        for (int64_t c = 0; c < d; ++c) num += phiq[c] * Sh[c * d + e];
        orow[e] = num / den;
      }
    }
    free(phiq);
  }
  return 0;
}

int oracle_forward(int64_t B, int64_t H, int64_t N, int64_t d,
                   oracle_tensor q, oracle_tensor k, oracle_tensor v,
                   double* o, double* S, double* z) {
  if (bad_args(B, H, N, d) || !o) return -1;
  double* Sb = S ? S : (double*)malloc(sizeof(double) * (size_t)(B * H * d * d));
  double* zb = z ? z : (double*)malloc(sizeof(double) * (size_t)(B * H * d));
  int rc = oracle_summary(B, H, N, d, k, v, Sb, zb);
  if (rc == 0) rc = oracle_apply(B, H, N, d, q, Sb, zb, o);
  if (!S) free(Sb);
  if (!z) free(zb);
  return rc;
}

/* Query side of the backward for one head: dnum_i and dden_i per query,
 * dS and dz (ordered sums over queries), and dQ.  dq may be NULL. */
static void backward_query_head(int64_t b, int64_t h, int64_t N, int64_t d,
                                const oracle_tensor* q, const oracle_tensor* g,
                                const double* S, const double* z, double* dS,
                                double* dz, double* dq) {
  /* Per query: dnum_i (d values) and dden_i, kept for the dS/dz sums. */
  double* dnum = (double*)malloc(sizeof(double) * (size_t)(N * d));
  double* dden = (double*)malloc(sizeof(double) * (size_t)N);

#pragma omp parallel
  {
    double* phiq = (double*)malloc(sizeof(double) * (size_t)d);
#pragma omp for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
      double den = 0.0;
      for (int64_t c = 0; c < d; ++c) {
        phiq[c] = oracle_phi(elem(q, b, h, i, c));
        den += phiq[c] * z[c];
      }
      double go = 0.0; /* G_i . O_i */
      for (int64_t e = 0; e < d; ++e) {
        double num = 0.0;
        for (int64_t c = 0; c < d; ++c) num += phiq[c] * S[c * d + e];
        const double gie = elem(g, b, h, i, e);
        go += gie * (num / den);
        dnum[i * d + e] = gie / den;
      }
      dden[i] = -go / den;
    }
    free(phiq);
  }

  /* dS and dz: one ordered sum over queries per entry; rows split. */
  const int64_t nblk = (d + ROWS_PER_TASK - 1) / ROWS_PER_TASK;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t blk = 0; blk < nblk; ++blk) {
    const int64_t c0 = blk * ROWS_PER_TASK;
    const int64_t c1 = c0 + ROWS_PER_TASK < d ? c0 + ROWS_PER_TASK : d;
    for (int64_t c = c0; c < c1; ++c) {
      dz[c] = 0.0;
      for (int64_t e = 0; e < d; ++e) dS[c * d + e] = 0.0;
    }
    for (int64_t i = 0; i < N; ++i) {
      for (int64_t c = c0; c < c1; ++c) {
        const double p = oracle_phi(elem(q, b, h, i, c));
        for (int64_t e = 0; e < d; ++e) dS[c * d + e] += p * dnum[i * d + e];
        dz[c] += dden[i] * p;
      }
    }
  }

  /* dQ_i = (S dnum_i + dden_i z) * phi'(q_i). */
  if (dq) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
      for (int64_t c = 0; c < d; ++c) {
        double acc = 0.0;
        for (int64_t e = 0; e < d; ++e) acc += S[c * d + e] * dnum[i * d + e];
        acc += dden[i] * z[c];
        dq[i * d + c] = acc * oracle_dphi(elem(q, b, h, i, c));
      }
    }
  }
  free(dnum);
  free(dden);
}

/* Key side of the backward for one head, given dS and dz. */
static void backward_key_head(int64_t b, int64_t h, int64_t N, int64_t d,
                              const oracle_tensor* k, const oracle_tensor* v,
                              const double* dS, const double* dz, double* dk,
                              double* dv) {
  /* dV_j = dS^T phi(k_j);  dK_j = (dS v_j + dz) * phi'(k_j). */
#pragma omp parallel
  {
    double* phik = (double*)malloc(sizeof(double) * (size_t)d);
    double* vrow = (double*)malloc(sizeof(double) * (size_t)d);
#pragma omp for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
      for (int64_t c = 0; c < d; ++c) phik[c] = oracle_phi(elem(k, b, h, j, c));
      for (int64_t e = 0; e < d; ++e) vrow[e] = elem(v, b, h, j, e);
      for (int64_t e = 0; e < d; ++e) {
        double acc = 0.0;
        for (int64_t c = 0; c < d; ++c) acc += phik[c] * dS[c * d + e];
        dv[j * d + e] = acc;
      }
      for (int64_t c = 0; c < d; ++c) {
        double acc = 0.0;
        for (int64_t e = 0; e < d; ++e) acc += dS[c * d + e] * vrow[e];
        acc += dz[c];
        dk[j * d + c] = acc * oracle_dphi(elem(k, b, h, j, c));
      }
    }
    free(phik);
    free(vrow);
  }
}

int oracle_backward_query(int64_t B, int64_t H, int64_t N, int64_t d,
                          oracle_tensor q, oracle_tensor g, const double* S,
                          const double* z, double* dq, double* dS, double* dz) {
  if (bad_args(B, H, N, d) || !S || !z || !dS || !dz) return -1;
  for (int64_t bh = 0; bh < B * H; ++bh)
    backward_query_head(bh / H, bh % H, N, d, &q, &g, S + bh * d * d, z + bh * d,
                        dS + bh * d * d, dz + bh * d, dq ? dq + bh * N * d : NULL);
  return 0;
}

int oracle_backward_key(int64_t B, int64_t H, int64_t N, int64_t d,
                        oracle_tensor k, oracle_tensor v, const double* dS,
                        const double* dz, double* dk, double* dv) {
  if (bad_args(B, H, N, d) || !dS || !dz || !dk || !dv) return -1;
  for (int64_t bh = 0; bh < B * H; ++bh)
    backward_key_head(bh / H, bh % H, N, d, &k, &v, dS + bh * d * d, dz + bh * d,
                      dk + bh * N * d, dv + bh * N * d);
  return 0;
}

int oracle_backward(int64_t B, int64_t H, int64_t N, int64_t d,
                    oracle_tensor q, oracle_tensor k, oracle_tensor v,
                    oracle_tensor g, double* dq, double* dk, double* dv,
                    double* dS, double* dz) {
  if (bad_args(B, H, N, d) || !dq || !dk || !dv) return -1;
  double* S = (double*)malloc(sizeof(double) * (size_t)(B * H * d * d));
  double* z = (double*)malloc(sizeof(double) * (size_t)(B * H * d));
  double* dSb = dS ? dS : (double*)malloc(sizeof(double) * (size_t)(B * H * d * d));
  double* dzb = dz ? dz : (double*)malloc(sizeof(double) * (size_t)(B * H * d));
  int rc = oracle_summary(B, H, N, d, k, v, S, z);
  if (rc == 0) rc = oracle_backward_query(B, H, N, d, q, g, S, z, dq, dSb, dzb);
  if (rc == 0) rc = oracle_backward_key(B, H, N, d, k, v, dSb, dzb, dk, dv);
  free(S);
  free(z);
  if (!dS) free(dSb);
  if (!dz) free(dzb);
  return rc;
}

/* ---- tiles with halos and Hann-weighted overlap averaging ------------- */

double oracle_hann(int64_t u, int64_t L) {
  const double pi = 3.14159265358979323846;
  const double sn = sin(pi * ((double)u + 0.5) / (double)L);
  return sn * sn;
}

static int tile_args_bad(const int64_t* dims, const int64_t* core, const int64_t* halo,
                         int64_t C) {
  if (C < 1) return 1;
  for (int k = 0; k < 3; ++k)
    if (dims[k] < 1 || core[k] < 1 || halo[k] < 0 || halo[k] > core[k]) return 1;
  return 0;
}

static int64_t ceil_div64(int64_t a, int64_t b) { return (a + b - 1) / b; }

static int64_t clamp64(int64_t v, int64_t lo, int64_t hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

int oracle_tile_extract(const int64_t* dims, const int64_t* core, const int64_t* halo,
                        int64_t C, const double* x, double* tiles) {
  if (tile_args_bad(dims, core, halo, C) || !x || !tiles) return -1;
  int64_t n[3], L[3];
  for (int k = 0; k < 3; ++k) {
    n[k] = ceil_div64(dims[k], core[k]);
    L[k] = core[k] + 2 * halo[k];
  }
  const int64_t tile_elems = L[0] * L[1] * L[2] * C;
#pragma omp parallel for schedule(static)
  for (int64_t tile = 0; tile < n[0] * n[1] * n[2]; ++tile) {
    const int64_t a = tile / (n[1] * n[2]), i = (tile / n[2]) % n[1], j = tile % n[2];
    double* dst = tiles + tile * tile_elems;
    for (int64_t ut = 0; ut < L[0]; ++ut)
      for (int64_t uy = 0; uy < L[1]; ++uy)
        for (int64_t ux = 0; ux < L[2]; ++ux) {
          const int64_t gt = clamp64(a * core[0] - halo[0] + ut, 0, dims[0] - 1);
          const int64_t gy = clamp64(i * core[1] - halo[1] + uy, 0, dims[1] - 1);
          const int64_t gx = clamp64(j * core[2] - halo[2] + ux, 0, dims[2] - 1);
          const double* src = x + ((gt * dims[1] + gy) * dims[2] + gx) * C;
          double* d = dst + ((ut * L[1] + uy) * L[2] + ux) * C;
          for (int64_t c = 0; c < C; ++c) d[c] = src[c];
        }
  }
  return 0;
}

int oracle_tile_blend(const int64_t* dims, const int64_t* core, const int64_t* halo,
                      int64_t C, const double* tiles, double* out) {
  if (tile_args_bad(dims, core, halo, C) || !tiles || !out) return -1;
  int64_t n[3], L[3];
  for (int k = 0; k < 3; ++k) {
    n[k] = ceil_div64(dims[k], core[k]);
    L[k] = core[k] + 2 * halo[k];
  }
  const int64_t tile_elems = L[0] * L[1] * L[2] * C;
  const int64_t npos = dims[0] * dims[1] * dims[2];
  double* wsum = (double*)calloc((size_t)npos, sizeof(double));
  for (int64_t p = 0; p < npos * C; ++p) out[p] = 0.0;
  /* every tile adds w * D into the positions it covers, tiles in order */
  for (int64_t tile = 0; tile < n[0] * n[1] * n[2]; ++tile) {
    const int64_t a = tile / (n[1] * n[2]), i = (tile / n[2]) % n[1], j = tile % n[2];
    const double* src = tiles + tile * tile_elems;
    for (int64_t ut = 0; ut < L[0]; ++ut) {
      const int64_t gt = a * core[0] - halo[0] + ut;
      if (gt < 0 || gt >= dims[0]) continue;
      for (int64_t uy = 0; uy < L[1]; ++uy) {
        const int64_t gy = i * core[1] - halo[1] + uy;
        if (gy < 0 || gy >= dims[1]) continue;
        for (int64_t ux = 0; ux < L[2]; ++ux) {
          const int64_t gx = j * core[2] - halo[2] + ux;
          if (gx < 0 || gx >= dims[2]) continue;
          const double w = oracle_hann(ut, L[0]) * oracle_hann(uy, L[1]) * oracle_hann(ux, L[2]);
          const int64_t p = (gt * dims[1] + gy) * dims[2] + gx;
          const double* d = src + ((ut * L[1] + uy) * L[2] + ux) * C;
          for (int64_t c = 0; c < C; ++c) out[p * C + c] += w * d[c];
          wsum[p] += w;
        }
      }
    }
  }
  for (int64_t p = 0; p < npos; ++p)
    for (int64_t c = 0; c < C; ++c) out[p * C + c] /= wsum[p];
  free(wsum);
  return 0;
}

/* ------------------------------------------------------------------------
 * Noise-gated mixing (Sec. III-B).  The spatial weight is the logistic
 * function of -(ln sigma - ln sigma_data), written as the ratio it equals;
 * sigma = 0 gives 1 and sigma = +inf gives 0.
 * ---------------------------------------------------------------------- */
double oracle_noise_gate(double sigma, double sigma_data) {
  return sigma_data / (sigma_data + sigma);
}

int oracle_gated_mix(int64_t B, int64_t H, int64_t N, int64_t d, const double* a,
                     oracle_tensor other, const double* sigma, double sigma_data, double* out) {
  if (B < 1 || H < 1 || N < 0 || d < 1 || !a || !sigma || !out || !(sigma_data > 0.0)) return -1;
  for (int64_t b = 0; b < B; ++b) {
    const double g = oracle_noise_gate(sigma[b], sigma_data);
    for (int64_t h = 0; h < H; ++h)
      for (int64_t n = 0; n < N; ++n)
        for (int64_t c = 0; c < d; ++c) {
          const int64_t i = ((b * H + h) * N + n) * d + c;
          out[i] = g * a[i] + (1.0 - g) * elem(&other, b, h, n, c);
        }
  }
  return 0;
}
