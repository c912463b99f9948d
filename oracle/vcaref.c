/*
 * vcaref.c -- TEST INFRASTRUCTURE ONLY: the plain CPU oracle of the VCA
 * features (Menon et al., GMSys 2023, Section 2).  Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no code
 * with the HIP library.
 *
 * The paper names the seven features of Section 2 (E_Y, h, L_Y, E_U, E_V,
 * L_U, L_V) and its low-pass DCT option (Section 2, optimisation (3)); their
 * formulas live in the VCA paper it cites, which is not reproduced here.  The
 * readings taken for what the paper leaves open are:
 *   - blocks: non-overlapping w x w blocks anchored at (0,0), only complete
 *     blocks counted, on Y and on each 4:2:0 chroma plane;
 *   - transform: the H.265 integer core-transform matrix C_w, applied as a
 *     horizontal pass T = floor((X C_w^T + 2^(s1-1)) / 2^s1) followed by a
 *     vertical pass Y = floor((C_w T + 2^(s2-1)) / 2^s2), with
 *     s1 = log2 w + B - 9 and s2 = log2 w + 6 on raw samples of bit depth B;
 *   - low-pass K: only the top-left K x K coefficients are computed, with the
 *     weights of the w x w transform;
 *   - block energy H = sum over (i,j) != (0,0), i,j < K of W_ij |Y(i,j)| with
 *     W_ij = exp(|((i+1)(j+1)/w^2)^2 - 1|);
 *   - block brightness sqrt(DC), DC = Y(0,0);
 *   - per frame: E_P = sum H / (C_P w^2), L_P = sum sqrt(DC) / (C_P w^2),
 *     h = sum |H_p - H_{p-1}| / (C_Y w^2) over luma, and h = 0 for the first
 *     frame.
 * Everything is written out in plain loops: int64 for the transform, double
 * for the features, sums taken sequentially in block raster order.
 */
#include "vcaref.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* Magnitudes of the 32-point integer DCT basis at angle a, i.e. the integer
 * stand-in for 64*sqrt(2)*cos(pi*a/64), a = 1..31 (H.265 core transform). */
static const int32_t kMag[32] = {0,  90, 90, 90, 89, 88, 87, 85, 83, 82, 80,
                                 78, 75, 73, 70, 67, 64, 61, 57, 54, 50, 46,
                                 43, 38, 36, 31, 25, 22, 18, 13, 9,  4};

/* Entry (k, n) of the 32-point matrix: row 0 is flat (64); for k > 0 the
 * angle k(2n+1) is folded into [0, 64] with the symmetries of the cosine. */
static int32_t c32(int k, int n) {
  if (k == 0) return 64;
  int a = (k * (2 * n + 1)) % 128;
  if (a > 64) a = 128 - a;       /* cos(pi a/64) = cos(pi (128 - a)/64) */
  if (a < 32) return kMag[a];
  if (a == 32) return 0;         /* does not occur for 0 < k < 32 */
  return -kMag[64 - a];          /* cos(pi a/64) = -cos(pi (64 - a)/64) */
}

static int valid_w(int32_t w) { return w == 4 || w == 8 || w == 16 || w == 32; }

static int ilog2(int32_t w) {
  int s = 0;
  while ((1 << s) < w) s++;
  return s;
}

/* floor(v / 2^s), written without relying on the sign behaviour of >>. */
static int64_t floor_div_pow2(int64_t v, int s) {
  int64_t d = (int64_t)1 << s;
  int64_t q = v / d;
  if (v % d != 0 && v < 0) q -= 1;
  return q;
}

int vcaref_dct_matrix(int32_t w, int32_t* out) {
  if (!valid_w(w) || !out) return VCAREF_EINVAL;
  /* The w-point matrix is the 32-point one sampled at every (32/w)-th row. */
  for (int k = 0; k < w; k++)
    for (int n = 0; n < w; n++) out[k * w + n] = c32(k * (32 / w), n);
  return 0;
}

int vcaref_weights(int32_t w, double* out) {
  if (!valid_w(w) || !out) return VCAREF_EINVAL;
  for (int i = 0; i < w; i++)
    for (int j = 0; j < w; j++) {
      double r = (double)((i + 1) * (j + 1)) / (double)(w * w);
      out[i * w + j] = exp(fabs(r * r - 1.0));
    }
  return 0;
}

/* Transform of one block: x is w x w (int64 scratch copy), y is K x K. */
static void transform(const int64_t* x, int w, int K, int B, const int32_t* C, int64_t* y) {
  int s1 = ilog2(w) + B - 9;
  int s2 = ilog2(w) + 6;
  int64_t T[32 * 32];
  /* horizontal pass: T[m][k] = sum_n X[m][n] C[k][n], rounded, k < K */
  for (int m = 0; m < w; m++)
    for (int k = 0; k < K; k++) {
      int64_t acc = 0;
      for (int n = 0; n < w; n++) acc += x[m * w + n] * (int64_t)C[k * w + n];
      T[m * 32 + k] = floor_div_pow2(acc + ((int64_t)1 << (s1 - 1)), s1);
    }
  /* vertical pass: Y[i][k] = sum_m C[i][m] T[m][k], rounded, i < K */
  for (int i = 0; i < K; i++)
    for (int k = 0; k < K; k++) {
      int64_t acc = 0;
      for (int m = 0; m < w; m++) acc += (int64_t)C[i * w + m] * T[m * 32 + k];
      y[i * K + k] = floor_div_pow2(acc + ((int64_t)1 << (s2 - 1)), s2);
    }
}

int vcaref_block_transform(const int32_t* x, int32_t w, int32_t K, int32_t bit_depth,
                           int64_t* y_out) {
  if (!x || !y_out || !valid_w(w) || K < 1 || K > w) return VCAREF_EINVAL;
  if (bit_depth != 8 && bit_depth != 10) return VCAREF_EINVAL;
  int32_t C[32 * 32];
  int64_t X[32 * 32];
  vcaref_dct_matrix(w, C);
  int32_t maxv = (1 << bit_depth) - 1;
  for (int t = 0; t < w * w; t++) {
    if (x[t] < 0 || x[t] > maxv) return VCAREF_ERANGE;
    X[t] = x[t];
  }
  transform(X, w, K, bit_depth, C, y_out);
  return 0;
}

static int check_config(const vcaref_config* cfg) {
  if (!cfg || !valid_w(cfg->block_size)) return VCAREF_EINVAL;
  if (cfg->bit_depth != 8 && cfg->bit_depth != 10) return VCAREF_EINVAL;
  if (cfg->width % 2 || cfg->height % 2) return VCAREF_EINVAL;
  /* every plane, chroma included, must hold at least one complete block */
  if (cfg->width / 2 < cfg->block_size || cfg->height / 2 < cfg->block_size) return VCAREF_EINVAL;
  if (cfg->lowpass_k < 0 || cfg->lowpass_k > cfg->block_size) return VCAREF_EINVAL;
  return 0;
}

int vcaref_block_counts(const vcaref_config* cfg, int32_t counts[3]) {
  if (check_config(cfg) || !counts) return VCAREF_EINVAL;
  int w = cfg->block_size;
  counts[0] = (cfg->width / w) * (cfg->height / w);
  counts[1] = ((cfg->width / 2) / w) * ((cfg->height / 2) / w);
  counts[2] = counts[1];
  return 0;
}

static int64_t sample_at(const void* base, int B, int64_t index) {
  if (B == 8) return ((const uint8_t*)base)[index];
  return ((const uint16_t*)base)[index];
}

int vcaref_analyze(const vcaref_config* cfg, const void* y, const void* u, const void* v,
                   int64_t pitch_y, int64_t pitch_uv, int64_t fstride_y, int64_t fstride_uv,
                   int32_t n_frames, int32_t n_threads, const double* h_prev,
                   double* features, double* block_h, int64_t* block_dc, int32_t* coeffs) {
  if (check_config(cfg)) return VCAREF_EINVAL;
  if (!y || !u || !v || !features || n_frames < 0 || n_threads < 1) return VCAREF_EINVAL;
  if (pitch_y < cfg->width || pitch_uv < cfg->width / 2) return VCAREF_EINVAL;
  if (fstride_y < 0 || fstride_uv < 0) return VCAREF_EINVAL;
  const int w = cfg->block_size, B = cfg->bit_depth;
  const int K = cfg->lowpass_k == 0 ? w : cfg->lowpass_k;
  int32_t cnt[3];
  vcaref_block_counts(cfg, cnt);
  const int64_t total = (int64_t)cnt[0] + cnt[1] + cnt[2];
  if (n_frames == 0) return 0;

  double* H = block_h ? block_h : (double*)malloc(sizeof(double) * total * n_frames);
  int64_t* DC = block_dc ? block_dc : (int64_t*)malloc(sizeof(int64_t) * total * n_frames);
  if (!H || !DC) {
    if (!block_h) free(H);
    if (!block_dc) free(DC);
    return VCAREF_EINVAL;
  }
  int32_t C[32 * 32];
  double W[32 * 32];
  vcaref_dct_matrix(w, C);
  vcaref_weights(w, W);
  const int64_t maxv = ((int64_t)1 << B) - 1;
  int range_error = 0;

#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
  for (int f = 0; f < n_frames; f++) {
    int64_t X[32 * 32];
    int64_t Yc[32 * 32];
    int64_t blk = (int64_t)f * total;
    for (int P = 0; P < 3; P++) {
      const void* base = P == 0 ? y : (P == 1 ? u : v);
      int64_t pitch = P == 0 ? pitch_y : pitch_uv;
      int64_t origin = (int64_t)f * (P == 0 ? fstride_y : fstride_uv);
      int pw = P == 0 ? cfg->width : cfg->width / 2;
      int ph = P == 0 ? cfg->height : cfg->height / 2;
      for (int by = 0; by < ph / w; by++)
        for (int bx = 0; bx < pw / w; bx++, blk++) {
          for (int m = 0; m < w; m++)
            for (int n = 0; n < w; n++) {
              int64_t s = sample_at(base, B, origin + (int64_t)(by * w + m) * pitch + bx * w + n);
              if (s > maxv) range_error = 1;
              X[m * w + n] = s;
            }
          transform(X, w, K, B, C, Yc);
          double e = 0.0;
          for (int i = 0; i < K; i++)
            for (int k = 0; k < K; k++)
              if (i != 0 || k != 0) e += W[i * w + k] * (double)llabs(Yc[i * K + k]);
          H[blk] = e;
          DC[blk] = Yc[0];
          if (coeffs)
            for (int t = 0; t < K * K; t++) coeffs[blk * K * K + t] = (int32_t)Yc[t];
        }
    }
  }

  if (!range_error) {
    const double ww = (double)w * (double)w;
    for (int f = 0; f < n_frames; f++) {
      const double* Hf = H + (int64_t)f * total;
      const int64_t* Df = DC + (int64_t)f * total;
      double sumH[3] = {0, 0, 0}, sumL[3] = {0, 0, 0}, dh = 0.0;
      int64_t off = 0;
      for (int P = 0; P < 3; P++) {
        for (int64_t b = 0; b < cnt[P]; b++) {
          sumH[P] += Hf[off + b];
          sumL[P] += sqrt((double)Df[off + b]);
        }
        off += cnt[P];
      }
      const double* prev = f > 0 ? H + (int64_t)(f - 1) * total : h_prev;
      if (prev)
        for (int64_t b = 0; b < cnt[0]; b++) dh += fabs(Hf[b] - prev[b]);
      double* out = features + (int64_t)f * 7;
      out[0] = sumH[0] / (cnt[0] * ww);  /* E_Y */
      out[1] = dh / (cnt[0] * ww);       /* h   */
      out[2] = sumL[0] / (cnt[0] * ww);  /* L_Y */
      out[3] = sumH[1] / (cnt[1] * ww);  /* E_U */
      out[4] = sumH[2] / (cnt[2] * ww);  /* E_V */
      out[5] = sumL[1] / (cnt[1] * ww);  /* L_U */
      out[6] = sumL[2] / (cnt[2] * ww);  /* L_V */
    }
  }
  if (!block_h) free(H);
  if (!block_dc) free(DC);
  return range_error ? VCAREF_ERANGE : 0;
}
