/*
 * vcaref.h -- TEST INFRASTRUCTURE ONLY.
 *
 * The plain, slow CPU oracle for the Video Complexity Analyzer (VCA) features
 * of Menon et al., "Green Video Complexity Analysis for Efficient Encoding in
 * Adaptive Video Streaming" (GMSys 2023), Section 2.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load this library;
 * the product (the HIP library declared in include/vca.h) never does, and the
 * two share no code.
 *
 * Integer transform in exact int64 arithmetic, features in FP64.
 * Return codes: 0 on success, VCAREF_EINVAL for a bad argument,
 * VCAREF_ERANGE for a sample above 2^bit_depth - 1.
 */
#ifndef VCAREF_H
#define VCAREF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VCAREF_EINVAL (-1)
#define VCAREF_ERANGE (-2)

typedef struct {
  int32_t width;       /* luma width in samples, even                          */
  int32_t height;      /* luma height in samples, even                         */
  int32_t bit_depth;   /* 8 (uint8 samples) or 10 (uint16 samples, 0..1023)    */
  int32_t block_size;  /* w in {4, 8, 16, 32}                                  */
  int32_t lowpass_k;   /* K: 0 or w for the full transform, else 1 <= K < w     */
} vcaref_config;

/* The w x w integer DCT matrix C_w (row k = frequency, column n = sample). */
int vcaref_dct_matrix(int32_t w, int32_t* out /* w*w, row-major */);

/* The w x w energy weights W[i][j] (FP64). */
int vcaref_weights(int32_t w, double* out /* w*w, row-major */);

/* Two-stage integer transform of one w x w block of raw samples x
 * (row-major, int32 values in [0, 2^B - 1]); writes the top-left K x K
 * coefficients Y[i][k] (i vertical, k horizontal frequency), row-major. */
int vcaref_block_transform(const int32_t* x, int32_t w, int32_t K, int32_t bit_depth,
                           int64_t* y_out);

/* Number of complete w x w blocks of the Y, U and V planes. */
int vcaref_block_counts(const vcaref_config* cfg, int32_t counts[3]);

/* Analyses n_frames frames of planar 4:2:0 video.
 *   y, u, v      first sample of frame 0 of each plane (uint8_t for 8-bit,
 *                uint16_t for 10-bit)
 *   pitch_*      samples per row; fstride_* samples between frames
 *   h_prev       luma block energies of the frame before frame 0 (C_Y
 *                doubles), or NULL: then frame 0 has h = 0
 *   features     out, n_frames x 7 doubles: E_Y, h, L_Y, E_U, E_V, L_U, L_V
 *   block_h      optional out, n_frames x (C_Y + C_U + C_V) block energies H
 *   block_dc     optional out, same shape, block DC coefficients
 *   coeffs       optional out, n_frames x (C_Y + C_U + C_V) x K x K coefficients
 *   n_threads    frames are spread over this many OpenMP threads (>= 1)      */
int vcaref_analyze(const vcaref_config* cfg, const void* y, const void* u, const void* v,
                   int64_t pitch_y, int64_t pitch_uv, int64_t fstride_y, int64_t fstride_uv,
                   int32_t n_frames, int32_t n_threads, const double* h_prev,
                   double* features, double* block_h, int64_t* block_dc, int32_t* coeffs);

#ifdef __cplusplus
}
#endif
#endif
