/*
 * dwt_oracle.h -- plain FP64 CPU reference for DWT-replacement pan-sharpening.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path; it
 * is never linked into, loaded by, or called from the product library.  Only
 * the test-suite, the smoke check and the benchmark's CPU-baseline leg use it.
 *
 * Method (Al-Oraiqat et al., "Fusion of multispectral satellite imagery using
 * a cluster of graphics processing unit", section 2):
 *   1. one-level 2D forward DWT of the PAN image: 1D transform over every row,
 *      then over every column;
 *   2. the approximation (LL) quadrant is replaced by one MS band;
 *   3. 2D inverse DWT: 1D inverse over every column, then over every row.
 * Wavelets: Haar (Eq. 1-2 forward, Eq. 11-12 inverse) and Daubechies-4 with
 * periodic wrap (Eq. 3-10 forward, Eq. 13-16 inverse).
 *
 * Readings where the text is garbled or silent (each is listed in the design
 * notes of the repository):
 *   - Eq. 9-10 print a high-pass filter that is not a wavelet filter (its taps
 *     do not sum to zero and the printed inverse does not invert the forward
 *     transform with it).  Read as the quadrature-mirror relation
 *     g_k = (-1)^k h_{3-k}.
 *   - Index ranges printed as closed intervals are half-open; Eq. 3-4 and
 *     15-16 cover the interior and Eq. 5-6 and 13-14 the wrap-around element.
 *   - In Eq. 13-14 the subscript "(N-1)k" is the product (N-1)*k.
 *   - The MS band replaces LL unscaled (kappa = 1).
 *   - An optional per-band gain multiplies the three detail quadrants before
 *     the inverse (gain 1 is the method as printed).
 *
 * Arrays are row-major, contiguous, double.  Every function returns 0 on
 * success and a negative value when its sizes are invalid (odd or < 2).
 */
#ifndef DWT_ORACLE_H
#define DWT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_HAAR = 0, ORACLE_D4 = 1 };

/* Filters of Eq. 7-10 (g per the reading above) and the synthesis tables
 * t, u defined after Eq. 16. */
int oracle_filters(double h[4], double g[4], double t[4], double u[4]);

/* 1D forward (Eq. 1-6) / inverse (Eq. 11-16) of a length-N vector. */
int oracle_dwt1_fwd(int wavelet, int64_t N, const double *s, double *out);
int oracle_dwt1_inv(int wavelet, int64_t N, const double *c, double *out);

/* Transposes of the two 1D maps above, applied to a vector. */
int oracle_dwt1_fwd_T(int wavelet, int64_t N, const double *y, double *out);
int oracle_dwt1_inv_T(int wavelet, int64_t N, const double *y, double *out);

/* 2D forward (rows, then columns) and inverse (columns, then rows) of an
 * H x W image; the LL quadrant is the top-left (H/2) x (W/2) block. */
int oracle_dwt2_fwd(int wavelet, int64_t H, int64_t W, const double *x, double *X);
int oracle_dwt2_inv(int wavelet, int64_t H, int64_t W, const double *X, double *x);

/* Fusion of one PAN (H x W) with B MS bands (B x H/2 x W/2) into B outputs
 * (B x H x W).  gain: B per-band detail gains, or NULL for all ones. */
int oracle_fuse(int wavelet, int64_t H, int64_t W, int64_t B,
                const double *pan, const double *ms, const double *gain,
                double *out);

/* The same fusion with the MS band scaled by kappa before it replaces LL
 * (kappa = 1 is the method as printed; kappa = (sum of the low-pass taps)^2
 * matches the DC gain of the analysis LL, i.e. 2 for D4 and 1 for the
 * divided-by-2 Haar of Eq. 1-2). */
int oracle_fuse_kappa(int wavelet, int64_t H, int64_t W, int64_t B,
                      const double *pan, const double *ms, const double *gain,
                      double kappa, double *out);

/* Eight-bit code of n values (the 8-bit-per-pixel image representation of
 * section 3): nearest integer with ties to the even neighbour, clamped to
 * [0, 255]; NaN becomes 0. */
int oracle_quantize_u8(int64_t n, const double *v, uint8_t *out);

/* Quality sums of B fused bands against B reference bands (H x W each):
 * sse[b] = sum of (fused - ref)^2, sum_ref[b] = sum of ref. */
int oracle_quality(int64_t H, int64_t W, int64_t B, const double *fused,
                   const double *ref, double *sse, double *sum_ref);

/* Rows row0 .. row1-1 (0 <= row0 <= row1 <= H) of every band of
 * oracle_fuse_kappa, equal to its rows bit for bit, computed from the
 * coefficient and PAN rows they need only.  out is B x (row1 - row0) x W. */
int oracle_fuse_rows(int wavelet, int64_t H, int64_t W, int64_t B, const double *pan,
                     const double *ms, const double *gain, double kappa,
                     int64_t row0, int64_t row1, double *out);

/* One output pixel (y, x) of the fusion with one MS band, evaluated from
 * the same 1D equations restricted to the coefficients that pixel needs. */
double oracle_fuse_point(int wavelet, int64_t H, int64_t W,
                         const double *pan, const double *ms_band, double gain,
                         int64_t y, int64_t x);

/* Transpose of the fusion map: given dL/d(out) (B x H x W), return
 * dL/d(pan) (H x W), dL/d(ms) (B x H/2 x W/2) and dL/d(gain) (B).
 * Any output pointer may be NULL to skip it. */
int oracle_fuse_backward(int wavelet, int64_t H, int64_t W, int64_t B,
                         const double *pan, const double *gain,
                         const double *grad_out,
                         double *grad_pan, double *grad_ms, double *grad_gain);

#ifdef __cplusplus
}
#endif
#endif
