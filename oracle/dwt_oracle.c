/*
 * dwt_oracle.c -- plain FP64 CPU reference for DWT-replacement
 * pan-sharpening (Al-Oraiqat et al., section 2, Eq. 1-16).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, to check and time the GPU path against.  It shares no code,
 * header or constant with the GPU library.
 *
 * Structure: each printed equation is written once, as a "taps" function
 * that lists which input elements (indices) and weights produce one output
 * element of a 1D transform.  The 1D and 2D transforms, the single-pixel
 * evaluation and the transposes (for gradients) are plain loops over those
 * taps.  Summation follows the order of the terms in each equation.  No
 * blocking, no reuse beyond what the method states.
 */
#include "dwt_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double h[4], g[4], t[4], u[4];
} filt_t;

/* Eq. 7-8 give h; Eq. 9-10 are read as g_k = (-1)^k h_{3-k}; the tables t
 * and u are defined after Eq. 16. */
static void make_filters(filt_t *f)
{
    const double r3 = sqrt(3.0);
    const double den = 4.0 * sqrt(2.0);
    for (int i = 0; i < 2; ++i) {
        f->h[i] = (1.0 + 2.0 * i + r3) / den;     /* Eq. 7 */
        f->h[i + 2] = (3.0 - 2.0 * i - r3) / den; /* Eq. 8 */
    }
    for (int k = 0; k < 4; ++k)
        f->g[k] = ((k & 1) ? -1.0 : 1.0) * f->h[3 - k];
    f->t[0] = f->h[2];
    f->t[1] = f->g[2];
    f->t[2] = f->h[0];
    f->t[3] = f->g[0];
    f->u[0] = f->h[3];
    f->u[1] = f->g[3];
    f->u[2] = f->h[1];
    f->u[3] = f->g[1];
}

static int valid_len(int64_t n) { return n >= 2 && (n % 2) == 0; }

/* Forward 1D transform of length N: taps of output element i (0 <= i < N).
 * The output is [approximations a_0..a_{N/2-1}, details d_0..d_{N/2-1}]. */
static int fwd1_taps(int w, int64_t N, int64_t i, const filt_t *f,
                     int64_t idx[4], double wt[4])
{
    const int64_t half = N / 2;
    if (w == ORACLE_HAAR) {
        const int64_t j = (i < half) ? i : i - half;
        idx[0] = 2 * j;
        idx[1] = 2 * j + 1;
        wt[0] = 0.5;
        wt[1] = (i < half) ? 0.5 : -0.5; /* Eq. 1 (sum) / Eq. 2 (difference) */
        return 2;
    }
    const double *flt = (i < half) ? f->h : f->g; /* Eq. 3,5: h; Eq. 4,6: g */
    const int64_t j = (i < half) ? i : i - half;
    if (j < half - 1) {
        for (int k = 0; k < 4; ++k) { /* Eq. 3-4: interior */
            idx[k] = 2 * j + k;
            wt[k] = flt[k];
        }
    } else {
        for (int m = 0; m < 2; ++m) { /* Eq. 5-6: last element wraps */
            idx[m] = N - 2 + m;
            wt[m] = flt[m];
        }
        for (int m = 0; m < 2; ++m) {
            idx[2 + m] = m;
            wt[2 + m] = flt[2 + m];
        }
    }
    return 4;
}

/* Inverse 1D transform of length N: taps (coefficient indices and weights)
 * of reconstructed sample n (0 <= n < N). */
static int inv1_taps(int w, int64_t N, int64_t n, const filt_t *f,
                     int64_t idx[4], double wt[4])
{
    const int64_t half = N / 2;
    if (w == ORACLE_HAAR) {
        const int64_t i = n / 2;
        idx[0] = i;
        idx[1] = half + i;
        wt[0] = 1.0;
        wt[1] = (n & 1) ? -1.0 : 1.0; /* Eq. 11 (even n) / Eq. 12 (odd n) */
        return 2;
    }
    const double *tab = (n & 1) ? f->u : f->t; /* Eq. 13,15: t; Eq. 14,16: u */
    if (n < 2) {
        for (int k = 0; k < 2; ++k) { /* Eq. 13-14: first pair wraps */
            idx[k] = half - 1 + k;
            wt[k] = tab[3 * k];
        }
        for (int k = 0; k < 2; ++k) {
            idx[2 + k] = (N - 1) * k;
            wt[2 + k] = tab[2 - k];
        }
    } else {
        const int64_t i = (n - 2) / 2; /* Eq. 15-16: interior */
        for (int k = 0; k < 2; ++k) {
            idx[k] = i + k;
            wt[k] = tab[2 * k];
        }
        for (int k = 0; k < 2; ++k) {
            idx[2 + k] = i + half + k;
            wt[2 + k] = tab[1 + 2 * k];
        }
    }
    return 4;
}

typedef int (*taps_fn)(int, int64_t, int64_t, const filt_t *, int64_t *, double *);

/* Apply a 1D map along every row of an H x W image. */
static void along_rows(taps_fn fn, int w, int64_t H, int64_t W, const filt_t *f,
                       const double *in, double *out)
{
    int64_t idx[4];
    double wt[4];
    for (int64_t y = 0; y < H; ++y)
        for (int64_t j = 0; j < W; ++j) {
            const int n = fn(w, W, j, f, idx, wt);
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += wt[k] * in[y * W + idx[k]];
            out[y * W + j] = acc;
        }
}

/* Apply a 1D map along every column of an H x W image (all columns share
 * the same taps for a given output row). */
static void along_cols(taps_fn fn, int w, int64_t H, int64_t W, const filt_t *f,
                       const double *in, double *out)
{
    int64_t idx[4];
    double wt[4];
    for (int64_t i = 0; i < H; ++i) {
        const int n = fn(w, H, i, f, idx, wt);
        for (int64_t x = 0; x < W; ++x) {
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += wt[k] * in[idx[k] * W + x];
            out[i * W + x] = acc;
        }
    }
}

/* Transpose of along_rows: scatter each output back onto its taps. */
static void along_rows_T(taps_fn fn, int w, int64_t H, int64_t W, const filt_t *f,
                         const double *in, double *out)
{
    int64_t idx[4];
    double wt[4];
    memset(out, 0, sizeof(double) * (size_t)(H * W));
    for (int64_t y = 0; y < H; ++y)
        for (int64_t j = 0; j < W; ++j) {
            const int n = fn(w, W, j, f, idx, wt);
            for (int k = 0; k < n; ++k) out[y * W + idx[k]] += wt[k] * in[y * W + j];
        }
}

/* Transpose of along_cols. */
static void along_cols_T(taps_fn fn, int w, int64_t H, int64_t W, const filt_t *f,
                         const double *in, double *out)
{
    int64_t idx[4];
    double wt[4];
    memset(out, 0, sizeof(double) * (size_t)(H * W));
    for (int64_t i = 0; i < H; ++i) {
        const int n = fn(w, H, i, f, idx, wt);
        for (int k = 0; k < n; ++k)
            for (int64_t x = 0; x < W; ++x) out[idx[k] * W + x] += wt[k] * in[i * W + x];
    }
}

static int valid_wavelet(int w) { return w == ORACLE_HAAR || w == ORACLE_D4; }

int oracle_filters(double h[4], double g[4], double t[4], double u[4])
{
    filt_t f;
    make_filters(&f);
    for (int k = 0; k < 4; ++k) {
        if (h) h[k] = f.h[k];
        if (g) g[k] = f.g[k];
        if (t) t[k] = f.t[k];
        if (u) u[k] = f.u[k];
    }
    return 0;
}

int oracle_dwt1_fwd(int w, int64_t N, const double *s, double *out)
{
    if (!valid_wavelet(w) || !valid_len(N)) return -1;
    filt_t f;
    make_filters(&f);
    along_rows(fwd1_taps, w, 1, N, &f, s, out);
    return 0;
}

int oracle_dwt1_inv(int w, int64_t N, const double *c, double *out)
{
    if (!valid_wavelet(w) || !valid_len(N)) return -1;
    filt_t f;
    make_filters(&f);
    along_rows(inv1_taps, w, 1, N, &f, c, out);
    return 0;
}

int oracle_dwt1_fwd_T(int w, int64_t N, const double *y, double *out)
{
    if (!valid_wavelet(w) || !valid_len(N)) return -1;
    filt_t f;
    make_filters(&f);
    along_rows_T(fwd1_taps, w, 1, N, &f, y, out);
    return 0;
}

int oracle_dwt1_inv_T(int w, int64_t N, const double *y, double *out)
{
    if (!valid_wavelet(w) || !valid_len(N)) return -1;
    filt_t f;
    make_filters(&f);
    along_rows_T(inv1_taps, w, 1, N, &f, y, out);
    return 0;
}

/* Section 2: forward 2D = rows, then columns. */
int oracle_dwt2_fwd(int w, int64_t H, int64_t W, const double *x, double *X)
{
    if (!valid_wavelet(w) || !valid_len(H) || !valid_len(W)) return -1;
    filt_t f;
    make_filters(&f);
    double *Z = (double *)malloc(sizeof(double) * (size_t)(H * W));
    if (!Z) return -2;
    along_rows(fwd1_taps, w, H, W, &f, x, Z);
    along_cols(fwd1_taps, w, H, W, &f, Z, X);
    free(Z);
    return 0;
}

/* Section 2: inverse 2D = columns, then rows. */
int oracle_dwt2_inv(int w, int64_t H, int64_t W, const double *X, double *x)
{
    if (!valid_wavelet(w) || !valid_len(H) || !valid_len(W)) return -1;
    filt_t f;
    make_filters(&f);
    double *Y = (double *)malloc(sizeof(double) * (size_t)(H * W));
    if (!Y) return -2;
    along_cols(inv1_taps, w, H, W, &f, X, Y);
    along_rows(inv1_taps, w, H, W, &f, Y, x);
    free(Y);
    return 0;
}

/* Section 2, method steps 1-3, for each band: forward 2D of PAN, LL replaced
 * by the band (times kappa), details scaled by the band's gain, inverse 2D. */
int oracle_fuse_kappa(int w, int64_t H, int64_t W, int64_t B, const double *pan,
                      const double *ms, const double *gain, double kappa, double *out)
{
    if (!valid_wavelet(w) || !valid_len(H) || !valid_len(W) || B < 0) return -1;
    const int64_t H2 = H / 2, W2 = W / 2, n = H * W;
    double *X = (double *)malloc(sizeof(double) * (size_t)n);
    double *Xb = (double *)malloc(sizeof(double) * (size_t)n);
    if (!X || !Xb) {
        free(X);
        free(Xb);
        return -2;
    }
    oracle_dwt2_fwd(w, H, W, pan, X);
    for (int64_t b = 0; b < B; ++b) {
        const double gb = gain ? gain[b] : 1.0;
        const double *m = ms + b * H2 * W2;
        for (int64_t i = 0; i < H; ++i)
            for (int64_t j = 0; j < W; ++j)
                Xb[i * W + j] = (i < H2 && j < W2) ? kappa * m[i * W2 + j] : gb * X[i * W + j];
        oracle_dwt2_inv(w, H, W, Xb, out + b * n);
    }
    free(X);
    free(Xb);
    return 0;
}

int oracle_fuse(int w, int64_t H, int64_t W, int64_t B, const double *pan,
                const double *ms, const double *gain, double *out)
{
    return oracle_fuse_kappa(w, H, W, B, pan, ms, gain, 1.0, out);
}

/* Rows row0 .. row1-1 of every fused band of oracle_fuse_kappa: the same
 * steps (forward along rows, then columns; LL replaced, details scaled;
 * inverse along columns, then rows) evaluated only for the 2D coefficient
 * rows that the column inverse of those output rows reads (Eq. 11-16), and
 * only for the PAN rows that the column forward of those coefficient rows
 * reads (Eq. 1-6).  Every value is formed by the same products and sums in
 * the same order as in the whole-image oracle, so the rows equal its rows
 * bit for bit.  out is B x (row1 - row0) x W. */
int oracle_fuse_rows(int w, int64_t H, int64_t W, int64_t B, const double *pan,
                     const double *ms, const double *gain, double kappa,
                     int64_t row0, int64_t row1, double *out)
{
    if (!valid_wavelet(w) || !valid_len(H) || !valid_len(W) || B < 0 || row0 < 0 ||
        row1 > H || row0 > row1)
        return -1;
    const int64_t H2 = H / 2, W2 = W / 2, R = row1 - row0;
    filt_t f;
    make_filters(&f);
    double **Z = (double **)calloc((size_t)H, sizeof(double *)); /* row-transformed PAN rows */
    double **X = (double **)calloc((size_t)H, sizeof(double *)); /* 2D forward coefficient rows */
    double *Y = (double *)malloc(sizeof(double) * (size_t)W);     /* one column-inverted row */
    int rc = 0;
    if (!Z || !X || !Y) {
        rc = -2;
        goto done;
    }
    int64_t ci[4], pi[4];
    double cw[4], pw[4];
    /* Step 1: the forward 2D transform, restricted to the rows needed. */
    for (int64_t y = row0; y < row1; ++y) {
        const int nc = inv1_taps(w, H, y, &f, ci, cw);
        for (int k = 0; k < nc; ++k) {
            const int64_t i = ci[k];
            if (X[i]) continue;
            const int np = fwd1_taps(w, H, i, &f, pi, pw);
            for (int t = 0; t < np; ++t) {
                const int64_t r = pi[t];
                if (Z[r]) continue;
                Z[r] = (double *)malloc(sizeof(double) * (size_t)W);
                if (!Z[r]) {
                    rc = -2;
                    goto done;
                }
                along_rows(fwd1_taps, w, 1, W, &f, pan + r * W, Z[r]);
            }
            X[i] = (double *)malloc(sizeof(double) * (size_t)W);
            if (!X[i]) {
                rc = -2;
                goto done;
            }
            for (int64_t x = 0; x < W; ++x) {
                double acc = 0.0;
                for (int t = 0; t < np; ++t) acc += pw[t] * Z[pi[t]][x];
                X[i][x] = acc;
            }
        }
    }
    /* Steps 2-3 per band: replaced coefficients, inverse along columns, then rows. */
    for (int64_t b = 0; b < B; ++b) {
        const double gb = gain ? gain[b] : 1.0;
        const double *m = ms + b * H2 * W2;
        for (int64_t y = row0; y < row1; ++y) {
            const int nc = inv1_taps(w, H, y, &f, ci, cw);
            for (int64_t x = 0; x < W; ++x) {
                double acc = 0.0;
                for (int k = 0; k < nc; ++k) {
                    const int64_t i = ci[k];
                    const double c = (i < H2 && x < W2) ? kappa * m[i * W2 + x] : gb * X[i][x];
                    acc += cw[k] * c;
                }
                Y[x] = acc;
            }
            along_rows(inv1_taps, w, 1, W, &f, Y, out + (b * R + (y - row0)) * W);
        }
    }
done:
    if (Z)
        for (int64_t r = 0; r < H; ++r) free(Z[r]);
    if (X)
        for (int64_t i = 0; i < H; ++i) free(X[i]);
    free(Z);
    free(X);
    free(Y);
    return rc;
}

/* Squared-error and reference sums per band, the inputs of RMSE and of an
 * ERGAS-style score (section 4 names ERGAS without a formula). */
int oracle_quality(int64_t H, int64_t W, int64_t B, const double *fused,
                   const double *ref, double *sse, double *sum_ref)
{
    if (H < 1 || W < 1 || B < 1) return -1;
    for (int64_t b = 0; b < B; ++b) {
        double e = 0.0, s = 0.0;
        for (int64_t i = 0; i < H * W; ++i) {
            const double d = fused[b * H * W + i] - ref[b * H * W + i];
            e += d * d;
            s += ref[b * H * W + i];
        }
        sse[b] = e;
        sum_ref[b] = s;
    }
    return 0;
}

/* Section 3 keeps images at 8 bits per pixel.  A fused value v becomes the
 * integer nearest to v (a value exactly halfway between two integers goes to
 * the even one), limited to [0, 255]. */
int oracle_quantize_u8(int64_t n, const double *v, uint8_t *out)
{
    if (n < 0) return -1;
    for (int64_t i = 0; i < n; ++i) {
        const double x = v[i];
        if (x != x) {  /* NaN */
            out[i] = 0;
            continue;
        }
        double r = floor(x);
        const double frac = x - r;  /* exact for |x| < 2^52 */
        if (frac > 0.5 || (frac == 0.5 && fmod(r, 2.0) != 0.0)) r += 1.0;
        if (r < 0.0) r = 0.0;
        if (r > 255.0) r = 255.0;
        out[i] = (uint8_t)r;
    }
    return 0;
}

/* ---- single output pixel: the same equations, evaluated on demand ---- */

typedef struct {
    int w;
    int64_t H, W;
    const double *pan, *ms;
    double gain;
    filt_t f;
} point_ctx;

/* Row-transformed PAN at (k, j): forward 1D along row k, element j. */
static double pt_rowfwd(const point_ctx *c, int64_t k, int64_t j)
{
    int64_t idx[4];
    double wt[4];
    const int n = fwd1_taps(c->w, c->W, j, &c->f, idx, wt);
    double acc = 0.0;
    for (int t = 0; t < n; ++t) acc += wt[t] * c->pan[k * c->W + idx[t]];
    return acc;
}

/* 2D forward coefficient at (i, j) after LL replacement and detail gain. */
static double pt_coef(const point_ctx *c, int64_t i, int64_t j)
{
    if (i < c->H / 2 && j < c->W / 2) return c->ms[i * (c->W / 2) + j];
    int64_t idx[4];
    double wt[4];
    const int n = fwd1_taps(c->w, c->H, i, &c->f, idx, wt);
    double acc = 0.0;
    for (int t = 0; t < n; ++t) acc += wt[t] * pt_rowfwd(c, idx[t], j);
    return c->gain * acc;
}

/* Column-inverted coefficients at (y, j): inverse 1D along column j. */
static double pt_colinv(const point_ctx *c, int64_t y, int64_t j)
{
    int64_t idx[4];
    double wt[4];
    const int n = inv1_taps(c->w, c->H, y, &c->f, idx, wt);
    double acc = 0.0;
    for (int t = 0; t < n; ++t) acc += wt[t] * pt_coef(c, idx[t], j);
    return acc;
}

double oracle_fuse_point(int w, int64_t H, int64_t W, const double *pan,
                         const double *ms_band, double gain, int64_t y, int64_t x)
{
    if (!valid_wavelet(w) || !valid_len(H) || !valid_len(W) || y < 0 || y >= H ||
        x < 0 || x >= W)
        return NAN;
    point_ctx c;
    c.w = w;
    c.H = H;
    c.W = W;
    c.pan = pan;
    c.ms = ms_band;
    c.gain = gain;
    make_filters(&c.f);
    int64_t idx[4];
    double wt[4];
    const int n = inv1_taps(w, W, x, &c.f, idx, wt);
    double acc = 0.0;
    for (int t = 0; t < n; ++t) acc += wt[t] * pt_colinv(&c, y, idx[t]);
    return acc;
}

/* ---- transpose of the fusion map ---- */

/* out_b = Srow(Scol(R_b(Acol(Arow(pan)), ms_b))), with R_b writing ms_b into
 * LL and gain_b times the PAN coefficients elsewhere.  The transpose applies
 * the transposed steps in reverse order. */
int oracle_fuse_backward(int w, int64_t H, int64_t W, int64_t B, const double *pan,
                         const double *gain, const double *grad_out,
                         double *grad_pan, double *grad_ms, double *grad_gain)
{
    if (!valid_wavelet(w) || !valid_len(H) || !valid_len(W) || B < 0) return -1;
    const int64_t H2 = H / 2, W2 = W / 2, n = H * W;
    filt_t f;
    make_filters(&f);
    double *X = (double *)malloc(sizeof(double) * (size_t)n);
    double *T1 = (double *)malloc(sizeof(double) * (size_t)n);
    double *Z = (double *)malloc(sizeof(double) * (size_t)n);
    double *acc = (double *)calloc((size_t)n, sizeof(double));
    if (!X || !T1 || !Z || !acc) {
        free(X);
        free(T1);
        free(Z);
        free(acc);
        return -2;
    }
    oracle_dwt2_fwd(w, H, W, pan, X);
    for (int64_t b = 0; b < B; ++b) {
        const double gb = gain ? gain[b] : 1.0;
        along_rows_T(inv1_taps, w, H, W, &f, grad_out + b * n, T1);
        along_cols_T(inv1_taps, w, H, W, &f, T1, Z); /* dL/d(replaced coefs) */
        double gg = 0.0;
        for (int64_t i = 0; i < H; ++i)
            for (int64_t j = 0; j < W; ++j) {
                const double z = Z[i * W + j];
                if (i < H2 && j < W2) {
                    if (grad_ms) grad_ms[b * H2 * W2 + i * W2 + j] = z;
                } else {
                    gg += z * X[i * W + j];
                    acc[i * W + j] += gb * z;
                }
            }
        if (grad_gain) grad_gain[b] = gg;
    }
    if (grad_pan) {
        along_cols_T(fwd1_taps, w, H, W, &f, acc, T1);
        along_rows_T(fwd1_taps, w, H, W, &f, T1, grad_pan);
    }
    free(X);
    free(T1);
    free(Z);
    free(acc);
    return 0;
}
