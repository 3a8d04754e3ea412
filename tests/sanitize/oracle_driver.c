/* Exercises every entry point of the C oracle on small images, for a build
 * under AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure:
 * run by tests/test_sanitizers.py).  Exit status 0 when every call returns 0
 * and the reconstructions hold; the sanitizers abort on any memory or
 * undefined-behaviour error. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "dwt_oracle.h"

static int fails = 0;

static void expect(int ok, const char *what, int w, long a, long b) {
    if (!ok) {
        fprintf(stderr, "FAIL %s (wavelet %d, %ld x %ld)\n", what, w, a, b);
        ++fails;
    }
}

static double *img(long n, unsigned seed) {
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    for (long i = 0; i < n; ++i) {
        seed = seed * 1103515245u + 12345u;
        p[i] = (double)((seed >> 16) & 255u);
    }
    return p;
}

int main(void) {
    double h[4], g[4], t[4], u[4];
    expect(oracle_filters(h, g, t, u) == 0, "filters", 1, 0, 0);
    const long sizes[][2] = {{2, 2}, {2, 4}, {4, 2}, {4, 6}, {6, 8}, {8, 8}, {10, 34}, {34, 10}};
    for (int w = 0; w < 2; ++w) {
        for (long n = 2; n <= 10; n += 2) {
            double *s = img(n, 7u + (unsigned)n), *c = img(n, 1u), *r = img(n, 2u), *y = img(n, 3u);
            expect(oracle_dwt1_fwd(w, n, s, c) == 0, "dwt1_fwd", w, n, 1);
            expect(oracle_dwt1_inv(w, n, c, r) == 0, "dwt1_inv", w, n, 1);
            for (long i = 0; i < n; ++i) expect(fabs(r[i] - s[i]) < 1e-9, "dwt1 round trip", w, n, i);
            expect(oracle_dwt1_fwd_T(w, n, s, y) == 0, "dwt1_fwd_T", w, n, 1);
            expect(oracle_dwt1_inv_T(w, n, s, y) == 0, "dwt1_inv_T", w, n, 1);
            free(s), free(c), free(r), free(y);
        }
        for (size_t k = 0; k < sizeof sizes / sizeof sizes[0]; ++k) {
            const long H = sizes[k][0], W = sizes[k][1], B = 3, q = (H / 2) * (W / 2);
            double *pan = img(H * W, 11u + (unsigned)k), *ms = img(B * q, 13u + (unsigned)k);
            double *X = img(H * W, 0u), *x = img(H * W, 0u), *out = img(B * H * W, 0u);
            double *gp = img(H * W, 0u), *gm = img(B * q, 0u), gg[3], gain[3] = {1.0, 0.5, 2.0};
            double sse[3], sref[3];
            unsigned char *u8 = (unsigned char *)malloc((size_t)(B * H * W));
            expect(oracle_dwt2_fwd(w, H, W, pan, X) == 0, "dwt2_fwd", w, H, W);
            expect(oracle_dwt2_inv(w, H, W, X, x) == 0, "dwt2_inv", w, H, W);
            for (long i = 0; i < H * W; ++i) expect(fabs(x[i] - pan[i]) < 1e-9, "dwt2 round trip", w, H, W);
            expect(oracle_fuse(w, H, W, B, pan, ms, gain, out) == 0, "fuse", w, H, W);
            expect(oracle_fuse(w, H, W, B, pan, ms, NULL, out) == 0, "fuse no gain", w, H, W);
            for (long y = 0; y < H; y += H - 1) {
                const double v = oracle_fuse_point(w, H, W, pan, ms, 1.0, y, W - 1);
                expect(fabs(v - out[y * W + W - 1]) < 1e-9, "fuse_point against fuse", w, H, W);
            }
            expect(oracle_fuse_kappa(w, H, W, B, pan, ms, gain, 2.0, out) == 0, "fuse_kappa", w, H, W);
            {
                /* rows 1 .. H-1 of every band (the first pair row at H = 2) equal the whole image's */
                const long r0 = H > 2 ? 1 : 0, r1 = H;
                double *rows = img(B * (r1 - r0) * W, 0u);
                expect(oracle_fuse_rows(w, H, W, B, pan, ms, gain, 2.0, r0, r1, rows) == 0, "fuse_rows", w, H, W);
                for (long b = 0; b < B; ++b)
                    for (long y = r0; y < r1; ++y)
                        for (long x = 0; x < W; ++x)
                            expect(rows[(b * (r1 - r0) + y - r0) * W + x] == out[(b * H + y) * W + x],
                                   "fuse_rows against fuse_kappa", w, H, W);
                expect(oracle_fuse_rows(w, H, W, B, pan, ms, NULL, 1.0, H / 2, H / 2, rows) == 0, "fuse_rows empty",
                       w, H, W);
                free(rows);
            }
            expect(oracle_quantize_u8(B * H * W, out, u8) == 0, "quantize_u8", w, H, W);
            expect(oracle_quality(H, W, B, out, out, sse, sref) == 0, "quality", w, H, W);
            for (int b = 0; b < 3; ++b) expect(sse[b] == 0.0, "quality of identical images", w, H, W);
            expect(oracle_fuse_backward(w, H, W, B, pan, gain, out, gp, gm, gg) == 0, "fuse_backward", w, H, W);
            expect(oracle_fuse_backward(w, H, W, B, pan, NULL, out, NULL, gm, NULL) == 0, "fuse_backward partial",
                   w, H, W);
            free(pan), free(ms), free(X), free(x), free(out), free(gp), free(gm), free(u8);
        }
    }
    if (fails) fprintf(stderr, "%d failures\n", fails);
    return fails ? 1 : 0;
}
