/* Drives the library's host-side validation (the dwt_fuse_check_* entry
 * points, which make no HIP call, and dwt_fuse_status_str) with valid and
 * invalid arguments, for a build of the host code under AddressSanitizer and
 * UndefinedBehaviorSanitizer (test infrastructure: run by
 * tests/test_sanitizers.py).  The pointers are host addresses that are never
 * dereferenced; only their values, alignment and overlap are checked.  Exit
 * status 0 when every call returns the expected class of status. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "dwt_fuse.h"

static int fails = 0;

static void expect(int ok, const char *what) {
    if (!ok) {
        fprintf(stderr, "FAIL %s\n", what);
        ++fails;
    }
}

static _Alignas(16) float arena[1 << 20];

int main(void) {
    const int64_t H = 64, W = 128, B = 3;
    const float *pan = arena, *ms = arena + 16384, *gain = arena + 32768;
    float *out = arena + 65536;
    expect(dwt_fuse_check_run(DWT_FUSE_D4, H, W, B, pan, W, ms, W / 2, (H / 2) * (W / 2), gain, out, W, H * W) ==
               DWT_FUSE_OK, "valid run");
    expect(dwt_fuse_check_run(DWT_FUSE_D4, H, W, B, NULL, W, ms, W / 2, (H / 2) * (W / 2), gain, out, W, H * W) !=
               DWT_FUSE_OK, "NULL pan");
    expect(dwt_fuse_check_run(DWT_FUSE_D4, H + 1, W, B, pan, W, ms, W / 2, (H / 2) * (W / 2), gain, out, W,
                              H * W) != DWT_FUSE_OK, "odd H");
    expect(dwt_fuse_check_run((dwt_fuse_wavelet)7, H, W, B, pan, W, ms, W / 2, (H / 2) * (W / 2), gain, out, W,
                              H * W) != DWT_FUSE_OK, "bad wavelet");
    expect(dwt_fuse_check_run(DWT_FUSE_HAAR, H, W, B, pan, W - 2, ms, W / 2, (H / 2) * (W / 2), gain, out, W,
                              H * W) != DWT_FUSE_OK, "pitch below width");
    expect(dwt_fuse_check_run(DWT_FUSE_HAAR, H, W, B, pan, W, ms, W / 2, (H / 2) * (W / 2), gain, (float *)pan, W,
                              H * W) != DWT_FUSE_OK, "output over input");
    expect(dwt_fuse_check_run(DWT_FUSE_HAAR, INT64_C(1) << 40, W, B, pan, W, ms, W / 2, (H / 2) * (W / 2), gain, out,
                              W, H * W) != DWT_FUSE_OK, "huge H");
    expect(dwt_fuse_check_backward(DWT_FUSE_D4, H, W, B, pan, W, gain, out, W, H * W, arena + 524288,
                                   arena + 589824, arena + 655360) == DWT_FUSE_OK, "valid backward");
    expect(dwt_fuse_check_backward(DWT_FUSE_D4, H, W, B, pan, W, gain, out, W, H * W, (float *)out, NULL, NULL) !=
               DWT_FUSE_OK, "backward output over input");
    expect(dwt_fuse_check_quality(H, W, B, out, W, H * W, pan, W, H * W, (const double *)(arena + 800000)) ==
               DWT_FUSE_OK, "valid quality");
    dwt_fuse_item items[3];
    memset(items, 0, sizeof items);
    for (int i = 0; i < 3; ++i) {
        items[i].wavelet = i & 1;
        items[i].B = 2;
        items[i].H = 32;
        items[i].W = 64;
        items[i].pan = arena + 100000 * i;
        items[i].ms = arena + 100000 * i + 4096;
        items[i].out = arena + 100000 * i + 8192;
        items[i].pan_ld = 64;
        items[i].ms_ld = 32;
        items[i].ms_band_stride = 16 * 32;
        items[i].out_ld = 64;
        items[i].out_band_stride = 32 * 64;
    }
    expect(dwt_fuse_check_batched(items, 3) == DWT_FUSE_OK, "valid batch");
    expect(dwt_fuse_check_batched(items, 0) == DWT_FUSE_OK, "empty batch");
    expect(dwt_fuse_check_batched(NULL, 2) != DWT_FUSE_OK, "NULL batch");
    items[2].out = arena + 8192; /* over item 0's output */
    expect(dwt_fuse_check_batched(items, 3) != DWT_FUSE_OK, "overlapping outputs in a batch");
    dwt_fuse_bwd_item bi[2];
    memset(bi, 0, sizeof bi);
    for (int i = 0; i < 2; ++i) {
        bi[i].wavelet = 1;
        bi[i].B = 2;
        bi[i].H = 32;
        bi[i].W = 64;
        bi[i].pan = arena + 200000 * i + 400000;
        bi[i].grad_out = arena + 200000 * i + 410000;
        bi[i].grad_pan = arena + 200000 * i + 420000;
        bi[i].grad_ms = arena + 200000 * i + 430000;
        bi[i].grad_gain = arena + 200000 * i + 440000;
        bi[i].pan_ld = 64;
        bi[i].go_ld = 64;
        bi[i].go_band_stride = 32 * 64;
    }
    expect(dwt_fuse_check_backward_batched(bi, 2) == DWT_FUSE_OK, "valid backward batch");
    bi[1].grad_ms = arena + 420000; /* over item 0's grad_pan */
    expect(dwt_fuse_check_backward_batched(bi, 2) != DWT_FUSE_OK, "overlapping backward outputs");
    for (int s = -3; s < 64; ++s) {
        const char *msg = dwt_fuse_status_str((dwt_fuse_status)s);
        expect(msg != NULL && strlen(msg) > 0, "status string");
    }
    if (fails) fprintf(stderr, "%d failures\n", fails);
    return fails ? 1 : 0;
}
