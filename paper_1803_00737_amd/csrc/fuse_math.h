// Per-pixel arithmetic shared by every forward kernel (float32 and 8-bit
// codec variants), so that all of them evaluate each output pixel with the
// same operations in the same order and agree bit for bit.  See
// fuse_kernels.hip for the derivation of the fused form.
#pragma once

#include <hip/hip_runtime.h>

#include "fuse_internal.h"

namespace dwtf {

typedef float f2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int wrap_idx(int q, int n) {
    q %= n;
    return q < 0 ? q + n : q;
}

// Workgroups are dispatched round-robin over the 8 XCDs.  Map hardware
// block b to a logical block so that XCD x gets a contiguous logical range.
__device__ __forceinline__ int xcd_remap(int b, int G) {
    constexpr int NX = 8;
    const int x = b % NX, i = b / NX, q = G / NX, rem = G % NX;
    return x * q + (x < rem ? x : rem) + i;
}

// Workgroup -> logical block.  Bit 1 of a launch's unit order clear:
// remapped so that each XCD takes a contiguous run of blocks; set: dispatch
// order (the hardware deals consecutive workgroups round-robin to the XCDs,
// so the whole GPU then advances through the units as one front).
__device__ __forceinline__ int block_unit(int order) {
    return (order & 2) ? (int)blockIdx.x : xcd_remap(blockIdx.x, gridDim.x);
}

// Row low-pass at coefficient columns pc[0..NC]: sum_l h_l PAN(y, 2s+l).
template <int NC>
__device__ __forceinline__ void rowfilt(const Filters &f, const f2 (&x)[NC + 2], float (&R)[NC + 1]) {
#pragma unroll
    for (int j = 0; j <= NC; ++j)
        R[j] = fmaf(f.h[3], x[j + 1].y, fmaf(f.h[2], x[j + 1].x, fmaf(f.h[1], x[j].y, f.h[0] * x[j].x)));
}

// Column low-pass of four consecutive row-filtered rows (one coefficient row
// of L PAN).  One fixed evaluation order, so every output is computed the
// same way whatever unit it falls in.
template <int NC>
__device__ __forceinline__ void colfilt(const Filters &f, const float (&R0)[NC + 1], const float (&R1)[NC + 1],
                                        const float (&R2)[NC + 1], const float (&R3)[NC + 1],
                                        float (&A)[NC + 1]) {
#pragma unroll
    for (int j = 0; j <= NC; ++j)
        A[j] = fmaf(f.h[3], R3[j], fmaf(f.h[2], R2[j], fmaf(f.h[1], R1[j], f.h[0] * R0[j])));
}

// Output rows 2r (q0) and 2r+1 (q1) of one band from the coefficient rows
// c(r-1) = cp, c(r) = cc of (kappa m - g L PAN) and the lane's PAN pixels of
// rows 2r (xa) and 2r+1 (xb).  kappa = 1 multiplies exactly.
template <int NC>
__device__ __forceinline__ void d4_out_rows(const Filters &f, float g, float kappa, const float (&mc)[NC + 1],
                                            const float (&mp)[NC + 1], const float (&A)[NC + 1],
                                            const float (&Ap)[NC + 1], const f2 (&xa)[NC + 2],
                                            const f2 (&xb)[NC + 2], f2 (&q0)[NC], f2 (&q1)[NC]) {
    const float h0 = f.h[0], h1 = f.h[1], h2 = f.h[2], h3 = f.h[3];
    float v0[NC + 1], v1[NC + 1];
#pragma unroll
    for (int j = 0; j <= NC; ++j) {
        const float cc = fmaf(-g, A[j], kappa * mc[j]);   // coefficient row r
        const float cp = fmaf(-g, Ap[j], kappa * mp[j]);  // coefficient row r-1
        v0[j] = fmaf(h2, cp, h0 * cc);             // output row 2r
        v1[j] = fmaf(h3, cp, h1 * cc);             // output row 2r+1
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        q0[i].x = fmaf(g, xa[i + 1].x, fmaf(h2, v0[i], h0 * v0[i + 1]));
        q0[i].y = fmaf(g, xa[i + 1].y, fmaf(h3, v0[i], h1 * v0[i + 1]));
        q1[i].x = fmaf(g, xb[i + 1].x, fmaf(h2, v1[i], h0 * v1[i + 1]));
        q1[i].y = fmaf(g, xb[i + 1].y, fmaf(h3, v1[i], h1 * v1[i + 1]));
    }
}

// Detail part of PAN: pixel minus the mean of its 2x2 block (the block mean is
// the LL coefficient of Eq. 1-2 applied to rows and columns).
template <int NC>
__device__ __forceinline__ void haar_details(const f2 (&a)[NC], const f2 (&c)[NC], f2 (&da)[NC], f2 (&dc)[NC]) {
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        const float mean = ((a[i].x + a[i].y) + (c[i].x + c[i].y)) * 0.25f;
        da[i] = f2{a[i].x - mean, a[i].y - mean};
        dc[i] = f2{c[i].x - mean, c[i].y - mean};
    }
}

// Output rows 2r, 2r+1 of one band: kappa m + g * detail.
template <int NC>
__device__ __forceinline__ void haar_out_rows(float g, float kappa, const float (&m)[NC], const f2 (&da)[NC], const f2 (&dc)[NC],
                                              f2 (&q0)[NC], f2 (&q1)[NC]) {
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        const float mk = kappa * m[i];
        q0[i] = f2{fmaf(g, da[i].x, mk), fmaf(g, da[i].y, mk)};
        q1[i] = f2{fmaf(g, dc[i].x, mk), fmaf(g, dc[i].y, mk)};
    }
}

}  // namespace dwtf
