// Adjoint (transpose) of the fused DWT pan-sharpening map, for gfx950.
//
// The forward map is linear in (PAN, MS) for fixed gains and linear in each
// gain:  out_b = g_b (PAN - P PAN) + S m_b, where P is the projection of an
// image onto its LL part and S is the synthesis of an LL-only coefficient
// image.  For D4 (orthonormal, Eq. 3-16 with wrap) S = L^T and P = L^T L;
// for Haar (Eq. 1-2, 11-12) S repeats each coefficient over its 2x2 block and
// P replaces each pixel by its block mean.  P is symmetric in both cases, so
// for an upstream gradient y_b = dLoss/d(out_b):
//     dLoss/d(m_b)   = S^T y_b            (D4: L y_b;  Haar: 2x2 block sum)
//     dLoss/d(PAN)   = Y - P Y,  Y = sum_b g_b y_b
//     dLoss/d(g_b)   = < y_b, PAN - P PAN >.
// The kernels walk the same work units as the forward kernels: rolling
// wavefronts (a strip of 64*NC coefficient columns, seg_rows coefficient rows,
// rows rolling in registers), one-shot wavefront tiles, and LDS-staged
// workgroup tiles.  The per-band gain products of each coefficient row of a
// strip are summed across the wavefront and written to their own slot
// (gain_row), and gain_chunk_kernel / gain_total_kernel add the slots in FP64
// in a fixed order, so grad_gain has the same bits whatever the unit length,
// order or variant with two coefficient columns per lane.  grad_pan and grad_ms are written
// with non-temporal stores (they are not read again by the kernel, except
// grad_pan by later band groups, and keeping them out of the caches leaves
// room for the upstream-gradient halo rows).
#include "fuse_internal.h"

namespace dwtf {

typedef float f2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kAdjMaxBands = 8;  // bands per launch; the host splits larger B

namespace {

__device__ __forceinline__ int wrap_idx(int q, int n) {
    q %= n;
    return q < 0 ? q + n : q;
}

// AL: the alignment class of a launch path's rows: 2 = 16-byte rows (pairs
// 8-byte aligned; two-column reads and writes as 16-byte accesses), 1 =
// 8-byte rows (pairs 8-byte aligned, rows of W/2 coefficients may be odd, so
// coefficient pairs are written one by one), 0 = 4-byte alignment only.
template <int AL>
__device__ __forceinline__ f2 ld2(const float *p) {
    if constexpr (AL >= 1) {
        return *reinterpret_cast<const f2 *>(p);
    } else {
        return f2{p[0], p[1]};
    }
}

template <int AL>
__device__ __forceinline__ void st2(float *p, f2 v) {
    if constexpr (AL >= 1) {
        __builtin_nontemporal_store(v, reinterpret_cast<f2 *>(p));
    } else {
        p[0] = v.x;
        p[1] = v.y;
    }
}

__device__ __forceinline__ int xcd_remap(int b, int G) {
    constexpr int NX = 8;
    const int x = b % NX, i = b / NX, q = G / NX, rem = G % NX;
    return x * q + (x < rem ? x : rem) + i;
}

// Workgroup -> logical block: bit 1 of the unit order set takes the dispatch
// order (one front across the GPU), clear the per-XCD contiguous runs above.
__device__ __forceinline__ int block_unit(int order) {
    return (order & 2) ? (int)blockIdx.x : xcd_remap(blockIdx.x, gridDim.x);
}

template <int CTRL>
__device__ __forceinline__ float dpp_move(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float lane_value(float x, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}

// Sum of v over the wavefront's 64 lanes (all of them must be active), the
// same value in every lane and the same bits for the same inputs.  Within
// each row of 16 lanes by data-parallel moves: pairs (quad_perm 1,0,3,2),
// quads (quad_perm 2,3,0,1), then the row's four quads (rotations by 4 and
// by 8; float addition commutes, so lane 0 of the row holds a fixed tree);
// then the four rows' sums, read from lanes 0, 16, 32, 48, in a fixed order.
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_move<0xB1>(v);
    v += dpp_move<0x4E>(v);
    v += dpp_move<0x124>(v);
    v += dpp_move<0x128>(v);
    return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// Gain partial of coefficient row r of a strip (two output rows, all of the
// strip's columns) for band b: the lanes' products summed across the
// wavefront, written to partial[(r * nstrips + strip) * pstride + b].  One
// entry per (row, strip) whatever unit holds the row, so the reduction over
// them gives the same bits for any unit length or order.  Every lane of the
// wavefront must take part (inactive columns contribute 0).
__device__ __forceinline__ void gain_row(const AdjParams &p, int strip, int r, int b, float dot) {
    if (!p.partial) return;
    const float s = wave_sum(dot);
    if ((threadIdx.x & 63) == 0) p.partial[((int64_t)r * p.nstrips + strip) * p.pstride + b] = s;
}

// Loads NC+2 column pairs (pc[0..NC+1]) of one row; pairs 1..NC are the
// lane's own pixels.
template <int NC, int AL>
__device__ __forceinline__ void load_pairs(const float *row, const int (&pc)[NC + 2], int s0, bool full,
                                           f2 (&x)[NC + 2]) {
    x[0] = ld2<AL>(row + 2 * pc[0]);
    if constexpr (NC == 2 && AL == 2) {
        if (full) {
            const f4 v = *reinterpret_cast<const f4 *>(row + 2 * s0);
            x[1] = f2{v.x, v.y};
            x[2] = f2{v.z, v.w};
        } else {
            x[1] = ld2<AL>(row + 2 * pc[1]);
            x[2] = ld2<AL>(row + 2 * pc[2]);
        }
    } else {
#pragma unroll
        for (int k = 1; k <= NC; ++k) x[k] = ld2<AL>(row + 2 * pc[k]);
    }
    x[NC + 1] = ld2<AL>(row + 2 * pc[NC + 1]);
}

// Per-pixel arithmetic of the D4 adjoint, written as explicit fma chains so
// that every kernel variant (rolling, one-shot, LDS-staged) forms each value
// with the same operations in the same order and they agree bit for bit
// (the compiler contracts free-standing a*b + c differently per kernel).

// Row low-pass at coefficient columns pc[0..NC]: sum_l h_l x(2s+l).
template <int NC>
__device__ __forceinline__ void rowfilt(const float (&h)[4], const f2 (&x)[NC + 2], float (&R)[NC + 1]) {
#pragma unroll
    for (int j = 0; j <= NC; ++j) R[j] = fmaf(h[3], x[j + 1].y, fmaf(h[2], x[j + 1].x, fmaf(h[1], x[j].y, h[0] * x[j].x)));
}

// Column low-pass of four row-filtered rows 2r .. 2r+3: coefficient row r of L.
__device__ __forceinline__ float col4(const float (&h)[4], float r0, float r1, float r2, float r3) {
    return fmaf(h[3], r3, fmaf(h[2], r2, fmaf(h[1], r1, h[0] * r0)));
}

// L^T of an LL-only coefficient image at the lane's pixels of rows 2r (s0)
// and 2r+1 (s1), from coefficient rows r (c) and r-1 (cp) at columns
// pc[0..NC]: pixel (2r+p, 2s+q) = sum_{a,b} h_{p+2a} h_{q+2b} c(r-a, s-b).
template <int NC>
__device__ __forceinline__ void synth_rows(const float (&h)[4], const float (&c)[NC + 1], const float (&cp)[NC + 1],
                                           f2 (&s0)[NC], f2 (&s1)[NC]) {
    float v0[NC + 1], v1[NC + 1];
#pragma unroll
    for (int j = 0; j <= NC; ++j) {
        v0[j] = fmaf(h[2], cp[j], h[0] * c[j]);
        v1[j] = fmaf(h[3], cp[j], h[1] * c[j]);
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        s0[i].x = fmaf(h[2], v0[i], h[0] * v0[i + 1]);
        s0[i].y = fmaf(h[3], v0[i], h[1] * v0[i + 1]);
        s1[i].x = fmaf(h[2], v1[i], h[0] * v1[i + 1]);
        s1[i].y = fmaf(h[3], v1[i], h[1] * v1[i + 1]);
    }
}

template <int NC, int AL>
__device__ __forceinline__ void store_pairs(float *row, int s0, int W2, bool full, const f2 (&q)[NC]) {
    if constexpr (NC == 2 && AL == 2) {
        if (full)
            __builtin_nontemporal_store(f4{q[0].x, q[0].y, q[1].x, q[1].y}, reinterpret_cast<f4 *>(row + 2 * s0));
        else if (s0 < W2)
            st2<AL>(row + 2 * s0, q[0]);
    } else {
#pragma unroll
        for (int i = 0; i < NC; ++i)
            if (s0 + i < W2) st2<AL>(row + 2 * (s0 + i), q[i]);
    }
}

template <int NC, int AL>
__device__ __forceinline__ void store_ms(float *row, int s0, int W2, bool full, const float (&v)[NC]) {
    if constexpr (NC == 2 && AL == 2) {
        if (full)
            __builtin_nontemporal_store(f2{v[0], v[1]}, reinterpret_cast<f2 *>(row + s0));
        else if (s0 < W2)
            row[s0] = v[0];
    } else {
#pragma unroll
        for (int i = 0; i < NC; ++i)
            if (s0 + i < W2) row[s0 + i] = v[i];
    }
}

// ---- D4 adjoint ----------------------------------------------------------

template <int NC, int AL>
__device__ __forceinline__ void d4_adj_unit(const AdjParams &p, const Filters &f, int strip, int seg, int lane) {
    const int W2 = p.W >> 1, H2 = p.H >> 1;
    const int s0 = (strip * 64 + lane) * NC;  // lanes past W2 load wrapped columns and store nothing
    const bool full = (s0 + NC) <= W2;
    bool valid[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) valid[i] = (s0 + i) < W2;
    int pc[NC + 2];
#pragma unroll
    for (int k = 0; k < NC + 2; ++k) pc[k] = wrap_idx(s0 - 1 + k, W2);
    const float h[4] = {f.h[0], f.h[1], f.h[2], f.h[3]};
    const int rb = seg * p.seg_rows;
    const int re = min(rb + p.seg_rows, H2);
    auto wrow = [&](int y) { return y < 0 ? y + p.H : (y >= p.H ? y - p.H : y); };

    // Row-filtered PAN rows 2r, 2r+1 (Ra, Rb), their pixels (xa, xb), and
    // L PAN / L Y at coefficient row r-1 (Ap, LYp), Y = sum_b g_b y_b.
    f2 xa[NC + 2], xb[NC + 2];
    float Ra[NC + 1], Rb[NC + 1], Ap[NC + 1], LYp[NC + 1];
    {
        f2 xt[NC + 2];
        float Rs[NC + 1], Rt[NC + 1];
        load_pairs<NC, AL>(p.pan + (int64_t)wrow(2 * rb - 2) * p.pan_ld, pc, s0, full, xt);
        rowfilt<NC>(h, xt, Rs);
        load_pairs<NC, AL>(p.pan + (int64_t)wrow(2 * rb - 1) * p.pan_ld, pc, s0, full, xt);
        rowfilt<NC>(h, xt, Rt);
        load_pairs<NC, AL>(p.pan + (int64_t)(2 * rb) * p.pan_ld, pc, s0, full, xa);
        load_pairs<NC, AL>(p.pan + (int64_t)(2 * rb + 1) * p.pan_ld, pc, s0, full, xb);
        rowfilt<NC>(h, xa, Ra);
        rowfilt<NC>(h, xb, Rb);
#pragma unroll
        for (int j = 0; j <= NC; ++j) {
            Ap[j] = col4(h, Rs[j], Rt[j], Ra[j], Rb[j]);
            LYp[j] = 0.f;
        }
        for (int b = 0; b < p.B; ++b) {
            const float g = p.gain ? p.gain[b] : 1.0f;
            const float *yb = p.gy + (int64_t)b * p.gy_bs;
            float R4[4][NC + 1];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                load_pairs<NC, AL>(yb + (int64_t)wrow(2 * rb - 2 + k) * p.gy_ld, pc, s0, full, xt);
                rowfilt<NC>(h, xt, R4[k]);
            }
#pragma unroll
            for (int j = 0; j <= NC; ++j) LYp[j] = fmaf(g, col4(h, R4[0][j], R4[1][j], R4[2][j], R4[3][j]), LYp[j]);
        }
    }

    for (int r = rb; r < re; ++r) {
        f2 xc[NC + 2], xd[NC + 2];
        float Rc[NC + 1], Rd[NC + 1], A[NC + 1];
        load_pairs<NC, AL>(p.pan + (int64_t)wrow(2 * r + 2) * p.pan_ld, pc, s0, full, xc);
        load_pairs<NC, AL>(p.pan + (int64_t)wrow(2 * r + 3) * p.pan_ld, pc, s0, full, xd);
        rowfilt<NC>(h, xc, Rc);
        rowfilt<NC>(h, xd, Rd);
#pragma unroll
        for (int j = 0; j <= NC; ++j) A[j] = col4(h, Ra[j], Rb[j], Rc[j], Rd[j]);
        // D = PAN - P PAN at output rows 2r, 2r+1 (own pixels).
        f2 Da[NC], Db[NC];
        {
            f2 sa[NC], sb[NC];
            synth_rows<NC>(h, A, Ap, sa, sb);
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                Da[i] = xa[i + 1] - sa[i];
                Db[i] = xb[i + 1] - sb[i];
            }
        }
        float LY[NC + 1];
        f2 Ya[NC], Yb[NC];
#pragma unroll
        for (int j = 0; j <= NC; ++j) LY[j] = 0.f;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            Ya[i] = f2{0.f, 0.f};
            Yb[i] = f2{0.f, 0.f};
        }
        for (int b = 0; b < p.B; ++b) {
            const float g = p.gain ? p.gain[b] : 1.0f;
            const float *yb = p.gy + (int64_t)b * p.gy_bs;
            f2 z0[NC + 2], z1[NC + 2], zt[NC + 2];
            float R0[NC + 1], R1[NC + 1], R2[NC + 1], R3[NC + 1], Ly[NC + 1];
            load_pairs<NC, AL>(yb + (int64_t)(2 * r) * p.gy_ld, pc, s0, full, z0);
            load_pairs<NC, AL>(yb + (int64_t)(2 * r + 1) * p.gy_ld, pc, s0, full, z1);
            rowfilt<NC>(h, z0, R0);
            rowfilt<NC>(h, z1, R1);
            load_pairs<NC, AL>(yb + (int64_t)wrow(2 * r + 2) * p.gy_ld, pc, s0, full, zt);
            rowfilt<NC>(h, zt, R2);
            load_pairs<NC, AL>(yb + (int64_t)wrow(2 * r + 3) * p.gy_ld, pc, s0, full, zt);
            rowfilt<NC>(h, zt, R3);
#pragma unroll
            for (int j = 0; j <= NC; ++j) Ly[j] = col4(h, R0[j], R1[j], R2[j], R3[j]);
            if (p.grad_ms) {
                float v[NC];
#pragma unroll
                for (int i = 0; i < NC; ++i) v[i] = Ly[i + 1];
                store_ms<NC, AL>(p.grad_ms + (int64_t)b * H2 * W2 + (int64_t)r * W2, s0, W2, full, v);
            }
#pragma unroll
            for (int j = 0; j <= NC; ++j) LY[j] = fmaf(g, Ly[j], LY[j]);
            float dot = 0.f;
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                if (!valid[i]) continue;
                Ya[i].x = fmaf(g, z0[i + 1].x, Ya[i].x);
                Ya[i].y = fmaf(g, z0[i + 1].y, Ya[i].y);
                Yb[i].x = fmaf(g, z1[i + 1].x, Yb[i].x);
                Yb[i].y = fmaf(g, z1[i + 1].y, Yb[i].y);
                dot = fmaf(z0[i + 1].x, Da[i].x, dot);
                dot = fmaf(z0[i + 1].y, Da[i].y, dot);
                dot = fmaf(z1[i + 1].x, Db[i].x, dot);
                dot = fmaf(z1[i + 1].y, Db[i].y, dot);
            }
            gain_row(p, strip, r, b, dot);
        }
        if (p.grad_pan) {
            f2 sa[NC], sb[NC], q0[NC], q1[NC];
            synth_rows<NC>(h, LY, LYp, sa, sb);
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                q0[i] = Ya[i] - sa[i];
                q1[i] = Yb[i] - sb[i];
            }
            float *g0 = p.grad_pan + (int64_t)(2 * r) * p.W;
            float *g1 = g0 + p.W;
            if (p.accumulate) {
#pragma unroll
                for (int i = 0; i < NC; ++i) {
                    if (!valid[i]) continue;
                    const f2 e0 = ld2<AL>(g0 + 2 * (s0 + i)), e1 = ld2<AL>(g1 + 2 * (s0 + i));
                    q0[i] += e0;
                    q1[i] += e1;
                }
            }
            store_pairs<NC, AL>(g0, s0, W2, full, q0);
            store_pairs<NC, AL>(g1, s0, W2, full, q1);
        }
#pragma unroll
        for (int j = 0; j <= NC; ++j) {
            Ap[j] = A[j];
            Ra[j] = Rc[j];
            Rb[j] = Rd[j];
            LYp[j] = LY[j];
        }
#pragma unroll
        for (int k = 0; k < NC + 2; ++k) {
            xa[k] = xc[k];
            xb[k] = xd[k];
        }
    }
}

// ---- D4 adjoint, rolling with a compile-time band group ------------------------
//
// As d4_adj_unit for BG (<= 4) bands, with the band loop unrolled so that the
// loads of all bands' rows are independent and issued together, and with each
// band's last two row-filtered upstream-gradient rows (and their own pixels)
// kept in registers: rows 2r+2, 2r+3 of one step are rows 2r, 2r+1 of the
// next, so every row of y_b is loaded once per unit.  Same fma chains as the
// other D4 adjoints (bit-identical grad_pan / grad_ms).

template <int NC, int AL, int BG>
__device__ __forceinline__ void d4_adj_unit_bg(const AdjParams &p, const Filters &f, int strip, int seg, int lane) {
    const int W2 = p.W >> 1, H2 = p.H >> 1;
    const int s0 = (strip * 64 + lane) * NC;  // lanes past W2 load wrapped columns and store nothing
    const bool full = (s0 + NC) <= W2;
    bool valid[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) valid[i] = (s0 + i) < W2;
    int pc[NC + 2];
#pragma unroll
    for (int k = 0; k < NC + 2; ++k) pc[k] = wrap_idx(s0 - 1 + k, W2);
    const float h[4] = {f.h[0], f.h[1], f.h[2], f.h[3]};
    const int rb = seg * p.seg_rows;
    const int re = min(rb + p.seg_rows, H2);
    auto wrow = [&](int y) { return y < 0 ? y + p.H : (y >= p.H ? y - p.H : y); };
    float g[BG];
    const float *yb[BG];
#pragma unroll
    for (int j = 0; j < BG; ++j) {
        g[j] = p.gain ? p.gain[j] : 1.0f;
        yb[j] = p.gy + (int64_t)j * p.gy_bs;
    }

    f2 xa[NC + 2], xb[NC + 2];
    float Ra[NC + 1], Rb[NC + 1], Ap[NC + 1], LYp[NC + 1];
    // Per band: row-filtered y rows 2r, 2r+1 and their own pixels.
    float Y0[BG][NC + 1], Y1[BG][NC + 1];
    f2 o0[BG][NC], o1[BG][NC];
    {
        f2 xt[NC + 2];
        float Rs[NC + 1], Rt[NC + 1];
        load_pairs<NC, AL>(p.pan + (int64_t)wrow(2 * rb - 2) * p.pan_ld, pc, s0, full, xt);
        rowfilt<NC>(h, xt, Rs);
        load_pairs<NC, AL>(p.pan + (int64_t)wrow(2 * rb - 1) * p.pan_ld, pc, s0, full, xt);
        rowfilt<NC>(h, xt, Rt);
        load_pairs<NC, AL>(p.pan + (int64_t)(2 * rb) * p.pan_ld, pc, s0, full, xa);
        load_pairs<NC, AL>(p.pan + (int64_t)(2 * rb + 1) * p.pan_ld, pc, s0, full, xb);
        rowfilt<NC>(h, xa, Ra);
        rowfilt<NC>(h, xb, Rb);
#pragma unroll
        for (int j = 0; j <= NC; ++j) {
            Ap[j] = col4(h, Rs[j], Rt[j], Ra[j], Rb[j]);
            LYp[j] = 0.f;
        }
#pragma unroll
        for (int bb = 0; bb < BG; ++bb) {
            f2 z[4][NC + 2];
            float R4[4][NC + 1];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                load_pairs<NC, AL>(yb[bb] + (int64_t)wrow(2 * rb - 2 + k) * p.gy_ld, pc, s0, full, z[k]);
                rowfilt<NC>(h, z[k], R4[k]);
            }
#pragma unroll
            for (int j = 0; j <= NC; ++j) {
                LYp[j] = fmaf(g[bb], col4(h, R4[0][j], R4[1][j], R4[2][j], R4[3][j]), LYp[j]);
                Y0[bb][j] = R4[2][j];
                Y1[bb][j] = R4[3][j];
            }
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                o0[bb][i] = z[2][i + 1];
                o1[bb][i] = z[3][i + 1];
            }
        }
    }

    for (int r = rb; r < re; ++r) {
        // Loads of this step: PAN rows 2r+2, 2r+3 and y rows 2r+2, 2r+3 of every band.
        f2 xc[NC + 2], xd[NC + 2];
        f2 zc[BG][NC + 2], zd[BG][NC + 2];
        load_pairs<NC, AL>(p.pan + (int64_t)wrow(2 * r + 2) * p.pan_ld, pc, s0, full, xc);
        load_pairs<NC, AL>(p.pan + (int64_t)wrow(2 * r + 3) * p.pan_ld, pc, s0, full, xd);
#pragma unroll
        for (int bb = 0; bb < BG; ++bb) {
            load_pairs<NC, AL>(yb[bb] + (int64_t)wrow(2 * r + 2) * p.gy_ld, pc, s0, full, zc[bb]);
            load_pairs<NC, AL>(yb[bb] + (int64_t)wrow(2 * r + 3) * p.gy_ld, pc, s0, full, zd[bb]);
        }
        float Rc[NC + 1], Rd[NC + 1], A[NC + 1];
        rowfilt<NC>(h, xc, Rc);
        rowfilt<NC>(h, xd, Rd);
#pragma unroll
        for (int j = 0; j <= NC; ++j) A[j] = col4(h, Ra[j], Rb[j], Rc[j], Rd[j]);
        f2 Da[NC], Db[NC];
        {
            f2 sa[NC], sb[NC];
            synth_rows<NC>(h, A, Ap, sa, sb);
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                Da[i] = xa[i + 1] - sa[i];
                Db[i] = xb[i + 1] - sb[i];
            }
        }
        float LY[NC + 1];
        f2 Ya[NC], Yb[NC];
#pragma unroll
        for (int j = 0; j <= NC; ++j) LY[j] = 0.f;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            Ya[i] = f2{0.f, 0.f};
            Yb[i] = f2{0.f, 0.f};
        }
#pragma unroll
        for (int bb = 0; bb < BG; ++bb) {
            float R2[NC + 1], R3[NC + 1], Ly[NC + 1];
            rowfilt<NC>(h, zc[bb], R2);
            rowfilt<NC>(h, zd[bb], R3);
#pragma unroll
            for (int j = 0; j <= NC; ++j) Ly[j] = col4(h, Y0[bb][j], Y1[bb][j], R2[j], R3[j]);
            if (p.grad_ms) {
                float v[NC];
#pragma unroll
                for (int i = 0; i < NC; ++i) v[i] = Ly[i + 1];
                store_ms<NC, AL>(p.grad_ms + (int64_t)bb * H2 * W2 + (int64_t)r * W2, s0, W2, full, v);
            }
#pragma unroll
            for (int j = 0; j <= NC; ++j) LY[j] = fmaf(g[bb], Ly[j], LY[j]);
            float dot = 0.f;
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                if (!valid[i]) continue;
                Ya[i].x = fmaf(g[bb], o0[bb][i].x, Ya[i].x);
                Ya[i].y = fmaf(g[bb], o0[bb][i].y, Ya[i].y);
                Yb[i].x = fmaf(g[bb], o1[bb][i].x, Yb[i].x);
                Yb[i].y = fmaf(g[bb], o1[bb][i].y, Yb[i].y);
                dot = fmaf(o0[bb][i].x, Da[i].x, dot);
                dot = fmaf(o0[bb][i].y, Da[i].y, dot);
                dot = fmaf(o1[bb][i].x, Db[i].x, dot);
                dot = fmaf(o1[bb][i].y, Db[i].y, dot);
            }
            gain_row(p, strip, r, bb, dot);
#pragma unroll
            for (int j = 0; j <= NC; ++j) {
                Y0[bb][j] = R2[j];
                Y1[bb][j] = R3[j];
            }
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                o0[bb][i] = zc[bb][i + 1];
                o1[bb][i] = zd[bb][i + 1];
            }
        }
        if (p.grad_pan) {
            f2 sa[NC], sb[NC], q0[NC], q1[NC];
            synth_rows<NC>(h, LY, LYp, sa, sb);
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                q0[i] = Ya[i] - sa[i];
                q1[i] = Yb[i] - sb[i];
            }
            float *g0 = p.grad_pan + (int64_t)(2 * r) * p.W;
            float *g1 = g0 + p.W;
            store_pairs<NC, AL>(g0, s0, W2, full, q0);
            store_pairs<NC, AL>(g1, s0, W2, full, q1);
        }
#pragma unroll
        for (int j = 0; j <= NC; ++j) {
            Ap[j] = A[j];
            Ra[j] = Rc[j];
            Rb[j] = Rd[j];
            LYp[j] = LY[j];
        }
#pragma unroll
        for (int k = 0; k < NC + 2; ++k) {
            xa[k] = xc[k];
            xb[k] = xd[k];
        }
    }
}

// ---- D4 adjoint, one-shot tile of KR coefficient rows ----------------------
//
// One wavefront covers KR coefficient rows of a strip: it issues all PAN rows
// 2rb-2 .. 2rb+2KR+1 at once, then, band after band, all of that band's
// upstream-gradient rows at once (the halo rows are re-read from L2).  The
// per-pixel values and the per-row gain products use the shared fma chains
// and operand order above, so all three gradients agree with the rolling
// units bit for bit.

template <int NC, int AL, int KR>
__device__ __forceinline__ void d4_adj_tile(const AdjParams &p, const Filters &f, int strip, int seg, int lane) {
    const int W2 = p.W >> 1, H2 = p.H >> 1;
    const int s0 = (strip * 64 + lane) * NC;  // lanes past W2 load wrapped columns and store nothing
    const bool full = (s0 + NC) <= W2;
    bool valid[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) valid[i] = (s0 + i) < W2;
    int pc[NC + 2];
#pragma unroll
    for (int k = 0; k < NC + 2; ++k) pc[k] = wrap_idx(s0 - 1 + k, W2);
    const float h[4] = {f.h[0], f.h[1], f.h[2], f.h[3]};
    const int rb = seg * KR;
    const int nr = min(KR, H2 - rb);
    constexpr int NR = 2 * KR + 4;  // image rows 2rb-2 .. 2rb+2KR+1
    auto wrow = [&](int y) { return wrap_idx(y, p.H); };

    // D = PAN - P PAN at the lane's pixels of the tile's 2*nr rows.
    f2 D[2 * KR][NC];
    {
        f2 x[NR][NC + 2];
#pragma unroll
        for (int k = 0; k < NR; ++k)
            load_pairs<NC, AL>(p.pan + (int64_t)wrow(2 * rb - 2 + k) * p.pan_ld, pc, s0, full, x[k]);
        float R[NR][NC + 1];
#pragma unroll
        for (int k = 0; k < NR; ++k) rowfilt<NC>(h, x[k], R[k]);
        float A[KR + 1][NC + 1];  // L PAN at coefficient rows rb-1 .. rb+KR-1
#pragma unroll
        for (int i = 0; i <= KR; ++i)
#pragma unroll
            for (int j = 0; j <= NC; ++j) A[i][j] = col4(h, R[2 * i][j], R[2 * i + 1][j], R[2 * i + 2][j], R[2 * i + 3][j]);
#pragma unroll
        for (int i = 0; i < KR; ++i) {
            f2 sa[NC], sb[NC];
            synth_rows<NC>(h, A[i + 1], A[i], sa, sb);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                D[2 * i][c] = x[2 * i + 2][c + 1] - sa[c];
                D[2 * i + 1][c] = x[2 * i + 3][c + 1] - sb[c];
            }
        }
    }
    float LY[KR + 1][NC + 1];
    f2 Y[2 * KR][NC];
#pragma unroll
    for (int i = 0; i <= KR; ++i)
#pragma unroll
        for (int j = 0; j <= NC; ++j) LY[i][j] = 0.f;
#pragma unroll
    for (int t = 0; t < 2 * KR; ++t)
#pragma unroll
        for (int c = 0; c < NC; ++c) Y[t][c] = f2{0.f, 0.f};

    for (int b = 0; b < p.B; ++b) {
        const float *yb = p.gy + (int64_t)b * p.gy_bs;
        f2 z[NR][NC + 2];
#pragma unroll
        for (int k = 0; k < NR; ++k)
            load_pairs<NC, AL>(yb + (int64_t)wrow(2 * rb - 2 + k) * p.gy_ld, pc, s0, full, z[k]);
        const float g = p.gain ? p.gain[b] : 1.0f;
        float R[NR][NC + 1];
#pragma unroll
        for (int k = 0; k < NR; ++k) rowfilt<NC>(h, z[k], R[k]);
#pragma unroll
        for (int i = 0; i <= KR; ++i) {
            // L y_b at coefficient row rb-1+i; rows rb .. rb+nr-1 are this tile's grad_ms.
            float Ly[NC + 1];
#pragma unroll
            for (int j = 0; j <= NC; ++j) Ly[j] = col4(h, R[2 * i][j], R[2 * i + 1][j], R[2 * i + 2][j], R[2 * i + 3][j]);
            if (i >= 1 && i - 1 < nr && p.grad_ms) {
                float v[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) v[c] = Ly[c + 1];
                store_ms<NC, AL>(p.grad_ms + (int64_t)b * H2 * W2 + (int64_t)(rb + i - 1) * W2, s0, W2, full, v);
            }
#pragma unroll
            for (int j = 0; j <= NC; ++j) LY[i][j] = fmaf(g, Ly[j], LY[i][j]);
        }
#pragma unroll
        for (int i = 0; i < KR; ++i) {
            if (i >= nr) break;
            // same operand order as the rolling units: per column, row 2r then 2r+1
            float dot = 0.f;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if (!valid[c]) continue;
                const f2 z0 = z[2 * i + 2][c + 1], z1 = z[2 * i + 3][c + 1];
                Y[2 * i][c].x = fmaf(g, z0.x, Y[2 * i][c].x);
                Y[2 * i][c].y = fmaf(g, z0.y, Y[2 * i][c].y);
                Y[2 * i + 1][c].x = fmaf(g, z1.x, Y[2 * i + 1][c].x);
                Y[2 * i + 1][c].y = fmaf(g, z1.y, Y[2 * i + 1][c].y);
                dot = fmaf(z0.x, D[2 * i][c].x, dot);
                dot = fmaf(z0.y, D[2 * i][c].y, dot);
                dot = fmaf(z1.x, D[2 * i + 1][c].x, dot);
                dot = fmaf(z1.y, D[2 * i + 1][c].y, dot);
            }
            gain_row(p, strip, rb + i, b, dot);
        }
    }
    if (p.grad_pan) {
#pragma unroll
        for (int i = 0; i < KR; ++i) {
            if (i >= nr) break;
            f2 sa[NC], sb[NC], q0[NC], q1[NC];
            synth_rows<NC>(h, LY[i + 1], LY[i], sa, sb);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                q0[c] = Y[2 * i][c] - sa[c];
                q1[c] = Y[2 * i + 1][c] - sb[c];
            }
            float *g0 = p.grad_pan + (int64_t)(2 * (rb + i)) * p.W;
            float *g1 = g0 + p.W;
            if (p.accumulate) {
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    if (!valid[c]) continue;
                    q0[c] += ld2<AL>(g0 + 2 * (s0 + c));
                    q1[c] += ld2<AL>(g1 + 2 * (s0 + c));
                }
            }
            store_pairs<NC, AL>(g0, s0, W2, full, q0);
            store_pairs<NC, AL>(g1, s0, W2, full, q1);
        }
    }
}

// ---- Haar adjoint --------------------------------------------------------

// BG = 0: any band count, in groups of 4 bands; BG = p.B (1..4): the band
// loop unrolled.  Either way a group's upstream-gradient rows are all loaded
// before any is used, and both forms take the same fma chains in the same
// order (bit-identical results).
template <int NC, int AL, int BG>
__device__ __forceinline__ void haar_adj_unit(const AdjParams &p, int strip, int seg, int lane) {
    const int W2 = p.W >> 1, H2 = p.H >> 1;
    const int s0 = (strip * 64 + lane) * NC;
    const bool full = (s0 + NC) <= W2;
    int pc[NC];
    // columns past W2 re-read an inside pair (pair s0, or W2-1 for lanes
    // wholly past the edge); they store nothing and add nothing
#pragma unroll
    for (int i = 0; i < NC; ++i) pc[i] = (s0 + i < W2) ? s0 + i : (s0 < W2 ? s0 : W2 - 1);
    bool valid[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) valid[i] = (s0 + i) < W2;
    const int rb = seg * p.seg_rows;
    const int re = min(rb + p.seg_rows, H2);
    auto load_own = [&](const float *row, f2(&x)[NC]) {
        if constexpr (NC == 2 && AL == 2) {
            if (full) {
                const f4 v = *reinterpret_cast<const f4 *>(row + 2 * s0);
                x[0] = f2{v.x, v.y};
                x[1] = f2{v.z, v.w};
                return;
            }
        }
#pragma unroll
        for (int i = 0; i < NC; ++i) x[i] = ld2<AL>(row + 2 * pc[i]);
    };
    // One band's contribution at coefficient row r: grad_ms (the 2x2 block
    // sums), Y += g y_b, and the gain product <y_b, D> over the lane's pixels.
    auto band = [&](int b, float g, const f2(&z0)[NC], const f2(&z1)[NC], const f2(&Da)[NC], const f2(&Dc)[NC],
                    f2(&Ya)[NC], f2(&Yc)[NC], int r) {
        float bs[NC];
        float dot = 0.f;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            bs[i] = (z0[i].x + z0[i].y) + (z1[i].x + z1[i].y);  // transpose of block repeat
            if (!valid[i]) continue;
            Ya[i].x = fmaf(g, z0[i].x, Ya[i].x);
            Ya[i].y = fmaf(g, z0[i].y, Ya[i].y);
            Yc[i].x = fmaf(g, z1[i].x, Yc[i].x);
            Yc[i].y = fmaf(g, z1[i].y, Yc[i].y);
            dot = fmaf(z0[i].x, Da[i].x, dot);
            dot = fmaf(z0[i].y, Da[i].y, dot);
            dot = fmaf(z1[i].x, Dc[i].x, dot);
            dot = fmaf(z1[i].y, Dc[i].y, dot);
        }
        if (p.grad_ms) store_ms<NC, AL>(p.grad_ms + (int64_t)b * H2 * W2 + (int64_t)r * W2, s0, W2, full, bs);
        gain_row(p, strip, r, b, dot);
    };
    for (int r = rb; r < re; ++r) {
        f2 a[NC], c[NC];
        load_own(p.pan + (int64_t)(2 * r) * p.pan_ld, a);
        load_own(p.pan + (int64_t)(2 * r + 1) * p.pan_ld, c);
        f2 Da[NC], Dc[NC];
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            const float mean = ((a[i].x + a[i].y) + (c[i].x + c[i].y)) * 0.25f;
            Da[i] = f2{a[i].x - mean, a[i].y - mean};
            Dc[i] = f2{c[i].x - mean, c[i].y - mean};
        }
        f2 Ya[NC], Yc[NC];
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            Ya[i] = f2{0.f, 0.f};
            Yc[i] = f2{0.f, 0.f};
        }
        if constexpr (BG > 0) {
            f2 z0[BG][NC], z1[BG][NC];
#pragma unroll
            for (int b = 0; b < BG; ++b) {
                const float *yb = p.gy + (int64_t)b * p.gy_bs;
                load_own(yb + (int64_t)(2 * r) * p.gy_ld, z0[b]);
                load_own(yb + (int64_t)(2 * r + 1) * p.gy_ld, z1[b]);
            }
#pragma unroll
            for (int b = 0; b < BG; ++b) band(b, p.gain ? p.gain[b] : 1.0f, z0[b], z1[b], Da, Dc, Ya, Yc, r);
        } else {
            // bands in groups of 4, each group's rows loaded before any is used
            for (int b0 = 0; b0 < p.B; b0 += 4) {
                f2 z0[4][NC], z1[4][NC];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (b0 + k >= p.B) break;
                    const float *yb = p.gy + (int64_t)(b0 + k) * p.gy_bs;
                    load_own(yb + (int64_t)(2 * r) * p.gy_ld, z0[k]);
                    load_own(yb + (int64_t)(2 * r + 1) * p.gy_ld, z1[k]);
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (b0 + k >= p.B) break;
                    band(b0 + k, p.gain ? p.gain[b0 + k] : 1.0f, z0[k], z1[k], Da, Dc, Ya, Yc, r);
                }
            }
        }
        if (p.grad_pan) {
            f2 q0[NC], q1[NC];
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                const float mean = ((Ya[i].x + Ya[i].y) + (Yc[i].x + Yc[i].y)) * 0.25f;
                q0[i] = f2{Ya[i].x - mean, Ya[i].y - mean};
                q1[i] = f2{Yc[i].x - mean, Yc[i].y - mean};
            }
            float *g0 = p.grad_pan + (int64_t)(2 * r) * p.W;
            float *g1 = g0 + p.W;
            if (p.accumulate) {
#pragma unroll
                for (int i = 0; i < NC; ++i) {
                    if (!valid[i]) continue;
                    q0[i] += ld2<AL>(g0 + 2 * (s0 + i));
                    q1[i] += ld2<AL>(g1 + 2 * (s0 + i));
                }
            }
            store_pairs<NC, AL>(g0, s0, W2, full, q0);
            store_pairs<NC, AL>(g1, s0, W2, full, q1);
        }
    }
}

__device__ __forceinline__ void unit_strip_seg(const AdjParams &p, int unit, int &strip, int &seg) {
    if (p.order & 1) {
        seg = unit / p.nstrips;
        strip = unit - seg * p.nstrips;
    } else {
        strip = unit / p.nseg;
        seg = unit - strip * p.nseg;
    }
}

// One work unit of each adjoint variant, by one wavefront (all 64 lanes).
// Its gain products go to p.partial, one entry per coefficient row and strip
// (gain_row).
//   KIND 0: rolling, any wavelet, p.B <= kAdjMaxBands (X unused)
//   KIND 1: rolling (D4 or Haar) with the band loop unrolled, p.B == X <= 4
//   KIND 2: one-shot D4 tile of X = p.seg_rows coefficient rows
template <int KIND, int NC, int AL, int X>
__device__ __forceinline__ void adj_unit(const AdjParams &p, const Filters &f, int unit, int lane) {
    int strip, seg;
    unit_strip_seg(p, unit, strip, seg);
    if constexpr (KIND == 0) {
        if (p.wavelet == 1)
            d4_adj_unit<NC, AL>(p, f, strip, seg, lane);
        else
            haar_adj_unit<NC, AL, 0>(p, strip, seg, lane);
    } else if constexpr (KIND == 1) {
        if (p.wavelet == 1)
            d4_adj_unit_bg<NC, AL, X>(p, f, strip, seg, lane);
        else
            haar_adj_unit<NC, AL, X>(p, strip, seg, lane);
    } else {
        d4_adj_tile<NC, AL, X>(p, f, strip, seg, lane);
    }
}

// One scene: one wavefront per work unit.
template <int KIND, int NC, int AL, int X>
__global__ __launch_bounds__(256) void adjoint_kernel(AdjParams p, Filters f) {
    const int wpb = blockDim.x >> 6;
    const int lane = threadIdx.x & 63;
    const int unit = block_unit(p.order) * wpb + (threadIdx.x >> 6);
    if (unit >= p.units) return;  // whole wavefront leaves together
    adj_unit<KIND, NC, AL, X>(p, f, unit, lane);
}

// Many scenes of one variant: workgroups of 4 wavefronts, wavefront u of the
// launch takes unit u - unit_begin of the scene whose range holds u.
__device__ __forceinline__ int find_adj_scene(const AdjScene *sc, int n, int u) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sc[mid].unit_begin <= u)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <int KIND, int NC, int AL, int X>
__global__ __launch_bounds__(256) void adjoint_batched_kernel(const AdjScene *__restrict__ scenes, int nscenes,
                                                              int total, Filters f) {
    const int lane = threadIdx.x & 63;
    const int u = xcd_remap(blockIdx.x, gridDim.x) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (u >= total) return;  // whole wavefront leaves together
    const int si = find_adj_scene(scenes, nscenes, u);
    const AdjParams p = scenes[si].p;
    adj_unit<KIND, NC, AL, X>(p, f, u - scenes[si].unit_begin, lane);
}

// ---- grad_gain reduction ----------------------------------------------------
//
// grad_gain[b] = sum over slots of partial[slot * pstride + b], in FP64 with
// a fixed order: chunks of kGainChunk consecutive slots, one workgroup each
// (thread t adds slots t, t + 256, ... of the chunk in turn, then a fixed
// tree over the workgroup), then a band's chunk sums (same scheme).  The
// single-scene and batched launches share both steps, so they agree bit for
// bit.

__device__ __forceinline__ double block_sum256(double a, double *sh) {
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    return sh[0];
}

__device__ __forceinline__ double chunk_sum(const float *partial, int pstride, int band, int units, int c,
                                            double *sh) {
    constexpr int K = kGainChunk / 256;
    const int u0 = c * kGainChunk + (int)threadIdx.x;
    float v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int u = u0 + k * 256;
        v[k] = u < units ? partial[(int64_t)u * pstride + band] : 0.f;
    }
    double a = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) a += (double)v[k];
    return block_sum256(a, sh);
}

__device__ __forceinline__ double chunks_total(const double *chunks, int n, double *sh) {
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) a += chunks[i];
    return block_sum256(a, sh);
}

// Workgroup g: chunk g % nch of band g / nch.
__global__ __launch_bounds__(256) void gain_chunk_kernel(const float *partial, int units, int B, int nch,
                                                         double *chunks) {
    __shared__ double sh[256];
    const int b = blockIdx.x / nch, c = blockIdx.x - b * nch;
    const double a = chunk_sum(partial, B, b, units, c, sh);
    if (threadIdx.x == 0) chunks[(int64_t)b * nch + c] = a;
}

__global__ __launch_bounds__(256) void gain_total_kernel(const double *chunks, int nch, float *grad_gain) {
    __shared__ double sh[256];
    const int b = blockIdx.x;
    const double a = chunks_total(chunks + (int64_t)b * nch, nch, sh);
    if (threadIdx.x == 0) grad_gain[b] = (float)a;
}

// Batched: workgroup g takes chunk g - chunk_begin of the job whose range
// holds g; then one workgroup per job.
__global__ __launch_bounds__(256) void gain_chunk_batched_kernel(const GainJob *__restrict__ jobs, int njobs) {
    __shared__ double sh[256];
    const int g = blockIdx.x;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].chunk_begin <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    const GainJob j = jobs[lo];
    const int c = g - j.chunk_begin;
    const double a = chunk_sum(j.partial, j.pstride, j.band, j.units, c, sh);
    if (threadIdx.x == 0) j.chunks[c] = a;
}

__global__ __launch_bounds__(256) void gain_total_batched_kernel(const GainJob *__restrict__ jobs) {
    __shared__ double sh[256];
    const GainJob j = jobs[blockIdx.x];
    const double a = chunks_total(j.chunks, (j.units + kGainChunk - 1) / kGainChunk, sh);
    if (threadIdx.x == 0) j.grad_gain[j.band] = (float)a;
}

// ---- D4 adjoint, LDS-staged workgroup tile (16- or 8-byte rows) -------------
//
// A workgroup of wpb wavefronts covers a strip of 128 coefficient columns and
// T = wpb * KR coefficient rows.  PAN rows 2r0-2 .. 2r0+2T+1 (with 2-column
// halos) are staged into LDS once; the same rows of each band's upstream
// gradient y_b are staged band after band into two alternating LDS buffers
// (band b+1 is in flight while band b is computed).  Each wavefront keeps
// Y = sum_b g_b y_b and L Y for its KR rows in registers and writes grad_pan
// once at the end, so any band count runs in one launch.  The per-band
// products <y_b, D> go out per coefficient row (gain_row), as in the rolling
// units.

constexpr int kAdjRow = 264;  // floats per staged row: [2,4) left halo, [4,260) own, [260,262) right halo

__device__ __forceinline__ void lds_load4(const float *g, float *l) {
    __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void *)l, 4, 0, 0);
}
__device__ __forceinline__ void lds_load16(const float *g, float *l) {
    __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void *)l, 16, 0, 0);
}

// Stage rows 2r0-2+k (k < 2T+4) of an H x W image (pitch ld) for strip sb:
// 16 bytes per lane on 16-byte rows (A16), else four 4-byte loads per lane,
// each column wrapped on its own.
template <bool A16>
__device__ __forceinline__ void adj_stage_rows(const float *img, int64_t ld, int H, int W, int r0, int T, int sb,
                                               float *dst, int w, int wpb, int lane) {
    for (int k = w; k < 2 * T + 4; k += wpb) {
        const float *row = img + (int64_t)wrap_idx(2 * r0 - 2 + k, H) * ld;
        float *d = dst + k * kAdjRow;
        if constexpr (A16) {
            lds_load16(row + wrap_idx(2 * sb + 4 * lane, W), d + 4);
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) lds_load4(row + wrap_idx(2 * sb + 64 * q + lane, W), d + 4 + 64 * q);
        }
        if (lane < 2) {
            lds_load4(row + wrap_idx(2 * sb - 2 + lane, W), d + 2);
            lds_load4(row + wrap_idx(2 * sb + 256 + lane, W), d + 260);
        }
    }
}

// grad_ms of a lane's two coefficients (one if !full): one 8-byte store on
// 16-byte rows; on 8-byte rows W/2 is odd, so two 4-byte stores.
template <bool A16>
__device__ __forceinline__ void staged_store_ms(float *gm, bool full, float v0, float v1) {
    if (!full) {
        gm[0] = v0;
    } else if constexpr (A16) {
        __builtin_nontemporal_store(f2{v0, v1}, reinterpret_cast<f2 *>(gm));
    } else {
        __builtin_nontemporal_store(v0, gm);
        __builtin_nontemporal_store(v1, gm + 1);
    }
}

// grad_pan of a lane's 2x2 (2x1 if !full) pixel pairs in rows g0 and g0 + W.
template <bool A16>
__device__ __forceinline__ void staged_store_pan(float *g0, int W, bool full, const f2 (&q0)[2], const f2 (&q1)[2]) {
    if (full) {
        if constexpr (A16) {
            __builtin_nontemporal_store(f4{q0[0].x, q0[0].y, q0[1].x, q0[1].y}, reinterpret_cast<f4 *>(g0));
            __builtin_nontemporal_store(f4{q1[0].x, q1[0].y, q1[1].x, q1[1].y}, reinterpret_cast<f4 *>(g0 + W));
        } else {
            __builtin_nontemporal_store(q0[0], reinterpret_cast<f2 *>(g0));
            __builtin_nontemporal_store(q0[1], reinterpret_cast<f2 *>(g0 + 2));
            __builtin_nontemporal_store(q1[0], reinterpret_cast<f2 *>(g0 + W));
            __builtin_nontemporal_store(q1[1], reinterpret_cast<f2 *>(g0 + W + 2));
        }
    } else {
        __builtin_nontemporal_store(q0[0], reinterpret_cast<f2 *>(g0));
        __builtin_nontemporal_store(q1[0], reinterpret_cast<f2 *>(g0 + W));
    }
}

template <int KR, bool A16>
__global__ __launch_bounds__(256) void d4_adjoint_staged_kernel(AdjParams p, Filters f) {
    extern __shared__ float lds[];
    const int wpb = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int T = wpb * KR;
    const int unit = block_unit(p.order);
    if (unit >= p.units) return;  // whole workgroup
    int strip, trow;
    if (p.order & 1) {
        trow = unit / p.nstrips;
        strip = unit - trow * p.nstrips;
    } else {
        strip = unit / p.nseg;
        trow = unit - strip * p.nseg;
    }
    const int W2 = p.W >> 1, H2 = p.H >> 1;
    const int sb = strip * 128, r0 = trow * T;
    const int rows = 2 * T + 4;
    float *Pl = lds;
    float *Yl[2] = {lds + rows * kAdjRow, lds + 2 * rows * kAdjRow};

    adj_stage_rows<A16>(p.pan, p.pan_ld, p.H, p.W, r0, T, sb, Pl, w, wpb, lane);
    adj_stage_rows<A16>(p.gy, p.gy_ld, p.H, p.W, r0, T, sb, Yl[0], w, wpb, lane);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    const int rb = r0 + KR * w;
    const int nr = max(0, min(KR, H2 - rb));
    const int s0 = sb + 2 * lane;
    const bool active = s0 < W2, full = s0 + 2 <= W2;
    const float h[4] = {f.h[0], f.h[1], f.h[2], f.h[3]};
    constexpr int NR = 2 * KR + 4;
    auto read_row = [&](const float *base, int t, f2 (&x)[4]) {
        const float *src = base + (2 * KR * w + t) * kAdjRow + 4 * lane;
        x[0] = *reinterpret_cast<const f2 *>(src + 2);
        const f4 v = *reinterpret_cast<const f4 *>(src + 4);
        x[1] = f2{v.x, v.y};
        x[2] = f2{v.z, v.w};
        x[3] = *reinterpret_cast<const f2 *>(src + 8);
    };
    // L PAN at rows rb-1 .. rb+KR-1, then D = PAN - P PAN at the lane's pixels.
    f2 D[2 * KR][2];
    {
        float R[NR][3];
        f2 own[2 * KR][2];
#pragma unroll
        for (int t = 0; t < NR; ++t) {
            f2 x[4];
            read_row(Pl, t, x);
            rowfilt<2>(h, x, R[t]);
            if (t >= 2 && t < 2 + 2 * KR) {
                own[t - 2][0] = x[1];
                own[t - 2][1] = x[2];
            }
        }
        float A[KR + 1][3];
#pragma unroll
        for (int i = 0; i <= KR; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) A[i][j] = col4(h, R[2 * i][j], R[2 * i + 1][j], R[2 * i + 2][j], R[2 * i + 3][j]);
#pragma unroll
        for (int i = 0; i < KR; ++i) {
            f2 sa[2], sb[2];
            synth_rows<2>(h, A[i + 1], A[i], sa, sb);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                D[2 * i][c] = own[2 * i][c] - sa[c];
                D[2 * i + 1][c] = own[2 * i + 1][c] - sb[c];
            }
        }
    }
    float LY[KR + 1][3];
    f2 Y[2 * KR][2];
#pragma unroll
    for (int i = 0; i <= KR; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) LY[i][j] = 0.f;
#pragma unroll
    for (int t = 0; t < 2 * KR; ++t) Y[t][0] = Y[t][1] = f2{0.f, 0.f};

    for (int b = 0; b < p.B; ++b) {
        const float *Yb = Yl[b & 1];
        if (b + 1 < p.B)  // next band into the other buffer, in flight during this band
            adj_stage_rows<A16>(p.gy + (int64_t)(b + 1) * p.gy_bs, p.gy_ld, p.H, p.W, r0, T, sb, Yl[(b + 1) & 1], w, wpb,
                           lane);
        const float g = p.gain ? p.gain[b] : 1.0f;
        float R[NR][3];
        f2 yo[2 * KR][2];
#pragma unroll
        for (int t = 0; t < NR; ++t) {
            f2 x[4];
            read_row(Yb, t, x);
            rowfilt<2>(h, x, R[t]);
            if (t >= 2 && t < 2 + 2 * KR) {
                yo[t - 2][0] = x[1];
                yo[t - 2][1] = x[2];
            }
        }
        float Ly[KR + 1][3];
#pragma unroll
        for (int i = 0; i <= KR; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) Ly[i][j] = col4(h, R[2 * i][j], R[2 * i + 1][j], R[2 * i + 2][j], R[2 * i + 3][j]);
#pragma unroll
        for (int i = 0; i < KR; ++i) {
            if (i >= nr) break;
            // same operand order as the rolling units: per column, row 2r then 2r+1
            float dot = 0.f;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                if (!active || (c == 1 && !full)) break;
                const f2 z0 = yo[2 * i][c], z1 = yo[2 * i + 1][c];
                Y[2 * i][c].x = fmaf(g, z0.x, Y[2 * i][c].x);
                Y[2 * i][c].y = fmaf(g, z0.y, Y[2 * i][c].y);
                Y[2 * i + 1][c].x = fmaf(g, z1.x, Y[2 * i + 1][c].x);
                Y[2 * i + 1][c].y = fmaf(g, z1.y, Y[2 * i + 1][c].y);
                dot = fmaf(z0.x, D[2 * i][c].x, dot);
                dot = fmaf(z0.y, D[2 * i][c].y, dot);
                dot = fmaf(z1.x, D[2 * i + 1][c].x, dot);
                dot = fmaf(z1.y, D[2 * i + 1][c].y, dot);
            }
            gain_row(p, strip, rb + i, b, dot);
        }
#pragma unroll
        for (int i = 0; i <= KR; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) LY[i][j] = fmaf(g, Ly[i][j], LY[i][j]);
        // Wait for band b+1's rows before this band's stores are issued, so
        // the wait does not include them (the counter also covers stores).
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();  // every wavefront is done with band b's buffer
        if (active && p.grad_ms) {
#pragma unroll
            for (int i = 0; i < KR; ++i) {
                if (i >= nr) break;
                float *gm = p.grad_ms + (int64_t)b * H2 * W2 + (int64_t)(rb + i) * W2 + s0;
                staged_store_ms<A16>(gm, full, Ly[i + 1][1], Ly[i + 1][2]);
            }
        }
    }
    // grad_pan = Y - L^T L Y at the lane's pixels.
    if (p.grad_pan && active) {
#pragma unroll
        for (int i = 0; i < KR; ++i) {
            if (i >= nr) break;
            f2 sa[2], sb[2], q0[2], q1[2];
            synth_rows<2>(h, LY[i + 1], LY[i], sa, sb);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                q0[c] = Y[2 * i][c] - sa[c];
                q1[c] = Y[2 * i + 1][c] - sb[c];
            }
            float *g0 = p.grad_pan + (int64_t)(2 * (rb + i)) * p.W + 2 * s0;
            staged_store_pan<A16>(g0, p.W, full, q0, q1);
        }
    }
}

// The same tile with the upstream gradients of a group of up to bg_all bands
// staged together: PAN and the group's y rows go to LDS at once, one barrier,
// then every band of the group is computed from LDS without further waits
// (per-pixel values as in the kernel above, so results are bit-identical).
template <int KR, bool A16>
__global__ __launch_bounds__(256) void d4_adjoint_staged_all_kernel(AdjParams p, Filters f, int bg_all) {
    extern __shared__ float lds[];
    const int wpb = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int T = wpb * KR;
    const int unit = block_unit(p.order);
    if (unit >= p.units) return;  // whole workgroup
    int strip, trow;
    if (p.order & 1) {
        trow = unit / p.nstrips;
        strip = unit - trow * p.nstrips;
    } else {
        strip = unit / p.nseg;
        trow = unit - strip * p.nseg;
    }
    const int W2 = p.W >> 1, H2 = p.H >> 1;
    const int sb = strip * 128, r0 = trow * T;
    const int rows = 2 * T + 4;
    float *Pl = lds;
    float *Yl = lds + rows * kAdjRow;                  // bg_all images of `rows` rows

    auto stage_group = [&](int g0, int bg) {
        for (int bi = 0; bi < bg; ++bi)
            adj_stage_rows<A16>(p.gy + (int64_t)(g0 + bi) * p.gy_bs, p.gy_ld, p.H, p.W, r0, T, sb, Yl + bi * rows * kAdjRow,
                           w, wpb, lane);
    };
    adj_stage_rows<A16>(p.pan, p.pan_ld, p.H, p.W, r0, T, sb, Pl, w, wpb, lane);
    stage_group(0, min(bg_all, p.B));
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    const int rb = r0 + KR * w;
    const int nr = max(0, min(KR, H2 - rb));
    const int s0 = sb + 2 * lane;
    const bool active = s0 < W2, full = s0 + 2 <= W2;
    const float h[4] = {f.h[0], f.h[1], f.h[2], f.h[3]};
    constexpr int NR = 2 * KR + 4;
    auto read_row = [&](const float *base, int t, f2 (&x)[4]) {
        const float *src = base + (2 * KR * w + t) * kAdjRow + 4 * lane;
        x[0] = *reinterpret_cast<const f2 *>(src + 2);
        const f4 v = *reinterpret_cast<const f4 *>(src + 4);
        x[1] = f2{v.x, v.y};
        x[2] = f2{v.z, v.w};
        x[3] = *reinterpret_cast<const f2 *>(src + 8);
    };
    f2 D[2 * KR][2];
    {
        float R[NR][3];
        f2 own[2 * KR][2];
#pragma unroll
        for (int t = 0; t < NR; ++t) {
            f2 x[4];
            read_row(Pl, t, x);
            rowfilt<2>(h, x, R[t]);
            if (t >= 2 && t < 2 + 2 * KR) {
                own[t - 2][0] = x[1];
                own[t - 2][1] = x[2];
            }
        }
        float A[KR + 1][3];
#pragma unroll
        for (int i = 0; i <= KR; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) A[i][j] = col4(h, R[2 * i][j], R[2 * i + 1][j], R[2 * i + 2][j], R[2 * i + 3][j]);
#pragma unroll
        for (int i = 0; i < KR; ++i) {
            f2 sa[2], sb2[2];
            synth_rows<2>(h, A[i + 1], A[i], sa, sb2);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                D[2 * i][c] = own[2 * i][c] - sa[c];
                D[2 * i + 1][c] = own[2 * i + 1][c] - sb2[c];
            }
        }
    }
    float LY[KR + 1][3];
    f2 Y[2 * KR][2];
#pragma unroll
    for (int i = 0; i <= KR; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) LY[i][j] = 0.f;
#pragma unroll
    for (int t = 0; t < 2 * KR; ++t) Y[t][0] = Y[t][1] = f2{0.f, 0.f};

    for (int g0 = 0; g0 < p.B; g0 += bg_all) {
        const int bg = min(bg_all, p.B - g0);
        if (g0 > 0) {  // every wavefront is done with the previous group's rows
            __syncthreads();
            stage_group(g0, bg);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        }
        for (int bi = 0; bi < bg; ++bi) {
            const int b = g0 + bi;
            const float *Yb = Yl + bi * rows * kAdjRow;
            const float g = p.gain ? p.gain[b] : 1.0f;
            float R[NR][3];
            f2 yo[2 * KR][2];
#pragma unroll
            for (int t = 0; t < NR; ++t) {
                f2 x[4];
                read_row(Yb, t, x);
                rowfilt<2>(h, x, R[t]);
                if (t >= 2 && t < 2 + 2 * KR) {
                    yo[t - 2][0] = x[1];
                    yo[t - 2][1] = x[2];
                }
            }
            float Ly[KR + 1][3];
#pragma unroll
            for (int i = 0; i <= KR; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    Ly[i][j] = col4(h, R[2 * i][j], R[2 * i + 1][j], R[2 * i + 2][j], R[2 * i + 3][j]);
#pragma unroll
            for (int i = 0; i < KR; ++i) {
                if (i >= nr) break;
                // same operand order as the rolling units: per column, row 2r then 2r+1
                float dot = 0.f;
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    if (!active || (c == 1 && !full)) break;
                    const f2 z0 = yo[2 * i][c], z1 = yo[2 * i + 1][c];
                    Y[2 * i][c].x = fmaf(g, z0.x, Y[2 * i][c].x);
                    Y[2 * i][c].y = fmaf(g, z0.y, Y[2 * i][c].y);
                    Y[2 * i + 1][c].x = fmaf(g, z1.x, Y[2 * i + 1][c].x);
                    Y[2 * i + 1][c].y = fmaf(g, z1.y, Y[2 * i + 1][c].y);
                    dot = fmaf(z0.x, D[2 * i][c].x, dot);
                    dot = fmaf(z0.y, D[2 * i][c].y, dot);
                    dot = fmaf(z1.x, D[2 * i + 1][c].x, dot);
                    dot = fmaf(z1.y, D[2 * i + 1][c].y, dot);
                }
                gain_row(p, strip, rb + i, b, dot);
            }
#pragma unroll
            for (int i = 0; i <= KR; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) LY[i][j] = fmaf(g, Ly[i][j], LY[i][j]);
            if (active && p.grad_ms) {
#pragma unroll
                for (int i = 0; i < KR; ++i) {
                    if (i >= nr) break;
                    float *gm = p.grad_ms + (int64_t)b * H2 * W2 + (int64_t)(rb + i) * W2 + s0;
                    staged_store_ms<A16>(gm, full, Ly[i + 1][1], Ly[i + 1][2]);
                }
            }
        }
    }
    if (p.grad_pan && active) {
#pragma unroll
        for (int i = 0; i < KR; ++i) {
            if (i >= nr) break;
            f2 sa[2], sb2[2], q0[2], q1[2];
            synth_rows<2>(h, LY[i + 1], LY[i], sa, sb2);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                q0[c] = Y[2 * i][c] - sa[c];
                q1[c] = Y[2 * i + 1][c] - sb2[c];
            }
            float *g0p = p.grad_pan + (int64_t)(2 * (rb + i)) * p.W + 2 * s0;
            staged_store_pan<A16>(g0p, p.W, full, q0, q1);
        }
    }
}

}  // namespace

// LDS bytes of the staged adjoint for T coefficient rows and B bands.
// Bands whose upstream-gradient rows a staged tile of T rows holds at once
// next to its PAN rows in 64 KB of LDS (all-bands form), at most B.
static int adjoint_staged_group(int T, int B) {
    const int img = (2 * T + 4) * kAdjRow;
    const int g = (16384 - img) / img;
    return g < B ? g : B;
}

size_t adjoint_staged_lds(int T, int B, bool all) {
    const size_t img = (size_t)(2 * T + 4) * kAdjRow;
    if (!all) return sizeof(float) * 3 * img;
    const int g = adjoint_staged_group(T, B);
    return g < 1 ? (size_t)1 << 30 : sizeof(float) * (1 + (size_t)g) * img;
}

hipError_t launch_adjoint_staged(const AdjParams &p, const Filters &f, int kr, int wpb, bool all, hipStream_t s) {
    if (p.units <= 0) return hipSuccess;
    if (p.wavelet != 1 || p.path == PATH_SCALAR || p.seg_rows != kr * wpb || p.nstrips != (p.W / 2 + 127) / 128)
        return hipErrorInvalidValue;
    const bool a16 = p.path == PATH_V4;
    const size_t lds = adjoint_staged_lds(p.seg_rows, p.B, all);
    if (lds > 65536) return hipErrorInvalidValue;
    const dim3 grid(p.units), block(64 * wpb);
    if (all) {
        const int g = adjoint_staged_group(p.seg_rows, p.B);
        switch (kr * 2 + (a16 ? 1 : 0)) {
            case 2: hipLaunchKernelGGL((d4_adjoint_staged_all_kernel<1, false>), grid, block, lds, s, p, f, g); break;
            case 3: hipLaunchKernelGGL((d4_adjoint_staged_all_kernel<1, true>), grid, block, lds, s, p, f, g); break;
            case 4: hipLaunchKernelGGL((d4_adjoint_staged_all_kernel<2, false>), grid, block, lds, s, p, f, g); break;
            case 5: hipLaunchKernelGGL((d4_adjoint_staged_all_kernel<2, true>), grid, block, lds, s, p, f, g); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (kr * 2 + (a16 ? 1 : 0)) {
        case 2: hipLaunchKernelGGL((d4_adjoint_staged_kernel<1, false>), grid, block, lds, s, p, f); break;
        case 3: hipLaunchKernelGGL((d4_adjoint_staged_kernel<1, true>), grid, block, lds, s, p, f); break;
        case 4: hipLaunchKernelGGL((d4_adjoint_staged_kernel<2, false>), grid, block, lds, s, p, f); break;
        case 5: hipLaunchKernelGGL((d4_adjoint_staged_kernel<2, true>), grid, block, lds, s, p, f); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_adjoint(const AdjParams &p, const Filters &f, int wpb, hipStream_t s) {
    if (p.units <= 0) return hipSuccess;
    if (p.B > kAdjMaxBands || p.B < 1) return hipErrorInvalidValue;
    const int grid = (p.units + wpb - 1) / wpb;
    const dim3 block(64 * wpb);
    switch (p.path) {
        case PATH_V4:
            hipLaunchKernelGGL((adjoint_kernel<0, 2, 2, 0>), dim3(grid), block, 0, s, p, f);
            break;
        case PATH_V2:
            hipLaunchKernelGGL((adjoint_kernel<0, 1, 1, 0>), dim3(grid), block, 0, s, p, f);
            break;
        case PATH_V2W:
            hipLaunchKernelGGL((adjoint_kernel<0, 2, 1, 0>), dim3(grid), block, 0, s, p, f);
            break;
        default:
            hipLaunchKernelGGL((adjoint_kernel<0, 1, 0, 0>), dim3(grid), block, 0, s, p, f);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_bg(const AdjParams &p, const Filters &f, int wpb, hipStream_t s) {
    if (p.units <= 0) return hipSuccess;
    if (p.B < 1 || p.B > 4 || p.accumulate || wpb < 1 || wpb > 4) return hipErrorInvalidValue;
    const int grid = (p.units + wpb - 1) / wpb;
    const dim3 block(64 * wpb);
#define ADJ_BG(NC, AL, BG) hipLaunchKernelGGL((adjoint_kernel<1, NC, AL, BG>), dim3(grid), block, 0, s, p, f)
#define ADJ_BG_PATH(BG)                                   \
    do {                                                  \
        if (p.path == PATH_V4) ADJ_BG(2, 2, BG);          \
        else if (p.path == PATH_V2W) ADJ_BG(2, 1, BG);    \
        else if (p.path == PATH_V2) ADJ_BG(1, 1, BG);     \
        else ADJ_BG(1, 0, BG);                            \
    } while (0)
    switch (p.B) {
        case 1: ADJ_BG_PATH(1); break;
        case 2: ADJ_BG_PATH(2); break;
        case 3: ADJ_BG_PATH(3); break;
        default: ADJ_BG_PATH(4); break;
    }
#undef ADJ_BG_PATH
#undef ADJ_BG
    return hipGetLastError();
}

hipError_t launch_adjoint_tile(const AdjParams &p, const Filters &f, int kr, int wpb, hipStream_t s) {
    if (p.units <= 0) return hipSuccess;
    if (p.B > kAdjMaxBands || p.B < 1 || p.wavelet != 1 || p.seg_rows != kr || wpb < 1 || wpb > 4)
        return hipErrorInvalidValue;
    const int grid = (p.units + wpb - 1) / wpb;
    const dim3 block(64 * wpb);
#define ADJ_TILE(NC, AL, KR) hipLaunchKernelGGL((adjoint_kernel<2, NC, AL, KR>), dim3(grid), block, 0, s, p, f)
    if (kr == 1) {
        if (p.path == PATH_V4) ADJ_TILE(2, 2, 1);
        else if (p.path == PATH_V2W) ADJ_TILE(2, 1, 1);
        else if (p.path == PATH_V2) ADJ_TILE(1, 1, 1);
        else ADJ_TILE(1, 0, 1);
    } else if (kr == 2) {
        if (p.path == PATH_V4) ADJ_TILE(2, 2, 2);
        else if (p.path == PATH_V2W) ADJ_TILE(2, 1, 2);
        else if (p.path == PATH_V2) ADJ_TILE(1, 1, 2);
        else ADJ_TILE(1, 0, 2);
    } else {
        return hipErrorInvalidValue;
    }
#undef ADJ_TILE
    return hipGetLastError();
}

hipError_t launch_adjoint_batched(const AdjScene *d_scenes, int nscenes, int total, int kind, int path, int x,
                                  const Filters &f, hipStream_t s) {
    if (nscenes <= 0 || total <= 0) return hipSuccess;
    if (kind < 0 || kind > 2) return hipErrorInvalidValue;
    if ((kind == 1 && (x < 1 || x > 4)) || (kind == 2 && x != 1 && x != 2)) return hipErrorInvalidValue;
    const dim3 grid((total + 3) / 4), block(256);
#define ADJ_B(K, NC, AL, X) \
    hipLaunchKernelGGL((adjoint_batched_kernel<K, NC, AL, X>), grid, block, 0, s, d_scenes, nscenes, total, f)
#define ADJ_B_PATH(K, X)                                  \
    do {                                                  \
        if (path == PATH_V4) ADJ_B(K, 2, 2, X);           \
        else if (path == PATH_V2W) ADJ_B(K, 2, 1, X);     \
        else if (path == PATH_V2) ADJ_B(K, 1, 1, X);      \
        else ADJ_B(K, 1, 0, X);                           \
    } while (0)
    if (kind == 0) {
        ADJ_B_PATH(0, 0);
    } else if (kind == 1) {
        switch (x) {
            case 1: ADJ_B_PATH(1, 1); break;
            case 2: ADJ_B_PATH(1, 2); break;
            case 3: ADJ_B_PATH(1, 3); break;
            default: ADJ_B_PATH(1, 4); break;
        }
    } else {
        if (x == 1) ADJ_B_PATH(2, 1);
        else ADJ_B_PATH(2, 2);
    }
#undef ADJ_B_PATH
#undef ADJ_B
    return hipGetLastError();
}

hipError_t launch_gain_reduce_batched(const GainJob *d_jobs, int njobs, int total_chunks, hipStream_t s) {
    if (njobs <= 0 || total_chunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(gain_chunk_batched_kernel, dim3(total_chunks), dim3(256), 0, s, d_jobs, njobs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gain_total_batched_kernel, dim3(njobs), dim3(256), 0, s, d_jobs);
    return hipGetLastError();
}

hipError_t launch_gain_reduce(const float *partial, int units, int B, double *chunks, float *grad_gain,
                              hipStream_t s) {
    if (B <= 0 || units <= 0) return hipSuccess;
    const int64_t nch = gain_chunks(units);
    if (nch * B > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gain_chunk_kernel, dim3((unsigned)(nch * B)), dim3(256), 0, s, partial, units, B, (int)nch,
                       chunks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gain_total_kernel, dim3(B), dim3(256), 0, s, chunks, (int)nch, grad_gain);
    return hipGetLastError();
}

int adjoint_max_bands() { return kAdjMaxBands; }

}  // namespace dwtf
