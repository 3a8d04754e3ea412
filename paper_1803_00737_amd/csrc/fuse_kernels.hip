// Fused forward-DWT -> replace-LL -> inverse-DWT kernels for gfx950.
//
// Method (section 2 of the paper): out_b = inverse2D(forward2D(PAN) with the
// LL quadrant replaced by MS band b).  The three detail quadrants are scaled
// by a per-band gain g_b (1 = the method as printed).
//
// The kernels evaluate the same linear map in a form that needs one pass and
// no stored coefficients.  Write L for the LL analysis operator (the rows of
// forward2D that produce the LL quadrant) and L^T for its transpose.
//   * D4 (Eq. 3-10 forward, Eq. 13-16 inverse): the 2D transform is
//     orthonormal and its inverse is its transpose, so inverting the detail
//     quadrants of PAN gives PAN - L^T L PAN, and
//         out_b = g_b * PAN + L^T (m_b - g_b * L PAN).
//     Coefficient (r, s) of L PAN is sum_{k,l} h_k h_l PAN(2r+k, 2s+l) with
//     indices taken modulo H and W (the periodic wrap of Eq. 5-6), and output
//     pixel (2r+p, 2s+q) of L^T c is
//         sum_{a,b in {0,1}} h_{p+2a} h_{q+2b} c(r-a, s-b)   (wrapped),
//     which is the transpose pattern of Eq. 13-16.
//   * Haar (Eq. 1-2, 11-12, divided-by-2 form): LL is the 2x2 block mean and
//     the inverse of an LL-only image repeats each coefficient over its block,
//         out_b = m_b(r, s) + g_b * (PAN - mean of its 2x2 block).
//     For integer-valued inputs every intermediate is a multiple of 1/4 below
//     2^10, so this is exact in float32 (and with g = 1 equals the printed
//     method bit for bit).
//
// Work decomposition: one wavefront handles a strip of 64*NC coefficient
// columns (each lane NC columns = 2*NC output columns, 128-bit rows for
// NC = 2) and walks down seg_rows coefficient rows.  D4 keeps a rolling
// window of two row-filtered PAN rows and one row of L PAN in registers, so
// every PAN row is read once per strip plus a 2-row halo at the top of each
// unit; the 1-column horizontal halos are neighbouring lanes' data and hit
// L1.  The PAN-dependent part (L PAN and the PAN pixels) is computed once
// per row pair and reused for all B bands.  Outputs go out with
// non-temporal stores.  Workgroups are remapped so that each XCD (one L2)
// takes a contiguous run of units, i.e. vertically adjacent units of a
// strip, whose halo rows then hit that L2.
#include "fuse_internal.h"

namespace dwtf {

typedef float f2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int wrap_idx(int q, int n) {
    q %= n;
    return q < 0 ? q + n : q;
}

template <bool AL>
__device__ __forceinline__ f2 ld2(const float *p) {
    if constexpr (AL) {
        return *reinterpret_cast<const f2 *>(p);
    } else {
        return f2{p[0], p[1]};
    }
}

template <bool AL>
__device__ __forceinline__ void st2(float *p, f2 v) {
    if constexpr (AL) {
        __builtin_nontemporal_store(v, reinterpret_cast<f2 *>(p));
    } else {
        __builtin_nontemporal_store(v.x, p);
        __builtin_nontemporal_store(v.y, p + 1);
    }
}

__device__ __forceinline__ void st4(float *p, f4 v) {
    __builtin_nontemporal_store(v, reinterpret_cast<f4 *>(p));
}

// Workgroups are dispatched round-robin over the 8 XCDs.  Map hardware
// block b to a logical block so that XCD x gets a contiguous logical range.
__device__ __forceinline__ int xcd_remap(int b, int G) {
    constexpr int NX = 8;
    const int x = b % NX, i = b / NX, q = G / NX, rem = G % NX;
    return x * q + (x < rem ? x : rem) + i;
}

// ---- Daubechies-4 ------------------------------------------------------

template <int NC, bool AL>
__device__ __forceinline__ void d4_unit(const FuseParams &p, const Filters &f, int strip, int seg,
                                        int lane) {
    const int W2 = p.W >> 1, H2 = p.H >> 1;
    const int s0 = (strip * 64 + lane) * NC;  // first own coefficient column
    if (s0 >= W2) return;
    const bool full = (s0 + NC) <= W2;
    // Column pairs (= coefficient columns) s0-1 .. s0+NC, wrapped (Eq. 5-6).
    int pc[NC + 2];
#pragma unroll
    for (int k = 0; k < NC + 2; ++k) pc[k] = wrap_idx(s0 - 1 + k, W2);
    const float h0 = f.h[0], h1 = f.h[1], h2 = f.h[2], h3 = f.h[3];
    const int rb = seg * p.seg_rows;
    const int re = min(rb + p.seg_rows, H2);

    // PAN row y at pairs pc[0..NC+1] (x[1..NC] are this lane's own pixels).
    auto load_row = [&](int y, f2(&x)[NC + 2]) {
        const float *row = p.pan + (int64_t)y * p.pan_ld;
        x[0] = ld2<AL>(row + 2 * pc[0]);
        if constexpr (NC == 2 && AL) {
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
    };
    // Row low-pass at coefficient columns pc[0..NC]: sum_l h_l PAN(y, 2s+l).
    auto rowfilt = [&](const f2(&x)[NC + 2], float(&R)[NC + 1]) {
#pragma unroll
        for (int j = 0; j <= NC; ++j)
            R[j] = fmaf(h3, x[j + 1].y, fmaf(h2, x[j + 1].x, fmaf(h1, x[j].y, h0 * x[j].x)));
    };
    // Column low-pass of four row-filtered rows: one fixed evaluation order,
    // so every output is computed the same way whatever unit it falls in.
    auto colfilt = [&](const float(&R0)[NC + 1], const float(&R1)[NC + 1], const float(&R2)[NC + 1],
                       const float(&R3)[NC + 1], float(&A)[NC + 1]) {
#pragma unroll
        for (int j = 0; j <= NC; ++j) A[j] = fmaf(h3, R3[j], fmaf(h2, R2[j], fmaf(h1, R1[j], h0 * R0[j])));
    };
    auto load_ms = [&](const float *mrow, float(&m)[NC + 1]) {
        m[0] = mrow[pc[0]];
        if constexpr (NC == 2 && AL) {
            if (full) {
                const f2 v = *reinterpret_cast<const f2 *>(mrow + s0);
                m[1] = v.x;
                m[2] = v.y;
            } else {
                m[1] = mrow[pc[1]];
                m[2] = mrow[pc[2]];
            }
        } else {
#pragma unroll
            for (int k = 1; k <= NC; ++k) m[k] = mrow[pc[k]];
        }
    };
    auto store_row = [&](float *orow, const f2(&q)[NC]) {
        if constexpr (NC == 2 && AL) {
            if (full)
                st4(orow + 2 * s0, f4{q[0].x, q[0].y, q[1].x, q[1].y});
            else
                st2<AL>(orow + 2 * s0, q[0]);  // s0 + 1 == W2: one pair left
        } else {
#pragma unroll
            for (int i = 0; i < NC; ++i)
                if (s0 + i < W2) st2<AL>(orow + 2 * (s0 + i), q[i]);
        }
    };

    // Prologue: rows 2rb-2 .. 2rb+1 give L PAN at coefficient row rb-1.
    f2 xa[NC + 2], xb[NC + 2];
    float Ra[NC + 1], Rb[NC + 1], Ap[NC + 1];
    {
        f2 xt[NC + 2];
        float Rs[NC + 1], Rt[NC + 1];
        int y = 2 * rb - 2;
        if (y < 0) y += p.H;
        load_row(y, xt);
        rowfilt(xt, Rs);
        y = 2 * rb - 1;
        if (y < 0) y += p.H;
        load_row(y, xt);
        rowfilt(xt, Rt);
        load_row(2 * rb, xa);
        load_row(2 * rb + 1, xb);
        rowfilt(xa, Ra);
        rowfilt(xb, Rb);
        colfilt(Rs, Rt, Ra, Rb, Ap);
    }

    for (int r = rb; r < re; ++r) {
        int y2 = 2 * r + 2;
        if (y2 >= p.H) y2 -= p.H;
        int y3 = 2 * r + 3;
        if (y3 >= p.H) y3 -= p.H;
        f2 xc[NC + 2], xd[NC + 2];
        load_row(y2, xc);
        load_row(y3, xd);
        float Rc[NC + 1], Rd[NC + 1], A[NC + 1];
        rowfilt(xc, Rc);
        rowfilt(xd, Rd);
        colfilt(Ra, Rb, Rc, Rd, A);
        const int rp = (r == 0) ? H2 - 1 : r - 1;
        for (int b = 0; b < p.B; ++b) {
            const float g = p.gain ? p.gain[b] : 1.0f;
            const float *mb = p.ms + (int64_t)b * p.ms_bs;
            float mc[NC + 1], mp[NC + 1];
            load_ms(mb + (int64_t)r * p.ms_ld, mc);
            load_ms(mb + (int64_t)rp * p.ms_ld, mp);
            float v0[NC + 1], v1[NC + 1];
#pragma unroll
            for (int j = 0; j <= NC; ++j) {
                const float cc = fmaf(-g, A[j], mc[j]);   // coefficient row r
                const float cp = fmaf(-g, Ap[j], mp[j]);  // coefficient row r-1
                v0[j] = fmaf(h2, cp, h0 * cc);             // output row 2r
                v1[j] = fmaf(h3, cp, h1 * cc);             // output row 2r+1
            }
            f2 q0[NC], q1[NC];
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                q0[i].x = fmaf(g, xa[i + 1].x, fmaf(h2, v0[i], h0 * v0[i + 1]));
                q0[i].y = fmaf(g, xa[i + 1].y, fmaf(h3, v0[i], h1 * v0[i + 1]));
                q1[i].x = fmaf(g, xb[i + 1].x, fmaf(h2, v1[i], h0 * v1[i + 1]));
                q1[i].y = fmaf(g, xb[i + 1].y, fmaf(h3, v1[i], h1 * v1[i + 1]));
            }
            float *o0 = p.out + (int64_t)b * p.out_bs + (int64_t)(2 * r) * p.out_ld;
            store_row(o0, q0);
            store_row(o0 + p.out_ld, q1);
        }
#pragma unroll
        for (int j = 0; j <= NC; ++j) {
            Ap[j] = A[j];
            Ra[j] = Rc[j];
            Rb[j] = Rd[j];
        }
#pragma unroll
        for (int k = 0; k < NC + 2; ++k) {
            xa[k] = xc[k];
            xb[k] = xd[k];
        }
    }
}

// ---- Haar ---------------------------------------------------------------

template <int NC, bool AL>
__device__ __forceinline__ void haar_unit(const FuseParams &p, int strip, int seg, int lane) {
    const int W2 = p.W >> 1, H2 = p.H >> 1;
    const int s0 = (strip * 64 + lane) * NC;
    if (s0 >= W2) return;
    const bool full = (s0 + NC) <= W2;
    const int rb = seg * p.seg_rows;
    const int re = min(rb + p.seg_rows, H2);
    for (int r = rb; r < re; ++r) {
        const float *p0 = p.pan + (int64_t)(2 * r) * p.pan_ld;
        const float *p1 = p0 + p.pan_ld;
        f2 a[NC], c[NC];
        if constexpr (NC == 2 && AL) {
            if (full) {
                const f4 u = *reinterpret_cast<const f4 *>(p0 + 2 * s0);
                const f4 v = *reinterpret_cast<const f4 *>(p1 + 2 * s0);
                a[0] = f2{u.x, u.y};
                a[1] = f2{u.z, u.w};
                c[0] = f2{v.x, v.y};
                c[1] = f2{v.z, v.w};
            } else {
                a[0] = ld2<AL>(p0 + 2 * s0);
                c[0] = ld2<AL>(p1 + 2 * s0);
                a[1] = f2{0.f, 0.f};
                c[1] = f2{0.f, 0.f};
            }
        } else {
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                a[i] = ld2<AL>(p0 + 2 * (s0 + i));
                c[i] = ld2<AL>(p1 + 2 * (s0 + i));
            }
        }
        // Detail part of PAN: pixel minus the mean of its 2x2 block (the
        // block mean is the LL coefficient of Eq. 1-2 applied to rows and
        // columns).
        f2 da[NC], dc[NC];
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            const float mean = ((a[i].x + a[i].y) + (c[i].x + c[i].y)) * 0.25f;
            da[i] = f2{a[i].x - mean, a[i].y - mean};
            dc[i] = f2{c[i].x - mean, c[i].y - mean};
        }
        for (int b = 0; b < p.B; ++b) {
            const float g = p.gain ? p.gain[b] : 1.0f;
            const float *mrow = p.ms + (int64_t)b * p.ms_bs + (int64_t)r * p.ms_ld;
            float m[NC];
            if constexpr (NC == 2 && AL) {
                if (full) {
                    const f2 v = *reinterpret_cast<const f2 *>(mrow + s0);
                    m[0] = v.x;
                    m[1] = v.y;
                } else {
                    m[0] = mrow[s0];
                    m[1] = 0.f;
                }
            } else {
#pragma unroll
                for (int i = 0; i < NC; ++i) m[i] = mrow[s0 + i];
            }
            float *o0 = p.out + (int64_t)b * p.out_bs + (int64_t)(2 * r) * p.out_ld;
            float *o1 = o0 + p.out_ld;
            f2 q0[NC], q1[NC];
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                q0[i] = f2{fmaf(g, da[i].x, m[i]), fmaf(g, da[i].y, m[i])};
                q1[i] = f2{fmaf(g, dc[i].x, m[i]), fmaf(g, dc[i].y, m[i])};
            }
            if constexpr (NC == 2 && AL) {
                if (full) {
                    st4(o0 + 2 * s0, f4{q0[0].x, q0[0].y, q0[1].x, q0[1].y});
                    st4(o1 + 2 * s0, f4{q1[0].x, q1[0].y, q1[1].x, q1[1].y});
                } else {
                    st2<AL>(o0 + 2 * s0, q0[0]);
                    st2<AL>(o1 + 2 * s0, q1[0]);
                }
            } else {
#pragma unroll
                for (int i = 0; i < NC; ++i) {
                    st2<AL>(o0 + 2 * (s0 + i), q0[i]);
                    st2<AL>(o1 + 2 * (s0 + i), q1[i]);
                }
            }
        }
    }
}

template <int NC, bool AL>
__device__ __forceinline__ void run_unit(const FuseParams &p, const Filters &f, int unit, int lane) {
    const int strip = unit / p.nseg;
    const int seg = unit - strip * p.nseg;
    if (p.wavelet == 1)
        d4_unit<NC, AL>(p, f, strip, seg, lane);
    else
        haar_unit<NC, AL>(p, strip, seg, lane);
}

// One scene: one wavefront per work unit.
template <int NC, bool AL>
__global__ __launch_bounds__(256) void fuse_kernel(FuseParams p, Filters f) {
    const int wpb = blockDim.x >> 6;
    const int lane = threadIdx.x & 63;
    const int unit = xcd_remap(blockIdx.x, gridDim.x) * wpb + (threadIdx.x >> 6);
    if (unit >= p.units) return;
    run_unit<NC, AL>(p, f, unit, lane);
}

hipError_t launch_fuse(const FuseParams &p, const Filters &f, int wpb, hipStream_t s) {
    if (p.units <= 0) return hipSuccess;
    const int grid = (p.units + wpb - 1) / wpb;
    const dim3 block(64 * wpb);
    switch (p.path) {
        case PATH_V4:
            hipLaunchKernelGGL((fuse_kernel<2, true>), dim3(grid), block, 0, s, p, f);
            break;
        case PATH_V2:
            hipLaunchKernelGGL((fuse_kernel<1, true>), dim3(grid), block, 0, s, p, f);
            break;
        default:
            hipLaunchKernelGGL((fuse_kernel<1, false>), dim3(grid), block, 0, s, p, f);
            break;
    }
    return hipGetLastError();
}

// ---- persistent batched kernel -----------------------------------------
//
// Many scenes of any size, band count, wavelet and alignment in one launch.
// Global work units are split into 8 contiguous queues of about equal bytes,
// one per XCD; a wavefront takes units from its own XCD's queue (so a
// scene's neighbouring units share that XCD's L2) and, when that queue is
// empty, from the others in turn.  The last wavefront to finish resets the
// counters, so the same launch can be replayed from a graph.

__device__ __forceinline__ int find_scene(const BatchScene *sc, int n, int u) {
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

__global__ __launch_bounds__(256) void fuse_batched_kernel(const BatchScene *__restrict__ scenes,
                                                           int nscenes, BatchQueues q,
                                                           uint32_t *counters, Filters f) {
    const int lane = threadIdx.x & 63;
    const int home = blockIdx.x % kQueues;  // the XCD this block runs on
    for (int k = 0; k < kQueues; ++k) {
        const int qi = (home + k) % kQueues;
        uint32_t *ctr = counters + qi * kQueueStride;
        const int qb = q.begin[qi], qe = q.end[qi];
        while (true) {
            int u = 0;
            if (lane == 0) u = qb + (int)atomicAdd(ctr, 1u);
            u = __shfl(u, 0);
            if (u >= qe) break;
            const int si = find_scene(scenes, nscenes, u);
            const FuseParams p = scenes[si].p;
            const int unit = u - scenes[si].unit_begin;
            switch (p.path) {
                case PATH_V4:
                    run_unit<2, true>(p, f, unit, lane);
                    break;
                case PATH_V2:
                    run_unit<1, true>(p, f, unit, lane);
                    break;
                default:
                    run_unit<1, false>(p, f, unit, lane);
                    break;
            }
        }
    }
    // Every wavefront has stopped taking work once it gets here; the last
    // one clears the queue counters and the exit counter for the next launch.
    if (lane == 0) {
        uint32_t *done = counters + kQueues * kQueueStride;
        const uint32_t total = gridDim.x * (blockDim.x >> 6);
        if (atomicAdd(done, 1u) == total - 1) {
            for (int k = 0; k < kQueues; ++k) atomicExch(counters + k * kQueueStride, 0u);
            atomicExch(done, 0u);
        }
    }
}

int batched_blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fuse_batched_kernel, 256, 0) != hipSuccess)
        return 4;
    return n > 0 ? n : 1;
}

hipError_t launch_fuse_batched(const BatchScene *d_scenes, int nscenes, const BatchQueues &q,
                               uint32_t *d_counters, int grid, const Filters &f, hipStream_t s) {
    if (nscenes <= 0 || grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(fuse_batched_kernel, dim3(grid), dim3(256), 0, s, d_scenes, nscenes, q,
                       d_counters, f);
    return hipGetLastError();
}

}  // namespace dwtf
