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
// Work decomposition: a strip of coefficient columns by a run of coefficient
// rows, every band.  Three variants:
//   * rolling (KR = 0): one wavefront walks seg_rows coefficient rows of a
//     strip of 64*NC columns (each lane NC columns = 2*NC output columns,
//     128-bit rows for NC = 2), keeping two row-filtered PAN rows and one row
//     of L PAN in registers, so each PAN row is read once per strip plus a
//     2-row halo per unit;
//   * one-shot (KR = 1 or 2): one wavefront covers KR coefficient rows, issues
//     all its PAN rows (with the 2-row halos) and band 0's MS rows at once,
//     and loads band b+1's MS rows while computing and storing band b; the
//     halo rows are re-read from L2;
//   * LDS-staged D4 tiles (d4_staged_tile): a workgroup of wpb wavefronts
//     copies the PAN rows of its wpb*KR coefficient rows (with the 2-row and
//     2-column halos) and a band group's MS rows straight into LDS, then each
//     wavefront computes its KR rows of every band from there, so the halos
//     are shared instead of re-read.
// All evaluate every output pixel with the same fixed fma chains, so they
// agree bit for bit whatever the tiling.  The PAN-dependent part (L PAN and
// the PAN pixels) is computed once and reused for all B bands.  Outputs go out
// with non-temporal stores.  Units are numbered down column strips or across
// row bands and handed to workgroups in dispatch order (the whole GPU as one
// front) or as one contiguous run per XCD; the LDS-staged tiles also have XCD
// slabs (slab_unit).  Output rows that do not start on a 64-byte boundary are
// covered by overlapped strips (strip_origin), so every stored run is 64-byte
// aligned.
#include "fuse_internal.h"
#include "fuse_math.h"

namespace dwtf {

template <int AL>
__device__ __forceinline__ f2 ld2(const float *p) {
    if constexpr (AL) {
        return *reinterpret_cast<const f2 *>(p);
    } else {
        return f2{p[0], p[1]};
    }
}

template <int AL>
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

// The columns one lane owns: coefficient columns s0 .. s0+NC-1 (output
// columns 2*s0 .. 2*s0+2*NC-1), plus the wrapped neighbours s0-1 and s0+NC
// that D4 needs (Eq. 5-6).  pc[k] = (s0 - 1 + k) mod W/2.
// AL: 0 = 4-byte rows; 1 = aligned rows (8-byte pairs, and with NC = 2
// 16-byte own groups and 8-byte MS pairs); 2 = NC = 2 on 8-byte rows, with
// 16-byte own groups on the rows that are 16-byte aligned and 8-byte MS pairs
// on the MS rows that are 8-byte aligned.  2*s0 is a multiple of 4 when
// NC = 2, so the alignment of a lane's group is that of its row (the same
// for the whole wavefront).
// Pixels [a, e) of the output row starting at orow that a strip stores: the
// strip's run [lo, lo + span) in a row starting on a 64-byte boundary,
// shifted left by the row's misalignment with overlapped strips (see
// strip_origin), and clipped to the image.
__device__ __forceinline__ void stored_span(const float *orow, int lo, int span, int W, int ovl, int &a, int &e) {
    const int phi = ovl ? (int)((reinterpret_cast<uintptr_t>(orow) >> 2) & 15) : 0;
    a = max(lo - phi, 0);
    e = min(lo - phi + span, W);
}

// Lane l receives lane l+1's value (lane 63 gets 0): DPP wave shift left.
__device__ __forceinline__ float from_next_lane(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, false));
}

// The pixel pairs q[0] (pixels x0, x0+1) and q[1] (x0+2, x0+3) of each lane
// (x0 = 2 s0, a multiple of 4 apart from lane to lane) on an output row that
// starts 8 bytes past a 16-byte boundary, as far as the strip stores them
// ([a, e)): each lane writes its second pair and its right neighbour's first
// pair with one 16-byte store (aligned there); a first pair that its left
// neighbour does not write that way is written alone.  Every active lane of
// the wavefront must call it (cross-lane move).
__device__ __forceinline__ void store_pairs_shifted(float *orow, int x0, int a, int e, int lane, const f2 (&q)[2]) {
    const float nx = from_next_lane(q[0].x), ny = from_next_lane(q[0].y);
    const bool in0 = x0 >= a && x0 < e, in1 = x0 + 2 >= a && x0 + 2 < e;
    const bool in2 = lane < 63 && x0 + 4 >= a && x0 + 4 < e;   // the right neighbour's first pair
    const bool left = lane > 0 && x0 - 2 >= a && x0 - 2 < e;    // the left neighbour writes pair x0
    if (in1 && in2) {
        st4(orow + x0 + 2, f4{q[1].x, q[1].y, nx, ny});
    } else if (in1) {
        st2<true>(orow + x0 + 2, q[1]);
    }
    if (in0 && !left) st2<true>(orow + x0, q[0]);
}

template <int NC, int AL>
struct LaneCols {
    int s0, W2;
    bool full;  // all NC own columns inside the image (vector access allowed)
    int ovl;    // overlapped strips
    int lo;     // first pixel of the strip's stored run in a row starting on a 64-byte boundary
    int pc[NC + 2];

    __device__ __forceinline__ LaneCols(int strip, int lane, int W2_, int ovl_) : W2(W2_), ovl(ovl_) {
        s0 = strip_origin(strip, NC, ovl_) + NC * lane;
        lo = 2 * strip * strip_stride_cols(NC, ovl_);
        full = s0 >= 0 && (s0 + NC) <= W2;
#pragma unroll
        for (int k = 0; k < NC + 2; ++k) pc[k] = wrap_idx(s0 - 1 + k, W2);
    }
    __device__ __forceinline__ bool active() const { return s0 < W2 && s0 + NC > 0; }

    static __device__ __forceinline__ bool wide(const float *row) {
        return AL == 1 || (AL == 2 && (reinterpret_cast<uintptr_t>(row) & 15) == 0);
    }
    static __device__ __forceinline__ bool wide_ms(const float *mrow) {
        return AL == 1 || (AL == 2 && (reinterpret_cast<uintptr_t>(mrow) & 7) == 0);
    }

    // Row pairs at pc[0..NC+1] (x[1..NC] are the lane's own pixels).
    __device__ __forceinline__ void load_row(const float *row, f2 (&x)[NC + 2]) const {
        x[0] = ld2<AL>(row + 2 * pc[0]);
        if constexpr (NC == 2 && AL) {
            if (full && wide(row)) {
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
    // Only the lane's own pairs (Haar).
    __device__ __forceinline__ void load_own(const float *row, f2 (&x)[NC]) const {
        if constexpr (NC == 2 && AL) {
            if (full && wide(row)) {
                const f4 v = *reinterpret_cast<const f4 *>(row + 2 * s0);
                x[0] = f2{v.x, v.y};
                x[1] = f2{v.z, v.w};
                return;
            }
        }
#pragma unroll
        for (int i = 0; i < NC; ++i) x[i] = ld2<AL>(row + 2 * pc[i + 1]);
    }
    // MS coefficients at pc[0..NC].
    __device__ __forceinline__ void load_ms(const float *mrow, float (&m)[NC + 1]) const {
        m[0] = mrow[pc[0]];
        if constexpr (NC == 2 && AL) {
            if (full && wide_ms(mrow)) {
                const f2 v = *reinterpret_cast<const f2 *>(mrow + s0);
                m[1] = v.x;
                m[2] = v.y;
                return;
            }
        }
#pragma unroll
        for (int k = 1; k <= NC; ++k) m[k] = mrow[pc[k]];
    }
    // MS coefficients at the lane's own columns only (Haar).
    __device__ __forceinline__ void load_ms_own(const float *mrow, float (&m)[NC]) const {
        if constexpr (NC == 2 && AL) {
            if (full && wide_ms(mrow)) {
                const f2 v = *reinterpret_cast<const f2 *>(mrow + s0);
                m[0] = v.x;
                m[1] = v.y;
                return;
            }
        }
#pragma unroll
        for (int i = 0; i < NC; ++i) m[i] = mrow[pc[i + 1]];
    }
    // orow: the start of the output row.  lane: the lane's index (AL 2:
    // rows 8 bytes off a 16-byte boundary are written with 16-byte stores
    // of pairs shifted by one, store_pairs_shifted).
    __device__ __forceinline__ void store_row(float *orow, const f2 (&q)[NC], int lane) const {
        int a, e;
        stored_span(orow, lo, 2 * strip_stride_cols(NC, ovl), 2 * W2, ovl, a, e);
        if constexpr (NC == 2 && AL == 2) {
            if (!wide(orow)) {
                store_pairs_shifted(orow, 2 * s0, a, e, lane, q);
                return;
            }
        }
        bool in[NC];
#pragma unroll
        for (int i = 0; i < NC; ++i) in[i] = 2 * (s0 + i) >= a && 2 * (s0 + i) < e;
        if constexpr (NC == 2 && AL) {
            if (in[0] && in[1] && wide(orow)) {
                st4(orow + 2 * s0, f4{q[0].x, q[0].y, q[1].x, q[1].y});
            } else {
                if (in[0]) st2<AL>(orow + 2 * s0, q[0]);
                if (in[1]) st2<AL>(orow + 2 * s0 + 2, q[1]);
            }
        } else {
#pragma unroll
            for (int i = 0; i < NC; ++i)
                if (in[i]) st2<AL>(orow + 2 * (s0 + i), q[i]);
        }
    }
};

// ---- Daubechies-4, rolling ----------------------------------------------

template <int NC, int AL>
__device__ __forceinline__ void d4_rolling(const FuseParams &p, const Filters &f, int strip, int seg, int lane) {
    const LaneCols<NC, AL> L(strip, lane, p.W >> 1, p.ovl);
    if (!L.active()) return;
    const int H2 = p.H >> 1;
    const int rb = seg * p.seg_rows;
    const int re = min(rb + p.seg_rows, H2);
    auto row = [&](int y) { return p.pan + (int64_t)y * p.pan_ld; };

    // Prologue: rows 2rb-2 .. 2rb+1 give L PAN at coefficient row rb-1.
    f2 xa[NC + 2], xb[NC + 2];
    float Ra[NC + 1], Rb[NC + 1], Ap[NC + 1];
    {
        f2 xs[NC + 2], xt[NC + 2];
        float Rs[NC + 1], Rt[NC + 1];
        L.load_row(row(wrap_idx(2 * rb - 2, p.H)), xs);
        L.load_row(row(wrap_idx(2 * rb - 1, p.H)), xt);
        L.load_row(row(2 * rb), xa);
        L.load_row(row(2 * rb + 1), xb);
        rowfilt<NC>(f, xs, Rs);
        rowfilt<NC>(f, xt, Rt);
        rowfilt<NC>(f, xa, Ra);
        rowfilt<NC>(f, xb, Rb);
        colfilt<NC>(f, Rs, Rt, Ra, Rb, Ap);
    }

    for (int r = rb; r < re; ++r) {
        f2 xc[NC + 2], xd[NC + 2];
        L.load_row(row(wrap_idx(2 * r + 2, p.H)), xc);
        L.load_row(row(wrap_idx(2 * r + 3, p.H)), xd);
        float Rc[NC + 1], Rd[NC + 1], A[NC + 1];
        rowfilt<NC>(f, xc, Rc);
        rowfilt<NC>(f, xd, Rd);
        colfilt<NC>(f, Ra, Rb, Rc, Rd, A);
        const int rp = (r == 0) ? H2 - 1 : r - 1;
        for (int b = 0; b < p.B; ++b) {
            const float g = p.gain ? p.gain[b] : 1.0f;
            const float *mb = p.ms + (int64_t)b * p.ms_bs;
            float mc[NC + 1], mp[NC + 1];
            L.load_ms(mb + (int64_t)r * p.ms_ld, mc);
            L.load_ms(mb + (int64_t)rp * p.ms_ld, mp);
            f2 q0[NC], q1[NC];
            d4_out_rows<NC>(f, g, p.kappa, mc, mp, A, Ap, xa, xb, q0, q1);
            float *o0 = p.out + (int64_t)b * p.out_bs + (int64_t)(2 * r) * p.out_ld;
            L.store_row(o0, q0, lane);
            L.store_row(o0 + p.out_ld, q1, lane);
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

// ---- Daubechies-4, one-shot tile of KR coefficient rows --------------------

template <int NC, int AL, int KR>
__device__ __forceinline__ void d4_tile(const FuseParams &p, const Filters &f, int strip, int seg, int lane) {
    const LaneCols<NC, AL> L(strip, lane, p.W >> 1, p.ovl);
    if (!L.active()) return;
    const int H2 = p.H >> 1;
    const int rb = seg * KR;
    const int nr = min(KR, H2 - rb);  // coefficient rows in this tile
    constexpr int NR = 2 * KR + 4;     // PAN rows 2rb-2 .. 2rb+2KR+1
    // Every load of the tile is issued before any arithmetic.
    f2 x[NR][NC + 2];
#pragma unroll
    for (int k = 0; k < NR; ++k) L.load_row(p.pan + (int64_t)wrap_idx(2 * rb - 2 + k, p.H) * p.pan_ld, x[k]);
    // MS coefficient rows rb-1 .. rb+KR-1 of one band.
    auto load_band = [&](int b, float(&m)[KR + 1][NC + 1]) {
        const float *mb = p.ms + (int64_t)b * p.ms_bs;
#pragma unroll
        for (int i = 0; i <= KR; ++i) L.load_ms(mb + (int64_t)wrap_idx(rb - 1 + i, H2) * p.ms_ld, m[i]);
    };
    float m[KR + 1][NC + 1];
    load_band(0, m);
    // L PAN at coefficient rows rb-1 .. rb+KR-1.
    float R[NR][NC + 1];
#pragma unroll
    for (int k = 0; k < NR; ++k) rowfilt<NC>(f, x[k], R[k]);
    float A[KR + 1][NC + 1];
#pragma unroll
    for (int i = 0; i <= KR; ++i) colfilt<NC>(f, R[2 * i], R[2 * i + 1], R[2 * i + 2], R[2 * i + 3], A[i]);

    for (int b = 0; b < p.B; ++b) {
        float mn[KR + 1][NC + 1];
        if (b + 1 < p.B) load_band(b + 1, mn);  // in flight while band b is computed and stored
        const float g = p.gain ? p.gain[b] : 1.0f;
        float *ob = p.out + (int64_t)b * p.out_bs;
#pragma unroll
        for (int i = 0; i < KR; ++i) {
            if (i >= nr) break;
            // Coefficient row rb+i: output rows 2(rb+i), 2(rb+i)+1 are PAN rows x[2i+2], x[2i+3].
            f2 q0[NC], q1[NC];
            d4_out_rows<NC>(f, g, p.kappa, m[i + 1], m[i], A[i + 1], A[i], x[2 * i + 2], x[2 * i + 3], q0, q1);
            float *o0 = ob + (int64_t)(2 * (rb + i)) * p.out_ld;
            L.store_row(o0, q0, lane);
            L.store_row(o0 + p.out_ld, q1, lane);
        }
        if (b + 1 < p.B) {
#pragma unroll
            for (int i = 0; i <= KR; ++i)
#pragma unroll
                for (int j = 0; j <= NC; ++j) m[i][j] = mn[i][j];
        }
    }
}

// ---- Haar -----------------------------------------------------------------

template <int NC, int AL>
__device__ __forceinline__ void haar_rolling(const FuseParams &p, int strip, int seg, int lane) {
    const LaneCols<NC, AL> L(strip, lane, p.W >> 1, p.ovl);
    if (!L.active()) return;
    const int H2 = p.H >> 1;
    const int rb = seg * p.seg_rows;
    const int re = min(rb + p.seg_rows, H2);
    for (int r = rb; r < re; ++r) {
        const float *p0 = p.pan + (int64_t)(2 * r) * p.pan_ld;
        f2 a[NC], c[NC], da[NC], dc[NC];
        L.load_own(p0, a);
        L.load_own(p0 + p.pan_ld, c);
        haar_details<NC>(a, c, da, dc);
        for (int b = 0; b < p.B; ++b) {
            const float g = p.gain ? p.gain[b] : 1.0f;
            float m[NC];
            L.load_ms_own(p.ms + (int64_t)b * p.ms_bs + (int64_t)r * p.ms_ld, m);
            f2 q0[NC], q1[NC];
            haar_out_rows<NC>(g, p.kappa, m, da, dc, q0, q1);
            float *o0 = p.out + (int64_t)b * p.out_bs + (int64_t)(2 * r) * p.out_ld;
            L.store_row(o0, q0, lane);
            L.store_row(o0 + p.out_ld, q1, lane);
        }
    }
}

template <int NC, int AL, int KR>
__device__ __forceinline__ void haar_tile(const FuseParams &p, int strip, int seg, int lane) {
    const LaneCols<NC, AL> L(strip, lane, p.W >> 1, p.ovl);
    if (!L.active()) return;
    const int H2 = p.H >> 1;
    const int rb = seg * KR;
    const int nr = min(KR, H2 - rb);
    f2 a[KR][NC], c[KR][NC];
#pragma unroll
    for (int i = 0; i < KR; ++i) {
        const int r = rb + (i < nr ? i : 0);  // rows past the image re-read row rb (unused)
        const float *p0 = p.pan + (int64_t)(2 * r) * p.pan_ld;
        L.load_own(p0, a[i]);
        L.load_own(p0 + p.pan_ld, c[i]);
    }
    auto load_band = [&](int b, float(&m)[KR][NC]) {
        const float *mb = p.ms + (int64_t)b * p.ms_bs;
#pragma unroll
        for (int i = 0; i < KR; ++i) L.load_ms_own(mb + (int64_t)(rb + (i < nr ? i : 0)) * p.ms_ld, m[i]);
    };
    f2 da[KR][NC], dc[KR][NC];
    constexpr int MB = 8;
    if (p.B <= MB) {
        // Up to 8 bands: every MS row of the tile is in flight together with
        // the PAN rows; the wavefront then only computes and stores.
        float mall[MB][KR][NC];
#pragma unroll
        for (int b = 0; b < MB; ++b)
            if (b < p.B) load_band(b, mall[b]);
#pragma unroll
        for (int i = 0; i < KR; ++i) haar_details<NC>(a[i], c[i], da[i], dc[i]);
#pragma unroll
        for (int b = 0; b < MB; ++b) {
            if (b >= p.B) break;
            const float g = p.gain ? p.gain[b] : 1.0f;
            float *ob = p.out + (int64_t)b * p.out_bs;
#pragma unroll
            for (int i = 0; i < KR; ++i) {
                if (i >= nr) break;
                f2 q0[NC], q1[NC];
                haar_out_rows<NC>(g, p.kappa, mall[b][i], da[i], dc[i], q0, q1);
                float *o0 = ob + (int64_t)(2 * (rb + i)) * p.out_ld;
                L.store_row(o0, q0, lane);
                L.store_row(o0 + p.out_ld, q1, lane);
            }
        }
        return;
    }
    float m[KR][NC];
    load_band(0, m);
#pragma unroll
    for (int i = 0; i < KR; ++i) haar_details<NC>(a[i], c[i], da[i], dc[i]);
    for (int b = 0; b < p.B; ++b) {
        float mn[KR][NC];
        if (b + 1 < p.B) load_band(b + 1, mn);
        const float g = p.gain ? p.gain[b] : 1.0f;
        float *ob = p.out + (int64_t)b * p.out_bs;
#pragma unroll
        for (int i = 0; i < KR; ++i) {
            if (i >= nr) break;
            f2 q0[NC], q1[NC];
            haar_out_rows<NC>(g, p.kappa, m[i], da[i], dc[i], q0, q1);
            float *o0 = ob + (int64_t)(2 * (rb + i)) * p.out_ld;
            L.store_row(o0, q0, lane);
            L.store_row(o0 + p.out_ld, q1, lane);
        }
        if (b + 1 < p.B) {
#pragma unroll
            for (int i = 0; i < KR; ++i)
#pragma unroll
                for (int j = 0; j < NC; ++j) m[i][j] = mn[i][j];
        }
    }
}

// Unit numbering.  Row-band-major (order bit 0 set) puts horizontally adjacent
// strips of the same rows next to each other, so with the XCD remap one
// XCD works on a band of rows across the whole width at a time and the
// 1-column halos of neighbouring strips are read while still in its L2.
__device__ __forceinline__ void unit_coords(int unit, int nstrips, int nseg, int order, int &strip, int &seg) {
    if (order & 1) {
        seg = unit / nstrips;
        strip = unit - seg * nstrips;
    } else {
        strip = unit / nseg;
        seg = unit - strip * nseg;
    }
}

// ---- Daubechies-4, LDS-staged workgroup tile --------------------------------
//
// A workgroup of wpb wavefronts covers one strip of 128 coefficient columns
// (256 output columns) and T = wpb * KR coefficient rows.  It stages, with
// direct global-to-LDS loads (no registers held), the T*2 + 4 PAN rows it
// needs (2-row halos above and below, 2-column halos left and right, all
// wrapped) and the T + 1 MS rows of a group of bands, waits once, and then
// each wavefront computes its KR coefficient rows from LDS and streams the
// outputs.  Halos are read once per workgroup instead of once per wavefront.

constexpr int kStagedPanRow = 264;  // floats: [2,4) left halo, [4,260) own, [260,262) right halo
constexpr int kStagedMsRow = 132;   // floats: [3] left halo, [4,132) own

__device__ __forceinline__ void lds_load4(const float *g, float *l) {
    __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void *)l, 4, 0, 0);
}
__device__ __forceinline__ void lds_load16(const float *g, float *l) {
    __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void *)l, 16, 0, 0);
}

// LDS floats for a tile of T coefficient rows and bg bands.
__host__ __device__ constexpr int staged_lds_floats(int T, int bg) {
    return (2 * T + 4) * kStagedPanRow + bg * (T + 1) * kStagedMsRow;
}

// The two pixel pairs of coefficient columns s0, s0+1 of the output row
// starting at orow, as far as this strip stores them (stored_span).
template <int LAY>
__device__ __forceinline__ void staged_store(float *orow, int s0, int lo, int span, int W, int ovl, int lane,
                                             const f2 (&q)[2]) {
    int a, e;
    stored_span(orow, lo, span, W, ovl, a, e);
    const int x = 2 * s0;
    if (LAY == 3 && (reinterpret_cast<uintptr_t>(orow) & 15) != 0) {  // 8-byte rows, this one 8 bytes off
        store_pairs_shifted(orow, x, a, e, lane, q);
        return;
    }
    const bool i0 = x >= a && x < e, i1 = x + 2 >= a && x + 2 < e;
    float *o = orow + x;
    if (i0 && i1 && (LAY == 0 || (reinterpret_cast<uintptr_t>(o) & 15) == 0)) {
        st4(o, f4{q[0].x, q[0].y, q[1].x, q[1].y});
    } else {
        if (i0) st2<true>(o, q[0]);
        if (i1) st2<true>(o + 2, q[1]);
    }
}

// One staged tile (`unit` of p) by the whole workgroup; every wavefront must
// call it (it contains barriers).  LAY follows the row alignment: 0 = 16-byte
// rows (PAN staged with 16-byte loads; a lane owns 2 adjacent coefficient
// columns and stores 16 bytes); 3 = 8-byte rows (PAN staged in 16-byte groups
// aligned per row in strips clear of the wrap, 4-byte loads elsewhere; a lane
// owns 2 adjacent columns and stores 16 bytes on rows 16-byte aligned there,
// 2 x 8 bytes on the others); 2 = 4-byte rows (4-byte staging; a lane owns
// coefficient columns sb+l and sb+64+l and stores their two pixels with two
// 4-byte stores, so each pair of store instructions of the wavefront covers
// one contiguous 512-byte run).
template <int KR, int LAY>
__device__ __forceinline__ void d4_staged_tile(const FuseParams &p, const Filters &f, int bg_max, int unit,
                                               float *lds, int wpb, int b_lo, int b_hi) {
    static_assert(LAY == 0 || LAY == 2 || LAY == 3, "row layouts: 16-, 4- or 8-byte rows");
    // The wavefront index is the same on all its lanes; saying so keeps the
    // tile's row bookkeeping on the scalar unit (about a quarter fewer vector
    // instructions in the kernel).
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int T = wpb * KR;
    int strip, trow;
    unit_coords(unit, p.nstrips, p.nseg, p.order, strip, trow);
    const int W2 = p.W >> 1, H2 = p.H >> 1;
    const int sb = strip_origin(strip, 2, p.ovl);  // first coefficient column of the strip
    const int lo = 2 * strip * strip_stride_cols(2, p.ovl), span = 2 * strip_stride_cols(2, p.ovl);
    const int r0 = trow * T;
    float *Pl = lds;
    float *Ml = lds + (2 * T + 4) * kStagedPanRow;

    // PAN rows 2r0-2 .. 2r0+2T+1.  On the 16-byte path column groups of 4
    // start at multiples of 4; a group straddles the wrap only when
    // W % 4 == 2 (16-byte rows with a pitch padded past an odd W/2), and only
    // in a strip that reaches the right border, which then stages single
    // floats (the group holding pixels W-2, W-1 would otherwise take the row
    // padding where Eq. 5-6 put pixels 0, 1, and its wrapped successors would
    // start 8 bytes off a 16-byte boundary).  The other paths stage single
    // floats, except that on 8-byte rows
    // (LAY 3) strips clear of the wrap stage 16-byte groups starting at pixel
    // 2sb (rows 16-byte aligned there) or 2sb-2 (rows 8 bytes off), the
    // latter placed 2 floats further right in LDS (row shift, see pan_shift).
    // 8-byte rows: a strip whose groups of 4 pixels from 2sb-2 to 2sb+257 all
    // lie inside the row.
    const bool fast = LAY == 3 && sb >= 128 && 2 * sb + 258 <= p.W;
    // 16-byte rows: every group of the strip is 16-byte aligned in the row.
    const bool groups16 = LAY == 0 && ((p.W & 3) == 0 || (sb >= 0 && 2 * sb + 256 <= p.W));
    for (int k = w; k < 2 * T + 4; k += wpb) {
        const float *row = p.pan + (int64_t)wrap_idx(2 * r0 - 2 + k, p.H) * p.pan_ld;
        float *dst = Pl + k * kStagedPanRow;
        if (LAY == 0 && groups16) {
            lds_load16(row + wrap_idx(2 * sb + 4 * lane, p.W), dst + 4);
        } else if (LAY == 3 && fast && (reinterpret_cast<uintptr_t>(row) & 15) != 0) {
            // groups from pixel 2sb-2: LDS 4 + 4l holds pixels 2sb-2+4l .. +3
            lds_load16(row + 2 * sb - 2 + 4 * lane, dst + 4);
            if (lane == 0) lds_load16(row + 2 * sb + 254, dst + 260);
            continue;  // both halos are inside the groups
        } else if (LAY == 3 && fast) {
            lds_load16(row + 2 * sb + 4 * lane, dst + 4);
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) lds_load4(row + wrap_idx(2 * sb + 64 * q + lane, p.W), dst + 4 + 64 * q);
        }
        if (lane < 2) {
            lds_load4(row + wrap_idx(2 * sb - 2 + lane, p.W), dst + 2);
            lds_load4(row + wrap_idx(2 * sb + 256 + lane, p.W), dst + 260);
        }
    }
    // MS rows r0-1 .. r0+T-1 of bands g0 .. g0+bg-1 (b_lo <= g0 < b_hi).
    auto stage_ms = [&](int g0, int bg) {
        for (int k = w; k < bg * (T + 1); k += wpb) {
            const int b = g0 + k / (T + 1), i = k - (k / (T + 1)) * (T + 1);
            const float *row = p.ms + (int64_t)b * p.ms_bs + (int64_t)wrap_idx(r0 - 1 + i, H2) * p.ms_ld;
            float *dst = Ml + k * kStagedMsRow;
            lds_load4(row + wrap_idx(sb + lane, W2), dst + 4);
            lds_load4(row + wrap_idx(sb + 64 + lane, W2), dst + 68);
            if (lane == 0) lds_load4(row + wrap_idx(sb - 1, W2), dst + 3);
        }
    };
    const int bg0 = min(b_hi - b_lo, bg_max);
    stage_ms(b_lo, bg0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    // This wavefront: coefficient rows rb .. rb+KR-1.
    const int rb = r0 + KR * w;
    const int nr = max(0, min(KR, H2 - rb));
    constexpr int NR = 2 * KR + 4;  // PAN rows 2rb-2 .. 2rb+2KR+1 = LDS rows 2KR*w + t
    constexpr int NC = (LAY == 0 || LAY == 3) ? 2 : 1;  // coefficient columns per lane and half
    constexpr int NH = (LAY == 0 || LAY == 3) ? 1 : 2;  // column halves per lane
    // LAY 3: staged row t sits 2 floats right when its row is 8 bytes off a
    // 16-byte boundary in a clear-of-the-wrap strip (the same test as staging).
    auto pan_shift = [&](int t) {
        if constexpr (LAY != 3) {
            return 0;
        } else {
            if (!fast) return 0;
            const float *row = p.pan + (int64_t)wrap_idx(2 * r0 - 2 + 2 * KR * w + t, p.H) * p.pan_ld;
            return (reinterpret_cast<uintptr_t>(row) & 15) != 0 ? 2 : 0;
        }
    };
    // Column layout of half h: first own coefficient column s0[h]; its PAN
    // pairs s0-1 .. s0+NC sit at LDS row positions pos[h] + 2k, MS columns
    // s0-1 .. s0+NC-1 at mpos[h] + k.
    int s0[NH], pos[NH], mpos[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        const int c = (LAY == 0 || LAY == 3) ? 2 * lane : 64 * h + lane;  // offset of s0 within the strip
        s0[h] = sb + c;
        pos[h] = 2 + 2 * c;
        mpos[h] = 3 + c;
    }
    f2 xo[NH][2 * KR][NC];  // the lane's PAN pixels of its output rows
    float A[NH][KR + 1][NC + 1];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        float R[NR][NC + 1];
#pragma unroll
        for (int t = 0; t < NR; ++t) {
            const float *src = Pl + (2 * KR * w + t) * kStagedPanRow + pos[h] + pan_shift(t);
            f2 x[NC + 2];
#pragma unroll
            for (int k = 0; k < NC + 2; ++k) x[k] = *reinterpret_cast<const f2 *>(src + 2 * k);
            rowfilt<NC>(f, x, R[t]);
            if (t >= 2 && t < 2 + 2 * KR) {
#pragma unroll
                for (int i = 0; i < NC; ++i) xo[h][t - 2][i] = x[i + 1];
            }
        }
#pragma unroll
        for (int i = 0; i <= KR; ++i)
            colfilt<NC>(f, R[2 * i], R[2 * i + 1], R[2 * i + 2], R[2 * i + 3], A[h][i]);
    }

    for (int g0 = b_lo; g0 < b_hi; g0 += bg_max) {
        const int bg = min(bg_max, b_hi - g0);
        if (g0 > b_lo) {  // next band group: every wavefront is done with the previous one
            __syncthreads();
            stage_ms(g0, bg);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        }
        for (int bi = 0; bi < bg; ++bi) {
            const int b = g0 + bi;
            const float g = p.gain ? p.gain[b] : 1.0f;
            float *ob = p.out + (int64_t)b * p.out_bs;
#pragma unroll
            for (int h = 0; h < NH; ++h) {
                if (s0[h] >= W2 || s0[h] + NC <= 0) continue;
                float m[KR + 1][NC + 1];
#pragma unroll
                for (int i = 0; i <= KR; ++i) {
                    const float *src = Ml + (bi * (T + 1) + KR * w + i) * kStagedMsRow + mpos[h];
#pragma unroll
                    for (int j = 0; j <= NC; ++j) m[i][j] = src[j];
                }
#pragma unroll
                for (int i = 0; i < KR; ++i) {
                    if (i >= nr) break;
                    // d4_out_rows reads the PAN pixels as pairs 1..NC of a chunk row
                    f2 xa[NC + 2], xb[NC + 2];
#pragma unroll
                    for (int k = 0; k < NC; ++k) {
                        xa[k + 1] = xo[h][2 * i][k];
                        xb[k + 1] = xo[h][2 * i + 1][k];
                    }
                    f2 q0[NC], q1[NC];
                    d4_out_rows<NC>(f, g, p.kappa, m[i + 1], m[i], A[h][i + 1], A[h][i], xa, xb, q0, q1);
                    float *r0 = ob + (int64_t)(2 * (rb + i)) * p.out_ld;  // output rows 2(rb+i), +1
                    if constexpr (LAY == 0 || LAY == 3) {
                        // 16-byte stores where both pairs are stored and the
                        // address is 16-byte aligned (every row on 16-byte rows,
                        // every other one on 8-byte rows), 8-byte ones elsewhere
                        staged_store<LAY>(r0, s0[h], lo, span, p.W, p.ovl, lane, q0);
                        staged_store<LAY>(r0 + p.out_ld, s0[h], lo, span, p.W, p.ovl, lane, q1);
                    } else {
                        float *o0 = r0 + 2 * s0[h];
                        st2<false>(o0, q0[0]);  // 4-byte rows
                        st2<false>(o0 + p.out_ld, q1[0]);
                    }
                }
            }
        }
    }
}

// Bit 2 of the unit order: XCD slabs.  The strips of every row band are cut
// into 8 contiguous chunks, chunk x for XCD x (workgroups are dealt
// round-robin to the 8 XCDs); XCD x walks its chunk row band after row band,
// so horizontally and vertically adjacent tiles share an L2 and the GPU still
// advances down the image together.  With nstrips = 8q + r, the r chunks of
// q + 1 strips go in row band t to XCDs t, t+1, .., t+r-1 (mod 8), so over
// any 8 consecutive row bands every XCD takes 8q + r tiles (fixed chunks would
// leave the XCDs holding the larger ones up to (q+1)/(q+r/8) times as much
// work).  The grid is 8 * slab_slots workgroups; those past their XCD's tiles
// leave at once.
__host__ __device__ inline int64_t slab_slots(int nstrips, int nseg) {
    return (int64_t)(nstrips >> 3) * nseg + (int64_t)(nstrips & 7) * ((nseg + 7) / 8);
}

__device__ __forceinline__ bool slab_unit(int b, int nstrips, int nseg, int &unit) {
    const int x = b & 7, i = b >> 3;
    const int q = nstrips >> 3, r = nstrips & 7;
    const int per = 8 * q + r;  // tiles of one XCD in 8 consecutive row bands
    const int P = i / per;
    int j = i - P * per;
    for (int k = 0; k < 8; ++k) {
        const int t = 8 * P + k;
        if (t >= nseg) return false;
        const int c = q + (((x - t) & 7) < r ? 1 : 0);  // XCD x's chunk in row band t
        if (j < c) {
            int below = 0;  // XCDs below x holding a larger chunk in row band t
            for (int m = 0; m < r; ++m) below += ((t + m) & 7) < x ? 1 : 0;
            unit = t * nstrips + x * q + below + j;  // row-band-major numbering
            return true;
        }
        j -= c;
    }
    return false;
}

template <int KR, int LAY>
__global__ __launch_bounds__(256) void d4_staged_kernel(FuseParams p, Filters f, int bg_max) {
    extern __shared__ float lds[];
    int unit = 0;
    if (p.order & 4) {
        if (!slab_unit(blockIdx.x, p.nstrips, p.nseg, unit)) return;  // whole workgroup
    } else {
        unit = block_unit(p.order);
    }
    if (unit >= p.units) return;  // whole workgroup
    if (p.bsplit > 0) {  // unit = tile * ngroups + group
        const int ng = (p.B + p.bsplit - 1) / p.bsplit;
        const int tile = unit / ng, g = unit - tile * ng;
        const int b_lo = g * p.bsplit;
        d4_staged_tile<KR, LAY>(p, f, bg_max, tile, lds, blockDim.x >> 6, b_lo, min(p.B, b_lo + p.bsplit));
    } else {
        d4_staged_tile<KR, LAY>(p, f, bg_max, unit, lds, blockDim.x >> 6, 0, p.B);
    }
}

template <int KR>
static void launch_staged(const FuseParams &p, const Filters &f, int wpb, size_t lds, int bgm, hipStream_t s) {
    const int grid = (p.order & 4) ? (int)(8 * slab_slots(p.nstrips, p.nseg)) : p.units;
    switch (p.path) {
        case PATH_V4:
            hipLaunchKernelGGL((d4_staged_kernel<KR, 0>), dim3(grid), dim3(64 * wpb), lds, s, p, f, bgm);
            break;
        case PATH_V2:
        case PATH_V2W:
            hipLaunchKernelGGL((d4_staged_kernel<KR, 3>), dim3(grid), dim3(64 * wpb), lds, s, p, f, bgm);
            break;
        default:
            hipLaunchKernelGGL((d4_staged_kernel<KR, 2>), dim3(grid), dim3(64 * wpb), lds, s, p, f, bgm);
            break;
    }
}

// KR = 0: rolling over p.seg_rows rows; KR = 1, 2: one-shot tile (seg_rows == KR).
// WAV = 0 Haar, 1 D4, -1 read from p.wavelet (batched launches mix wavelets).
template <int NC, int AL, int KR, int WAV = -1>
__device__ __forceinline__ void run_unit(const FuseParams &p, const Filters &f, int unit, int lane) {
    int strip, seg;
    unit_coords(unit, p.nstrips, p.nseg, p.order, strip, seg);
    const bool d4 = WAV < 0 ? p.wavelet == 1 : WAV == 1;
    if constexpr (KR == 0) {
        if (d4) {
            if constexpr (WAV != 0) d4_rolling<NC, AL>(p, f, strip, seg, lane);
        } else {
            if constexpr (WAV != 1) haar_rolling<NC, AL>(p, strip, seg, lane);
        }
    } else {
        if (d4) {
            if constexpr (WAV != 0) d4_tile<NC, AL, KR>(p, f, strip, seg, lane);
        } else {
            if constexpr (WAV != 1) haar_tile<NC, AL, KR>(p, strip, seg, lane);
        }
    }
}

// One scene: one wavefront per work unit.  Specialised per wavelet so each
// gets its own register allocation.
template <int WAV, int NC, int AL, int KR>
__global__ __launch_bounds__(256) void fuse_kernel(FuseParams p, Filters f) {
    const int wpb = blockDim.x >> 6;
    const int lane = threadIdx.x & 63;
    const int unit = block_unit(p.order) * wpb + (threadIdx.x >> 6);
    if (unit >= p.units) return;
    run_unit<NC, AL, KR, WAV>(p, f, unit, lane);
}

template <int WAV, int KR>
static void launch_path_w(const FuseParams &p, const Filters &f, int grid, dim3 block, hipStream_t s) {
    switch (p.path) {
        case PATH_V4:
            hipLaunchKernelGGL((fuse_kernel<WAV, 2, true, KR>), dim3(grid), block, 0, s, p, f);
            break;
        case PATH_V2:
            hipLaunchKernelGGL((fuse_kernel<WAV, 1, true, KR>), dim3(grid), block, 0, s, p, f);
            break;
        case PATH_V2W:
            hipLaunchKernelGGL((fuse_kernel<WAV, 2, 2, KR>), dim3(grid), block, 0, s, p, f);
            break;
        default:
            hipLaunchKernelGGL((fuse_kernel<WAV, 1, false, KR>), dim3(grid), block, 0, s, p, f);
            break;
    }
}

template <int KR>
static void launch_path(const FuseParams &p, const Filters &f, int grid, dim3 block, hipStream_t s) {
    if (p.wavelet == 1)
        launch_path_w<1, KR>(p, f, grid, block, s);
    else
        launch_path_w<0, KR>(p, f, grid, block, s);
}

// Largest band group whose MS rows fit next to the PAN rows in 64 KB of LDS.
int staged_bg_max(int T) {
    const int pan = (2 * T + 4) * kStagedPanRow;
    const int per_band = (T + 1) * kStagedMsRow;
    const int bg = (16384 - pan) / per_band;
    return bg < 1 ? 0 : (bg > 8 ? 8 : bg);
}

hipError_t launch_fuse(const FuseParams &p, const Filters &f, int wpb, hipStream_t s) {
    if (p.units <= 0) return hipSuccess;
    if (p.mode >= 3) {  // LDS-staged: one workgroup per unit, KR = mode - 2 rows per wavefront
        const int kr = p.mode - 2;
        if (p.wavelet != 1 || p.seg_rows != wpb * kr || p.nstrips != strip_count(p.W, 2, p.ovl) ||
            (p.ovl && p.path == PATH_SCALAR))
            return hipErrorInvalidValue;
        const int bgm = p.bg > 0 && p.bg < staged_bg_max(p.seg_rows) ? p.bg : staged_bg_max(p.seg_rows);
        if (bgm < 1 || p.bsplit < 0) return hipErrorInvalidValue;
        if ((p.order & 4) && (p.bsplit > 0 || (p.order & 1) == 0 || 8 * slab_slots(p.nstrips, p.nseg) > INT32_MAX))
            return hipErrorInvalidValue;  // slabs: whole tiles, row-band-major numbering
        const int per_unit = p.bsplit > 0 && p.bsplit < p.B ? p.bsplit : p.B;  // bands one unit handles
        const size_t lds = sizeof(float) * staged_lds_floats(p.seg_rows, per_unit < bgm ? per_unit : bgm);
        switch (kr) {
            case 1: launch_staged<1>(p, f, wpb, lds, bgm, s); break;
            case 2: launch_staged<2>(p, f, wpb, lds, bgm, s); break;
            case 4: launch_staged<4>(p, f, wpb, lds, bgm, s); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    const int grid = (p.units + wpb - 1) / wpb;
    const dim3 block(64 * wpb);
    switch (p.mode) {
        case 0: launch_path<0>(p, f, grid, block, s); break;
        case 1: launch_path<1>(p, f, grid, block, s); break;
        case 2: launch_path<2>(p, f, grid, block, s); break;
        default: return hipErrorInvalidValue;
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
// counters, so the same launch can be replayed from a graph.  All scenes of
// one launch use the same variant KR (the host sets seg_rows accordingly).

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

template <int KR>
__global__ __launch_bounds__(256) void fuse_batched_kernel(const BatchScene *__restrict__ scenes, int nscenes,
                                                           BatchQueues q, uint32_t *counters, Filters f) {
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
                    run_unit<2, true, KR>(p, f, unit, lane);
                    break;
                case PATH_V2:
                    run_unit<1, true, KR>(p, f, unit, lane);
                    break;
                case PATH_V2W:
                    run_unit<2, 2, KR>(p, f, unit, lane);
                    break;
                default:
                    run_unit<1, false, KR>(p, f, unit, lane);
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

int batched_blocks_per_cu(int mode) {
    int n = 0;
    hipError_t e;
    switch (mode) {
        case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fuse_batched_kernel<1>, 256, 0); break;
        case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fuse_batched_kernel<2>, 256, 0); break;
        default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fuse_batched_kernel<0>, 256, 0); break;
    }
    if (e != hipSuccess) return 4;
    return n > 0 ? n : 1;
}

hipError_t launch_fuse_batched(const BatchScene *d_scenes, int nscenes, const BatchQueues &q, uint32_t *d_counters,
                               int grid, int mode, const Filters &f, hipStream_t s) {
    if (nscenes <= 0 || grid <= 0) return hipSuccess;
    switch (mode) {
        case 1:
            hipLaunchKernelGGL(fuse_batched_kernel<1>, dim3(grid), dim3(256), 0, s, d_scenes, nscenes, q, d_counters, f);
            break;
        case 2:
            hipLaunchKernelGGL(fuse_batched_kernel<2>, dim3(grid), dim3(256), 0, s, d_scenes, nscenes, q, d_counters, f);
            break;
        default:
            hipLaunchKernelGGL(fuse_batched_kernel<0>, dim3(grid), dim3(256), 0, s, d_scenes, nscenes, q, d_counters, f);
            break;
    }
    return hipGetLastError();
}

// ---- flat batched kernel ------------------------------------------------
//
// One launch, one workgroup of 4 wavefronts per work item: the item is a
// staged LDS tile (mode >= 3 scenes) or 4 consecutive one-shot wavefront units
// (other scenes).  Items of all scenes are numbered consecutively (scene by
// scene, row bands across the width inside a scene) and remapped so that each
// XCD takes a contiguous run; a workgroup finds its scene by binary search.
// Short-lived workgroups keep the memory system busier than a persistent
// queue on this GPU.

__global__ __launch_bounds__(256) void fuse_batched_flat_kernel(const BatchScene *__restrict__ scenes, int nscenes,
                                                                int total, int bg_max, int order, Filters f) {
    extern __shared__ float lds[];
    const int u = block_unit(order);
    if (u >= total) return;
    const int si = find_scene(scenes, nscenes, u);
    const FuseParams p = scenes[si].p;
    const int item = u - scenes[si].unit_begin;
    if (p.mode == 4) {  // staged, 4 wavefronts x 2 rows
        if (p.path == PATH_V4)
            d4_staged_tile<2, 0>(p, f, bg_max, item, lds, 4, 0, p.B);
        else if (p.path == PATH_V2 || p.path == PATH_V2W)
            d4_staged_tile<2, 3>(p, f, bg_max, item, lds, 4, 0, p.B);
        else
            d4_staged_tile<2, 2>(p, f, bg_max, item, lds, 4, 0, p.B);
        return;
    }
    if (p.mode == 3) {  // staged, 4 wavefronts x 1 row
        if (p.path == PATH_V4)
            d4_staged_tile<1, 0>(p, f, bg_max, item, lds, 4, 0, p.B);
        else if (p.path == PATH_V2 || p.path == PATH_V2W)
            d4_staged_tile<1, 3>(p, f, bg_max, item, lds, 4, 0, p.B);
        else
            d4_staged_tile<1, 2>(p, f, bg_max, item, lds, 4, 0, p.B);
        return;
    }
    const int unit = item * 4 + (threadIdx.x >> 6);
    if (unit >= p.units) return;
    const int lane = threadIdx.x & 63;
    switch (p.path) {
        case PATH_V4:
            run_unit<2, true, 1>(p, f, unit, lane);
            break;
        case PATH_V2:
            run_unit<1, true, 1>(p, f, unit, lane);
            break;
        case PATH_V2W:
            run_unit<2, 2, 1>(p, f, unit, lane);
            break;
        default:
            run_unit<1, false, 1>(p, f, unit, lane);
            break;
    }
}

hipError_t launch_fuse_batched_flat(const BatchScene *d_scenes, int nscenes, int total, int staged_bands,
                                    int staged_rows, int order, const Filters &f, hipStream_t s) {
    if (nscenes <= 0 || total <= 0) return hipSuccess;
    if (staged_rows != 1 && staged_rows != 2) return hipErrorInvalidValue;
    const int T = 4 * staged_rows;
    const int bgm = staged_bg_max(T);
    const int bg = staged_bands < bgm ? staged_bands : bgm;
    const size_t lds = bg > 0 ? sizeof(float) * staged_lds_floats(T, bg) : 0;
    hipLaunchKernelGGL(fuse_batched_flat_kernel, dim3(total), dim3(256), lds, s, d_scenes, nscenes, total,
                       bg > 0 ? bg : 1, order, f);
    return hipGetLastError();
}

}  // namespace dwtf
