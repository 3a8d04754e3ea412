// Format variants of the fused kernels for gfx950: 8-bit PAN/MS with 8-bit
// or float32 output, and float32 PAN/MS with 8-bit output, with the scale
// kappa on the MS band where it replaces the LL quadrant (kappa = 1 is the
// method as printed).  Float in and out runs on the float kernels.
//
// The paper moves images at 8 bits per pixel (section 3).  With 8-bit input
// and output a fused pixel costs 1/B + 1/4 + 1 bytes of HBM traffic instead
// of 4/B + 1 + 4, so the same bandwidth carries about four times the pixels.
// Every pixel is computed with the float32 arithmetic of the float kernels
// (fuse_math.h): 8-bit inputs are converted exactly, so the float32 output of
// this path equals dwt_fuse_run's on the same values bit for bit, and the
// 8-bit output is that float32 value rounded to the nearest integer (ties to
// even) and clamped to [0, 255] (NaN -> 0).
//
// Work decomposition: a wavefront covers a strip of 64*NC coefficient columns
// (each lane NC coefficient columns = 2*NC pixels per row: 8 or 16 bytes of
// 8-bit PAN, 16 bytes of float PAN) and a run of coefficient rows of every
// band.  One-shot tiles (KR = 1, 2 rows) issue all their PAN rows (with the
// D4 halo rows and columns, Eq. 5-6 wrap) and the first band's MS rows before
// computing; the float-output tiles load band b+1's MS rows while band b is
// computed and stored, the 8-bit D4 tiles two bands ahead (three rotating
// register sets), the 8-bit Haar tiles every band's rows (up to 8) up front.
// D4 also has rolling units (KR = 0: seg_rows rows, each PAN row filtered
// once) and an LDS-staged form (a workgroup converts its strip's PAN and MS
// rows to float32 in LDS once).
#include "fuse_internal.h"
#include "fuse_math.h"

namespace dwtf {
namespace {

typedef uint32_t u2 __attribute__((ext_vector_type(2)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float byte_at(uint32_t w, int i) { return (float)((w >> (8 * i)) & 0xffu); }

// q mod n for q in [-n, 2n) (two compare/selects instead of an integer divide).
__device__ __forceinline__ int wrap_near(int q, int n) {
    q = q < 0 ? q + n : q;
    return q >= n ? q - n : q;
}

// q mod n for a row index that is the same on every lane of the wavefront
// and lies within a few n of [0, n) (n >= 1): a short scalar loop, no
// integer divide.
__device__ __forceinline__ int wrap_row(int q, int n) {
    while (q < 0) q += n;
    while (q >= n) q -= n;
    return q;
}

// 8-bit code of a fused value: nearest integer, ties to even, clamped to
// [0, 255], NaN -> 0.  The gfx950 float-to-packed-byte conversion does
// exactly this in one instruction per pixel (rounding in the default
// nearest-even mode, saturating, NaN to 0); the parity tests check every
// code against that definition.
__device__ __forceinline__ uint32_t q8(float v) { return __builtin_amdgcn_cvt_pk_u8_f32(v, 0, 0u); }

__device__ __forceinline__ uint32_t pack4(float a, float b, float c, float d) {
    uint32_t w = __builtin_amdgcn_cvt_pk_u8_f32(a, 0, 0u);
    w = __builtin_amdgcn_cvt_pk_u8_f32(b, 1, w);
    w = __builtin_amdgcn_cvt_pk_u8_f32(c, 2, w);
    return __builtin_amdgcn_cvt_pk_u8_f32(d, 3, w);
}

// One pair of pixels (2 elements) starting at p.
template <typename T, bool AL>
__device__ __forceinline__ f2 ld_pair(const T *p) {
    if constexpr (sizeof(T) == 1) {
        if constexpr (AL) {
            const uint32_t v = *reinterpret_cast<const uint16_t *>(p);
            return f2{(float)(v & 0xffu), (float)(v >> 8)};
        } else {
            return f2{(float)p[0], (float)p[1]};
        }
    } else {
        if constexpr (AL) {
            return *reinterpret_cast<const f2 *>(p);
        } else {
            return f2{p[0], p[1]};
        }
    }
}

// The 2*NC pixels a lane owns in one row, as NC pairs (vector load).
template <typename T, int NC>
__device__ __forceinline__ void ld_own_vec(const T *p, f2 *x) {
    if constexpr (sizeof(T) == 1) {
        static_assert(NC == 4 || NC == 8, "8-bit rows: 8 or 16 bytes per lane");
        uint32_t w[NC / 2];
        if constexpr (NC == 4) {
            const u2 v = *reinterpret_cast<const u2 *>(p);
            w[0] = v.x;
            w[1] = v.y;
        } else {
            const u4 v = *reinterpret_cast<const u4 *>(p);
            w[0] = v.x;
            w[1] = v.y;
            w[2] = v.z;
            w[3] = v.w;
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) x[k] = f2{byte_at(w[k >> 1], 2 * (k & 1)), byte_at(w[k >> 1], 2 * (k & 1) + 1)};
    } else {
        static_assert(NC == 2, "float rows: 16 bytes per lane");
        const f4 v = *reinterpret_cast<const f4 *>(p);
        x[0] = f2{v.x, v.y};
        x[1] = f2{v.z, v.w};
    }
}

// The NC MS coefficients a lane owns in one row (vector load).
template <typename T, int NC>
__device__ __forceinline__ void ld_ms_vec(const T *p, float *m) {
    if constexpr (sizeof(T) == 1) {
        if constexpr (NC == 4) {
            const uint32_t v = *reinterpret_cast<const uint32_t *>(p);
#pragma unroll
            for (int k = 0; k < 4; ++k) m[k] = byte_at(v, k);
        } else {
            const u2 v = *reinterpret_cast<const u2 *>(p);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                m[k] = byte_at(v.x, k);
                m[4 + k] = byte_at(v.y, k);
            }
        }
    } else {
        const f2 v = *reinterpret_cast<const f2 *>(p);
        m[0] = v.x;
        m[1] = v.y;
    }
}

// Columns of one lane: coefficient columns s0 .. s0+NC-1 and the wrapped
// neighbours s0-1, s0+NC (pc[k] = (s0 - 1 + k) mod W/2).
template <typename TI, int NC, bool AL>
struct CodecCols {
    int s0, W2;
    bool full;
    int pc[NC + 2];

    __device__ __forceinline__ CodecCols(int strip, int lane, int W2_) : W2(W2_) {
        s0 = (strip * 64 + lane) * NC;
        full = (s0 + NC) <= W2;
        if (W2 > NC + 1) {  // s0 - 1 + k lies in [-1, W2 + NC] within [-W2, 2 W2)
#pragma unroll
            for (int k = 0; k < NC + 2; ++k) pc[k] = wrap_near(s0 - 1 + k, W2);
        } else {
#pragma unroll
            for (int k = 0; k < NC + 2; ++k) pc[k] = wrap_idx(s0 - 1 + k, W2);
        }
    }
    __device__ __forceinline__ bool active() const { return s0 < W2; }
    // Byte offsets of the lane's 8-bit accesses within a row, as opaque 32-bit
    // values: added to a wavefront-uniform row address they make loads and
    // stores of the scalar-base, vector-offset form (no 64-bit vector address
    // arithmetic per access).
    __device__ __forceinline__ static unsigned opaque(unsigned v) {
        asm volatile("" : "+v"(v));
        return v;
    }

    __device__ __forceinline__ void load_row(const TI *row, f2 (&x)[NC + 2]) const {
        x[0] = ld_pair<TI, AL>(row + 2 * pc[0]);
        if (AL && full) {
            ld_own_vec<TI, NC>(row + 2 * s0, &x[1]);
        } else {
#pragma unroll
            for (int k = 1; k <= NC; ++k) x[k] = ld_pair<TI, AL>(row + 2 * pc[k]);
        }
        x[NC + 1] = ld_pair<TI, AL>(row + 2 * pc[NC + 1]);
    }
    // 8-bit rows: the lane's own 2*NC pixels as packed words, and the two halo
    // pairs as 16-bit words (low byte first).
    __device__ __forceinline__ void load_row_raw(const TI *row, uint32_t (&w)[NC / 2], uint32_t &hl,
                                                 uint32_t &hr) const {
        if constexpr (AL) {
            hl = *reinterpret_cast<const uint16_t *>(row + opaque(2u * pc[0]));
            hr = *reinterpret_cast<const uint16_t *>(row + opaque(2u * pc[NC + 1]));
        } else {
            hl = (uint32_t)row[2 * pc[0]] | ((uint32_t)row[2 * pc[0] + 1] << 8);
            hr = (uint32_t)row[2 * pc[NC + 1]] | ((uint32_t)row[2 * pc[NC + 1] + 1] << 8);
        }
        if (AL && full) {
            if constexpr (NC == 4) {
                const u2 v = *reinterpret_cast<const u2 *>(row + opaque(2u * s0));
                w[0] = v.x;
                w[1] = v.y;
            } else {
                const u4 v = *reinterpret_cast<const u4 *>(row + opaque(2u * s0));
                w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
            }
        } else {
#pragma unroll
            for (int j = 0; j < NC / 2; ++j) {
                const uint32_t a0 = row[2 * pc[2 * j + 1]], a1 = row[2 * pc[2 * j + 1] + 1];
                const uint32_t b0 = row[2 * pc[2 * j + 2]], b1 = row[2 * pc[2 * j + 2] + 1];
                w[j] = a0 | (a1 << 8) | (b0 << 16) | (b1 << 24);
            }
        }
    }
    // 8-bit MS row: halo coefficient pc[0] in w[0], own NC coefficients packed in w[1..].
    __device__ __forceinline__ void load_ms_raw(const TI *mrow, uint32_t (&w)[1 + NC / 4]) const {
        w[0] = mrow[opaque(pc[0])];
        if (AL && full) {
            if constexpr (NC == 4) {
                w[1] = *reinterpret_cast<const uint32_t *>(mrow + opaque(s0));
            } else {
                const u2 v = *reinterpret_cast<const u2 *>(mrow + opaque(s0));
                w[1] = v.x;
                w[2] = v.y;
            }
        } else {
#pragma unroll
            for (int j = 0; j < NC / 4; ++j)
                w[1 + j] = (uint32_t)mrow[pc[4 * j + 1]] | ((uint32_t)mrow[pc[4 * j + 2]] << 8) |
                           ((uint32_t)mrow[pc[4 * j + 3]] << 16) | ((uint32_t)mrow[pc[4 * j + 4]] << 24);
        }
    }
    __device__ __forceinline__ void load_own(const TI *row, f2 (&x)[NC]) const {
        if (AL && full) {
            ld_own_vec<TI, NC>(row + 2 * s0, &x[0]);
        } else {
#pragma unroll
            for (int i = 0; i < NC; ++i) x[i] = ld_pair<TI, AL>(row + 2 * pc[i + 1]);
        }
    }
    // MS coefficients at pc[0..NC].
    __device__ __forceinline__ void load_ms(const TI *mrow, float (&m)[NC + 1]) const {
        m[0] = (float)mrow[pc[0]];
        if (AL && full) {
            ld_ms_vec<TI, NC>(mrow + s0, &m[1]);
        } else {
#pragma unroll
            for (int k = 1; k <= NC; ++k) m[k] = (float)mrow[pc[k]];
        }
    }
    // 8-bit MS row: the lane's own NC coefficients packed 4 per word.
    __device__ __forceinline__ void load_ms_own_raw(const TI *mrow, uint32_t (&w)[NC / 4]) const {
        if (AL && full) {
            if constexpr (NC == 4) {
                w[0] = *reinterpret_cast<const uint32_t *>(mrow + s0);
            } else {
                const u2 v = *reinterpret_cast<const u2 *>(mrow + s0);
                w[0] = v.x;
                w[1] = v.y;
            }
        } else {
#pragma unroll
            for (int j = 0; j < NC / 4; ++j)
                w[j] = (uint32_t)mrow[pc[4 * j + 1]] | ((uint32_t)mrow[pc[4 * j + 2]] << 8) |
                       ((uint32_t)mrow[pc[4 * j + 3]] << 16) | ((uint32_t)mrow[pc[4 * j + 4]] << 24);
        }
    }
    __device__ __forceinline__ void load_ms_own(const TI *mrow, float (&m)[NC]) const {
        if (AL && full) {
            ld_ms_vec<TI, NC>(mrow + s0, &m[0]);
        } else {
#pragma unroll
            for (int i = 0; i < NC; ++i) m[i] = (float)mrow[pc[i + 1]];
        }
    }
};

// Store the lane's 2*NC pixels of one output row.
template <typename TO, int NC, bool AL>
__device__ __forceinline__ void store_out(TO *orow, int s0, int W2, bool full, const f2 (&q)[NC]) {
    if constexpr (sizeof(TO) == 1) {
        if (AL && full) {
            uint32_t w[NC / 2];
#pragma unroll
            for (int k = 0; k < NC / 2; ++k) w[k] = pack4(q[2 * k].x, q[2 * k].y, q[2 * k + 1].x, q[2 * k + 1].y);
            unsigned off = 2u * s0;  // opaque 32-bit offset: scalar-base store (see CodecCols::opaque)
            asm volatile("" : "+v"(off));
            if constexpr (NC == 2) {
                __builtin_nontemporal_store(w[0], reinterpret_cast<uint32_t *>(orow + off));
            } else if constexpr (NC == 4) {
                __builtin_nontemporal_store(u2{w[0], w[1]}, reinterpret_cast<u2 *>(orow + off));
            } else {
                __builtin_nontemporal_store(u4{w[0], w[1], w[2], w[3]}, reinterpret_cast<u4 *>(orow + off));
            }
        } else {
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                if (s0 + i < W2) {
                    orow[2 * (s0 + i)] = (uint8_t)q8(q[i].x);
                    orow[2 * (s0 + i) + 1] = (uint8_t)q8(q[i].y);
                }
            }
        }
    } else {
        if (AL && full) {
#pragma unroll
            for (int k = 0; k < NC / 2; ++k)
                __builtin_nontemporal_store(f4{q[2 * k].x, q[2 * k].y, q[2 * k + 1].x, q[2 * k + 1].y},
                                            reinterpret_cast<f4 *>(orow + 2 * (s0 + 2 * k)));
        } else {
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                if (s0 + i < W2) {
                    orow[2 * (s0 + i)] = q[i].x;
                    orow[2 * (s0 + i) + 1] = q[i].y;
                }
            }
        }
    }
}

template <typename TI, typename TO, int NC, int KR, bool AL>
__device__ __forceinline__ void d4_codec_tile(const CodecParams &p, const Filters &f, int strip, int seg, int lane) {
    const CodecCols<TI, NC, AL> L(strip, lane, p.W >> 1);
    if (!L.active()) return;
    const TI *pan = static_cast<const TI *>(p.pan);
    const TI *ms = static_cast<const TI *>(p.ms);
    TO *out = static_cast<TO *>(p.out);
    const int H2 = p.H >> 1;
    const int rb = seg * KR;
    const int nr = min(KR, H2 - rb);
    constexpr int NR = 2 * KR + 4;  // PAN rows 2rb-2 .. 2rb+2KR+1
    // Rows lie in [-2, H + 2KR - 1] and [-1, H2 + KR - 1].
    auto wrow = [](int y, int n) { return wrap_row(y, n); };
    f2 x[NR][NC + 2];
#pragma unroll
    for (int k = 0; k < NR; ++k) L.load_row(pan + (int64_t)wrow(2 * rb - 2 + k, p.H) * p.pan_ld, x[k]);
    int64_t mrow[KR + 1];  // MS row offsets, the same for every band
#pragma unroll
    for (int i = 0; i <= KR; ++i) mrow[i] = (int64_t)wrow(rb - 1 + i, H2) * p.ms_ld;
    auto load_band = [&](int b, float(&m)[KR + 1][NC + 1]) {
        const TI *mb = ms + (int64_t)b * p.ms_bs;
#pragma unroll
        for (int i = 0; i <= KR; ++i) L.load_ms(mb + mrow[i], m[i]);
    };
    const bool unit_kappa = p.kappa == 1.0f;  // kappa * m == m exactly: skip the multiply
    float m[KR + 1][NC + 1];
    load_band(0, m);
    float A[KR + 1][NC + 1];
    {
        float R[NR][NC + 1];
#pragma unroll
        for (int k = 0; k < NR; ++k) rowfilt<NC>(f, x[k], R[k]);
#pragma unroll
        for (int i = 0; i <= KR; ++i) colfilt<NC>(f, R[2 * i], R[2 * i + 1], R[2 * i + 2], R[2 * i + 3], A[i]);
    }
    const float h0 = f.h[0], h1 = f.h[1], h2 = f.h[2], h3 = f.h[3];
    for (int b = 0; b < p.B; ++b) {
        float mn[KR + 1][NC + 1];
        if (b + 1 < p.B) load_band(b + 1, mn);
        const float g = p.gain ? p.gain[b] : 1.0f;
        TO *ob = out + (int64_t)b * p.out_bs;
        // Coefficient rows rb-1 .. rb+KR-1 of (kappa m - g L PAN), each formed
        // once; then the synthesis of d4_out_rows, operation for operation.
        float c[KR + 1][NC + 1];
#pragma unroll
        for (int i = 0; i <= KR; ++i)
#pragma unroll
            for (int j = 0; j <= NC; ++j) c[i][j] = fmaf(-g, A[i][j], unit_kappa ? m[i][j] : p.kappa * m[i][j]);
#pragma unroll
        for (int i = 0; i < KR; ++i) {
            if (i >= nr) break;
            float v0[NC + 1], v1[NC + 1];
#pragma unroll
            for (int j = 0; j <= NC; ++j) {
                v0[j] = fmaf(h2, c[i][j], h0 * c[i + 1][j]);
                v1[j] = fmaf(h3, c[i][j], h1 * c[i + 1][j]);
            }
            const f2(&xa)[NC + 2] = x[2 * i + 2];
            const f2(&xb)[NC + 2] = x[2 * i + 3];
            f2 q0[NC], q1[NC];
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                q0[k].x = fmaf(g, xa[k + 1].x, fmaf(h2, v0[k], h0 * v0[k + 1]));
                q0[k].y = fmaf(g, xa[k + 1].y, fmaf(h3, v0[k], h1 * v0[k + 1]));
                q1[k].x = fmaf(g, xb[k + 1].x, fmaf(h2, v1[k], h0 * v1[k + 1]));
                q1[k].y = fmaf(g, xb[k + 1].y, fmaf(h3, v1[k], h1 * v1[k + 1]));
            }
            TO *o0 = ob + (int64_t)(2 * (rb + i)) * p.out_ld;
            store_out<TO, NC, AL>(o0, L.s0, L.W2, L.full, q0);
            store_out<TO, NC, AL>(o0 + p.out_ld, L.s0, L.W2, L.full, q1);
        }
        if (b + 1 < p.B) {
#pragma unroll
            for (int i = 0; i <= KR; ++i)
#pragma unroll
                for (int j = 0; j <= NC; ++j) m[i][j] = mn[i][j];
        }
    }
}

// D4, 8-bit in and out, one-shot tile: as d4_codec_tile, with the PAN pixels of
// the output rows and the MS rows kept as packed bytes (4 per register) and
// converted where they are used, which keeps the register count low enough
// for three wavefronts per SIMD at 8 coefficient columns and 2 rows per
// lane; the MS rows of later bands are loaded kMsAhead bands ahead (the
// 8-bit path is bound by load latency at its occupancy: two bands ahead
// measured 25-30% faster than one).  Same operations in the same order, so
// the same results.
constexpr int kMsAhead = 2;

// A tile's inputs as loaded: every PAN row (own pixels 4 per word, the two
// halo pairs 2 per word) and the first band's MS rows (halo coefficient in
// word 0, own coefficients 4 per word after it).
template <int NC, int KR>
struct U8Tile {
    static constexpr int NR = 2 * KR + 4;  // PAN rows 2rb-2 .. 2rb+2KR+1
    static constexpr int MW = 1 + NC / 4;
    uint32_t rw[NR][NC / 2], hl[NR], hr[NR];
    uint32_t m[KR + 1][MW];
};

// The tile's inputs straight from global memory.  Rows lie in
// [-2, H + 2KR - 1] and [-1, H2 + KR - 1].
template <int NC, int KR, bool AL>
__device__ __forceinline__ void u8_tile_load(const CodecParams &p, const CodecCols<uint8_t, NC, AL> &L, int rb,
                                             U8Tile<NC, KR> &t) {
    const uint8_t *pan = static_cast<const uint8_t *>(p.pan);
    const uint8_t *ms = static_cast<const uint8_t *>(p.ms);
#pragma unroll
    for (int k = 0; k < U8Tile<NC, KR>::NR; ++k)
        L.load_row_raw(pan + (int64_t)wrap_row(2 * rb - 2 + k, p.H) * p.pan_ld, t.rw[k], t.hl[k], t.hr[k]);
#pragma unroll
    for (int i = 0; i <= KR; ++i) L.load_ms_raw(ms + (int64_t)wrap_row(rb - 1 + i, p.H >> 1) * p.ms_ld, t.m[i]);
}

// Coefficient rows rb .. rb+nr-1 of every band from a loaded tile (the MS
// rows of bands after the first are loaded here).
template <typename TO, int NC, int KR, bool AL>
__device__ __forceinline__ void u8_tile_compute(const CodecParams &p, const Filters &f,
                                                const CodecCols<uint8_t, NC, AL> &L, int rb, int nr,
                                                U8Tile<NC, KR> &t) {
    static_assert(sizeof(TO) == 1 && (NC == 4 || NC == 8), "8-bit in and out");
    const uint8_t *ms = static_cast<const uint8_t *>(p.ms);
    TO *out = static_cast<TO *>(p.out);
    const int H2 = p.H >> 1;
    constexpr int NR = U8Tile<NC, KR>::NR;
    constexpr int MW = U8Tile<NC, KR>::MW;
    uint32_t raw[2 * KR][NC / 2];  // own pixels of the output rows
#pragma unroll
    for (int r = 0; r < 2 * KR; ++r)
#pragma unroll
        for (int j = 0; j < NC / 2; ++j) raw[r][j] = t.rw[r + 2][j];
    int64_t mrow[KR + 1];  // MS row offsets, the same for every band
#pragma unroll
    for (int i = 0; i <= KR; ++i) mrow[i] = (int64_t)wrap_row(rb - 1 + i, H2) * p.ms_ld;
    auto load_band = [&](int b, uint32_t(&m)[KR + 1][MW]) {
        const uint8_t *mb = ms + (int64_t)b * p.ms_bs;
#pragma unroll
        for (int i = 0; i <= KR; ++i) L.load_ms_raw(mb + mrow[i], m[i]);
    };
    const bool unit_kappa = p.kappa == 1.0f;  // kappa * m == m exactly: skip the multiply
    float A[KR + 1][NC + 1];
    {
        float R[NR][NC + 1];
#pragma unroll
        for (int k = 0; k < NR; ++k) {  // each row converted just before it is filtered
            f2 x[NC + 2];
            x[0] = f2{byte_at(t.hl[k], 0), byte_at(t.hl[k], 1)};
#pragma unroll
            for (int j = 0; j < NC; ++j)
                x[j + 1] = f2{byte_at(t.rw[k][j >> 1], 2 * (j & 1)), byte_at(t.rw[k][j >> 1], 2 * (j & 1) + 1)};
            x[NC + 1] = f2{byte_at(t.hr[k], 0), byte_at(t.hr[k], 1)};
            rowfilt<NC>(f, x, R[k]);
        }
#pragma unroll
        for (int i = 0; i <= KR; ++i) colfilt<NC>(f, R[2 * i], R[2 * i + 1], R[2 * i + 2], R[2 * i + 3], A[i]);
    }
    const float h0 = f.h[0], h1 = f.h[1], h2 = f.h[2], h3 = f.h[3];
    // One band from its MS rows mb: coefficient rows rb-1 .. rb+KR-1 of
    // (kappa m - g L PAN), each formed once; then the synthesis of
    // d4_out_rows, operation for operation.
    auto band = [&](int b, const uint32_t(&mb)[KR + 1][MW]) {
        const float g = p.gain ? p.gain[b] : 1.0f;
        TO *ob = out + (int64_t)b * p.out_bs;
        float c[KR + 1][NC + 1];
#pragma unroll
        for (int i = 0; i <= KR; ++i)
#pragma unroll
            for (int j = 0; j <= NC; ++j) {
                const float mv = j == 0 ? (float)mb[i][0] : byte_at(mb[i][1 + ((j - 1) >> 2)], (j - 1) & 3);
                c[i][j] = fmaf(-g, A[i][j], unit_kappa ? mv : p.kappa * mv);
            }
#pragma unroll
        for (int i = 0; i < KR; ++i) {
            if (i >= nr) break;
            float v0[NC + 1], v1[NC + 1];
#pragma unroll
            for (int j = 0; j <= NC; ++j) {
                v0[j] = fmaf(h2, c[i][j], h0 * c[i + 1][j]);
                v1[j] = fmaf(h3, c[i][j], h1 * c[i + 1][j]);
            }
            // The PAN pixels stay packed across the band loop and are converted
            // again for every band: the empty asm makes the packed words look
            // changed here, so the compiler does not hoist the conversions out of
            // the loop and hold the floats (which costs the occupancy).
            f2 xa[NC + 1], xb[NC + 1];
#pragma unroll
            for (int j = 0; j < NC / 2; ++j) {
                asm volatile("" : "+v"(raw[2 * i][j]));
                asm volatile("" : "+v"(raw[2 * i + 1][j]));
            }
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                xa[j + 1] = f2{byte_at(raw[2 * i][j >> 1], 2 * (j & 1)), byte_at(raw[2 * i][j >> 1], 2 * (j & 1) + 1)};
                xb[j + 1] = f2{byte_at(raw[2 * i + 1][j >> 1], 2 * (j & 1)),
                               byte_at(raw[2 * i + 1][j >> 1], 2 * (j & 1) + 1)};
            }
            f2 q0[NC], q1[NC];
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                q0[k].x = fmaf(g, xa[k + 1].x, fmaf(h2, v0[k], h0 * v0[k + 1]));
                q0[k].y = fmaf(g, xa[k + 1].y, fmaf(h3, v0[k], h1 * v0[k + 1]));
                q1[k].x = fmaf(g, xb[k + 1].x, fmaf(h2, v1[k], h0 * v1[k + 1]));
                q1[k].y = fmaf(g, xb[k + 1].y, fmaf(h3, v1[k], h1 * v1[k + 1]));
            }
            TO *o0 = ob + (int64_t)(2 * (rb + i)) * p.out_ld;
            store_out<TO, NC, AL>(o0, L.s0, L.W2, L.full, q0);
            store_out<TO, NC, AL>(o0 + p.out_ld, L.s0, L.W2, L.full, q1);
        }
    };
    // MS rows are loaded kMsAhead bands ahead into kMsAhead + 1 rotating
    // register sets (one band of arithmetic does not cover their latency).  The
    // loop is unrolled by the set count so the sets rotate without register
    // copies (a copy would wait for its load), and past the last band the
    // last band is loaded again (a cache hit), so every path issues the same
    // loads and the wait before each band covers only that band's rows.
    constexpr int D = kMsAhead;
    const int last = p.B - 1;
    uint32_t mset[D + 1][KR + 1][MW];
#pragma unroll
    for (int i = 0; i <= KR; ++i)
#pragma unroll
        for (int j = 0; j < MW; ++j) mset[0][i][j] = t.m[i][j];  // band 0 (renamed, not copied)
#pragma unroll
    for (int k = 1; k < D; ++k) load_band(min(k, last), mset[k]);
    for (int b = 0; b <= last; b += D + 1) {
#pragma unroll
        for (int r = 0; r <= D; ++r) {
            if (b + r > last) break;
            load_band(min(b + r + D, last), mset[(r + D) % (D + 1)]);
            band(b + r, mset[r]);
        }
    }
}

template <typename TI, typename TO, int NC, int KR, bool AL>
__device__ __forceinline__ void d4_codec_tile_u8(const CodecParams &p, const Filters &f, int strip, int seg, int lane) {
    static_assert(sizeof(TI) == 1 && sizeof(TO) == 1 && (NC == 4 || NC == 8), "8-bit in and out");
    const CodecCols<TI, NC, AL> L(strip, lane, p.W >> 1);
    if (!L.active()) return;
    const int rb = seg * KR;
    const int nr = min(KR, (p.H >> 1) - rb);
    U8Tile<NC, KR> t;
    u8_tile_load<NC, KR, AL>(p, L, rb, t);
    u8_tile_compute<TO, NC, KR, AL>(p, f, L, rb, nr, t);
}

// D4, rolling: the wavefront walks p.seg_rows coefficient rows of its strip,
// keeping two row-filtered PAN rows, the PAN pixels of the current row pair
// and one row of L PAN in registers, so each PAN row is unpacked and
// filtered once per unit (the one-shot tiles filter the halo rows again in
// every tile).  Same per-pixel arithmetic as the tiles.
template <typename TI, typename TO, int NC, bool AL>
__device__ __forceinline__ void d4_codec_rolling(const CodecParams &p, const Filters &f, int strip, int seg, int lane) {
    const CodecCols<TI, NC, AL> L(strip, lane, p.W >> 1);
    if (!L.active()) return;
    const TI *pan = static_cast<const TI *>(p.pan);
    const TI *ms = static_cast<const TI *>(p.ms);
    TO *out = static_cast<TO *>(p.out);
    const int H2 = p.H >> 1;
    const int rb = seg * p.seg_rows;
    const int re = min(rb + p.seg_rows, H2);
    // rows needed lie in [-2, H+1]: one conditional wrap (Eq. 5-6) suffices
    auto row = [&](int y) {
        y = y < 0 ? y + p.H : (y >= p.H ? y - p.H : y);
        return pan + (int64_t)y * p.pan_ld;
    };
    f2 xa[NC + 2], xb[NC + 2];
    float Ra[NC + 1], Rb[NC + 1], Ap[NC + 1];
    {
        f2 xs[NC + 2], xt[NC + 2];
        float Rs[NC + 1], Rt[NC + 1];
        L.load_row(row(2 * rb - 2), xs);
        L.load_row(row(2 * rb - 1), xt);
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
        L.load_row(row(2 * r + 2), xc);
        L.load_row(row(2 * r + 3), xd);
        float Rc[NC + 1], Rd[NC + 1], A[NC + 1];
        rowfilt<NC>(f, xc, Rc);
        rowfilt<NC>(f, xd, Rd);
        colfilt<NC>(f, Ra, Rb, Rc, Rd, A);
        const int rp = (r == 0) ? H2 - 1 : r - 1;
        for (int b = 0; b < p.B; ++b) {
            const float g = p.gain ? p.gain[b] : 1.0f;
            const TI *mb = ms + (int64_t)b * p.ms_bs;
            float mc[NC + 1], mp[NC + 1];
            L.load_ms(mb + (int64_t)r * p.ms_ld, mc);
            L.load_ms(mb + (int64_t)rp * p.ms_ld, mp);
            f2 q0[NC], q1[NC];
            d4_out_rows<NC>(f, g, p.kappa, mc, mp, A, Ap, xa, xb, q0, q1);
            TO *o0 = out + (int64_t)b * p.out_bs + (int64_t)(2 * r) * p.out_ld;
            store_out<TO, NC, AL>(o0, L.s0, L.W2, L.full, q0);
            store_out<TO, NC, AL>(o0 + p.out_ld, L.s0, L.W2, L.full, q1);
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

template <typename TI, typename TO, int NC, int KR, bool AL>
__device__ __forceinline__ void haar_codec_tile(const CodecParams &p, int strip, int seg, int lane) {
    const CodecCols<TI, NC, AL> L(strip, lane, p.W >> 1);
    if (!L.active()) return;
    const TI *pan = static_cast<const TI *>(p.pan);
    const TI *ms = static_cast<const TI *>(p.ms);
    TO *out = static_cast<TO *>(p.out);
    const int H2 = p.H >> 1;
    const int rb = seg * KR;
    const int nr = min(KR, H2 - rb);
    f2 da[KR][NC], dc[KR][NC];
    {
        f2 a[KR][NC], c[KR][NC];
#pragma unroll
        for (int i = 0; i < KR; ++i) {
            const int r = rb + (i < nr ? i : 0);  // rows past the image re-read row rb (unused)
            const TI *p0 = pan + (int64_t)(2 * r) * p.pan_ld;
            L.load_own(p0, a[i]);
            L.load_own(p0 + p.pan_ld, c[i]);
        }
#pragma unroll
        for (int i = 0; i < KR; ++i) haar_details<NC>(a[i], c[i], da[i], dc[i]);
    }
    auto load_band = [&](int b, float(&m)[KR][NC]) {
        const TI *mb = ms + (int64_t)b * p.ms_bs;
#pragma unroll
        for (int i = 0; i < KR; ++i) L.load_ms_own(mb + (int64_t)(rb + (i < nr ? i : 0)) * p.ms_ld, m[i]);
    };
    if constexpr (sizeof(TI) == 1 && (NC == 4 || NC == 8)) {
        // 8-bit MS, up to 8 bands: every band's rows of the tile are loaded up
        // front as packed bytes (NC / 4 registers a row) and converted where
        // they are used, so no band waits for its own loads.
        constexpr int MB = 8;
        if (p.B <= MB) {
            uint32_t mall[MB][KR][NC / 4];
#pragma unroll
            for (int b = 0; b < MB; ++b) {
                if (b >= p.B) break;
                const TI *mb = ms + (int64_t)b * p.ms_bs;
#pragma unroll
                for (int i = 0; i < KR; ++i) L.load_ms_own_raw(mb + (int64_t)(rb + (i < nr ? i : 0)) * p.ms_ld, mall[b][i]);
            }
#pragma unroll
            for (int b = 0; b < MB; ++b) {
                if (b >= p.B) break;
                const float g = p.gain ? p.gain[b] : 1.0f;
                TO *ob = out + (int64_t)b * p.out_bs;
#pragma unroll
                for (int i = 0; i < KR; ++i) {
                    if (i >= nr) break;
                    float mv[NC];
#pragma unroll
                    for (int j = 0; j < NC; ++j) mv[j] = byte_at(mall[b][i][j >> 2], j & 3);
                    f2 q0[NC], q1[NC];
                    haar_out_rows<NC>(g, p.kappa, mv, da[i], dc[i], q0, q1);
                    TO *o0 = ob + (int64_t)(2 * (rb + i)) * p.out_ld;
                    store_out<TO, NC, AL>(o0, L.s0, L.W2, L.full, q0);
                    store_out<TO, NC, AL>(o0 + p.out_ld, L.s0, L.W2, L.full, q1);
                }
            }
            return;
        }
    }
    float m[KR][NC];
    load_band(0, m);
    for (int b = 0; b < p.B; ++b) {
        float mn[KR][NC];
        if (b + 1 < p.B) load_band(b + 1, mn);
        const float g = p.gain ? p.gain[b] : 1.0f;
        TO *ob = out + (int64_t)b * p.out_bs;
#pragma unroll
        for (int i = 0; i < KR; ++i) {
            if (i >= nr) break;
            f2 q0[NC], q1[NC];
            haar_out_rows<NC>(g, p.kappa, m[i], da[i], dc[i], q0, q1);
            TO *o0 = ob + (int64_t)(2 * (rb + i)) * p.out_ld;
            store_out<TO, NC, AL>(o0, L.s0, L.W2, L.full, q0);
            store_out<TO, NC, AL>(o0 + p.out_ld, L.s0, L.W2, L.full, q1);
        }
        if (b + 1 < p.B) {
#pragma unroll
            for (int i = 0; i < KR; ++i)
#pragma unroll
                for (int j = 0; j < NC; ++j) m[i][j] = mn[i][j];
        }
    }
}

template <typename TI, typename TO, int NC, int KR, bool AL, int WAV>
__global__ __launch_bounds__(256) void codec_kernel(CodecParams p, Filters f) {
    const int wpb = blockDim.x >> 6;
    const int lane = threadIdx.x & 63;
    // The wavefront's index is the same on all its lanes; saying so keeps the
    // unit's row and column bookkeeping in scalar registers.
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int unit = block_unit(p.order) * wpb + wave;
    if (unit >= p.units) return;  // whole wavefront; no barriers in this kernel
    int strip, seg;
    if (p.order & 1) {
        seg = unit / p.nstrips;
        strip = unit - seg * p.nstrips;
    } else {
        strip = unit / p.nseg;
        seg = unit - strip * p.nseg;
    }
    if constexpr (WAV == 1) {
        if constexpr (KR == 0)
            d4_codec_rolling<TI, TO, NC, AL>(p, f, strip, seg, lane);
        else if constexpr (sizeof(TI) == 1 && sizeof(TO) == 1)
            d4_codec_tile_u8<TI, TO, NC, KR, AL>(p, f, strip, seg, lane);
        else
            d4_codec_tile<TI, TO, NC, KR, AL>(p, f, strip, seg, lane);
    } else {
        haar_codec_tile<TI, TO, NC, KR, AL>(p, strip, seg, lane);
    }
}

// ---- D4, 8-bit input, LDS-staged workgroup tiles -----------------------------
//
// As the float LDS-staged kernel: a workgroup of wpb wavefronts covers a strip
// of 128 coefficient columns and T = wpb * KR coefficient rows.  Its PAN rows
// 2r0-2 .. 2r0+2T+1 (2-column halos, all wrapped) and the MS rows r0-1 ..
// r0+T-1 of a group of bands are read once, converted to float32 and written
// to LDS; after one barrier each wavefront computes its KR rows from LDS
// (two coefficient columns per lane) with the same fma chains as every other
// kernel, so its results equal theirs bit for bit.  Only the rows a
// wavefront is computing sit in its registers, so many more wavefronts fit
// on a CU than with the one-shot 8-bit tiles, which hold every PAN row of
// their unit as floats.
constexpr int kCPanRow = 264;  // floats: [2,4) left halo, [4,260) own 256 pixels, [260,262) right halo
constexpr int kCMsRow = 132;   // floats: [3] left halo, [4,132) own 128 coefficients

template <typename TO, int KR, bool AL>
__global__ __launch_bounds__(256) void d4_codec_staged_kernel(CodecParams p, Filters f, int bg_max) {
    extern __shared__ float lds[];
    const int wpb = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int unit = block_unit(p.order);
    if (unit >= p.units) return;  // whole workgroup
    const int T = wpb * KR;
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
    const uint8_t *pan = static_cast<const uint8_t *>(p.pan);
    const uint8_t *ms = static_cast<const uint8_t *>(p.ms);
    TO *out = static_cast<TO *>(p.out);
    float *Pl = lds;
    float *Ml = lds + (2 * T + 4) * kCPanRow;
    // The strip's 256 pixels lie inside every row (no wrap within them).
    const bool clear = 2 * sb + 256 <= p.W;

    for (int k = w; k < 2 * T + 4; k += wpb) {
        const uint8_t *row = pan + (int64_t)wrap_row(2 * r0 - 2 + k, p.H) * p.pan_ld;
        float *dst = Pl + k * kCPanRow;
        if (clear && (reinterpret_cast<uintptr_t>(row) & 3) == 0) {
            const uint32_t v = *reinterpret_cast<const uint32_t *>(row + 2 * sb + 4 * lane);
            *reinterpret_cast<f4 *>(dst + 4 + 4 * lane) = f4{byte_at(v, 0), byte_at(v, 1), byte_at(v, 2), byte_at(v, 3)};
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[4 + 4 * lane + q] = (float)row[wrap_idx(2 * sb + 4 * lane + q, p.W)];
        }
        if (lane < 2) {
            dst[2 + lane] = (float)row[wrap_idx(2 * sb - 2 + lane, p.W)];
            dst[260 + lane] = (float)row[wrap_idx(2 * sb + 256 + lane, p.W)];
        }
    }
    const bool mclear = sb + 128 <= W2;
    auto stage_ms = [&](int g0, int bg) {
        for (int k = w; k < bg * (T + 1); k += wpb) {
            const int b = g0 + k / (T + 1), i = k - (k / (T + 1)) * (T + 1);
            const uint8_t *row = ms + (int64_t)b * p.ms_bs + (int64_t)wrap_row(r0 - 1 + i, H2) * p.ms_ld;
            float *dst = Ml + k * kCMsRow;
            if (mclear && (reinterpret_cast<uintptr_t>(row) & 1) == 0) {
                const uint32_t v = *reinterpret_cast<const uint16_t *>(row + sb + 2 * lane);
                *reinterpret_cast<f2 *>(dst + 4 + 2 * lane) = f2{byte_at(v, 0), byte_at(v, 1)};
            } else {
                dst[4 + 2 * lane] = (float)row[wrap_idx(sb + 2 * lane, W2)];
                dst[5 + 2 * lane] = (float)row[wrap_idx(sb + 2 * lane + 1, W2)];
            }
            if (lane == 0) dst[3] = (float)row[wrap_idx(sb - 1, W2)];
        }
    };
    const int bg0 = min(p.B, bg_max);
    stage_ms(0, bg0);
    __syncthreads();

    // This wavefront: coefficient rows rb .. rb+KR-1, coefficient columns
    // s0 = sb + 2*lane and s0 + 1; its PAN pairs s0-1 .. s0+2 start at LDS
    // float 2 + 4*lane of a staged row, its MS columns s0-1 .. s0+1 at 3 + 2*lane.
    const int rb = r0 + KR * w;
    const int nr = max(0, min(KR, H2 - rb));
    constexpr int NR = 2 * KR + 4;  // PAN rows 2rb-2 .. 2rb+2KR+1 = staged rows 2KR*w + t
    const int s0 = sb + 2 * lane;
    const bool full = s0 + 2 <= W2;
    f2 xo[2 * KR][2];  // the lane's PAN pixels of its output rows
    float A[KR + 1][3];
    {
        float R[NR][3];
#pragma unroll
        for (int t = 0; t < NR; ++t) {
            const float *src = Pl + (2 * KR * w + t) * kCPanRow + 2 + 4 * lane;
            f2 x[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) x[k] = *reinterpret_cast<const f2 *>(src + 2 * k);
            rowfilt<2>(f, x, R[t]);
            if (t >= 2 && t < 2 + 2 * KR) {
                xo[t - 2][0] = x[1];
                xo[t - 2][1] = x[2];
            }
        }
#pragma unroll
        for (int i = 0; i <= KR; ++i) colfilt<2>(f, R[2 * i], R[2 * i + 1], R[2 * i + 2], R[2 * i + 3], A[i]);
    }

    for (int g0 = 0; g0 < p.B; g0 += bg_max) {
        const int bg = min(bg_max, p.B - g0);
        if (g0 > 0) {  // next band group: every wavefront is done with the previous one
            __syncthreads();
            stage_ms(g0, bg);
            __syncthreads();
        }
        for (int bi = 0; bi < bg && s0 < W2; ++bi) {
            const int b = g0 + bi;
            const float g = p.gain ? p.gain[b] : 1.0f;
            TO *ob = out + (int64_t)b * p.out_bs;
            float m[KR + 1][3];
#pragma unroll
            for (int i = 0; i <= KR; ++i) {
                const float *src = Ml + (bi * (T + 1) + KR * w + i) * kCMsRow + 3 + 2 * lane;
#pragma unroll
                for (int j = 0; j < 3; ++j) m[i][j] = src[j];
            }
#pragma unroll
            for (int i = 0; i < KR; ++i) {
                if (i >= nr) break;
                f2 xa[4], xb[4];
                xa[1] = xo[2 * i][0];
                xa[2] = xo[2 * i][1];
                xb[1] = xo[2 * i + 1][0];
                xb[2] = xo[2 * i + 1][1];
                f2 q0[2], q1[2];
                d4_out_rows<2>(f, g, p.kappa, m[i + 1], m[i], A[i + 1], A[i], xa, xb, q0, q1);
                TO *o0 = ob + (int64_t)(2 * (rb + i)) * p.out_ld;
                store_out<TO, 2, AL>(o0, s0, W2, full, q0);
                store_out<TO, 2, AL>(o0 + p.out_ld, s0, W2, full, q1);
            }
        }
    }
}

// Largest band group a staged 8-bit tile of T rows holds in 64 KB of LDS (<= 8).
int codec_staged_bg_max(int T) {
    const int pan = (2 * T + 4) * kCPanRow, per_band = (T + 1) * kCMsRow;
    const int bg = (16384 - pan) / per_band;
    return bg < 1 ? 0 : (bg > 8 ? 8 : bg);
}

template <typename TO>
hipError_t launch_staged_io(const CodecParams &p, const Filters &f, int kr, bool al, int wpb, hipStream_t s) {
    const int T = kr * wpb;
    const int bgm = codec_staged_bg_max(T);
    if (bgm < 1) return hipErrorInvalidValue;
    const int bg = p.B < bgm ? p.B : bgm;
    const size_t lds = sizeof(float) * ((size_t)(2 * T + 4) * kCPanRow + (size_t)bg * (T + 1) * kCMsRow);
    const dim3 grid(p.units), block(64 * wpb);
#define CODEC_STAGED(KR, AL) \
    hipLaunchKernelGGL((d4_codec_staged_kernel<TO, KR, AL>), grid, block, lds, s, p, f, bgm)
    if (kr == 1) {
        if (al) CODEC_STAGED(1, true);
        else CODEC_STAGED(1, false);
    } else {
        if (al) CODEC_STAGED(2, true);
        else CODEC_STAGED(2, false);
    }
#undef CODEC_STAGED
    return hipGetLastError();
}

template <typename TI, typename TO, int NC, int KR, bool AL>
hipError_t launch_t(const CodecParams &p, const Filters &f, int wpb, hipStream_t s) {
    const int grid = (p.units + wpb - 1) / wpb;
    if constexpr (KR == 0) {  // rolling exists for D4 only
        if (p.wavelet != 1) return hipErrorInvalidValue;
        hipLaunchKernelGGL((codec_kernel<TI, TO, NC, 0, AL, 1>), dim3(grid), dim3(64 * wpb), 0, s, p, f);
    } else {
        if (p.wavelet == 1)
            hipLaunchKernelGGL((codec_kernel<TI, TO, NC, KR, AL, 1>), dim3(grid), dim3(64 * wpb), 0, s, p, f);
        else
            hipLaunchKernelGGL((codec_kernel<TI, TO, NC, KR, AL, 0>), dim3(grid), dim3(64 * wpb), 0, s, p, f);
    }
    return hipGetLastError();
}

template <typename TI, typename TO>
hipError_t launch_io(const CodecParams &p, const Filters &f, int nc, int kr, bool al, int wpb, hipStream_t s) {
    if constexpr (sizeof(TI) == 1) {
        if (!al) return (nc == 4 && kr == 1) ? launch_t<TI, TO, 4, 1, false>(p, f, wpb, s) : hipErrorInvalidValue;
        if (nc == 4 && kr == 1) return launch_t<TI, TO, 4, 1, true>(p, f, wpb, s);
        if (nc == 4 && kr == 2) return launch_t<TI, TO, 4, 2, true>(p, f, wpb, s);
        if (nc == 8 && kr == 1) return launch_t<TI, TO, 8, 1, true>(p, f, wpb, s);
        if (nc == 8 && kr == 2) return launch_t<TI, TO, 8, 2, true>(p, f, wpb, s);
        if (nc == 4 && kr == 0) return launch_t<TI, TO, 4, 0, true>(p, f, wpb, s);
        if (nc == 8 && kr == 0) return launch_t<TI, TO, 8, 0, true>(p, f, wpb, s);
    } else {
        if (!al) return (nc == 2 && kr == 1) ? launch_t<TI, TO, 2, 1, false>(p, f, wpb, s) : hipErrorInvalidValue;
        if (nc == 2 && kr == 1) return launch_t<TI, TO, 2, 1, true>(p, f, wpb, s);
        if (nc == 2 && kr == 2) return launch_t<TI, TO, 2, 2, true>(p, f, wpb, s);
        if (nc == 2 && kr == 0) return launch_t<TI, TO, 2, 0, true>(p, f, wpb, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

bool codec_shape_ok(int in_u8, int nc, int kr, bool al, int wavelet) {
    if (kr >= 3) return in_u8 && wavelet == 1 && nc == 2 && kr <= 4;  // LDS-staged (al: output stores)
    if (kr == 0 && (wavelet != 1 || !al)) return false;  // rolling: D4, aligned buffers
    if (in_u8) return al ? ((nc == 4 || nc == 8) && kr >= 0 && kr <= 2) : (nc == 4 && kr == 1);
    return al ? (nc == 2 && kr >= 0 && kr <= 2) : (nc == 2 && kr == 1);
}

hipError_t launch_codec(const CodecParams &p, const Filters &f, int in_u8, int out_u8, int nc, int kr, bool al,
                        int wpb, hipStream_t s) {
    if (p.units <= 0) return hipSuccess;
    if (wpb < 1 || wpb > 4 || !codec_shape_ok(in_u8, nc, kr, al, p.wavelet)) return hipErrorInvalidValue;
    if (kr >= 3) {  // LDS-staged D4 tiles of (kr - 2) * wpb rows, 8-bit input
        if (p.seg_rows != (kr - 2) * wpb || p.nstrips != (p.W / 2 + 127) / 128 ||
            p.nseg != (p.H / 2 + p.seg_rows - 1) / p.seg_rows)
            return hipErrorInvalidValue;
        return out_u8 ? launch_staged_io<uint8_t>(p, f, kr - 2, al, wpb, s)
                      : launch_staged_io<float>(p, f, kr - 2, al, wpb, s);
    }
    if (p.seg_rows < 1 || (kr > 0 && p.seg_rows != kr)) return hipErrorInvalidValue;
    if (p.nstrips != (p.W / 2 + 64 * nc - 1) / (64 * nc) || p.nseg != (p.H / 2 + p.seg_rows - 1) / p.seg_rows)
        return hipErrorInvalidValue;
    if (in_u8) {
        return out_u8 ? launch_io<uint8_t, uint8_t>(p, f, nc, kr, al, wpb, s)
                      : launch_io<uint8_t, float>(p, f, nc, kr, al, wpb, s);
    }
    // float in and out is the tuned float path (fuse_kernels.hip)
    return out_u8 ? launch_io<float, uint8_t>(p, f, nc, kr, al, wpb, s) : hipErrorInvalidValue;
}

}  // namespace dwtf
