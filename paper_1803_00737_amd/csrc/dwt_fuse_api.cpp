// Host side of the C ABI declared in include/dwt_fuse.h: argument
// validation, the context (stream, workspace, batch tables, captured graphs,
// tuning table), work decomposition and kernel dispatch.
#pragma GCC visibility push(default)
#include "dwt_fuse.h"
#pragma GCC visibility pop

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "fuse_internal.h"

#ifndef DWT_FUSE_BUILD_ID
#define DWT_FUSE_BUILD_ID "dev"
#endif

using namespace dwtf;

static_assert(DWT_FUSE_STATIC_SCRATCH_BYTES == kStaticScratchBytes, "header and library disagree on the static scratch size");

namespace {

// ---------------------------------------------------------------- validation

struct Span {
    uintptr_t lo = 0, hi = 0;  // byte range [lo, hi); empty if lo == hi
    bool overlaps(const Span &o) const { return lo < o.hi && o.lo < hi && lo != hi && o.lo != o.hi; }
};

// Elements spanned by nb bands of rows x cols with pitch ld and band stride
// bs: (nb-1)*bs + (rows-1)*ld + cols.  False on overflow.
bool extent(int64_t nb, int64_t rows, int64_t cols, int64_t ld, int64_t bs, int64_t *elems) {
    int64_t a = 0, b = 0, c = 0;
    if (__builtin_mul_overflow(nb - 1, bs, &a)) return false;
    if (__builtin_mul_overflow(rows - 1, ld, &b)) return false;
    if (__builtin_add_overflow(a, b, &c)) return false;
    if (__builtin_add_overflow(c, cols, &c)) return false;
    if (c > INT64_MAX / 4) return false;
    *elems = c;
    return true;
}

// The byte range [p, p + elems * esize) does not wrap past the end of the
// address space.
bool fits_address_space(const void *p, int64_t elems, int64_t esize = sizeof(float)) {
    const uintptr_t lo = reinterpret_cast<uintptr_t>(p);
    return elems >= 0 && (uintptr_t)elems <= (UINTPTR_MAX - lo) / (uintptr_t)esize;
}

Span span_of(const void *p, int64_t elems, int64_t esize = sizeof(float)) {
    Span s;
    s.lo = reinterpret_cast<uintptr_t>(p);
    s.hi = s.lo + static_cast<uintptr_t>(elems) * static_cast<uintptr_t>(esize);
    return s;
}

constexpr int64_t kMaxSide = int64_t(1) << 30;  // kernels index rows/columns in int32
constexpr int64_t kMaxBands = int64_t(1) << 20;

dwt_fuse_status check_shape(int64_t H, int64_t W, int64_t B, std::string *err) {
    if (H < 2 || W < 2 || (H & 1) || (W & 1) || H > kMaxSide || W > kMaxSide) {
        if (err) *err = "H and W must be even, >= 2 and <= 2^30";
        return DWT_FUSE_E_SHAPE;
    }
    if (B < 1 || B > kMaxBands) {
        if (err) *err = "B must be in [1, 2^20]";
        return DWT_FUSE_E_SHAPE;
    }
    int64_t hw = 0, hwb = 0;
    if (__builtin_mul_overflow(H, W, &hw) || __builtin_mul_overflow(hw, B, &hwb) || hwb > INT64_MAX / 4) {
        if (err) *err = "H*W*B overflows";
        return DWT_FUSE_E_SHAPE;
    }
    return DWT_FUSE_OK;
}

dwt_fuse_status check_strided(const char *name, int64_t nb, int64_t rows, int64_t cols, int64_t ld, int64_t bs,
                              const void *ptr, Span *sp, std::string *err, int64_t esize = sizeof(float)) {
    if (ld < cols || (nb > 1 && (bs < 0 || bs / ld < rows))) {
        if (err) *err = std::string(name) + ": pitch smaller than the row width, or band stride smaller than rows*pitch";
        return DWT_FUSE_E_STRIDE;
    }
    if (nb > 1) {
        int64_t rl = 0;
        if (__builtin_mul_overflow(rows, ld, &rl) || bs < rl) {
            if (err) *err = std::string(name) + ": band stride smaller than rows*pitch";
            return DWT_FUSE_E_STRIDE;
        }
    }
    int64_t e = 0;
    if (!extent(nb, rows, cols, ld, bs, &e) || !fits_address_space(ptr, e, esize)) {
        if (err) *err = std::string(name) + ": extent overflows";
        return DWT_FUSE_E_SHAPE;
    }
    *sp = span_of(ptr, e, esize);
    return DWT_FUSE_OK;
}

struct RunArgs {
    int wavelet;
    int64_t H, W, B;
    const float *pan;
    int64_t pan_ld;
    const float *ms;
    int64_t ms_ld, ms_bs;
    const float *gain;
    const float *out;
    int64_t out_ld, out_bs;
};

struct RunSpans {
    Span pan, ms, gain, out;
};

dwt_fuse_status check_run_args(const RunArgs &a, RunSpans *sp, std::string *err) {
    if (!a.pan || !a.ms || !a.out) {
        if (err) *err = "pan, ms and out must not be NULL";
        return DWT_FUSE_E_NULL;
    }
    dwt_fuse_status st = check_shape(a.H, a.W, a.B, err);
    if (st) return st;
    if (a.wavelet != DWT_FUSE_HAAR && a.wavelet != DWT_FUSE_D4) {
        if (err) *err = "unknown wavelet";
        return DWT_FUSE_E_WAVELET;
    }
    RunSpans s;
    if ((st = check_strided("pan", 1, a.H, a.W, a.pan_ld, 0, a.pan, &s.pan, err))) return st;
    if ((st = check_strided("ms", a.B, a.H / 2, a.W / 2, a.ms_ld, a.ms_bs, a.ms, &s.ms, err))) return st;
    if ((st = check_strided("out", a.B, a.H, a.W, a.out_ld, a.out_bs, a.out, &s.out, err))) return st;
    if (a.gain && !fits_address_space(a.gain, a.B)) {
        if (err) *err = "gain: extent overflows";
        return DWT_FUSE_E_SHAPE;
    }
    s.gain = a.gain ? span_of(a.gain, a.B) : Span{};
    if (s.out.overlaps(s.pan) || s.out.overlaps(s.ms) || s.out.overlaps(s.gain)) {
        if (err) *err = "out overlaps an input";
        return DWT_FUSE_E_ALIAS;
    }
    if (sp) *sp = s;
    return DWT_FUSE_OK;
}

// dwt_fuse_run_ex: formats and kappa on top of RunArgs' geometry.
struct ExArgs {
    int wavelet;
    int64_t H, W, B;
    const void *pan;
    int64_t pan_ld;
    const void *ms;
    int64_t ms_ld, ms_bs;
    const float *gain;
    const void *out;
    int64_t out_ld, out_bs;
    int in_format, out_format;
    float kappa;
};

int64_t format_size(int fmt) { return fmt == DWT_FUSE_U8 ? 1 : (int64_t)sizeof(float); }

dwt_fuse_status check_ex_args(const ExArgs &a, std::string *err) {
    if (!a.pan || !a.ms || !a.out) {
        if (err) *err = "pan, ms and out must not be NULL";
        return DWT_FUSE_E_NULL;
    }
    dwt_fuse_status st = check_shape(a.H, a.W, a.B, err);
    if (st) return st;
    if (a.wavelet != DWT_FUSE_HAAR && a.wavelet != DWT_FUSE_D4) {
        if (err) *err = "unknown wavelet";
        return DWT_FUSE_E_WAVELET;
    }
    const auto known = [](int f) { return f == DWT_FUSE_F32 || f == DWT_FUSE_U8; };
    if (!known(a.in_format) || !known(a.out_format)) {
        if (err) *err = "unknown element format";
        return DWT_FUSE_E_FORMAT;
    }
    const int64_t ei = format_size(a.in_format), eo = format_size(a.out_format);
    Span pan, ms, out;
    if ((st = check_strided("pan", 1, a.H, a.W, a.pan_ld, 0, a.pan, &pan, err, ei))) return st;
    if ((st = check_strided("ms", a.B, a.H / 2, a.W / 2, a.ms_ld, a.ms_bs, a.ms, &ms, err, ei))) return st;
    if ((st = check_strided("out", a.B, a.H, a.W, a.out_ld, a.out_bs, a.out, &out, err, eo))) return st;
    if (a.gain && !fits_address_space(a.gain, a.B)) {
        if (err) *err = "gain: extent overflows";
        return DWT_FUSE_E_SHAPE;
    }
    const Span gain = a.gain ? span_of(a.gain, a.B) : Span{};
    if (out.overlaps(pan) || out.overlaps(ms) || out.overlaps(gain)) {
        if (err) *err = "out overlaps an input";
        return DWT_FUSE_E_ALIAS;
    }
    return DWT_FUSE_OK;
}

struct BwdArgs {
    int wavelet;
    int64_t H, W, B;
    const float *pan;
    int64_t pan_ld;
    const float *gain;
    const float *gy;
    int64_t gy_ld, gy_bs;
    const float *grad_pan, *grad_ms, *grad_gain;
};

// Byte ranges of a backward call's inputs and (possibly empty) outputs.
struct BwdSpans {
    Span pan, gy, gain;
    Span outs[3];  // grad_pan, grad_ms, grad_gain
};

dwt_fuse_status check_bwd_args(const BwdArgs &a, std::string *err, BwdSpans *sp = nullptr) {
    if (!a.pan || !a.gy) {
        if (err) *err = "pan and grad_out must not be NULL";
        return DWT_FUSE_E_NULL;
    }
    dwt_fuse_status st = check_shape(a.H, a.W, a.B, err);
    if (st) return st;
    if (a.wavelet != DWT_FUSE_HAAR && a.wavelet != DWT_FUSE_D4) {
        if (err) *err = "unknown wavelet";
        return DWT_FUSE_E_WAVELET;
    }
    Span pan, gy;
    if ((st = check_strided("pan", 1, a.H, a.W, a.pan_ld, 0, a.pan, &pan, err))) return st;
    if ((st = check_strided("grad_out", a.B, a.H, a.W, a.gy_ld, a.gy_bs, a.gy, &gy, err))) return st;
    if ((a.gain && !fits_address_space(a.gain, a.B)) || (a.grad_pan && !fits_address_space(a.grad_pan, a.H * a.W)) ||
        (a.grad_ms && !fits_address_space(a.grad_ms, a.B * (a.H / 2) * (a.W / 2))) ||
        (a.grad_gain && !fits_address_space(a.grad_gain, a.B))) {
        if (err) *err = "a gain or gradient extent overflows";
        return DWT_FUSE_E_SHAPE;
    }
    const Span gain = a.gain ? span_of(a.gain, a.B) : Span{};
    const Span outs[3] = {a.grad_pan ? span_of(a.grad_pan, a.H * a.W) : Span{},
                          a.grad_ms ? span_of(a.grad_ms, a.B * (a.H / 2) * (a.W / 2)) : Span{},
                          a.grad_gain ? span_of(a.grad_gain, a.B) : Span{}};
    for (int i = 0; i < 3; ++i) {
        if (outs[i].overlaps(pan) || outs[i].overlaps(gy) || outs[i].overlaps(gain)) {
            if (err) *err = "a gradient output overlaps an input";
            return DWT_FUSE_E_ALIAS;
        }
        for (int j = i + 1; j < 3; ++j)
            if (outs[i].overlaps(outs[j])) {
                if (err) *err = "gradient outputs overlap each other";
                return DWT_FUSE_E_ALIAS;
            }
    }
    if (sp) {
        sp->pan = pan;
        sp->gy = gy;
        sp->gain = gain;
        for (int i = 0; i < 3; ++i) sp->outs[i] = outs[i];
    }
    return DWT_FUSE_OK;
}

BwdArgs bwd_item_args(const dwt_fuse_bwd_item &it) {
    return BwdArgs{it.wavelet, it.H,       it.W,        it.B,       it.pan,      it.pan_ld,   it.gain,
                   it.grad_out, it.go_ld, it.go_band_stride, it.grad_pan, it.grad_ms, it.grad_gain};
}

// True if any two spans of `v` overlap (empty spans never do).
bool any_overlap(std::vector<Span> v) {
    v.erase(std::remove_if(v.begin(), v.end(), [](const Span &x) { return x.lo == x.hi; }), v.end());
    std::sort(v.begin(), v.end(), [](const Span &a, const Span &b) { return a.lo < b.lo; });
    for (size_t i = 1; i < v.size(); ++i)
        if (v[i].lo < v[i - 1].hi) return true;
    return false;
}

dwt_fuse_status check_bwd_batch(const dwt_fuse_bwd_item *items, int64_t n, std::string *err) {
    if (n < 0) {
        if (err) *err = "n < 0";
        return DWT_FUSE_E_SHAPE;
    }
    if (n == 0) return DWT_FUSE_OK;
    if (!items) {
        if (err) *err = "items is NULL";
        return DWT_FUSE_E_NULL;
    }
    if (n > (int64_t(1) << 24)) {
        if (err) *err = "too many items";
        return DWT_FUSE_E_SHAPE;
    }
    std::vector<Span> outs, ins;
    outs.reserve(3 * n);
    ins.reserve(3 * n);
    for (int64_t i = 0; i < n; ++i) {
        BwdSpans sp;
        std::string e;
        const dwt_fuse_status st = check_bwd_args(bwd_item_args(items[i]), &e, &sp);
        if (st) {
            if (err) *err = "item " + std::to_string(i) + ": " + e;
            return st;
        }
        for (const Span &o : sp.outs)
            if (o.lo != o.hi) outs.push_back(o);
        ins.push_back(sp.pan);
        ins.push_back(sp.gy);
        if (sp.gain.lo != sp.gain.hi) ins.push_back(sp.gain);
    }
    if (any_overlap(outs)) {
        if (err) *err = "gradient outputs of two items overlap";
        return DWT_FUSE_E_ALIAS;
    }
    // No output overlaps any input (inputs may overlap each other).
    std::sort(ins.begin(), ins.end(), [](const Span &a, const Span &b) { return a.lo < b.lo; });
    std::vector<uintptr_t> pmax(ins.size());
    uintptr_t m = 0;
    for (size_t i = 0; i < ins.size(); ++i) pmax[i] = m = std::max(m, ins[i].hi);
    for (const Span &o : outs) {
        // inputs starting before o.hi; the furthest-reaching of them must end at or before o.lo
        const size_t k = std::lower_bound(ins.begin(), ins.end(), o.hi,
                                          [](const Span &a, uintptr_t v) { return a.lo < v; }) -
                         ins.begin();
        if (k > 0 && pmax[k - 1] > o.lo) {
            if (err) *err = "a gradient output overlaps an input of another item";
            return DWT_FUSE_E_ALIAS;
        }
    }
    return DWT_FUSE_OK;
}

RunArgs item_args(const dwt_fuse_item &it) {
    return RunArgs{it.wavelet, it.H, it.W, it.B, it.pan, it.pan_ld, it.ms, it.ms_ld, it.ms_band_stride,
                   it.gain, it.out, it.out_ld, it.out_band_stride};
}

dwt_fuse_status check_batch(const dwt_fuse_item *items, int64_t n, std::string *err) {
    if (n < 0) {
        if (err) *err = "n < 0";
        return DWT_FUSE_E_SHAPE;
    }
    if (n == 0) return DWT_FUSE_OK;
    if (!items) {
        if (err) *err = "items is NULL";
        return DWT_FUSE_E_NULL;
    }
    if (n > (int64_t(1) << 24)) {
        if (err) *err = "too many items";
        return DWT_FUSE_E_SHAPE;
    }
    std::vector<Span> outs, ins;
    outs.reserve(n);
    ins.reserve(3 * n);
    for (int64_t i = 0; i < n; ++i) {
        RunSpans s;
        std::string e;
        const dwt_fuse_status st = check_run_args(item_args(items[i]), &s, &e);
        if (st) {
            if (err) *err = "item " + std::to_string(i) + ": " + e;
            return st;
        }
        outs.push_back(s.out);
        ins.push_back(s.pan);
        ins.push_back(s.ms);
        if (s.gain.lo != s.gain.hi) ins.push_back(s.gain);
    }
    // Outputs pairwise disjoint: sort by start, compare neighbours.
    std::vector<Span> o = outs;
    std::sort(o.begin(), o.end(), [](const Span &a, const Span &b) { return a.lo < b.lo; });
    for (size_t i = 1; i < o.size(); ++i)
        if (o[i].lo < o[i - 1].hi) {
            if (err) *err = "outputs of two items overlap";
            return DWT_FUSE_E_ALIAS;
        }
    // No output overlaps any input (inputs may overlap each other).
    std::sort(ins.begin(), ins.end(), [](const Span &a, const Span &b) { return a.lo < b.lo; });
    std::vector<uintptr_t> pmax(ins.size());
    uintptr_t m = 0;
    for (size_t i = 0; i < ins.size(); ++i) pmax[i] = m = std::max(m, ins[i].hi);
    for (const Span &s : outs) {
        // last input starting before s.hi
        size_t lo = 0, hi = ins.size();
        while (lo < hi) {
            const size_t mid = (lo + hi) / 2;
            if (ins[mid].lo < s.hi)
                lo = mid + 1;
            else
                hi = mid;
        }
        if (lo > 0 && pmax[lo - 1] > s.lo) {
            if (err) *err = "an item's output overlaps an input";
            return DWT_FUSE_E_ALIAS;
        }
    }
    return DWT_FUSE_OK;
}

// ---------------------------------------------------------------- tiling

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

Path choose_path(const RunArgs &a) {
    const bool b1 = a.B == 1;
    if (aligned(a.pan, 16) && aligned(a.out, 16) && a.pan_ld % 4 == 0 && a.out_ld % 4 == 0 &&
        (b1 || a.out_bs % 4 == 0) && aligned(a.ms, 8) && a.ms_ld % 2 == 0 && (b1 || a.ms_bs % 2 == 0))
        return PATH_V4;
    if (aligned(a.pan, 8) && aligned(a.out, 8) && a.pan_ld % 2 == 0 && a.out_ld % 2 == 0 &&
        (b1 || a.out_bs % 2 == 0))
        return PATH_V2;
    return PATH_SCALAR;
}

// Forward launches store in overlapped strips (strip_origin) when some
// output row does not start on a 64-byte boundary; never on 4-byte rows
// (their pixel pairs are not 8-byte aligned).
bool overlap_strips(const RunArgs &a, Path path, int forced = -1) {
    if (path == PATH_SCALAR) return false;
    if (forced >= 0) return forced == 1;
    return !(aligned(a.out, 64) && a.out_ld % 16 == 0 && (a.B == 1 || a.out_bs % 16 == 0));
}

Path choose_bwd_path(const BwdArgs &a) {
    const bool b1 = a.B == 1;
    const bool gp = !a.grad_pan || aligned(a.grad_pan, 16);
    const bool gm = !a.grad_ms || aligned(a.grad_ms, 8);
    if (aligned(a.pan, 16) && aligned(a.gy, 16) && gp && gm && a.pan_ld % 4 == 0 && a.gy_ld % 4 == 0 &&
        (b1 || a.gy_bs % 4 == 0) && a.W % 4 == 0)
        return PATH_V4;
    const bool gp2 = !a.grad_pan || aligned(a.grad_pan, 8);
    if (aligned(a.pan, 8) && aligned(a.gy, 8) && gp2 && a.pan_ld % 2 == 0 && a.gy_ld % 2 == 0 &&
        (b1 || a.gy_bs % 2 == 0))
        return PATH_V2;
    return PATH_SCALAR;
}

// Launch shape of one scene.  mode 0: rolling wavefronts over seg_rows
// coefficient rows; mode 1 or 2: one-shot wavefronts of `mode` rows; mode
// 2 + KR (KR = 1, 2, 4): LDS-staged workgroups of wpb wavefronts with KR rows
// each (D4, 128-bit path only).  seg_rows is ignored unless mode == 0.
struct Tile {
    int seg_rows = 0, wpb = 0, nc = 0;
    int order = 1;  // bit 0: row-band-major (else strip-major); bit 1: dispatch order (else per-XCD runs)
    int mode = 0;
    int split = 0;  // LDS-staged: bands per unit (0 = all)
    int bg = 0;     // LDS-staged: bands staged at once (0 = as many as fit)
    int rows() const { return mode >= 3 ? wpb * (mode - 2) : (mode > 0 ? mode : seg_rows); }
};

// Forced launch shape (0 = automatic for each field); variant 1 = rolling,
// 2 = one-shot, 3 = LDS-staged (where it applies); split = bands per
// LDS-staged unit.
struct Forced {
    int seg_rows = 0, wpb = 0, nc = 0, variant = 0, split = 0;
    int order = -1;  // unit order of forward launches (-1 = the shape's own)
    int ovl = -1;    // overlapped strips (-1 = by the output's alignment)
    int bg = 0;      // LDS-staged: bands staged at once (0 = the shape's own)
};

struct Decomp {
    int32_t nstrips = 0, nseg = 0, units = 0;
    int32_t ovl = 0;  // overlapped strips (strip_origin)
};

bool decompose(int64_t H, int64_t W, const Tile &t, Decomp *d, bool ovl = false) {
    const int64_t H2 = H / 2;
    const int seg_rows = t.rows();
    if (seg_rows < 1 || t.nc < 1 || t.nc > 2) return false;
    const int64_t ns = strip_count(W, t.nc, ovl ? 1 : 0);
    d->ovl = ovl ? 1 : 0;
    const int64_t ng = (H2 + seg_rows - 1) / seg_rows;
    if (ns * ng > INT32_MAX) return false;
    d->nstrips = (int32_t)ns;
    d->nseg = (int32_t)ng;
    d->units = (int32_t)(ns * ng);
    return true;
}

// Rolling shape (the adjoint kernels and the persistent batch kernel's
// rolling variant): 4 waves per workgroup, nc coefficient columns per lane
// (the widest the caller's kernels have on the path), units of 32
// coefficient rows shortened until the launch has at least 8192 wavefronts
// (32 per CU) or 4 rows.
Tile rolling_tile(int64_t H, int64_t W, int nc) {
    Tile t;
    t.nc = nc;
    t.wpb = 4;
    t.seg_rows = 32;
    t.mode = 0;
    Decomp d;
    while (t.seg_rows > 4 && decompose(H, W, t, &d) && d.units < 8192) t.seg_rows /= 2;
    return t;
}

// Default forward shape (what the tuner picks on the large workloads):
// D4 -> LDS-staged workgroups of 4 wavefronts x 2 coefficient rows, except on
// 8-byte rows below 2^25 pixels, where one-shot single-row wavefronts with 2
// coefficient columns per lane measured faster (the staged tile then stages
// half of its rows in 16-byte groups shifted by 2 floats); Haar -> one-shot
// single-row wavefronts.  Units row-band-major in dispatch order (order 3):
// the whole GPU writes one narrow band of rows of every output band at a
// time, which HBM absorbs faster than the same stores spread over per-XCD
// runs or down column strips (Landsat-shaped D4, 6 bands: 1.36 against
// 1.56 ms strip-major with per-XCD runs; Haar 1.35 against 1.42 ms).  The
// staged D4 tiles go one step further (order 7, XCD slabs): the band still
// advances across the whole GPU, but each XCD takes a contiguous chunk of its
// strips, so a tile's left, right, upper and lower neighbours share its L2
// and the halo columns and rows are not fetched again from HBM (reads 1.25
// -> 1.04 x algorithmic; 8192^2 B = 3 0.224 -> 0.209 ms, Landsat-shaped
// 1.36 -> 1.35 ms).  The small-image one-shot D4 shape keeps per-XCD runs
// (order 1), whose halo rows then stay in one L2.
Tile default_tile(int wavelet, int64_t H, int64_t W, Path path) {
    Tile t;
    if (wavelet == DWT_FUSE_D4 && !(path == PATH_V2 && H * W < ((int64_t)1 << 25))) {
        t.nc = 2;
        t.mode = 4;
        t.seg_rows = 2;
        t.wpb = 4;
        t.order = 7;
        t.bg = 2;
    } else {
        t.nc = path_nc(path);
        t.mode = 1;
        t.seg_rows = 1;
        t.wpb = wavelet == DWT_FUSE_D4 ? 4 : 1;
        t.order = wavelet == DWT_FUSE_D4 ? 1 : 3;
    }
    return t;
}

int ceil_log2(int64_t v) {
    int k = 0;
    while ((int64_t(1) << k) < v) ++k;
    return k;
}

std::string tune_key(int kind, int wavelet, int64_t H, int64_t W, int64_t B, Path path) {
    char buf[96];
    std::snprintf(buf, sizeof(buf), "%c%d_h%d_w%d_b%d_p%d", kind == 0 ? 'f' : 'b', wavelet, ceil_log2(H),
                  ceil_log2(W), (int)std::min<int64_t>(B, 8), (int)path);
    return buf;
}

Filters make_filters() {
    // Eq. 7-8: h_i = (1 + 2i + sqrt3)/(4 sqrt2), h_{i+2} = (3 - 2i - sqrt3)/(4 sqrt2),
    // evaluated in double and rounded once to float.
    const double r3 = std::sqrt(3.0), den = 4.0 * std::sqrt(2.0);
    Filters f;
    for (int i = 0; i < 2; ++i) {
        f.h[i] = (float)((1.0 + 2.0 * i + r3) / den);
        f.h[i + 2] = (float)((3.0 - 2.0 * i - r3) / den);
    }
    return f;
}

}  // namespace

// ---------------------------------------------------------------- context

// Form of a batched forward launch: persistent queues (mode 0 rolling, 1-2
// one-shot rows) or the flat grid (mode 3) with its unit order and the band
// group size of its LDS-staged tiles (0 = every band of the batch at once).
struct BatchChoice {
    int mode = 3;
    int order = 3;
    int bg = 2;
    int staged = 1;  // flat: D4 scenes as LDS-staged tiles of kr rows per wavefront (1), one-shot single-row
                     // wavefronts (0), or staged with each scene's own (per-image tuned) rows per wavefront (2)
    int kr = 2;      // flat: coefficient rows per wavefront of a staged tile (1 or 2; 4 wavefronts)
};

struct dwt_fuse_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string last_error;
    Filters filt{};
    int num_cu = 256;
    std::string device_name;
    // tiling
    bool tuning = false;
    Forced forced;
    bool force_batch = false;  // DWT_FUSE_FORCE_BATCH: every batch takes forced_batch
    BatchChoice forced_batch;
    std::map<std::string, Tile> table;
    std::map<std::string, BatchChoice> batch_modes;  // tuned form per batch signature
    // backward workspace
    float *ws = nullptr;
    size_t ws_bytes = 0;
    // multi-pass comparator work arrays (2 x H x W floats)
    float *mp = nullptr;
    size_t mp_bytes = 0;
    // batched
    BatchScene *d_scenes = nullptr;
    BatchScene *h_scenes = nullptr;  // pinned staging
    size_t scenes_cap = 0;
    uint32_t *d_counters = nullptr;
    hipEvent_t staged = nullptr;     // last upload of h_scenes finished
    bool staged_pending = false;
    std::map<std::string, hipGraphExec_t> graphs;
    hipStream_t cap_stream = nullptr;  // capture only (the null stream cannot be captured)
    // batched backward: adjoint scene table and gain jobs (device + pinned staging)
    void *d_bwd = nullptr;
    void *h_bwd = nullptr;
    size_t bwd_bytes = 0;
    hipEvent_t bwd_staged = nullptr;  // last upload of h_bwd finished
    bool bwd_pending = false;
    hipEvent_t switched = nullptr;  // recorded on the old stream by dwt_fuse_set_stream
    // the device's static scratch (dwt_fuse_backward_noalloc); NULL if the
    // lookup at creation failed (scratch_err says why)
    void *scratch = nullptr;
    std::string scratch_err;
};

namespace {

dwt_fuse_status fail(dwt_fuse_ctx *c, dwt_fuse_status st, const std::string &msg) {
    if (c) c->last_error = msg;
    return st;
}

dwt_fuse_status hip_fail(dwt_fuse_ctx *c, hipError_t e, const char *what) {
    return fail(c, DWT_FUSE_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

dwt_fuse_status use_device(dwt_fuse_ctx *c) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(c, e, "hipGetDevice");
    if (cur != c->device) {
        e = hipSetDevice(c->device);
        if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    }
    return DWT_FUSE_OK;
}

void clear_graphs(dwt_fuse_ctx *c) {
    for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
}

FuseParams make_params(const RunArgs &a, Path path, const Tile &t, const Decomp &d) {
    FuseParams p{};
    p.pan = a.pan;
    p.ms = a.ms;
    p.gain = a.gain;
    p.out = const_cast<float *>(a.out);
    p.pan_ld = a.pan_ld;
    p.ms_ld = a.ms_ld;
    p.ms_bs = a.ms_bs;
    p.out_ld = a.out_ld;
    p.out_bs = a.out_bs;
    p.H = (int32_t)a.H;
    p.W = (int32_t)a.W;
    p.B = (int32_t)a.B;
    p.seg_rows = t.rows();
    p.nseg = d.nseg;
    p.units = d.units;
    p.wavelet = a.wavelet;
    p.path = path;
    p.nstrips = d.nstrips;
    p.order = t.order;
    p.mode = t.mode;
    p.kappa = 1.0f;
    // XCD slabs exist for LDS-staged tiles without band split, numbered by row bands
    if (p.order & 4) p.order = (t.mode >= 3 && !(t.split > 0 && t.split < a.B)) ? (p.order | 1) : (p.order & 3);
    p.ovl = d.ovl;
    p.bg = t.mode >= 3 ? t.bg : 0;
    if (t.mode >= 3 && t.split > 0 && t.split < a.B) {  // (tile, band group) units
        p.bsplit = t.split;
        p.units = d.units * (int32_t)((a.B + t.split - 1) / t.split);  // bounded by split_fits
    }
    return p;
}

// The (tile, band group) unit count of a band-split staged launch fits int32.
bool split_fits(const Tile &t, const Decomp &d, int64_t B) {
    if (!(t.mode >= 3 && t.split > 0 && t.split < B)) return true;
    return (int64_t)d.units * ((B + t.split - 1) / t.split) <= INT32_MAX;
}

// LDS-staged tiles exist for D4 on every path (their strips are always 128
// coefficient columns wide, i.e. nc = 2 in the decomposition).
bool staged_allowed(int wavelet, Path, int) { return wavelet == DWT_FUSE_D4; }

// max_nc: the widest lane layout the caller's kernels have on this path.
Tile apply_forced(const dwt_fuse_ctx *c, Tile t, Path path, int wavelet, int max_nc) {
    const Forced &fo = c->forced;
    if (fo.seg_rows > 0) t.seg_rows = fo.seg_rows;
    if (fo.wpb > 0) t.wpb = fo.wpb;
    if (fo.nc > 0) t.nc = std::min(fo.nc, max_nc);
    int variant = fo.variant;
    if (variant == 3 && !staged_allowed(wavelet, path, t.nc)) variant = 2;
    if (variant == 0 && t.mode >= 3 && !staged_allowed(wavelet, path, t.nc)) variant = 2;
    if (variant == 1) t.mode = 0;
    if (variant == 2) t.mode = std::min(2, std::max(1, fo.seg_rows > 0 ? fo.seg_rows : 2));
    if (variant == 3) {
        const int kr = fo.seg_rows >= 4 ? 4 : (fo.seg_rows >= 2 ? 2 : (fo.seg_rows == 1 ? 1 : 2));
        t.mode = 2 + kr;
    }
    if (t.mode >= 3) {
        t.nc = 2;  // staged strips are 128 coefficient columns on every path
        if (t.wpb < 1) t.wpb = 4;
    } else if (t.mode > 0 || variant == 1) {
        if (t.nc > max_nc || t.nc < 1) t.nc = max_nc;
    }
    if (t.wpb < 1) t.wpb = 4;
    if (t.mode == 0 && t.seg_rows < 1) t.seg_rows = 1;
    if (fo.split > 0) t.split = fo.split;
    if (t.mode < 3) t.split = 0;
    if (fo.order >= 0) t.order = fo.order;
    if (fo.bg > 0) t.bg = fo.bg;
    return t;
}

// The path a launch runs: NC = 1 on 128-bit rows takes the 64-bit kernels,
// NC = 2 on 64-bit rows the mixed 64/128-bit ones.
Path path_for_nc(Path path, int nc) {
    if (path == PATH_V4 && nc == 1) return PATH_V2;
    if (path == PATH_V2 && nc == 2) return PATH_V2W;
    return path;
}

// Median of 3 timed runs of `launch` on stream s (ms), after one warm-up;
// 1e30 if any launch or event call fails, so a failing candidate is never
// chosen.
template <class F>
float time_median3(hipStream_t s, F launch) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return 1e30f;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return 1e30f;
    }
    float t[3] = {1e30f, 1e30f, 1e30f};
    bool ok = launch() == hipSuccess;
    for (int k = 0; ok && k < 3; ++k)
        ok = hipEventRecord(e0, s) == hipSuccess && launch() == hipSuccess && hipEventRecord(e1, s) == hipSuccess &&
             hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&t[k], e0, e1) == hipSuccess;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!ok) return 1e30f;
    std::sort(t, t + 3);
    return t[1];
}

// One forward launch of shape t on the caller's buffers.
hipError_t launch_tile(dwt_fuse_ctx *c, const RunArgs &a, Path path, const Tile &t) {
    Decomp d;
    if (!decompose(a.H, a.W, t, &d, overlap_strips(a, path, c->forced.ovl)) || !split_fits(t, d, a.B)) return hipErrorInvalidValue;
    const FuseParams p = make_params(a, path_for_nc(path, t.nc), t, d);
    return launch_fuse(p, c->filt, t.wpb, c->stream);
}

// Time one forward launch configuration on the caller's buffers (ms, median of 3).
float time_fuse(dwt_fuse_ctx *c, const RunArgs &a, Path path, const Tile &t) {
    Decomp d;
    if (!decompose(a.H, a.W, t, &d, overlap_strips(a, path, c->forced.ovl)) || !split_fits(t, d, a.B)) return 1e30f;
    return time_median3(c->stream, [&] { return launch_tile(c, a, path, t); });
}

// Second pass over the fastest few shapes of a first pass: 7 timed runs of
// each, interleaved across the shapes (clock or thermal drift during the
// pass then affects them alike), each run a burst of 4 back-to-back
// launches (the steady state of repeated calls, where one launch's tail
// overlaps the next one's start; isolated launches ranked a 1-row staged
// shape first on the 8192^2 workload, 14% slower back to back than the
// 2-row one); the lowest median wins, near-ties going to the smallest
// tie_key.  A single pass over ~100 shapes with 3 runs each also tends to
// keep whichever shape happened to run fast.
template <class T, class L, class K>
T confirm_best(hipStream_t stream, std::vector<std::pair<float, T>> &cands, L launch, K tie_key, float *best_ms) {
    std::stable_sort(cands.begin(), cands.end(),
                     [](const std::pair<float, T> &x, const std::pair<float, T> &y) { return x.first < y.first; });
    size_t k = 0;
    while (k < cands.size() && k < 4 && cands[k].first < 1e29f) ++k;
    *best_ms = cands[0].first;
    if (k < 2) return cands[0].second;
    constexpr int R = 7;
    std::vector<float> t(k * R, 1e30f);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return cands[0].second;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return cands[0].second;
    }
    constexpr int BURST = 4;
    bool ok = true;
    for (int r = 0; ok && r < R; ++r)
        for (size_t i = 0; ok && i < k; ++i) {
            ok = hipEventRecord(e0, stream) == hipSuccess;
            for (int q = 0; ok && q < BURST; ++q) ok = launch(cands[i].second) == hipSuccess;
            ok = ok && hipEventRecord(e1, stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                 hipEventElapsedTime(&t[i * R + r], e0, e1) == hipSuccess;
            t[i * R + r] /= BURST;
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!ok) return cands[0].second;
    std::vector<float> med(k);
    float bm = 1e30f;
    for (size_t i = 0; i < k; ++i) {
        std::sort(t.begin() + i * R, t.begin() + (i + 1) * R);
        med[i] = t[i * R + R / 2];
        bm = std::min(bm, med[i]);
    }
    // Shapes within 1% of the best burst median are taken as equal; of those
    // the one with the smallest tie_key wins (first-pass order among equal
    // keys), so that repeated tuning settles on the same shape.
    size_t best = k;
    for (size_t i = 0; i < k; ++i)
        if (med[i] <= 1.01f * bm && (best == k || tie_key(cands[i].second) < tie_key(cands[best].second))) best = i;
    *best_ms = med[best];
    return cands[best].second;
}

Tile tune_fuse(dwt_fuse_ctx *c, const RunArgs &a, Path path) {
    std::vector<std::pair<float, Tile>> cands;
    {
        const Tile t = default_tile(a.wavelet, a.H, a.W, path);
        cands.emplace_back(time_fuse(c, a, path, t), t);
    }
    // Candidates: rolling units of 2..64 rows and one-shot units of 1 or 2
    // rows, each with 1, 2 or 4 waves per workgroup, three unit orders
    // (strip-major and row-band-major in per-XCD runs, row-band-major in
    // dispatch order) and
    // (on 128- and 64-bit rows) 1 or 2 coefficient columns per lane.
    const int ncs[2] = {2, 1};
    const int rows_cand[8] = {-1, -2, 2, 4, 8, 16, 32, 64};  // negative: one-shot of that many rows
    for (int nc : ncs) {
        if (nc > path_nc(path)) continue;
        for (int rc : rows_cand) {
            for (int wpb : {1, 2, 4}) {
                for (int order : {1, 0, 3}) {
                    Tile t;
                    t.nc = nc;
                    t.mode = rc < 0 ? -rc : 0;
                    t.seg_rows = rc < 0 ? -rc : rc;
                    t.wpb = wpb;
                    t.order = order;
                    cands.emplace_back(time_fuse(c, a, path, t), t);
                }
            }
        }
    }
    // LDS-staged workgroups (D4): KR rows per wavefront, all bands of a tile
    // per unit (units split into band groups, dwt_fuse_force_band_split,
    // measured slower on every workload, so they are not candidates), the
    // MS rows of every band or of 2 bands at a time in LDS.
    if (staged_allowed(a.wavelet, path, 2)) {
        for (int kr : {1, 2, 4}) {
            for (int wpb : {1, 2, 4}) {
                for (int order : {1, 0, 3, 7}) {
                    for (int bg : {0, 2}) {  // bands staged at once: as many as fit, or 2 (less LDS)
                        if (bg > 0 && bg >= a.B) continue;
                        Tile t;
                        t.nc = 2;
                        t.mode = 2 + kr;
                        t.seg_rows = kr;
                        t.wpb = wpb;
                        t.order = order;
                        t.bg = bg;
                        cands.emplace_back(time_fuse(c, a, path, t), t);
                    }
                }
            }
        }
    }
    float bestms = 0.f;
    // near-ties: fewest work units (larger tiles re-read fewer halo rows and
    // stay ahead when launches do not overlap, e.g. one call at a time)
    auto units = [&](const Tile &t) {
        Decomp d;
        return decompose(a.H, a.W, t, &d, overlap_strips(a, path, c->forced.ovl)) ? (int64_t)d.units : INT64_MAX;
    };
    const Tile bestt =
        confirm_best(c->stream, cands, [&](const Tile &t) { return launch_tile(c, a, path, t); }, units, &bestms);
    if (std::getenv("DWT_FUSE_LOG"))
        std::fprintf(stderr, "[dwt_fuse] tuned %s: mode=%d seg_rows=%d wpb=%d nc=%d order=%d split=%d bg=%d (%.3f ms)\n",
                     tune_key(0, a.wavelet, a.H, a.W, a.B, path).c_str(), bestt.mode, bestt.seg_rows, bestt.wpb,
                     bestt.nc, bestt.order, bestt.split, bestt.bg, bestms);
    return bestt;
}

Tile tile_for_run(dwt_fuse_ctx *c, const RunArgs &a, Path path, bool allow_tune) {
    const std::string key = tune_key(0, a.wavelet, a.H, a.W, a.B, path);
    auto it = c->table.find(key);
    Tile t;
    if (it != c->table.end()) {
        t = it->second;
    } else if (c->tuning && allow_tune) {
        t = tune_fuse(c, a, path);
        c->table[key] = t;
    } else {
        t = default_tile(a.wavelet, a.H, a.W, path);
    }
    return apply_forced(c, t, path, a.wavelet, path_nc(path));
}

dwt_fuse_status ensure_ws(dwt_fuse_ctx *c, size_t bytes) {
    if (bytes <= c->ws_bytes) return DWT_FUSE_OK;
    if (c->ws) {
        // earlier work may still use the buffer; a failed wait leaves it in place
        const hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize before growing the workspace");
        (void)hipFree(c->ws);
        c->ws = nullptr;
        c->ws_bytes = 0;
    }
    const size_t nb = std::max<size_t>(bytes, 1 << 16);
    if (hipMalloc(reinterpret_cast<void **>(&c->ws), nb) != hipSuccess) {
        c->ws = nullptr;
        return fail(c, DWT_FUSE_E_NOMEM, "workspace allocation failed");
    }
    c->ws_bytes = nb;
    return DWT_FUSE_OK;
}

dwt_fuse_status ensure_batch_tables(dwt_fuse_ctx *c, size_t n) {
    if (!c->d_counters) {
        const size_t bytes = (kQueues + 1) * kQueueStride * sizeof(uint32_t);
        if (hipMalloc(reinterpret_cast<void **>(&c->d_counters), bytes) != hipSuccess) {
            c->d_counters = nullptr;
            return fail(c, DWT_FUSE_E_NOMEM, "counter allocation failed");
        }
        hipError_t e = hipMemsetAsync(c->d_counters, 0, bytes, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "hipMemsetAsync");
    }
    if (!c->staged) {
        hipError_t e = hipEventCreateWithFlags(&c->staged, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(c, e, "hipEventCreate");
    }
    if (n <= c->scenes_cap) return DWT_FUSE_OK;
    // Growing moves the device table: captured graphs point at the old one.
    const hipError_t se = hipStreamSynchronize(c->stream);
    if (se != hipSuccess) return hip_fail(c, se, "hipStreamSynchronize before growing the scene table");
    clear_graphs(c);
    if (c->d_scenes) (void)hipFree(c->d_scenes);
    if (c->h_scenes) (void)hipHostFree(c->h_scenes);
    c->d_scenes = nullptr;
    c->h_scenes = nullptr;
    c->scenes_cap = 0;
    const size_t cap = std::max<size_t>(n, 128);
    if (hipMalloc(reinterpret_cast<void **>(&c->d_scenes), cap * sizeof(BatchScene)) != hipSuccess) {
        c->d_scenes = nullptr;
        return fail(c, DWT_FUSE_E_NOMEM, "scene table allocation failed");
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&c->h_scenes), cap * sizeof(BatchScene), hipHostMallocDefault) !=
        hipSuccess) {
        c->h_scenes = nullptr;
        return fail(c, DWT_FUSE_E_NOMEM, "pinned staging allocation failed");
    }
    c->scenes_cap = cap;
    c->staged_pending = false;
    return DWT_FUSE_OK;
}


// ---- batched launch planning ----

// Batch variants: 0, 1, 2 = persistent work-queue kernel with rolling or
// one-shot (1 or 2 rows) wavefront units; 3 = flat grid, one workgroup per
// work item (LDS-staged D4 tiles, one-shot wavefronts otherwise).
constexpr int kFlatBatch = 3;

struct BatchPlan {
    std::vector<BatchScene> sc;
    BatchQueues q;
    int grid = 0;
    int mode = 0;
    int total = 0;          // work items (flat) or wavefront units (persistent)
    int staged_bands = 0;   // flat: largest band count among staged scenes
    int flat_order = 3;     // flat: unit order of the items (bit 0 row-band-major, bit 1 dispatch order)
    int flat_bg = 0;        // flat: bands staged at once by an LDS-staged tile (0 = all)
    int flat_kr = 2;        // flat: coefficient rows per wavefront of a staged tile
    std::string sig;  // batch signature (graph cache key), includes the variant and grid
};

// Per-scene tiles (tuned per size class with the per-image kernel when tuning
// is on), forced to the batch's variant `mode`, then 8 contiguous queues of
// about equal bytes.
dwt_fuse_status plan_batch(dwt_fuse_ctx *ctx, const dwt_fuse_item *items, int64_t n, const BatchChoice &ch,
                           BatchPlan *pl) {
    const int mode = ch.mode;
    pl->sc.assign((size_t)n, BatchScene{});
    pl->mode = mode;
    pl->flat_order = ctx->forced.order >= 0 ? ctx->forced.order : ch.order;
    pl->flat_bg = ch.bg;
    pl->flat_kr = ch.kr == 1 ? 1 : 2;
    int max_kr = 0;  // per-scene shapes: the largest staged rows per wavefront (sizes the launch's LDS)
    pl->staged_bands = 0;
    pl->sig.clear();
    pl->sig.reserve((size_t)n * 48);
    std::vector<double> unit_bytes((size_t)n);
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) {
        const RunArgs a = item_args(items[i]);
        const Path path = choose_path(a);
        Tile t;
        int items_of_scene = 0;
        Decomp d;
        if (mode == kFlatBatch) {
            t.order = pl->flat_order & 1;
            t.wpb = 4;
            // Every D4 scene staged, also on 8-byte rows where one-shot
            // wavefronts win per image: the launch reserves the staged
            // tiles' LDS for every workgroup, and one-shot items at that
            // occupancy measured slower than staged ones.
            // Per-scene shapes: every D4 scene staged, with the rows per
            // wavefront of its per-image tile (tuned for its size class when
            // tuning is on): 1 where that tile is staged with 1 row, else 2.
            int kr = pl->flat_kr;
            const bool stage = ch.staged >= 1 && staged_allowed(a.wavelet, path, 2);
            if (ch.staged == 2 && stage) kr = tile_for_run(ctx, a, path, true).mode == 3 ? 1 : 2;
            if (stage) {
                t.nc = 2;
                t.mode = 2 + kr;  // staged, 1 or 2 rows per wavefront, 4 wavefronts
                t.seg_rows = kr;
                pl->staged_bands = std::max<int>(pl->staged_bands, (int)a.B);
                max_kr = std::max(max_kr, kr);
            } else {
                t.nc = path_nc(path);
                t.mode = 1;
                t.seg_rows = 1;
            }
            if (!decompose(a.H, a.W, t, &d, overlap_strips(a, path, ctx->forced.ovl)))
                return fail(ctx, DWT_FUSE_E_SHAPE, "too many work units");
            items_of_scene = t.mode >= 3 ? d.units : (d.units + 3) / 4;
        } else {
            t = tile_for_run(ctx, a, path, true);
            if (mode > 0) {
                t.mode = mode;
            } else if (t.mode > 0) {  // one-shot or staged per-image tiles: rolling here
                t = rolling_tile(a.H, a.W, path_nc(path));
            }
            if (!decompose(a.H, a.W, t, &d, overlap_strips(a, path, ctx->forced.ovl)))
                return fail(ctx, DWT_FUSE_E_SHAPE, "too many work units");
            items_of_scene = d.units;
        }
        BatchScene &b = pl->sc[(size_t)i];
        t.split = 0;  // batched launches keep every band of a tile in one work item
        b.p = make_params(a, path_for_nc(path, t.nc), t, d);
        b.unit_begin = (int32_t)total;
        b.pad_ = 0;
        total += items_of_scene;
        if (total > INT32_MAX) return fail(ctx, DWT_FUSE_E_SHAPE, "too many work units in batch");
        unit_bytes[(size_t)i] = (double)a.H * a.W * (4.0 + 5.0 * a.B) / std::max(1, items_of_scene);
        char buf[200];
        std::snprintf(buf, sizeof(buf), "%d.%lld.%lld.%lld.%lld.%lld.%lld.%lld.%lld.%d.%d.%d.%d.%d|", a.wavelet,
                      (long long)a.H, (long long)a.W, (long long)a.B, (long long)a.pan_ld, (long long)a.ms_ld,
                      (long long)a.ms_bs, (long long)a.out_ld, (long long)a.out_bs, (int)b.p.path, t.rows(),
                      t.order, t.mode, a.gain ? 1 : 0);
        pl->sig += buf;
    }
    pl->total = (int)total;
    if (mode == kFlatBatch) {
        if (ch.staged == 2 && max_kr > 0) pl->flat_kr = max_kr;  // LDS for the largest staged tile
        pl->grid = (int)total;
        char gb[64];
        std::snprintf(gb, sizeof(gb), "#flat#%d#o%d#g%d#s%d#k%d", pl->staged_bands, pl->flat_order, pl->flat_bg,
                      ch.staged, pl->flat_kr);
        pl->sig += gb;
        return DWT_FUSE_OK;
    }
    BatchQueues &q = pl->q;
    double all = 0;
    for (int64_t i = 0; i < n; ++i) all += unit_bytes[(size_t)i] * pl->sc[(size_t)i].p.units;
    int qi = 0;
    double acc = 0;
    q.begin[0] = 0;
    for (int64_t i = 0; i < n && qi < kQueues - 1; ++i) {
        const BatchScene &b = pl->sc[(size_t)i];
        for (int32_t u = 0; u < b.p.units && qi < kQueues - 1; ++u) {
            acc += unit_bytes[(size_t)i];
            if (acc >= all * (qi + 1) / kQueues) {
                q.end[qi] = b.unit_begin + u + 1;
                ++qi;
                q.begin[qi] = b.unit_begin + u + 1;
            }
        }
    }
    for (; qi < kQueues; ++qi) {
        q.end[qi] = (int32_t)total;
        if (qi + 1 < kQueues) q.begin[qi + 1] = (int32_t)total;
    }
    const int resident = ctx->num_cu * batched_blocks_per_cu(mode);
    pl->grid = std::max(kQueues, (int)std::min<int64_t>(resident, (total + 3) / 4 + kQueues));
    char gb[64];
    std::snprintf(gb, sizeof(gb), "#m%d#g%d", mode, pl->grid);
    pl->sig += gb;
    return DWT_FUSE_OK;
}

// Upload the scene table (after the previous upload has left the staging buffer).
dwt_fuse_status stage_batch(dwt_fuse_ctx *ctx, const BatchPlan &pl) {
    const size_t n = pl.sc.size();
    if (ctx->staged_pending) {
        hipError_t e = hipEventSynchronize(ctx->staged);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipEventSynchronize");
    }
    std::memcpy(ctx->h_scenes, pl.sc.data(), sizeof(BatchScene) * n);
    hipError_t e = hipMemcpyAsync(ctx->d_scenes, ctx->h_scenes, sizeof(BatchScene) * n, hipMemcpyHostToDevice,
                                  ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "scene table upload");
    e = hipEventRecord(ctx->staged, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipEventRecord");
    ctx->staged_pending = true;
    return DWT_FUSE_OK;
}

hipError_t launch_plan(dwt_fuse_ctx *ctx, const BatchPlan &pl, hipStream_t s) {
    const int n = (int)pl.sc.size();
    if (pl.mode == kFlatBatch)
        return launch_fuse_batched_flat(ctx->d_scenes, n, pl.total,
                                        pl.flat_bg > 0 ? std::min(pl.flat_bg, pl.staged_bands) : pl.staged_bands,
                                        pl.flat_kr, pl.flat_order, ctx->filt, s);
    return launch_fuse_batched(ctx->d_scenes, n, pl.q, ctx->d_counters, pl.grid, pl.mode, ctx->filt, s);
}

// Median of 3 timed launches of a planned batch (ms), after one warm-up.
float time_batch(dwt_fuse_ctx *ctx, const BatchPlan &pl) {
    if (stage_batch(ctx, pl) != DWT_FUSE_OK) return 1e30f;
    return time_median3(ctx->stream, [&] { return launch_plan(ctx, pl, ctx->stream); });
}

}  // namespace

// ---------------------------------------------------------------- C ABI

// The public entry points below take C linkage from their declarations in
// dwt_fuse.h; the helpers between them are internal C++.

const char *dwt_fuse_status_str(dwt_fuse_status s) {
    switch (s) {
        case DWT_FUSE_OK: return "ok";
        case DWT_FUSE_E_NULL: return "null pointer";
        case DWT_FUSE_E_SHAPE: return "invalid shape";
        case DWT_FUSE_E_WAVELET: return "unknown wavelet";
        case DWT_FUSE_E_STRIDE: return "invalid pitch or band stride";
        case DWT_FUSE_E_ALIAS: return "output overlaps an input";
        case DWT_FUSE_E_NOMEM: return "out of device memory";
        case DWT_FUSE_E_DEVICE: return "HIP device error";
        case DWT_FUSE_E_STATE: return "invalid context state";
        case DWT_FUSE_E_FORMAT: return "unknown element format";
    }
    return "unknown status";
}

const char *dwt_fuse_last_error(const dwt_fuse_ctx *ctx) { return ctx ? ctx->last_error.c_str() : ""; }

dwt_fuse_status dwt_fuse_check_run(dwt_fuse_wavelet wavelet, int64_t H, int64_t W, int64_t B, const float *pan,
                                   int64_t pan_ld, const float *ms, int64_t ms_ld, int64_t ms_band_stride,
                                   const float *gain, const float *out, int64_t out_ld,
                                   int64_t out_band_stride) {
    const RunArgs a{(int)wavelet, H, W, B, pan, pan_ld, ms, ms_ld, ms_band_stride, gain, out, out_ld,
                    out_band_stride};
    return check_run_args(a, nullptr, nullptr);
}

dwt_fuse_status dwt_fuse_check_batched(const dwt_fuse_item *items, int64_t n) {
    return check_batch(items, n, nullptr);
}

dwt_fuse_status dwt_fuse_check_backward(dwt_fuse_wavelet wavelet, int64_t H, int64_t W, int64_t B,
                                        const float *pan, int64_t pan_ld, const float *gain,
                                        const float *grad_out, int64_t go_ld, int64_t go_band_stride,
                                        const float *grad_pan, const float *grad_ms, const float *grad_gain) {
    const BwdArgs a{(int)wavelet, H, W, B, pan, pan_ld, gain, grad_out, go_ld, go_band_stride,
                    grad_pan, grad_ms, grad_gain};
    return check_bwd_args(a, nullptr);
}

dwt_fuse_status dwt_fuse_create(dwt_fuse_ctx **ctx, int device, void *hip_stream) {
    if (!ctx) return DWT_FUSE_E_NULL;
    *ctx = nullptr;
    try {
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return DWT_FUSE_E_DEVICE;
        if (hipSetDevice(device) != hipSuccess) return DWT_FUSE_E_DEVICE;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) != hipSuccess) return DWT_FUSE_E_DEVICE;
        dwt_fuse_ctx *c = new dwt_fuse_ctx();
        c->device = device;
        c->stream = reinterpret_cast<hipStream_t>(hip_stream);
        c->filt = make_filters();
        c->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
        c->device_name = prop.gcnArchName;
        // once per device (cached), with the device current: the static
        // scratch's device address for the entry points that allocate nothing
        if (const hipError_t e = static_scratch_address(device, &c->scratch)) {
            c->scratch = nullptr;
            c->scratch_err = std::string("hipGetSymbolAddress of the static scratch failed: ") + hipGetErrorString(e);
        }
        if (const char *f = std::getenv("DWT_FUSE_FORCE_TILE")) {
            int a = 0, b = 0, d = 0, v = 0;
            if (std::sscanf(f, "%d,%d,%d,%d", &a, &b, &d, &v) >= 1 && a >= 0 && a <= 4096 && b >= 0 && b <= 4 &&
                d >= 0 && d <= 2 && v >= 0 && v <= 3) {
                c->forced.seg_rows = a;
                c->forced.wpb = b;
                c->forced.nc = d;
                c->forced.variant = v;
            }
        }
        if (const char *f = std::getenv("DWT_FUSE_FORCE_BG")) {
            const int o = std::atoi(f);
            if (o >= 0 && o <= 8) c->forced.bg = o;
        }
        if (const char *f = std::getenv("DWT_FUSE_FORCE_OVERLAP")) {
            const int o = std::atoi(f);
            if (o >= 0 && o <= 1) c->forced.ovl = o;
        }
        if (const char *f = std::getenv("DWT_FUSE_FORCE_BATCH")) {  // "mode,order,bg,staged,kr"
            BatchChoice b;
            if (std::sscanf(f, "%d,%d,%d,%d,%d", &b.mode, &b.order, &b.bg, &b.staged, &b.kr) == 5 && b.mode >= 0 &&
                b.mode <= kFlatBatch && b.order >= 0 && b.order <= 3 && b.bg >= 0 && b.bg <= 8 && b.staged >= 0 &&
                b.staged <= 2 && (b.kr == 1 || b.kr == 2)) {
                c->force_batch = true;
                c->forced_batch = b;
            }
        }
        if (const char *f = std::getenv("DWT_FUSE_FORCE_ORDER")) {
            const int o = std::atoi(f);
            if (o >= 0 && o <= 7) c->forced.order = o;
        }
        if (const char *f = std::getenv("DWT_FUSE_TUNE_CACHE")) dwt_fuse_tune_load(c, f);
        *ctx = c;
        return DWT_FUSE_OK;
    } catch (const std::bad_alloc &) {
        return DWT_FUSE_E_NOMEM;
    } catch (...) {
        return DWT_FUSE_E_STATE;
    }
}

void dwt_fuse_destroy(dwt_fuse_ctx *ctx) {
    if (!ctx) return;
    try {
        int cur = -1;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(ctx->device);
        // Work issued through the context may still read its workspace and
        // tables; wait for the device (the context's stream may already be gone).
        (void)hipDeviceSynchronize();
        clear_graphs(ctx);
        if (ctx->ws) (void)hipFree(ctx->ws);
        if (ctx->mp) (void)hipFree(ctx->mp);
        if (ctx->d_scenes) (void)hipFree(ctx->d_scenes);
        if (ctx->h_scenes) (void)hipHostFree(ctx->h_scenes);
        if (ctx->d_counters) (void)hipFree(ctx->d_counters);
        if (ctx->staged) (void)hipEventDestroy(ctx->staged);
        if (ctx->d_bwd) (void)hipFree(ctx->d_bwd);
        if (ctx->h_bwd) (void)hipHostFree(ctx->h_bwd);
        if (ctx->bwd_staged) (void)hipEventDestroy(ctx->bwd_staged);
        if (ctx->switched) (void)hipEventDestroy(ctx->switched);
        if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
        if (cur >= 0) (void)hipSetDevice(cur);
    } catch (...) {
    }
    delete ctx;
}

dwt_fuse_status dwt_fuse_set_stream(dwt_fuse_ctx *ctx, void *hip_stream) {
    if (!ctx) return DWT_FUSE_E_NULL;
    const hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    if (s == ctx->stream) return DWT_FUSE_OK;
    try {
        dwt_fuse_status st = use_device(ctx);
        if (st) return st;
        if (!ctx->switched) {
            const hipError_t e = hipEventCreateWithFlags(&ctx->switched, hipEventDisableTiming);
            if (e != hipSuccess) {
                ctx->switched = nullptr;
                return hip_fail(ctx, e, "hipEventCreate");
            }
        }
        // Work issued later on the new stream runs after the context's work
        // on the old one (workspace, descriptor tables and graphs are shared).
        hipError_t e = hipEventRecord(ctx->switched, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipEventRecord");
        e = hipStreamWaitEvent(s, ctx->switched, 0);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamWaitEvent");
        ctx->stream = s;
        return DWT_FUSE_OK;
    } catch (...) {
        return fail(ctx, DWT_FUSE_E_STATE, "unexpected exception");
    }
}

dwt_fuse_status dwt_fuse_set_tuning(dwt_fuse_ctx *ctx, int enable) {
    if (!ctx) return DWT_FUSE_E_NULL;
    ctx->tuning = enable != 0;
    return DWT_FUSE_OK;
}

dwt_fuse_status dwt_fuse_force_tile(dwt_fuse_ctx *ctx, int seg_rows, int wpb, int nc, int variant) {
    if (!ctx) return DWT_FUSE_E_NULL;
    if (seg_rows < 0 || seg_rows > 4096 || wpb < 0 || wpb > 4 || nc < 0 || nc > 2 || variant < 0 || variant > 3)
        return fail(ctx, DWT_FUSE_E_SHAPE,
                    "tile out of range (seg_rows <= 4096, wpb <= 4, nc <= 2, variant <= 3)");
    ctx->forced.seg_rows = seg_rows;
    ctx->forced.wpb = wpb;
    ctx->forced.nc = nc;
    ctx->forced.variant = variant;
    return DWT_FUSE_OK;
}

dwt_fuse_status dwt_fuse_force_band_split(dwt_fuse_ctx *ctx, int bands_per_unit) {
    if (!ctx) return DWT_FUSE_E_NULL;
    if (bands_per_unit < 0 || bands_per_unit > 8)
        return fail(ctx, DWT_FUSE_E_SHAPE, "bands per unit out of range (0 .. 8)");
    ctx->forced.split = bands_per_unit;
    return DWT_FUSE_OK;
}

dwt_fuse_status dwt_fuse_force_order(dwt_fuse_ctx *ctx, int order) {
    if (!ctx) return DWT_FUSE_E_NULL;
    if (order < -1 || order > 7) return fail(ctx, DWT_FUSE_E_SHAPE, "unit order out of range (-1 .. 7)");
    ctx->forced.order = order;
    return DWT_FUSE_OK;
}

dwt_fuse_status dwt_fuse_tune_save(const dwt_fuse_ctx *ctx, const char *path) {
    if (!ctx || !path) return DWT_FUSE_E_NULL;
    FILE *f = std::fopen(path, "w");
    if (!f) return DWT_FUSE_E_STATE;
    std::fprintf(f, "dwt_fuse_tune 5 %s %s\n", DWT_FUSE_BUILD_ID, ctx->device_name.c_str());
    for (const auto &kv : ctx->table)
        std::fprintf(f, "%s %d %d %d %d %d %d %d\n", kv.first.c_str(), kv.second.seg_rows, kv.second.wpb, kv.second.nc,
                     kv.second.order, kv.second.mode, kv.second.split, kv.second.bg);
    std::fclose(f);
    return DWT_FUSE_OK;
}

dwt_fuse_status dwt_fuse_tune_load(dwt_fuse_ctx *ctx, const char *path) {
    if (!ctx || !path) return DWT_FUSE_E_NULL;
    FILE *f = std::fopen(path, "r");
    if (!f) return fail(ctx, DWT_FUSE_E_STATE, "cannot open tuning file");
    char magic[32] = {0}, build[128] = {0}, dev[128] = {0};
    int ver = 0;
    std::map<std::string, Tile> tab;
    bool ok = std::fscanf(f, "%31s %d %127s %127s", magic, &ver, build, dev) == 4 &&
              std::strcmp(magic, "dwt_fuse_tune") == 0 && ver == 5 && std::strcmp(build, DWT_FUSE_BUILD_ID) == 0 &&
              ctx->device_name == dev;
    while (ok) {
        char key[96] = {0};
        Tile t;
        const int r = std::fscanf(f, "%95s %d %d %d %d %d %d %d", key, &t.seg_rows, &t.wpb, &t.nc, &t.order, &t.mode,
                                  &t.split, &t.bg);
        if (r == EOF) break;
        // 'f' / 'b': float-path tiles (mode 0 rolling, 1-2 one-shot, 3/4/6
        // LDS-staged); 'c': format-variant shapes (nc 2/4/8, mode = rows of a
        // one-shot tile, 0 = rolling).
        const bool codec = key[0] == 'c';
        const bool shape_ok = codec ? ((t.nc == 2 || t.nc == 4 || t.nc == 8) && t.mode >= 0 && t.mode <= 4 &&
                                              (t.mode < 3 || t.nc == 2))
                                    : (t.nc >= 1 && t.nc <= 2 && t.mode >= 0 && t.mode <= 6 && t.mode != 5);
        if (r != 8 || t.split < 0 || t.split > 8 || t.bg < 0 || t.bg > 8 || (key[0] != 'f' && key[0] != 'b' && !codec) || t.seg_rows < 1 || t.seg_rows > 4096 ||
            t.wpb < 1 || t.wpb > 4 || t.order < 0 || t.order > 7 || !shape_ok) {
            ok = false;
            break;
        }
        tab[key] = t;
    }
    std::fclose(f);
    if (!ok) return fail(ctx, DWT_FUSE_E_STATE, "tuning file does not match this library version/device or is corrupt; ignored");
    for (const auto &kv : tab) ctx->table[kv.first] = kv.second;
    return DWT_FUSE_OK;
}

namespace {

// Float PAN/MS/out: the tuned fused kernels, LL <- kappa * MS.
dwt_fuse_status run_float(dwt_fuse_ctx *ctx, const RunArgs &a, float kappa) {
    try {
        std::string err;
        dwt_fuse_status st = check_run_args(a, nullptr, &err);
        if (st) return fail(ctx, st, err);
        if ((st = use_device(ctx))) return st;
        const Path path = choose_path(a);
        const Tile t = tile_for_run(ctx, a, path, true);
        Decomp d;
        if (!decompose(a.H, a.W, t, &d, overlap_strips(a, path, ctx->forced.ovl)) || !split_fits(t, d, a.B))
            return fail(ctx, DWT_FUSE_E_SHAPE, "too many work units");
        FuseParams p = make_params(a, path_for_nc(path, t.nc), t, d);
        p.kappa = kappa;
        const hipError_t e = launch_fuse(p, ctx->filt, t.wpb, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "fuse launch");
        return DWT_FUSE_OK;
    } catch (const std::bad_alloc &) {
        return fail(ctx, DWT_FUSE_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(ctx, DWT_FUSE_E_STATE, "unexpected exception");
    }
}

}  // namespace

dwt_fuse_status dwt_fuse_run(dwt_fuse_ctx *ctx, dwt_fuse_wavelet wavelet, int64_t H, int64_t W, int64_t B,
                             const float *pan, int64_t pan_ld, const float *ms, int64_t ms_ld,
                             int64_t ms_band_stride, const float *gain, float *out, int64_t out_ld,
                             int64_t out_band_stride) {
    if (!ctx) return DWT_FUSE_E_NULL;
    const RunArgs a{(int)wavelet, H, W, B, pan, pan_ld, ms, ms_ld, ms_band_stride, gain, out, out_ld,
                    out_band_stride};
    return run_float(ctx, a, 1.0f);
}

namespace {

// ------------------------------------------------------------ format variants

struct CodecShape {
    int nc = 4, kr = 1, wpb = 4, order = 3;
    // coefficient rows per unit: kr for one-shot tiles (kr 1, 2), seg_rows when
    // rolling (kr 0), (kr - 2) * wpb for LDS-staged tiles (kr 3, 4: D4, 8-bit
    // input, nc 2)
    int rows = 1;
    bool aligned = false;  // vector access (LDS-staged: output stores only)
};

bool is_aligned(const void *p, int64_t ld, int64_t bs, int64_t nb, int64_t esize, int64_t a) {
    if (reinterpret_cast<uintptr_t>(p) % (uintptr_t)a) return false;
    if ((ld * esize) % a) return false;
    return nb <= 1 || (bs * esize) % a == 0;
}

// Vector access for nc coefficient columns per lane: own PAN pixels (2*nc
// elements), own MS coefficients (nc elements) and output pixels (2*nc
// elements, at most 16 bytes per store) in one access each.
bool codec_aligned(const ExArgs &a, int nc) {
    const int64_t ei = format_size(a.in_format), eo = format_size(a.out_format);
    return is_aligned(a.pan, a.pan_ld, 0, 1, ei, 2 * nc * ei) &&
           is_aligned(a.ms, a.ms_ld, a.ms_bs, a.B, ei, nc * ei) &&
           is_aligned(a.out, a.out_ld, a.out_bs, a.B, eo, std::min<int64_t>(2 * nc * eo, 16));
}

// LDS-staged 8-bit tiles: 4-byte (8-bit) or 16-byte (float) output stores.
bool codec_staged_aligned(const ExArgs &a) {
    const int64_t eo = format_size(a.out_format);
    return is_aligned(a.out, a.out_ld, a.out_bs, a.B, eo, 4 * eo);
}

// Recompute the alignment flag of a shape for these buffers.
void codec_set_aligned(const ExArgs &a, CodecShape *t) {
    t->aligned = t->kr >= 3 ? codec_staged_aligned(a) : codec_aligned(a, t->nc);
}

std::string codec_key(const ExArgs &a, bool aligned) {
    char buf[96];
    std::snprintf(buf, sizeof(buf), "c%d%d%d_h%d_w%d_b%d_a%d", a.in_format, a.out_format, a.wavelet, ceil_log2(a.H),
                  ceil_log2(a.W), (int)std::min<int64_t>(a.B, 8), aligned ? 1 : 0);
    return buf;
}

// Untuned shape: one coefficient row per wavefront, 16-byte 8-bit rows for
// Haar, 8-byte ones for D4; D4 with 8-bit input and output: 16-byte rows, 2
// coefficient rows per wavefront, one wavefront per workgroup, row bands in
// per-XCD runs (unit order 1; among the fastest measured on both 8-bit D4
// workloads).
CodecShape codec_default(const ExArgs &a) {
    CodecShape t;
    const bool u8 = a.in_format == DWT_FUSE_U8;
    const bool u8io = u8 && a.out_format == DWT_FUSE_U8 && a.wavelet == DWT_FUSE_D4;
    t.nc = u8 ? (a.wavelet == DWT_FUSE_D4 && !u8io ? 4 : 8) : 2;
    t.kr = u8io ? 2 : 1;
    t.rows = t.kr;
    if (u8io) {
        t.wpb = 1;
        t.order = 1;
    }
    if (!codec_aligned(a, t.nc) && u8) t.nc = 4;
    t.aligned = codec_aligned(a, t.nc);
    if (!t.aligned) {
        t.nc = u8 ? 4 : 2;
        t.kr = 1;
        t.rows = 1;
    }
    return t;
}

bool codec_params(const ExArgs &a, const CodecShape &t, CodecParams *p) {
    const int64_t W2 = a.W / 2, H2 = a.H / 2;
    const int rows = t.kr >= 3 ? (t.kr - 2) * t.wpb : (t.kr > 0 ? t.kr : std::max(1, t.rows));
    const int64_t ns = (W2 + 64 * t.nc - 1) / (64 * t.nc), ng = (H2 + rows - 1) / rows;
    if (ns * ng > INT32_MAX - 4) return false;
    CodecParams q{};
    q.pan = a.pan;
    q.ms = a.ms;
    q.gain = a.gain;
    q.out = const_cast<void *>(a.out);
    q.pan_ld = a.pan_ld;
    q.ms_ld = a.ms_ld;
    q.ms_bs = a.ms_bs;
    q.out_ld = a.out_ld;
    q.out_bs = a.out_bs;
    q.kappa = a.kappa;
    q.H = (int32_t)a.H;
    q.W = (int32_t)a.W;
    q.B = (int32_t)a.B;
    q.nstrips = (int32_t)ns;
    q.seg_rows = rows;
    q.nseg = (int32_t)ng;
    q.units = (int32_t)(ns * ng);
    q.order = t.order;
    q.wavelet = a.wavelet;
    *p = q;
    return true;
}

hipError_t launch_codec_shape(dwt_fuse_ctx *c, const ExArgs &a, const CodecShape &t) {
    CodecParams p;
    if (!codec_params(a, t, &p)) return hipErrorInvalidValue;
    return launch_codec(p, c->filt, a.in_format == DWT_FUSE_U8, a.out_format == DWT_FUSE_U8, t.nc, t.kr, t.aligned,
                        t.wpb, c->stream);
}

float time_codec(dwt_fuse_ctx *c, const ExArgs &a, const CodecShape &t) {
    return time_median3(c->stream, [&] { return launch_codec_shape(c, a, t); });
}

CodecShape codec_shape_of(dwt_fuse_ctx *c, const ExArgs &a);

// The launch shape of a format call, with a forced unit order applied.
CodecShape codec_shape(dwt_fuse_ctx *c, const ExArgs &a) {
    CodecShape t = codec_shape_of(c, a);
    if (c->forced.order >= 0) t.order = c->forced.order;
    return t;
}

CodecShape codec_shape_of(dwt_fuse_ctx *c, const ExArgs &a) {
    CodecShape t = codec_default(a);
    const bool u8 = a.in_format == DWT_FUSE_U8;
    const std::string key = codec_key(a, t.aligned);
    auto it = c->table.find(key);
    if (it != c->table.end()) {
        t.nc = it->second.nc;
        t.kr = it->second.mode;  // 0 = rolling
        t.rows = it->second.seg_rows;
        t.wpb = it->second.wpb;
        t.order = it->second.order;
    } else if (c->tuning && t.aligned) {
        std::vector<std::pair<float, CodecShape>> cands;
        cands.emplace_back(time_codec(c, a, t), t);
        // one-shot tiles of 1 or 2 rows (rolling D4 units, forced variant 1,
        // measured slower on every 8-bit workload, so they are not candidates)
        const int rows_cand[2] = {-1, -2};  // negative: one-shot of that many rows
        for (int nc : {2, 4, 8}) {
            if (!codec_shape_ok(u8, nc, 1, true, a.wavelet) || !codec_aligned(a, nc)) continue;
            for (int rc : rows_cand) {
                if (rc > 0 && a.wavelet != DWT_FUSE_D4) continue;
                for (int wpb : {1, 2, 4})
                    for (int order : {1, 0, 3}) {
                        CodecShape s = t;
                        s.nc = nc;
                        s.kr = rc < 0 ? -rc : 0;
                        s.rows = rc < 0 ? -rc : rc;
                        s.wpb = wpb;
                        s.order = order;
                        cands.emplace_back(time_codec(c, a, s), s);
                    }
            }
        }
        // LDS-staged D4 tiles (8-bit input): 1 or 2 rows per wavefront
        if (u8 && a.wavelet == DWT_FUSE_D4) {
            for (int kr : {3, 4})
                for (int wpb : {2, 4})
                    for (int order : {0, 1, 3}) {
                        CodecShape s = t;
                        s.nc = 2;
                        s.kr = kr;
                        s.wpb = wpb;
                        s.rows = (kr - 2) * wpb;
                        s.order = order;
                        codec_set_aligned(a, &s);
                        cands.emplace_back(time_codec(c, a, s), s);
                    }
        }
        float bestms = 0.f;
        // near-ties: D4 one-shot tiles in per-XCD runs of row bands (order 1),
        // whose vertically adjacent tiles share an L2 and so fetch each halo
        // row once (1.0 x the algorithmic reads against up to 2.1 x otherwise)
        const bool d4 = a.wavelet == DWT_FUSE_D4;
        t = confirm_best(
            c->stream, cands, [&](const CodecShape &s) { return launch_codec_shape(c, a, s); },
            [d4](const CodecShape &s) { return d4 && s.kr > 0 && s.kr < 3 && s.order != 1 ? 1 : 0; }, &bestms);
        Tile rec;
        rec.nc = t.nc;
        rec.seg_rows = t.rows;
        rec.wpb = t.wpb;
        rec.order = t.order;
        rec.mode = t.kr;
        c->table[key] = rec;
        if (std::getenv("DWT_FUSE_LOG"))
            std::fprintf(stderr, "[dwt_fuse] tuned %s: nc=%d kr=%d rows=%d wpb=%d order=%d (%.3f ms)\n", key.c_str(),
                         t.nc, t.kr, t.rows, t.wpb, t.order, bestms);
    }
    // Forced fields: variant 1 = rolling (D4) of seg_rows rows (default 16),
    // otherwise one-shot tiles of 1 or 2 rows; waves; columns 1/2 -> nc 4/8
    // for 8-bit input.
    // Forced variant 3: LDS-staged D4 tiles (8-bit input) of seg_rows (1 or 2,
    // default 2) rows per wavefront.
    const Forced &fo = c->forced;
    if (fo.variant == 3 && u8 && a.wavelet == DWT_FUSE_D4) {
        t.kr = 2 + (fo.seg_rows == 1 ? 1 : 2);
        t.nc = 2;
        if (fo.wpb > 0) t.wpb = fo.wpb;
        t.rows = (t.kr - 2) * t.wpb;
        codec_set_aligned(a, &t);
        return t;
    }
    if (fo.variant == 1 && a.wavelet == DWT_FUSE_D4) {
        t.kr = 0;
        t.rows = fo.seg_rows > 0 ? fo.seg_rows : 16;
    } else if (fo.variant != 0 || fo.seg_rows > 0) {
        if (t.kr == 0 || t.kr >= 3 || fo.seg_rows > 0) t.kr = fo.seg_rows >= 2 ? 2 : 1;
        t.rows = t.kr;
    }
    if (fo.wpb > 0) t.wpb = fo.wpb;
    if (t.kr >= 3) {  // a staged shape from the table
        t.rows = (t.kr - 2) * t.wpb;
        codec_set_aligned(a, &t);
        if (codec_shape_ok(u8, t.nc, t.kr, t.aligned, a.wavelet)) return t;
        t.kr = 1;
        t.rows = 1;
    }
    if ((t.nc == 2 && u8) || (fo.nc > 0 && u8)) t.nc = fo.nc == 2 ? 8 : 4;
    if (t.aligned && !codec_aligned(a, t.nc)) t.nc = 4;
    t.aligned = codec_aligned(a, t.nc);
    if (!codec_shape_ok(u8, t.nc, t.kr, t.aligned, a.wavelet)) {
        t.nc = u8 ? 4 : 2;
        t.kr = 1;
        t.rows = 1;
        t.aligned = codec_aligned(a, t.nc);
    }
    return t;
}

}  // namespace

dwt_fuse_status dwt_fuse_run_ex(dwt_fuse_ctx *ctx, dwt_fuse_wavelet wavelet, int64_t H, int64_t W, int64_t B,
                                const void *pan, int64_t pan_ld, const void *ms, int64_t ms_ld, int64_t ms_band_stride,
                                const float *gain, void *out, int64_t out_ld, int64_t out_band_stride,
                                const dwt_fuse_opts *opts) {
    if (!ctx) return DWT_FUSE_E_NULL;
    const dwt_fuse_opts o = opts ? *opts : dwt_fuse_opts{DWT_FUSE_F32, DWT_FUSE_F32, 1.0f};
    if (o.in_format == DWT_FUSE_F32 && o.out_format == DWT_FUSE_F32) {
        const RunArgs a{(int)wavelet, H, W, B, static_cast<const float *>(pan), pan_ld,
                        static_cast<const float *>(ms), ms_ld, ms_band_stride, gain,
                        static_cast<const float *>(out), out_ld, out_band_stride};
        return run_float(ctx, a, o.kappa);
    }
    try {
        const ExArgs a{(int)wavelet, H, W, B, pan, pan_ld, ms, ms_ld, ms_band_stride, gain, out, out_ld,
                       out_band_stride, o.in_format, o.out_format, o.kappa};
        std::string err;
        dwt_fuse_status st = check_ex_args(a, &err);
        if (st) return fail(ctx, st, err);
        if ((st = use_device(ctx))) return st;
        const CodecShape t = codec_shape(ctx, a);
        CodecParams p;
        if (!codec_params(a, t, &p)) return fail(ctx, DWT_FUSE_E_SHAPE, "too many work units");
        const hipError_t e = launch_codec(p, ctx->filt, a.in_format == DWT_FUSE_U8, a.out_format == DWT_FUSE_U8,
                                          t.nc, t.kr, t.aligned, t.wpb, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "format-variant launch");
        return DWT_FUSE_OK;
    } catch (const std::bad_alloc &) {
        return fail(ctx, DWT_FUSE_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(ctx, DWT_FUSE_E_STATE, "unexpected exception");
    }
}

dwt_fuse_status dwt_fuse_check_run_ex(dwt_fuse_wavelet wavelet, int64_t H, int64_t W, int64_t B, const void *pan,
                                      int64_t pan_ld, const void *ms, int64_t ms_ld, int64_t ms_band_stride,
                                      const float *gain, const void *out, int64_t out_ld, int64_t out_band_stride,
                                      const dwt_fuse_opts *opts) {
    const dwt_fuse_opts o = opts ? *opts : dwt_fuse_opts{DWT_FUSE_F32, DWT_FUSE_F32, 1.0f};
    const ExArgs a{(int)wavelet, H, W, B, pan, pan_ld, ms, ms_ld, ms_band_stride, gain, out, out_ld,
                   out_band_stride, o.in_format, o.out_format, o.kappa};
    return check_ex_args(a, nullptr);
}

namespace {

dwt_fuse_status check_quality_args(int64_t H, int64_t W, int64_t B, const float *fused, int64_t f_ld, int64_t f_bs,
                                   const float *ref, int64_t r_ld, int64_t r_bs, const double *out,
                                   std::string *err, bool scores = false) {
    if (!fused || !ref || !out) {
        if (err) *err = "fused, ref and out must not be NULL";
        return DWT_FUSE_E_NULL;
    }
    if (H < 1 || W < 1 || H > kMaxSide || W > kMaxSide || B < 1 || B > kQualityMaxBands) {
        if (err) *err = "H, W must be in [1, 2^30] and B in [1, 65535]";
        return DWT_FUSE_E_SHAPE;
    }
    Span fs, rs;
    dwt_fuse_status st;
    if ((st = check_strided("fused", B, H, W, f_ld, f_bs, fused, &fs, err))) return st;
    if ((st = check_strided("ref", B, H, W, r_ld, r_bs, ref, &rs, err))) return st;
    const int64_t nout = scores ? 4 * B + 1 : 2 * B;
    if (!fits_address_space(out, nout, sizeof(double))) {
        if (err) *err = "out: extent overflows";
        return DWT_FUSE_E_SHAPE;
    }
    const Span os = span_of(out, nout, sizeof(double));
    if (os.overlaps(fs) || os.overlaps(rs)) {
        if (err) *err = "out overlaps an input";
        return DWT_FUSE_E_ALIAS;
    }
    return DWT_FUSE_OK;
}

}  // namespace

namespace {

dwt_fuse_status quality_impl(dwt_fuse_ctx *ctx, int64_t H, int64_t W, int64_t B, const float *fused,
                             int64_t fused_ld, int64_t fused_band_stride, const float *ref, int64_t ref_ld,
                             int64_t ref_band_stride, double *out, bool scores) {
    if (!ctx) return DWT_FUSE_E_NULL;
    try {
        std::string err;
        dwt_fuse_status st = check_quality_args(H, W, B, fused, fused_ld, fused_band_stride, ref, ref_ld,
                                                ref_band_stride, out, &err, scores);
        if (st) return fail(ctx, st, err);
        if ((st = use_device(ctx))) return st;
        if ((st = ensure_ws(ctx, sizeof(double) * 2 * (size_t)kQualityBlocks * (size_t)B))) return st;
        QualityParams p{};
        p.fused = fused;
        p.ref = ref;
        p.f_ld = fused_ld;
        p.f_bs = fused_band_stride;
        p.r_ld = ref_ld;
        p.r_bs = ref_band_stride;
        p.H = (int32_t)H;
        p.W = (int32_t)W;
        p.B = (int32_t)B;
        double *partial = reinterpret_cast<double *>(ctx->ws);
        const hipError_t e = scores ? launch_quality_scores(p, partial, out, ctx->stream)
                                    : launch_quality(p, partial, out, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "quality launch");
        return DWT_FUSE_OK;
    } catch (const std::bad_alloc &) {
        return fail(ctx, DWT_FUSE_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(ctx, DWT_FUSE_E_STATE, "unexpected exception");
    }
}

}  // namespace

dwt_fuse_status dwt_fuse_quality(dwt_fuse_ctx *ctx, int64_t H, int64_t W, int64_t B, const float *fused,
                                 int64_t fused_ld, int64_t fused_band_stride, const float *ref, int64_t ref_ld,
                                 int64_t ref_band_stride, double *out) {
    return quality_impl(ctx, H, W, B, fused, fused_ld, fused_band_stride, ref, ref_ld, ref_band_stride, out, false);
}

dwt_fuse_status dwt_fuse_quality_scores(dwt_fuse_ctx *ctx, int64_t H, int64_t W, int64_t B, const float *fused,
                                        int64_t fused_ld, int64_t fused_band_stride, const float *ref,
                                        int64_t ref_ld, int64_t ref_band_stride, double *out) {
    return quality_impl(ctx, H, W, B, fused, fused_ld, fused_band_stride, ref, ref_ld, ref_band_stride, out, true);
}

dwt_fuse_status dwt_fuse_check_quality(int64_t H, int64_t W, int64_t B, const float *fused, int64_t fused_ld,
                                       int64_t fused_band_stride, const float *ref, int64_t ref_ld,
                                       int64_t ref_band_stride, const double *out) {
    return check_quality_args(H, W, B, fused, fused_ld, fused_band_stride, ref, ref_ld, ref_band_stride, out,
                              nullptr);
}

dwt_fuse_status dwt_fuse_run_batched(dwt_fuse_ctx *ctx, const dwt_fuse_item *items, int64_t n, uint32_t flags) {
    if (!ctx) return DWT_FUSE_E_NULL;
    try {
        std::string err;
        dwt_fuse_status st = check_batch(items, n, &err);
        if (st) return fail(ctx, st, err);
        if (n == 0) return DWT_FUSE_OK;
        if ((st = use_device(ctx))) return st;
        if ((st = ensure_batch_tables(ctx, (size_t)n))) return st;

        BatchPlan plan;
        BatchChoice ch;
        if (ctx->force_batch) {
            ch = ctx->forced_batch;
        } else if (ctx->forced.variant == 1) {
            ch.mode = 0;
        } else if (ctx->forced.variant == 2) {
            ch.mode = std::min(2, std::max(1, ctx->forced.seg_rows > 0 ? ctx->forced.seg_rows : 2));
        } else if (ctx->forced.variant == 3) {
            // forced flat grid: seg_rows = rows per wavefront of its staged
            // tiles (1 or 2), band split = bands they stage at once (0 = all)
            ch.mode = kFlatBatch;
            ch.kr = ctx->forced.seg_rows == 1 ? 1 : 2;
            ch.bg = ctx->forced.split;
        } else {
            // The form is chosen per batch signature (sizes, bands, wavelets,
            // pitches); with tuning on, each candidate is timed once on the
            // batch: the flat grid in dispatch order or per-XCD runs, with
            // its staged tiles holding every band, 3 or 2 bands at once (less
            // LDS per workgroup: more of the batch's one-shot Haar items
            // resident per CU), with 1 or 2 rows per wavefront for every
            // scene or each scene's own (per-image tuned) rows, and the
            // persistent queue kernels.  (Taking each D4 scene's whole
            // per-image shape, one-shot wavefronts where those won alone,
            // measured 1.43 against 1.09 ms on the 96-scene batch: the launch
            // reserves the staged tiles' LDS for every workgroup.)
            if ((st = plan_batch(ctx, items, n, BatchChoice{}, &plan))) return st;
            auto it = ctx->batch_modes.find(plan.sig);
            if (it != ctx->batch_modes.end()) {
                ch = it->second;
            } else if (ctx->tuning) {
                std::vector<BatchChoice> cands;
                for (int kr : {2, 1})
                    for (int bg : {2, 0, 3, 1}) cands.push_back(BatchChoice{kFlatBatch, 3, bg, 1, kr});
                cands.push_back(BatchChoice{kFlatBatch, 1, 2, 1, 2});
                cands.push_back(BatchChoice{kFlatBatch, 3, 0, 0, 2});
                cands.push_back(BatchChoice{kFlatBatch, 3, 2, 2, 2});  // per-scene rows per wavefront
                for (int m : {0, 1, 2}) cands.push_back(BatchChoice{m, 1, 0, 1, 2});
                float best = 1e30f;
                for (const BatchChoice &c : cands) {
                    BatchPlan pm;
                    if ((st = plan_batch(ctx, items, n, c, &pm))) return st;
                    const float ms = time_batch(ctx, pm);
                    if (std::getenv("DWT_FUSE_LOG"))
                        std::fprintf(stderr,
                                     "[dwt_fuse]   batch candidate mode=%d order=%d bg=%d staged=%d kr=%d: %.3f ms\n",
                                     c.mode, c.order, c.bg, c.staged, c.kr, ms);
                    if (ms < best) {
                        best = ms;
                        ch = c;
                    }
                }
                ctx->batch_modes[plan.sig] = ch;
                if (std::getenv("DWT_FUSE_LOG"))
                    std::fprintf(stderr, "[dwt_fuse] tuned batch of %lld scenes: mode=%d order=%d bg=%d (%.3f ms)\n",
                                 (long long)n, ch.mode, ch.order, ch.bg, best);
            }
        }
        if ((st = plan_batch(ctx, items, n, ch, &plan))) return st;
        if ((st = stage_batch(ctx, plan))) return st;

        hipError_t e;
        if (!(flags & DWT_FUSE_GRAPH)) {
            e = launch_plan(ctx, plan, ctx->stream);
            if (e != hipSuccess) return hip_fail(ctx, e, "batched launch");
            return DWT_FUSE_OK;
        }
        auto it = ctx->graphs.find(plan.sig);
        if (it == ctx->graphs.end()) {
            if (!ctx->cap_stream) {
                e = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking);
                if (e != hipSuccess) {
                    ctx->cap_stream = nullptr;
                    return hip_fail(ctx, e, "hipStreamCreate");
                }
            }
            // Capture records the launch without running it; the graph is
            // then launched on the caller's stream, after the table upload.
            hipGraph_t g = nullptr;
            e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamBeginCapture");
            const hipError_t le = launch_plan(ctx, plan, ctx->cap_stream);
            e = hipStreamEndCapture(ctx->cap_stream, &g);
            if (le != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return hip_fail(ctx, le, "batched launch (capture)");
            }
            if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamEndCapture");
            hipGraphExec_t ge = nullptr;
            e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return hip_fail(ctx, e, "hipGraphInstantiate");
            if (ctx->graphs.size() >= 64) clear_graphs(ctx);
            it = ctx->graphs.emplace(plan.sig, ge).first;
        }
        e = hipGraphLaunch(it->second, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipGraphLaunch");
        return DWT_FUSE_OK;
    } catch (const std::bad_alloc &) {
        return fail(ctx, DWT_FUSE_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(ctx, DWT_FUSE_E_STATE, "unexpected exception");
    }
}

dwt_fuse_status dwt_fuse_run_multipass(dwt_fuse_ctx *ctx, dwt_fuse_wavelet wavelet, int64_t H, int64_t W, int64_t B,
                                       const float *pan, int64_t pan_ld, const float *ms, int64_t ms_ld,
                                       int64_t ms_band_stride, float *out, int64_t out_ld, int64_t out_band_stride) {
    if (!ctx) return DWT_FUSE_E_NULL;
    try {
        const RunArgs a{(int)wavelet, H, W, B, pan, pan_ld, ms, ms_ld, ms_band_stride, nullptr, out, out_ld,
                        out_band_stride};
        std::string err;
        dwt_fuse_status st = check_run_args(a, nullptr, &err);
        if (st) return fail(ctx, st, err);
        if (H > 65535) return fail(ctx, DWT_FUSE_E_SHAPE, "the multi-pass pipeline needs H <= 65535");
        if ((st = use_device(ctx))) return st;
        const size_t need = sizeof(float) * 2 * (size_t)H * (size_t)W;
        if (need > ctx->mp_bytes) {
            if (ctx->mp) {
                const hipError_t e = hipStreamSynchronize(ctx->stream);
                if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize before growing the work arrays");
                (void)hipFree(ctx->mp);
                ctx->mp = nullptr;
                ctx->mp_bytes = 0;
            }
            if (hipMalloc(reinterpret_cast<void **>(&ctx->mp), need) != hipSuccess) {
                ctx->mp = nullptr;
                return fail(ctx, DWT_FUSE_E_NOMEM, "multi-pass work arrays could not be allocated");
            }
            ctx->mp_bytes = need;
        }
        const hipError_t e = launch_multipass((int)wavelet, (int)H, (int)W, (int)B, pan, pan_ld, ms, ms_ld,
                                              ms_band_stride, out, out_ld, out_band_stride, ctx->mp,
                                              ctx->mp + (size_t)H * (size_t)W, ctx->filt, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "multi-pass launch");
        return DWT_FUSE_OK;
    } catch (const std::bad_alloc &) {
        return fail(ctx, DWT_FUSE_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(ctx, DWT_FUSE_E_STATE, "unexpected exception");
    }
}

// True when the backward shape of this call comes from the defaults (no
// tuned or loaded table entry).
static bool it_bwd_default(const dwt_fuse_ctx *ctx, const BwdArgs &a, Path path) {
    return ctx->table.find(tune_key(1, a.wavelet, a.H, a.W, a.B, path)) == ctx->table.end();
}

// Work units of the rolling / one-shot adjoint of one scene (everything but
// the LDS-staged form): tile, launch path, decomposition and kernel variant
// (kind 0 rolling, 1 rolling with x = B <= 4 bands unrolled, 2 one-shot
// D4 tiles of x rows).
struct BwdTile {
    Tile t;
    Path pp = PATH_SCALAR;
    Decomp d;
    int kind = 0, x = 0;
    bool auto_seg = false;  // unit length chosen by the default rule below (no tuned or forced one)
};

// Gain partial slots of an adjoint launch: one per (coefficient row, strip),
// B floats each, whatever the unit length (see gain_row).
static int64_t gain_slots(int64_t H, int64_t nstrips) { return (H / 2) * nstrips; }

// Workspace of a single-scene gain reduction: the slots' B floats each, then
// (256-byte aligned) the B * gain_chunks(slots) chunk sums.
static size_t gain_ws_chunk_off(int64_t slots, int64_t B) { return ((size_t)(slots * B) * sizeof(float) + 255) / 256 * 256; }
static size_t gain_ws_bytes(int64_t slots, int64_t B) {
    return gain_ws_chunk_off(slots, B) + (size_t)(gain_chunks(slots) * B) * sizeof(double);
}

// Rows per unit of the band-unrolled D4 adjoint over scenes (H[i], W[i])
// that share one launch: 64 if that still gives >= 1536 units (about one
// round of wavefronts at the kernel's 2-3 waves per SIMD), else the longest
// of 16, 8, 4 that does (4 at least).  Measured: 64 best at 7680^2 and
// 8192^2; below 1536 units at 64 rows, 32-row units lost to 16-row ones
// (6144^2 B = 3: 0.216 vs 0.194 ms; 4096^2 B = 4: 0.113 vs 0.101 ms).
struct SegScene {
    int64_t H, W;
    Tile t;
};
static int bwd_auto_seg(const std::vector<SegScene> &sc) {
    auto units = [&](int seg) {
        int64_t n = 0;
        for (const SegScene &s : sc) {
            Tile t = s.t;
            t.seg_rows = seg;
            Decomp d;
            if (!decompose(s.H, s.W, t, &d)) return (int64_t)-1;
            n += d.units;
        }
        return n;
    };
    if (units(64) >= 1536) return 64;
    for (int seg : {16, 8})
        if (units(seg) >= 1536) return seg;
    return 4;
}
static int bwd_auto_seg(int64_t H, int64_t W, const Tile &t) { return bwd_auto_seg(std::vector<SegScene>{{H, W, t}}); }

static bool plan_bwd(const dwt_fuse_ctx *ctx, const BwdArgs &a, Path path, BwdTile *out) {
    const int64_t H = a.H, W = a.W, B = a.B;
    Tile t = rolling_tile(H, W, path_nc(path));
    {
        auto it = ctx->table.find(tune_key(1, a.wavelet, H, W, B, path));
        if (it != ctx->table.end()) t = it->second;
    }
    if (a.wavelet == DWT_FUSE_D4 && B <= 4 && ctx->forced.seg_rows == 0 && it_bwd_default(ctx, a, path)) {
        t.seg_rows = bwd_auto_seg(H, W, t);
        out->auto_seg = true;
    } else {
        out->auto_seg = false;
    }
    t = apply_forced(ctx, t, path, a.wavelet, path_nc(path));
    // Adjoint kernels: rolling units (mode 0) and, for D4, one-shot tiles of
    // 1 or 2 rows (mode 1, 2); no LDS-staged form here.
    if (t.mode != 0 && !(a.wavelet == DWT_FUSE_D4 && (t.mode == 1 || t.mode == 2))) {
        const Tile r = rolling_tile(H, W, path_nc(path));
        t.mode = 0;
        t.seg_rows = r.seg_rows;
        t.nc = std::min(t.nc, path_nc(path));
        if (t.nc < 1) t.nc = r.nc;
    }
    if (t.mode == 1 || t.mode == 2) t.seg_rows = t.mode;
    if (t.seg_rows < 1) t.seg_rows = 1;
    if (t.nc > path_nc(path)) t.nc = path_nc(path);
    out->t = t;
    out->pp = path_for_nc(path, t.nc);
    if (!decompose(H, W, t, &out->d)) return false;
    if (gain_slots(H, out->d.nstrips) > INT32_MAX - kGainChunk) return false;
    // At most 4 bands: the rolling kernel with the band loop unrolled
    // (unless the dynamic-band rolling kernel is forced).
    if (t.mode != 0) {
        out->kind = 2;
        out->x = t.mode;
    } else if (B <= 4 && ctx->forced.variant != 1) {
        out->kind = 1;
        out->x = (int)B;
    } else {
        out->kind = 0;
        out->x = 0;
    }
    return true;
}

// Parameters of the adjoint launch over bands b0 .. b0 + min(maxb, B - b0) - 1
// (later band groups add into grad_pan).
static AdjParams bwd_params(const BwdArgs &a, const BwdTile &bt, float *partial, int64_t b0) {
    const int64_t nb = std::min<int64_t>(adjoint_max_bands(), a.B - b0);
    AdjParams p{};
    p.pan = a.pan;
    p.gain = a.gain ? a.gain + b0 : nullptr;
    p.gy = a.gy + b0 * a.gy_bs;
    p.grad_pan = const_cast<float *>(a.grad_pan);
    p.grad_ms = a.grad_ms ? const_cast<float *>(a.grad_ms) + b0 * (a.H / 2) * (a.W / 2) : nullptr;
    p.partial = partial ? partial + b0 : nullptr;
    p.pan_ld = a.pan_ld;
    p.gy_ld = a.gy_ld;
    p.gy_bs = a.gy_bs;
    p.H = (int32_t)a.H;
    p.W = (int32_t)a.W;
    p.B = (int32_t)nb;
    p.seg_rows = bt.t.seg_rows;
    p.nseg = bt.d.nseg;
    p.units = bt.d.units;
    p.wavelet = a.wavelet;
    p.path = bt.pp;
    p.nstrips = bt.d.nstrips;
    p.order = bt.t.order;
    p.pstride = (int32_t)a.B;
    p.accumulate = b0 > 0 ? 1 : 0;
    return p;
}

// The LDS-staged D4 adjoint (16- or 8-byte rows): workgroups of wpb wavefronts x
// kr coefficient rows over a 128-column strip; `all` stages the upstream
// gradients of as many bands as fit at once (else band after band in two
// buffers).
struct StagedBwd {
    int kr = 0, wpb = 0;
    bool all = true;
    int order = 0;
};

static int64_t staged_strips(const BwdArgs &a) { return (a.W / 2 + 127) / 128; }

// Fewer than 1536 rolling units even at 4 rows per unit (two columns per lane).
static bool small_for_rolling(const BwdArgs &a, Path path) {
    Tile t = rolling_tile(a.H, a.W, path_nc(path));
    t.seg_rows = 4;
    Decomp d;
    return decompose(a.H, a.W, t, &d) && d.units < 1536;
}

// Whether a scene takes the staged adjoint: on request (forced variant 3,
// with the forced rows and waves), or by default with no tuned or forced
// shape: for D4 with 5 or more bands, where it measured faster than the
// rolling adjoint (whose band loop is unrolled only up to 4 bands), 2 rows
// x 4 wavefronts, every band staged; and, in a call of its own (`single`),
// for a D4 scene too small to fill the GPU with 4-row rolling units
// (< 1536 of them), 1 row x 4 wavefronts (1024^2: 10-25% faster).  A batch
// keeps rolling units for the latter, its scenes filling the GPU together;
// up to 8 bands both kernels give the same bits.
static bool staged_bwd(const dwt_fuse_ctx *ctx, const BwdArgs &a, Path path, bool single, StagedBwd *sb) {
    if (a.wavelet != DWT_FUSE_D4 || path == PATH_SCALAR) return false;
    const Forced &fc = ctx->forced;
    const bool unforced = fc.variant == 0 && fc.seg_rows == 0 && fc.wpb == 0 && fc.nc == 0;
    const bool dflt = unforced && it_bwd_default(ctx, a, path);
    auto it = ctx->table.find(tune_key(1, a.wavelet, a.H, a.W, a.B, path));
    if (fc.variant == 3) {
        sb->kr = fc.seg_rows == 2 ? 2 : 1;
        sb->wpb = fc.wpb >= 1 && fc.wpb <= 4 ? fc.wpb : 4;
        sb->all = fc.nc != 1;
    } else if (unforced && it != ctx->table.end()) {  // tuned (or loaded) shape
        if (it->second.mode < 3) return false;
        sb->kr = it->second.mode - 2;
        sb->wpb = it->second.wpb;
        sb->all = true;
        sb->order = it->second.order;
    } else if (dflt && a.B >= 5) {
        sb->kr = 2;
        sb->wpb = 4;
        sb->all = true;
    } else if (dflt && single && small_for_rolling(a, path)) {
        sb->kr = 1;
        sb->wpb = 4;
        sb->all = true;
    } else {
        return false;
    }
    return adjoint_staged_lds(sb->kr * sb->wpb, (int)a.B, sb->all) <= 65536;
}

// Launches the staged adjoint of one scene; gain slots go to `partial` (NULL:
// no grad_gain).
static dwt_fuse_status run_staged_bwd(dwt_fuse_ctx *ctx, const BwdArgs &a, Path path, const StagedBwd &sb,
                                      float *partial) {
    const int T = sb.kr * sb.wpb;
    const int64_t ns = staged_strips(a), ng = (a.H / 2 + T - 1) / T;
    if (ns * ng > INT32_MAX) return fail(ctx, DWT_FUSE_E_SHAPE, "too many work units");
    AdjParams p{};
    p.pan = a.pan;
    p.gain = a.gain;
    p.gy = a.gy;
    p.grad_pan = const_cast<float *>(a.grad_pan);
    p.grad_ms = const_cast<float *>(a.grad_ms);
    p.partial = partial;
    p.pan_ld = a.pan_ld;
    p.gy_ld = a.gy_ld;
    p.gy_bs = a.gy_bs;
    p.H = (int32_t)a.H;
    p.W = (int32_t)a.W;
    p.B = (int32_t)a.B;
    p.seg_rows = T;
    p.nseg = (int32_t)ng;
    p.units = (int32_t)(ns * ng);
    p.wavelet = a.wavelet;
    p.path = path;
    p.nstrips = (int32_t)ns;
    p.order = ctx->forced.order >= 0 ? ctx->forced.order : sb.order;
    p.pstride = (int32_t)a.B;
    p.accumulate = 0;
    const hipError_t e = launch_adjoint_staged(p, ctx->filt, sb.kr, sb.wpb, sb.all, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "staged adjoint launch");
    return DWT_FUSE_OK;
}

// Gain-reduction workspace of one backward call (slots' partial sums, then
// the chunk sums): context workspace, grown on demand, or with `noalloc` the
// device's static scratch, checked against its size (nothing is launched if
// it does not fit).
static dwt_fuse_status gain_workspace(dwt_fuse_ctx *ctx, bool noalloc, int64_t slots, int64_t B, float **partial,
                                      double **chunks) {
    const size_t bytes = gain_ws_bytes(slots, B);
    char *base = nullptr;
    if (noalloc) {
        if (!ctx->scratch) return fail(ctx, DWT_FUSE_E_DEVICE, ctx->scratch_err);
        if (bytes > kStaticScratchBytes)
            return fail(ctx, DWT_FUSE_E_SHAPE,
                        "grad_gain of this scene needs " + std::to_string(bytes) +
                            " bytes of scratch, more than the static scratch's " +
                            std::to_string(kStaticScratchBytes) + " (use dwt_fuse_backward)");
        base = static_cast<char *>(ctx->scratch);
    } else {
        if (const dwt_fuse_status st = ensure_ws(ctx, bytes)) return st;
        base = reinterpret_cast<char *>(ctx->ws);
    }
    *partial = reinterpret_cast<float *>(base);
    *chunks = reinterpret_cast<double *>(base + gain_ws_chunk_off(slots, B));
    return DWT_FUSE_OK;
}

// The adjoint kernels of one call with launch shape t (rolling mode 0,
// one-shot D4 mode 1-2, LDS-staged D4 mode >= 3), gain slots to `partial`
// (NULL: none); no gain reduction.
static hipError_t launch_bwd_shape(dwt_fuse_ctx *ctx, const BwdArgs &a, Path path, const Tile &t, float *partial) {
    if (t.mode >= 3) {
        StagedBwd sb;
        sb.kr = t.mode - 2;
        sb.wpb = t.wpb;
        sb.all = true;
        sb.order = t.order;
        if (adjoint_staged_lds(sb.kr * sb.wpb, (int)a.B, true) > 65536) return hipErrorInvalidValue;
        return run_staged_bwd(ctx, a, path, sb, partial) == DWT_FUSE_OK ? hipSuccess : hipErrorLaunchFailure;
    }
    BwdTile bt;
    bt.t = t;
    bt.pp = path_for_nc(path, t.nc);
    if (!decompose(a.H, a.W, t, &bt.d)) return hipErrorInvalidValue;
    if (t.mode != 0) {
        bt.kind = 2;
        bt.x = t.mode;
    } else {
        bt.kind = a.B <= 4 ? 1 : 0;
        bt.x = a.B <= 4 ? (int)a.B : 0;
    }
    const int maxb = adjoint_max_bands();
    for (int64_t b0 = 0; b0 < a.B; b0 += maxb) {
        const AdjParams p = bwd_params(a, bt, partial, b0);
        const hipError_t e = bt.kind == 2   ? launch_adjoint_tile(p, ctx->filt, bt.x, t.wpb, ctx->stream)
                             : bt.kind == 1 ? launch_adjoint_bg(p, ctx->filt, t.wpb, ctx->stream)
                                            : launch_adjoint(p, ctx->filt, t.wpb, ctx->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Adjoint tuner (first call of a (wavelet, size class, bands, path) key with
// tuning on): times, on the call's own buffers, rolling units of 4 .. 64
// rows in three unit orders, one-shot D4 tiles of 1 or 2 rows and LDS-staged
// D4 tiles of 1 or 2 rows x 4 wavefronts, every one with the path's widest
// lane layout (so grad_gain keeps the same partial-slot layout and bits),
// then confirms the fastest few as the forward tuner does.
static Tile tune_bwd(dwt_fuse_ctx *ctx, const BwdArgs &a, Path path, float *partial) {
    std::vector<std::pair<float, Tile>> cands;
    const int nc = path_nc(path);
    auto timed = [&](const Tile &t) {
        return time_median3(ctx->stream, [&] { return launch_bwd_shape(ctx, a, path, t, partial); });
    };
    for (int seg : {64, 32, 16, 8, 4})
        for (int order : {1, 0, 3}) {
            Tile t;
            t.mode = 0;
            t.seg_rows = seg;
            t.wpb = 4;
            t.nc = nc;
            t.order = order;
            cands.emplace_back(timed(t), t);
        }
    if (a.wavelet == DWT_FUSE_D4) {
        for (int kr : {1, 2})
            for (int order : {1, 3}) {
                Tile t;
                t.mode = kr;
                t.seg_rows = kr;
                t.wpb = 4;
                t.nc = nc;
                t.order = order;
                cands.emplace_back(timed(t), t);
            }
        if (path != PATH_SCALAR)
            for (int kr : {1, 2})
                for (int order : {0, 3}) {
                    Tile t;
                    t.mode = 2 + kr;
                    t.seg_rows = kr;
                    t.wpb = 4;
                    t.nc = 2;
                    t.order = order;
                    cands.emplace_back(timed(t), t);
                }
    }
    float bestms = 0.f;
    const Tile best = confirm_best(
        ctx->stream, cands, [&](const Tile &t) { return launch_bwd_shape(ctx, a, path, t, partial); },
        [](const Tile &t) { return t.mode >= 3 ? 0 : t.mode > 0 ? 1 : 2 + 64 / std::max(1, t.seg_rows); }, &bestms);
    if (std::getenv("DWT_FUSE_LOG"))
        std::fprintf(stderr, "[dwt_fuse] tuned %s: mode=%d seg_rows=%d wpb=%d nc=%d order=%d (%.3f ms)\n",
                     tune_key(1, a.wavelet, a.H, a.W, a.B, path).c_str(), best.mode, best.seg_rows, best.wpb, best.nc,
                     best.order, bestms);
    return best;
}

static dwt_fuse_status backward_impl(dwt_fuse_ctx *ctx, const BwdArgs &a, bool noalloc) {
    const int64_t H = a.H, B = a.B;
    std::string err;
    dwt_fuse_status st = check_bwd_args(a, &err);
    if (st) return fail(ctx, st, err);
    if (!a.grad_pan && !a.grad_ms && !a.grad_gain) return DWT_FUSE_OK;
    if ((st = use_device(ctx))) return st;
    const Path path = choose_bwd_path(a);
    {
        const Forced &fc = ctx->forced;
        if (ctx->tuning && !noalloc && fc.variant == 0 && fc.seg_rows == 0 && fc.wpb == 0 && fc.nc == 0 &&
            it_bwd_default(ctx, a, path)) {
            // gain slots for the widest strip layout a candidate uses (128 columns)
            float *partial = nullptr;
            double *chunks = nullptr;
            const int64_t slots = gain_slots(H, (a.W / 2 + 63) / 64);
            if (a.grad_gain && slots <= INT32_MAX - kGainChunk &&
                (st = gain_workspace(ctx, false, slots, B, &partial, &chunks)))
                return st;
            ctx->table[tune_key(1, a.wavelet, a.H, a.W, a.B, path)] = tune_bwd(ctx, a, path, partial);
        }
    }
    StagedBwd sb;
    if (staged_bwd(ctx, a, path, true, &sb)) {
        const int64_t slots = gain_slots(H, staged_strips(a));
        if (slots > INT32_MAX - kGainChunk) return fail(ctx, DWT_FUSE_E_SHAPE, "too many gain partial slots");
        float *partial = nullptr;
        double *chunks = nullptr;
        if (a.grad_gain && (st = gain_workspace(ctx, noalloc, slots, B, &partial, &chunks))) return st;
        if ((st = run_staged_bwd(ctx, a, path, sb, partial))) return st;
        if (a.grad_gain) {
            const hipError_t e = launch_gain_reduce(partial, (int)slots, (int)B, chunks, const_cast<float *>(a.grad_gain), ctx->stream);
            if (e != hipSuccess) return hip_fail(ctx, e, "gain reduction launch");
        }
        return DWT_FUSE_OK;
    }
    BwdTile bt;
    if (!plan_bwd(ctx, a, path, &bt)) return fail(ctx, DWT_FUSE_E_SHAPE, "too many work units");
    const int64_t slots = gain_slots(H, bt.d.nstrips);
    float *partial = nullptr;
    double *chunks = nullptr;
    if (a.grad_gain && (st = gain_workspace(ctx, noalloc, slots, B, &partial, &chunks))) return st;
    const int maxb = adjoint_max_bands();
    for (int64_t b0 = 0; b0 < B; b0 += maxb) {
        const AdjParams p = bwd_params(a, bt, partial, b0);
        const hipError_t e = bt.kind == 2   ? launch_adjoint_tile(p, ctx->filt, bt.x, bt.t.wpb, ctx->stream)
                             : bt.kind == 1 ? launch_adjoint_bg(p, ctx->filt, bt.t.wpb, ctx->stream)
                                            : launch_adjoint(p, ctx->filt, bt.t.wpb, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "adjoint launch");
    }
    if (a.grad_gain) {
        const hipError_t e = launch_gain_reduce(partial, (int)slots, (int)B, chunks, const_cast<float *>(a.grad_gain), ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "gain reduction launch");
    }
    return DWT_FUSE_OK;
}

dwt_fuse_status dwt_fuse_backward(dwt_fuse_ctx *ctx, dwt_fuse_wavelet wavelet, int64_t H, int64_t W, int64_t B,
                                  const float *pan, int64_t pan_ld, const float *gain, const float *grad_out,
                                  int64_t go_ld, int64_t go_band_stride, float *grad_pan, float *grad_ms,
                                  float *grad_gain) {
    if (!ctx) return DWT_FUSE_E_NULL;
    try {
        const BwdArgs a{(int)wavelet, H, W, B, pan, pan_ld, gain, grad_out, go_ld, go_band_stride,
                        grad_pan, grad_ms, grad_gain};
        return backward_impl(ctx, a, false);
    } catch (const std::bad_alloc &) {
        return fail(ctx, DWT_FUSE_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(ctx, DWT_FUSE_E_STATE, "unexpected exception");
    }
}

dwt_fuse_status dwt_fuse_backward_noalloc(dwt_fuse_ctx *ctx, dwt_fuse_wavelet wavelet, int64_t H, int64_t W,
                                          int64_t B, const float *pan, int64_t pan_ld, const float *gain,
                                          const float *grad_out, int64_t go_ld, int64_t go_band_stride,
                                          float *grad_pan, float *grad_ms, float *grad_gain) {
    if (!ctx) return DWT_FUSE_E_NULL;
    try {
        const BwdArgs a{(int)wavelet, H, W, B, pan, pan_ld, gain, grad_out, go_ld, go_band_stride,
                        grad_pan, grad_ms, grad_gain};
        return backward_impl(ctx, a, true);
    } catch (const std::bad_alloc &) {
        return fail(ctx, DWT_FUSE_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(ctx, DWT_FUSE_E_STATE, "unexpected exception");
    }
}

dwt_fuse_status dwt_fuse_check_backward_batched(const dwt_fuse_bwd_item *items, int64_t n) {
    return check_bwd_batch(items, n, nullptr);
}

namespace {

// Grow the batched-backward tables to `bytes` (device and pinned staging).
dwt_fuse_status ensure_bwd_tables(dwt_fuse_ctx *c, size_t bytes) {
    if (!c->bwd_staged) {
        const hipError_t e = hipEventCreateWithFlags(&c->bwd_staged, hipEventDisableTiming);
        if (e != hipSuccess) {
            c->bwd_staged = nullptr;
            return hip_fail(c, e, "hipEventCreate");
        }
    }
    if (bytes <= c->bwd_bytes) return DWT_FUSE_OK;
    const hipError_t se = hipStreamSynchronize(c->stream);
    if (se != hipSuccess) return hip_fail(c, se, "hipStreamSynchronize before growing the backward tables");
    if (c->d_bwd) (void)hipFree(c->d_bwd);
    if (c->h_bwd) (void)hipHostFree(c->h_bwd);
    c->d_bwd = nullptr;
    c->h_bwd = nullptr;
    c->bwd_bytes = 0;
    c->bwd_pending = false;
    const size_t cap = std::max<size_t>(bytes, 16384);
    if (hipMalloc(&c->d_bwd, cap) != hipSuccess) {
        c->d_bwd = nullptr;
        return fail(c, DWT_FUSE_E_NOMEM, "backward scene table allocation failed");
    }
    if (hipHostMalloc(&c->h_bwd, cap, hipHostMallocDefault) != hipSuccess) {
        c->h_bwd = nullptr;
        return fail(c, DWT_FUSE_E_NOMEM, "pinned staging allocation failed");
    }
    c->bwd_bytes = cap;
    return DWT_FUSE_OK;
}

// Adjoint launches of one kernel variant and band group.
struct BwdGroup {
    int kind, path, x, chunk;
    std::vector<AdjScene> sc;
    int64_t total = 0;
};

}  // namespace

dwt_fuse_status dwt_fuse_backward_batched(dwt_fuse_ctx *ctx, const dwt_fuse_bwd_item *items, int64_t n) {
    if (!ctx) return DWT_FUSE_E_NULL;
    try {
        std::string err;
        dwt_fuse_status st = check_bwd_batch(items, n, &err);
        if (st) return fail(ctx, st, err);
        if (n == 0) return DWT_FUSE_OK;
        if ((st = use_device(ctx))) return st;
        // Plan every scene as dwt_fuse_backward would, then group the rolling
        // and one-shot launches by kernel variant and band group; scenes on
        // the LDS-staged adjoint get a launch of their own each.
        std::vector<BwdTile> tiles((size_t)n);
        std::vector<StagedBwd> stg((size_t)n);
        std::vector<char> is_staged((size_t)n, 0);
        std::vector<int64_t> nslots((size_t)n, 0);
        std::vector<int64_t> poff((size_t)n, -1);  // float offset of a scene's partials in ws
        std::vector<int64_t> doff((size_t)n, -1);  // offset of its chunk sums in the double part
        int64_t pfloats = 0, pdoubles = 0;
        for (int64_t i = 0; i < n; ++i) {
            const BwdArgs a = bwd_item_args(items[i]);
            if (!a.grad_pan && !a.grad_ms && !a.grad_gain) continue;
            const Path path = choose_bwd_path(a);
            if (staged_bwd(ctx, a, path, false, &stg[(size_t)i])) {
                is_staged[(size_t)i] = 1;
                nslots[(size_t)i] = gain_slots(a.H, staged_strips(a));
                const int T = stg[(size_t)i].kr * stg[(size_t)i].wpb;
                if (staged_strips(a) * ((a.H / 2 + T - 1) / T) > INT32_MAX)
                    return fail(ctx, DWT_FUSE_E_SHAPE, "item " + std::to_string(i) + ": too many work units");
                if (nslots[(size_t)i] > INT32_MAX - kGainChunk)
                    return fail(ctx, DWT_FUSE_E_SHAPE, "item " + std::to_string(i) + ": too many gain partial slots");
            } else {
                if (!plan_bwd(ctx, a, path, &tiles[(size_t)i]))
                    return fail(ctx, DWT_FUSE_E_SHAPE, "item " + std::to_string(i) + ": too many work units");
                nslots[(size_t)i] = gain_slots(a.H, tiles[(size_t)i].d.nstrips);
            }
            if (a.grad_gain) {
                const int64_t slots = nslots[(size_t)i];
                poff[(size_t)i] = pfloats;
                pfloats += slots * a.B;
                doff[(size_t)i] = pdoubles;
                pdoubles += gain_chunks(slots) * a.B;
            }
        }
        // workspace: every scene's slot partials, then (256-byte aligned) their chunk sums
        const size_t dbyte = ((size_t)pfloats * sizeof(float) + 255) / 256 * 256;
        if (pfloats > 0 && (st = ensure_ws(ctx, dbyte + (size_t)pdoubles * sizeof(double)))) return st;
        double *dbase = pfloats > 0 ? reinterpret_cast<double *>(reinterpret_cast<char *>(ctx->ws) + dbyte) : nullptr;
        // Scenes on the default band-unrolled D4 plan run in one launch, so
        // their units are lengthened together: the single-scene rule
        // (bwd_auto_seg) over all of them, never shorter than a scene would
        // take alone.  Gradients do not depend on the unit length (the gain
        // products are kept per row), so every scene's results still equal
        // its single call's bit for bit.
        {
            std::vector<int64_t> joint;
            std::vector<SegScene> hw;
            for (int64_t i = 0; i < n; ++i)
                if (!is_staged[(size_t)i] && tiles[(size_t)i].auto_seg && tiles[(size_t)i].kind == 1 &&
                    tiles[(size_t)i].t.mode == 0) {
                    const BwdArgs a = bwd_item_args(items[i]);
                    if (a.grad_pan || a.grad_ms || a.grad_gain) {
                        joint.push_back(i);
                        hw.push_back(SegScene{a.H, a.W, tiles[(size_t)i].t});
                    }
                }
            if (joint.size() > 1) {
                const int seg = bwd_auto_seg(hw);
                for (const int64_t i : joint) {
                    BwdTile &bt = tiles[(size_t)i];
                    if (seg <= bt.t.seg_rows) continue;
                    Tile t = bt.t;
                    t.seg_rows = seg;
                    Decomp d;
                    if (!decompose(items[i].H, items[i].W, t, &d)) continue;
                    bt.t = t;
                    bt.d = d;
                }
            }
        }
        const int maxb = adjoint_max_bands();
        std::map<std::tuple<int, int, int, int>, BwdGroup> groups;  // (chunk, kind, path, x): chunk first
        std::vector<GainJob> jobs;
        int64_t total_chunks = 0;
        for (int64_t i = 0; i < n; ++i) {
            const BwdArgs a = bwd_item_args(items[i]);
            if (!a.grad_pan && !a.grad_ms && !a.grad_gain) continue;
            const BwdTile &bt = tiles[(size_t)i];
            float *partial = poff[(size_t)i] >= 0 ? ctx->ws + poff[(size_t)i] : nullptr;
            for (int64_t b0 = 0; b0 < a.B && !is_staged[(size_t)i]; b0 += maxb) {
                const int chunk = (int)(b0 / maxb);
                BwdGroup &g = groups[std::make_tuple(chunk, bt.kind, (int)bt.pp, bt.x)];
                g.kind = bt.kind;
                g.path = bt.pp;
                g.x = bt.x;
                g.chunk = chunk;
                AdjScene sc{};
                sc.p = bwd_params(a, bt, partial, b0);
                sc.unit_begin = (int32_t)g.total;
                g.total += bt.d.units;
                if (g.total > INT32_MAX) return fail(ctx, DWT_FUSE_E_SHAPE, "too many work units in batch");
                g.sc.push_back(sc);
            }
            if (partial) {
                const int64_t slots = nslots[(size_t)i], nch = gain_chunks(slots);
                for (int64_t b = 0; b < a.B; ++b) {
                    jobs.push_back(GainJob{partial, const_cast<float *>(a.grad_gain),
                                           dbase + doff[(size_t)i] + b * nch, (int32_t)slots, (int32_t)a.B,
                                           (int32_t)b, (int32_t)total_chunks});
                    total_chunks += nch;
                    if (total_chunks > INT32_MAX)
                        return fail(ctx, DWT_FUSE_E_SHAPE, "too many gain reduction chunks in batch");
                }
            }
        }
        if (jobs.size() > (size_t)INT32_MAX) return fail(ctx, DWT_FUSE_E_SHAPE, "too many gain reductions in batch");
        size_t nsc = 0;
        for (const auto &kv : groups) nsc += kv.second.sc.size();
        const size_t sc_bytes = nsc * sizeof(AdjScene);
        const size_t job_off = (sc_bytes + 255) / 256 * 256;
        const size_t bytes = job_off + jobs.size() * sizeof(GainJob);
        hipError_t e = hipSuccess;
        if (nsc > 0 || !jobs.empty()) {
            if ((st = ensure_bwd_tables(ctx, bytes))) return st;
            if (ctx->bwd_pending) {  // the previous upload has left the pinned buffer
                e = hipEventSynchronize(ctx->bwd_staged);
                if (e != hipSuccess) return hip_fail(ctx, e, "hipEventSynchronize");
            }
            char *h = static_cast<char *>(ctx->h_bwd);
            size_t off = 0;
            for (const auto &kv : groups) {
                std::memcpy(h + off, kv.second.sc.data(), kv.second.sc.size() * sizeof(AdjScene));
                off += kv.second.sc.size() * sizeof(AdjScene);
            }
            if (!jobs.empty()) std::memcpy(h + job_off, jobs.data(), jobs.size() * sizeof(GainJob));
            e = hipMemcpyAsync(ctx->d_bwd, ctx->h_bwd, bytes, hipMemcpyHostToDevice, ctx->stream);
            if (e != hipSuccess) return hip_fail(ctx, e, "backward table upload");
            e = hipEventRecord(ctx->bwd_staged, ctx->stream);
            if (e != hipSuccess) return hip_fail(ctx, e, "hipEventRecord");
            ctx->bwd_pending = true;
        }
        // Band group 0 of every scene first (the map is ordered by chunk), so
        // later groups, which add into grad_pan, run after it on the stream.
        const AdjScene *d_sc = static_cast<const AdjScene *>(ctx->d_bwd);
        for (const auto &kv : groups) {
            const BwdGroup &g = kv.second;
            e = launch_adjoint_batched(d_sc, (int)g.sc.size(), (int)g.total, g.kind, g.path, g.x, ctx->filt,
                                       ctx->stream);
            if (e != hipSuccess) return hip_fail(ctx, e, "batched adjoint launch");
            d_sc += g.sc.size();
        }
        for (int64_t i = 0; i < n; ++i) {
            if (!is_staged[(size_t)i]) continue;
            const BwdArgs a = bwd_item_args(items[i]);
            float *partial = poff[(size_t)i] >= 0 ? ctx->ws + poff[(size_t)i] : nullptr;
            if ((st = run_staged_bwd(ctx, a, choose_bwd_path(a), stg[(size_t)i], partial))) return st;
        }
        if (!jobs.empty()) {
            e = launch_gain_reduce_batched(
                reinterpret_cast<const GainJob *>(static_cast<const char *>(ctx->d_bwd) + job_off), (int)jobs.size(),
                (int)total_chunks, ctx->stream);
            if (e != hipSuccess) return hip_fail(ctx, e, "batched gain reduction launch");
        }
        return DWT_FUSE_OK;
    } catch (const std::bad_alloc &) {
        return fail(ctx, DWT_FUSE_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(ctx, DWT_FUSE_E_STATE, "unexpected exception");
    }
}


