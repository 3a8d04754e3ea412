// Internal interface between the host library (dwt_fuse_api.cpp) and the
// gfx950 kernels (fuse_kernels.hip, adjoint_kernels.hip, codec_kernels.hip,
// multipass_kernels.hip).  Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dwtf {

// Column layout of one lane: NC coefficient columns = 2*NC output columns.
//   PATH_V4     NC = 2, 128-bit PAN/out rows, 64-bit MS rows (all aligned)
//   PATH_V2     NC = 1, 64-bit PAN/out rows, scalar MS
//   PATH_SCALAR NC = 1, scalar everything (odd pointer offsets or pitches)
//   PATH_V2W    NC = 2 on 64-bit rows (forward only): 128-bit accesses on the
//               rows that happen to be 16-byte aligned, 64-bit on the others;
//               64-bit MS on 8-byte aligned MS rows, scalar otherwise
// The LDS-staged D4 kernels read only the row alignment from the path
// (PATH_V2 and PATH_V2W both mean 8-byte rows).
enum Path : int32_t { PATH_V4 = 0, PATH_V2 = 1, PATH_SCALAR = 2, PATH_V2W = 3 };

// Widest lane layout of a path chosen from the alignment of the arguments:
// two coefficient columns per lane on 128- and 64-bit rows (the latter as
// PATH_V2W, see path_for_nc), one on 32-bit rows.
inline int path_nc(Path p) { return p == PATH_SCALAR ? 1 : 2; }

// One scene as the kernels see it.  A work unit is one wavefront (64 lanes)
// covering a strip of 64*NC coefficient columns and seg_rows coefficient
// rows (2*seg_rows output rows) of every band; for the LDS-staged D4 tiles
// (mode >= 3) it is one workgroup covering 128 coefficient columns and
// seg_rows = wavefronts x rows per wavefront coefficient rows.
struct FuseParams {
    const float *pan;
    const float *ms;
    const float *gain;  // NULL = all ones
    float *out;
    int64_t pan_ld, ms_ld, ms_bs, out_ld, out_bs;
    int32_t H, W, B;
    int32_t seg_rows;  // coefficient rows per work unit
    int32_t nseg;      // work units per strip = ceil((H/2) / seg_rows)
    int32_t units;     // nstrips * nseg
    int32_t wavelet;   // 0 Haar, 1 D4
    int32_t path;      // Path
    int32_t nstrips;   // ceil((W/2) / (64*NC))
    int32_t order;     // unit numbering, bit 0: row-band-major (else strip-major); bit 1:
                       // workgroups in dispatch order (else each XCD a contiguous run);
                       // bit 2 (LDS-staged D4 tiles without band split, with bit 0): XCD
                       // slabs, each XCD walking its own chunk of every row band's strips
    int32_t mode;      // 0 rolling over seg_rows rows; 1, 2 one-shot tile of that many rows
    float kappa;       // LL <- kappa * MS band (1 = as printed)
    int32_t bsplit;    // LDS-staged D4: bands per unit (0 = every band in one unit); units
                       // are then (tile, band group) with the groups of a tile adjacent
    int32_t ovl;       // 1: overlapped strips (see strip_origin); 0: strips side by side
    int32_t bg;        // LDS-staged D4: bands staged at once (0 = as many as fit in 64 KB)
    int32_t pad_;
};

// Column strips of a launch.  Side by side (ovl 0), strip k's wavefront
// computes and stores coefficient columns [64 NC k, 64 NC (k+1)).  With output
// rows that do not start on a 64-byte boundary, such strips split a 64-byte
// line of every row between two wavefronts that write their parts at
// different times, which HBM absorbs as slower partial writes.  Overlapped
// strips (ovl 1) advance by S = 64 NC - 8 coefficient columns (2S = 128 NC -
// 16 output pixels, a multiple of 64 bytes); strip k computes the 64 NC
// columns from k S - 8 on, and stores, of every output row, the pixels
// [2 S k - phi, 2 S (k+1) - phi) inside the image, where phi (< 16, even on
// 8-byte aligned rows) is the row's start address in floats modulo 16, so
// every stored run starts on a 64-byte boundary and covers whole lines.  The
// overlap recomputes 16 pixels per strip; the results do not change (each
// pixel is evaluated by the same arithmetic wherever it is computed).
__host__ __device__ inline int strip_stride_cols(int nc, int ovl) { return ovl ? 64 * nc - 8 : 64 * nc; }
// First coefficient column computed by strip k.
__host__ __device__ inline int strip_origin(int k, int nc, int ovl) {
    return ovl ? k * (64 * nc - 8) - 8 : k * 64 * nc;
}
// Number of strips for W output columns.
__host__ __device__ inline int64_t strip_count(int64_t W, int nc, int ovl) {
    return ovl ? (W + 14 + 2 * (64 * nc - 8) - 1) / (2 * (64 * nc - 8)) : (W / 2 + 64 * nc - 1) / (64 * nc);
}

// Daubechies-4 low-pass taps (Eq. 7-8), rounded once from double.
struct Filters {
    float h[4];
};

// Batched (persistent) launch: device table of scenes plus 8 work queues,
// one per XCD, each a contiguous range of the global unit index.
struct BatchScene {
    FuseParams p;
    int32_t unit_begin;  // first global unit index of this scene
    int32_t pad_;
};

constexpr int kQueues = 8;           // = XCDs of an MI355X
constexpr int kQueueStride = 64;     // uint32 slots between counters (256 B)

struct BatchQueues {
    int32_t begin[kQueues];
    int32_t end[kQueues];
};

// Adjoint.  grad_ms / grad_pan are contiguous; grad-gain partial sums are
// written per (coefficient row r, strip, band b) into
// partial[(r * nstrips + strip) * pstride + b] and reduced in a fixed order.
struct AdjParams {
    const float *pan;
    const float *gain;
    const float *gy;  // dL/d(out)
    float *grad_pan;  // may be NULL
    float *grad_ms;   // may be NULL
    float *partial;   // (H/2) * nstrips * pstride floats, may be NULL (no grad_gain)
    int64_t pan_ld, gy_ld, gy_bs;
    int32_t H, W, B;
    int32_t seg_rows, nseg, units;
    int32_t wavelet, path;
    int32_t nstrips, order;  // as in FuseParams
    int32_t pstride;     // floats between consecutive (row, strip) slots
    int32_t accumulate;  // 1: add into grad_pan instead of overwriting
};

hipError_t launch_fuse(const FuseParams &p, const Filters &f, int waves_per_block, hipStream_t s);

// All scenes of one batched launch use the same variant `mode` (see FuseParams).
hipError_t launch_fuse_batched(const BatchScene *d_scenes, int nscenes, const BatchQueues &q,
                               uint32_t *d_counters, int grid, int mode, const Filters &f, hipStream_t s);

// Blocks per CU the batched kernel of a variant can keep resident (grid sizing).
int batched_blocks_per_cu(int mode);

// Flat batched launch: `total` workgroups of 256 threads, one work item each
// (scene unit_begin counts items).  Scenes with mode >= 3 are LDS-staged D4
// tiles of 8 coefficient rows (4 wavefronts x 2 rows, band groups of at most
// `staged_bands`); all others are one-shot single-row wavefront units, 4 per
// item.
hipError_t launch_fuse_batched_flat(const BatchScene *d_scenes, int nscenes, int total, int staged_bands,
                                    int staged_rows, int order, const Filters &f, hipStream_t s);

// Largest band group a staged tile of T coefficient rows can hold in 64 KB of LDS.
int staged_bg_max(int T);

hipError_t launch_adjoint(const AdjParams &p, const Filters &f, int waves_per_block, hipStream_t s);

// Rolling adjoint (D4 or Haar) with the band loop unrolled for p.B <= 4
// bands (whole band set in one launch, no accumulate); same units and
// results as launch_adjoint.
hipError_t launch_adjoint_bg(const AdjParams &p, const Filters &f, int waves_per_block, hipStream_t s);

// One-shot D4 adjoint: units of kr (1 or 2) coefficient rows (p.seg_rows == kr),
// same decomposition and band-group rules as launch_adjoint.
hipError_t launch_adjoint_tile(const AdjParams &p, const Filters &f, int kr, int waves_per_block, hipStream_t s);

// grad_gain[b] = sum_u partial[u * B + b] over slots u < units, b < B, in
// FP64 and a fixed order: first per chunk of kGainChunk consecutive slots
// (one workgroup each; the chunk sums go to `chunks`, B * gain_chunks(units)
// doubles of device workspace, band-major), then each band's chunk sums.
constexpr int kGainChunk = 2048;
inline int64_t gain_chunks(int64_t units) { return (units + kGainChunk - 1) / kGainChunk; }
hipError_t launch_gain_reduce(const float *partial, int units, int B, double *chunks, float *grad_gain,
                              hipStream_t s);

// One scene of a batched adjoint launch: its parameters (as for the
// single-scene launchers) and the first launch-wide unit it owns.
struct AdjScene {
    AdjParams p;
    int32_t unit_begin;
    int32_t pad_;
};

// Adjoint units of many scenes that share one kernel variant, in one launch
// of 4-wavefront workgroups (scenes sorted by unit_begin, units of scene i
// are unit_begin[i] .. unit_begin[i] + p.units - 1, total in all).  kind 0:
// rolling, any wavelet, B <= adjoint_max_bands(); kind 1: rolling, any
// wavelet, x = B <= 4 bands unrolled (no accumulate); kind 2: one-shot D4 tiles of
// x = seg_rows (1 or 2) rows.  path: PATH_V4, PATH_V2W (two columns per lane
// on 8-byte rows), PATH_V2 or PATH_SCALAR, the same for every scene.  Results
// per scene equal the single-scene launch.
hipError_t launch_adjoint_batched(const AdjScene *d_scenes, int nscenes, int total, int kind, int path, int x,
                                  const Filters &f, hipStream_t s);

// One band of one scene's gain reduction: grad_gain[band] = sum over the
// scene's slots u of partial[u * pstride + band], with the chunks, order and
// rounding of launch_gain_reduce.  `chunks` holds the job's
// gain_chunks(units) chunk sums; chunk_begin numbers the job's first chunk
// among all chunks of the launch (jobs in increasing order, total_chunks in
// all).
struct GainJob {
    const float *partial;
    float *grad_gain;
    double *chunks;
    int32_t units, pstride, band, chunk_begin;
};
hipError_t launch_gain_reduce_batched(const GainJob *d_jobs, int njobs, int total_chunks, hipStream_t s);

// Bands one rolling adjoint launch handles (the host splits larger band counts).
int adjoint_max_bands();

// LDS-staged D4 adjoint (p.path PATH_V4: 16-byte rows; PATH_V2 or PATH_V2W:
// 8-byte rows, staged with 4-byte loads): units are strips of 128 coefficient
// columns x (kr * wpb) coefficient rows, one workgroup each; any band count.
// all: the upstream gradients of a group of bands are staged together (one
// barrier per group) instead of band after band into two alternating buffers.
hipError_t launch_adjoint_staged(const AdjParams &p, const Filters &f, int kr, int wpb, bool all, hipStream_t s);
size_t adjoint_staged_lds(int T, int B, bool all);

// Format variants (codec_kernels.hip): pan/ms 8-bit with out float32 or 8-bit,
// or pan/ms float32 with out 8-bit; MS scaled by kappa.  Units are one-shot wavefronts over a strip of
// 64*nc coefficient columns and kr coefficient rows; pitches and band
// strides in elements of each buffer's format.
struct CodecParams {
    const void *pan;
    const void *ms;
    const float *gain;  // NULL = all ones
    void *out;
    int64_t pan_ld, ms_ld, ms_bs, out_ld, out_bs;
    float kappa;
    int32_t H, W, B;
    int32_t nstrips;   // ceil((W/2) / (64*nc))
    int32_t seg_rows;  // coefficient rows per unit (= kr for one-shot tiles)
    int32_t nseg;      // ceil((H/2) / seg_rows)
    int32_t units;     // nstrips * nseg
    int32_t order;     // as in FuseParams
    int32_t wavelet;   // 0 Haar, 1 D4
};

// Shapes that exist: 8-bit input nc 4 or 8 (kr 1, 2, or 0 = rolling for D4)
// on aligned buffers, nc 4 kr 1 otherwise; float input nc 2 (likewise).
bool codec_shape_ok(int in_u8, int nc, int kr, bool aligned, int wavelet);
hipError_t launch_codec(const CodecParams &p, const Filters &f, int in_u8, int out_u8, int nc, int kr, bool aligned,
                        int waves_per_block, hipStream_t s);

// Quality diagnostics (quality_kernels.hip): per band, sum of squared
// differences fused - ref and sum of ref, FP64, fixed order.
struct QualityParams {
    const float *fused;
    const float *ref;
    int64_t f_ld, f_bs, r_ld, r_bs;
    int32_t H, W, B;
};
constexpr int kQualityBlocks = 256;       // blocks per band
constexpr int kQualityMaxBands = 65535;  // grid y limit
// partial: B * kQualityBlocks * 2 doubles of workspace; out: 2 * B doubles.
hipError_t launch_quality(const QualityParams &p, double *partial, double *out, hipStream_t s);
// The same sums followed by RMSE, mean and the ERGAS-style score: out holds
// 4*B + 1 doubles (sse, sum_ref, rmse, mean per band, then the score).
hipError_t launch_quality_scores(const QualityParams &p, double *partial, double *out, hipStream_t s);

// Static device scratch of the entry points that allocate nothing
// (static_scratch.hip): kStaticScratchBytes per GPU, held from the library's
// load until the process ends.  static_scratch_address gives its address on
// `device` (looked up once per device, then cached).
constexpr size_t kStaticScratchBytes = size_t(16) << 20;
hipError_t static_scratch_address(int device, void **ptr);

// The paper's multi-pass pipeline (comparator); work and scratch are H x W.
hipError_t launch_multipass(int wavelet, int H, int W, int B, const float *pan, int64_t pan_ld, const float *ms,
                            int64_t ms_ld, int64_t ms_bs, float *out, int64_t out_ld, int64_t out_bs, float *work,
                            float *scratch, const Filters &f, hipStream_t s);

}  // namespace dwtf
