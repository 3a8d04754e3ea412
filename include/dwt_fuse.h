/*
 * dwt_fuse.h -- C ABI of the MI355X (gfx950) DWT pan-sharpening library.
 *
 * The operation (Al-Oraiqat et al., "Fusion of multispectral satellite
 * imagery using a cluster of graphics processing unit", section 2): for a
 * panchromatic image PAN of H x W pixels and B multispectral bands of
 * (H/2) x (W/2) pixels each (the 4:1 pixel ratio of section 2), output band b
 * is
 *     inverse2D( forward2D(PAN) with its approximation (LL) quadrant
 *                replaced by MS band b )
 * where forward2D is the 1D transform over every row and then every column,
 * and inverse2D is the 1D inverse over every column and then every row.
 *   - DWT_FUSE_HAAR: Eq. 1-2 (forward, divided by 2) and Eq. 11-12 (inverse).
 *   - DWT_FUSE_D4:   Daubechies-4 with periodic wrap, Eq. 3-10 (forward) and
 *                    Eq. 13-16 (inverse), with the high-pass filter read as
 *                    g_k = (-1)^k h_{3-k} (Eq. 9-10 are garbled in print).
 * The MS band is inserted unscaled.  An optional per-band gain multiplies the
 * three detail quadrants of PAN before the inverse (gain 1 = the method as
 * printed); it is the "injection gain" that the backward pass differentiates.
 *
 * Conventions for every entry point:
 *   - All image pointers are DEVICE pointers to float32, owned by the caller,
 *     row-major.  "ld" is the row pitch and "band_stride" the distance between
 *     consecutive bands, both in elements (not bytes).
 *   - H and W must be even and >= 2.  Any even size is valid for both
 *     wavelets (a side of 2 makes D4 reduce to orthonormal Haar along it).
 *   - Pointers and pitches need no particular alignment; 16-byte aligned
 *     rows take the 128-bit path, others a narrower one, with identical results.
 *   - Calls are asynchronous and ordered on the context's HIP stream.  The
 *     returned status covers argument validation (done on the host before any
 *     HIP call) and launch errors; a fault inside a kernel is reported as
 *     DWT_FUSE_E_DEVICE by a later call.
 *   - No call throws or aborts.  A context is not thread-safe; use one per
 *     host thread / stream.
 */
#ifndef DWT_FUSE_H
#define DWT_FUSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { DWT_FUSE_HAAR = 0, DWT_FUSE_D4 = 1 } dwt_fuse_wavelet;

typedef enum {
    DWT_FUSE_OK = 0,
    DWT_FUSE_E_NULL = 1,    /* a required pointer is NULL */
    DWT_FUSE_E_SHAPE = 2,   /* H or W odd or < 2, B < 1, n < 0, or a size overflows */
    DWT_FUSE_E_WAVELET = 3, /* wavelet not in dwt_fuse_wavelet */
    DWT_FUSE_E_STRIDE = 4,  /* ld < row width, or band_stride < rows * ld */
    DWT_FUSE_E_ALIAS = 5,   /* an output's byte range overlaps an input's */
    DWT_FUSE_E_NOMEM = 6,   /* context workspace could not be allocated */
    DWT_FUSE_E_DEVICE = 7,  /* HIP error (bad device, launch failure, earlier fault) */
    DWT_FUSE_E_STATE = 8,   /* context unusable (e.g. created for another device) */
    DWT_FUSE_E_FORMAT = 9   /* element format not in dwt_fuse_format */
} dwt_fuse_status;

typedef struct dwt_fuse_ctx dwt_fuse_ctx; /* opaque */

/* Create a context bound to HIP device `device` and stream `hip_stream`
 * (a hipStream_t; NULL = the default stream).  The context owns its
 * workspace (gradient partial sums, batch descriptor tables, captured
 * graphs, the tuning table).  On failure *ctx is set to NULL. */
dwt_fuse_status dwt_fuse_create(dwt_fuse_ctx **ctx, int device, void *hip_stream);

/* Release a context and everything it owns.  NULL is ignored.  Waits for
 * all work on the context's device first (hipDeviceSynchronize), so work
 * issued through the context never reads freed memory. */
void dwt_fuse_destroy(dwt_fuse_ctx *ctx);

/* Make subsequent calls use `hip_stream` (same device).  When the stream
 * changes, the new stream is made to wait (hipStreamWaitEvent, no host
 * wait) for everything already issued through the context on the old one,
 * so the context's workspace and tables are never rewritten while earlier
 * work still reads them.  DWT_FUSE_E_DEVICE if that ordering cannot be
 * set up. */
dwt_fuse_status dwt_fuse_set_stream(dwt_fuse_ctx *ctx, void *hip_stream);

/* Fuse one scene (section 2, method steps 1-3, for every band).
 *   pan   H x W, pitch pan_ld (>= W).
 *   ms    B bands of (H/2) x (W/2), pitch ms_ld (>= W/2), band_stride
 *         ms_band_stride (>= (H/2) * ms_ld when B > 1).
 *   gain  NULL (all ones) or B floats on the device: detail gain per band.
 *   out   B bands of H x W, pitch out_ld (>= W), band stride
 *         out_band_stride (>= H * out_ld when B > 1).  Must not overlap pan,
 *         ms or gain (DWT_FUSE_E_ALIAS).
 * The PAN detail part is computed once and reused for all bands.  Haar
 * results on integer-valued inputs are exact (every intermediate is a
 * multiple of 1/4); D4 results are float32 evaluations of the same map.
 * Allocates nothing. */
dwt_fuse_status dwt_fuse_run(dwt_fuse_ctx *ctx, dwt_fuse_wavelet wavelet,
                             int64_t H, int64_t W, int64_t B,
                             const float *pan, int64_t pan_ld,
                             const float *ms, int64_t ms_ld, int64_t ms_band_stride,
                             const float *gain,
                             float *out, int64_t out_ld, int64_t out_band_stride);

/* Element formats of dwt_fuse_run_ex. */
typedef enum { DWT_FUSE_F32 = 0, DWT_FUSE_U8 = 1 } dwt_fuse_format;

typedef struct {
    int32_t in_format;  /* dwt_fuse_format of pan and ms */
    int32_t out_format; /* dwt_fuse_format of out */
    float kappa;        /* LL <- kappa * MS band (1 = as printed) */
} dwt_fuse_opts;

/* dwt_fuse_run with a choice of element formats and of the scale of the
 * inserted MS band.
 *   - in_format DWT_FUSE_U8: pan and ms hold 8-bit pixels (uint8_t), the
 *     8-bit-per-pixel representation the paper moves images in (section 3).
 *   - out_format DWT_FUSE_U8: each output pixel is the float32 value that
 *     out_format DWT_FUSE_F32 gives, rounded to the nearest integer (ties to
 *     the even one), clamped to [0, 255], NaN -> 0.
 *   - kappa scales the MS band where it replaces LL (section 2, step 2).  1 is
 *     the method as printed; 2 = (sum of the D4 low-pass taps of Eq. 7-8)^2
 *     matches the DC gain of the D4 analysis LL, so that a band at MS
 *     radiometry keeps its mean level (with 1, D4 output has half the MS mean).
 * Pitches and band strides are in elements of each buffer's own format.
 * opts NULL = {F32, F32, 1}.  With opts {F32, F32, 1} this is dwt_fuse_run.
 * For every format the float32 values equal dwt_fuse_run's on the same
 * (converted) inputs and gains times kappa on the MS band, bit for bit.
 * DWT_FUSE_E_FORMAT for a format outside the enum; other errors as in
 * dwt_fuse_run, with byte ranges computed from each format's element size.
 * Allocates nothing. */
dwt_fuse_status dwt_fuse_run_ex(dwt_fuse_ctx *ctx, dwt_fuse_wavelet wavelet,
                                int64_t H, int64_t W, int64_t B,
                                const void *pan, int64_t pan_ld,
                                const void *ms, int64_t ms_ld, int64_t ms_band_stride,
                                const float *gain,
                                void *out, int64_t out_ld, int64_t out_band_stride,
                                const dwt_fuse_opts *opts);

/* Quality diagnostics of B fused bands against B reference bands (e.g. the
 * full-resolution truth of a synthetic scene), both H x W float32 on the
 * device with their own pitches and band strides:
 *     out[b]     = sum over pixels of (fused_b - ref_b)^2
 *     out[B + b] = sum over pixels of ref_b
 * accumulated in FP64 in a fixed order (reproducible bit for bit); out is a
 * device array of 2*B doubles.  From these, RMSE_b = sqrt(out[b] / (H*W)),
 * mean_b = out[B+b] / (H*W), and an ERGAS-style score
 * 100 * (1/2) * sqrt(mean over b of (RMSE_b / mean_b)^2) for the 1:2 PAN:MS
 * pixel-size ratio of section 2 (the paper names ERGAS in section 4 without
 * defining it).  H, W >= 1; 1 <= B <= 65535.  Uses context workspace
 * (DWT_FUSE_E_NOMEM if it cannot grow); out must not overlap the inputs. */
dwt_fuse_status dwt_fuse_quality(dwt_fuse_ctx *ctx, int64_t H, int64_t W, int64_t B,
                                 const float *fused, int64_t fused_ld, int64_t fused_band_stride,
                                 const float *ref, int64_t ref_ld, int64_t ref_band_stride,
                                 double *out);

/* As dwt_fuse_quality, with the scores formed on the device in FP64 (bands
 * in order, reproducible bit for bit): out is a device array of 4*B + 1
 * doubles, out[0 .. 2B) the sums above, out[2B + b] = RMSE_b, out[3B + b] =
 * mean_b, out[4B] = the ERGAS-style score (+inf if some mean_b is 0). */
dwt_fuse_status dwt_fuse_quality_scores(dwt_fuse_ctx *ctx, int64_t H, int64_t W, int64_t B,
                                        const float *fused, int64_t fused_ld, int64_t fused_band_stride,
                                        const float *ref, int64_t ref_ld, int64_t ref_band_stride,
                                        double *out);

/* One independent scene of a batch; fields as in dwt_fuse_run. */
typedef struct {
    int32_t wavelet; /* dwt_fuse_wavelet */
    int32_t B;
    int64_t H, W;
    const float *pan, *ms, *gain; /* gain may be NULL */
    float *out;
    int64_t pan_ld, ms_ld, ms_band_stride, out_ld, out_band_stride;
} dwt_fuse_item;

enum { DWT_FUSE_GRAPH = 1 /* capture into / replay from a cached hipGraph */ };

/* Fuse n independent scenes of any sizes, band counts and wavelets in ONE
 * kernel launch.  The launch is either a flat grid, one workgroup per
 * (scene, tile) work item (LDS-staged D4 tiles, one-shot Haar wavefronts),
 * or a persistent kernel whose workgroups take work units from per-XCD
 * device queues; with tuning on, the form (grid or queue, unit order, rows
 * per wavefront, bands staged at once) is timed on the batch itself and
 * kept per batch signature, else the flat grid with 2-row staged tiles
 * runs.  The environment variable DWT_FUSE_FORCE_BATCH = "mode,order,bg,
 * staged,kr" read at dwt_fuse_create fixes the form (mode 3 = flat grid;
 * staged 2 = each D4 scene with its own per-image tuned rows per
 * wavefront).  `items` is a HOST array of n descriptors (read during the
 * call only); the pointers inside are device pointers.  Every item is
 * validated as in dwt_fuse_run (first failure returned, nothing launched);
 * outputs must not overlap any item's inputs or each other.  Results are
 * bit-identical to one dwt_fuse_run call per scene, in every form.  With
 * DWT_FUSE_GRAPH the launch is captured once per batch signature (sizes,
 * bands, wavelets, pitches) and replayed afterwards; scene pointers live in
 * a device table refreshed before each replay, so new tensors of the same
 * signature replay safely.  n == 0 is a no-op.  The context grows its
 * descriptor tables on first use of a larger batch (DWT_FUSE_E_NOMEM on
 * failure). */
dwt_fuse_status dwt_fuse_run_batched(dwt_fuse_ctx *ctx, const dwt_fuse_item *items,
                                     int64_t n, uint32_t flags);

/* Transpose (adjoint) of dwt_fuse_run with respect to PAN, MS and the
 * per-band gains, for a given upstream gradient grad_out = dL/d(out).
 *   pan       H x W, pitch pan_ld (needed for dL/dgain).
 *   gain      NULL (all ones) or B device floats (the forward's gains).
 *   grad_out  B x H x W, pitch go_ld, band stride go_band_stride.
 *   grad_pan  NULL or H x W contiguous:      sum_b gain_b (y_b - P y_b)
 *   grad_ms   NULL or B x H/2 x W/2 contiguous: LL part of forward2D(y_b)
 *             (Haar: the 2x2 block sum of y_b, the transpose of Eq. 11-12)
 *   grad_gain NULL or B floats:              < y_b, PAN - P PAN >
 * where P is the projection of an image onto its LL part.  grad_gain is
 * reduced in a fixed order (bitwise reproducible, whatever the rows per work
 * unit).  D4 on 8-byte aligned rows runs the LDS-staged adjoint (all bands
 * in one launch) with 5 or more bands or when the scene is too small to
 * fill the GPU with 4-row rolling units; other cases the rolling adjoint.
 * Outputs must not overlap inputs.  Uses context workspace (DWT_FUSE_E_NOMEM
 * if it cannot grow). */
dwt_fuse_status dwt_fuse_backward(dwt_fuse_ctx *ctx, dwt_fuse_wavelet wavelet,
                                  int64_t H, int64_t W, int64_t B,
                                  const float *pan, int64_t pan_ld, const float *gain,
                                  const float *grad_out, int64_t go_ld, int64_t go_band_stride,
                                  float *grad_pan, float *grad_ms, float *grad_gain);

/* Size of the static device scratch used by dwt_fuse_backward_noalloc, per GPU. */
#define DWT_FUSE_STATIC_SCRATCH_BYTES (16u * 1024u * 1024u)

/* dwt_fuse_backward for callers that cannot allocate device memory: code
 * under hipGraph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, validation and kernels as dwt_fuse_backward
 * on the same context, so the same results bit for bit; it calls no
 * hipMalloc, hipFree or other allocating routine.  The only scratch it needs,
 * the grad_gain reduction's partial sums, lives in a static device array of
 * DWT_FUSE_STATIC_SCRATCH_BYTES that every GPU the library runs on holds
 * from the library's load until the process ends (its address is looked up
 * once per device in dwt_fuse_create).  That is
 *   4 * B * (H/2) * S  bytes (rounded up to 256) + 8 * B * ceil((H/2) * S / 2048)
 * with S = ceil((W/2) / 128) column strips, or ceil((W/2) / 64) where the
 * adjoint runs one column per lane (pointers or pitches not 8-byte aligned,
 * or such a shape forced), e.g. 10.7 MB for 15872 x 14336 with 6 bands; a call needing more returns DWT_FUSE_E_SHAPE before launching
 * anything.  Without grad_gain no scratch is used.  Every call on one GPU
 * shares that GPU's array (each call overwrites every slot it reads, so
 * nothing needs clearing): calls that may overlap in time on one GPU (other
 * streams, contexts or threads) race on it and must be ordered by the
 * caller. */
dwt_fuse_status dwt_fuse_backward_noalloc(dwt_fuse_ctx *ctx, dwt_fuse_wavelet wavelet,
                                          int64_t H, int64_t W, int64_t B,
                                          const float *pan, int64_t pan_ld, const float *gain,
                                          const float *grad_out, int64_t go_ld, int64_t go_band_stride,
                                          float *grad_pan, float *grad_ms, float *grad_gain);

/* One scene of a batched backward; fields as in dwt_fuse_backward (grad_pan
 * H x W and grad_ms B x H/2 x W/2 contiguous; each output may be NULL). */
typedef struct {
    int32_t wavelet; /* dwt_fuse_wavelet */
    int32_t B;
    int64_t H, W;
    const float *pan;
    const float *gain; /* NULL = all ones */
    const float *grad_out;
    float *grad_pan, *grad_ms, *grad_gain;
    int64_t pan_ld, go_ld, go_band_stride;
} dwt_fuse_bwd_item;

/* dwt_fuse_backward of n independent scenes (any sizes, band counts and
 * wavelets; the adjoint of a dwt_fuse_run_batched call, for instance) with
 * one adjoint launch per kernel variant present in the batch (scenes of the
 * same variant share a launch, so small scenes fill the GPU together) and
 * two launches for every grad_gain reduction.  Each scene gets the kernel
 * variant dwt_fuse_backward would give it on this context (a scene on the
 * LDS-staged adjoint gets a launch of its own); scenes on the default
 * band-unrolled D4 plan (at most 4 bands, no tuned or forced shape) may take
 * longer work units than alone, since the batch fills the GPU together.  No
 * gradient depends on the unit length, so every scene's results are
 * bit-identical to that call's.  `items` is a HOST array of n descriptors
 * (read during the call only); the pointers inside are device pointers.
 * Every item is validated as in dwt_fuse_backward (first failure returned,
 * nothing launched); no output of any item may overlap any input or another
 * output of any item.  n == 0 is a no-op.  Uses context workspace for the
 * per-row gain partials of all scenes and a context-owned scene table, grown
 * on first use of a larger batch (DWT_FUSE_E_NOMEM on failure). */
dwt_fuse_status dwt_fuse_backward_batched(dwt_fuse_ctx *ctx, const dwt_fuse_bwd_item *items, int64_t n);

/* The paper's own GPU pipeline, kept as a comparator for dwt_fuse_run
 * (section 3, the per-channel step list): for each band, PAN is copied into a
 * working array, then full-image passes run one after another -- forward 1D
 * over rows, copy, forward 1D over columns, LL replaced by the band, copy,
 * inverse 1D over columns, copy, inverse 1D over rows into the output band --
 * one thread per output element.  Same arguments and results as
 * dwt_fuse_run without gains (Haar bit-identical; D4 within float32
 * rounding).  Uses two H x W float work arrays owned by the context,
 * allocated on first use of a larger size (DWT_FUSE_E_NOMEM on failure).
 * H must be <= 65535. */
dwt_fuse_status dwt_fuse_run_multipass(dwt_fuse_ctx *ctx, dwt_fuse_wavelet wavelet,
                                       int64_t H, int64_t W, int64_t B,
                                       const float *pan, int64_t pan_ld,
                                       const float *ms, int64_t ms_ld, int64_t ms_band_stride,
                                       float *out, int64_t out_ld, int64_t out_band_stride);

/* Argument validation only, exactly as the calls above perform it; no HIP
 * call is made, so these work without a GPU. */
dwt_fuse_status dwt_fuse_check_run(dwt_fuse_wavelet wavelet, int64_t H, int64_t W, int64_t B,
                                   const float *pan, int64_t pan_ld,
                                   const float *ms, int64_t ms_ld, int64_t ms_band_stride,
                                   const float *gain,
                                   const float *out, int64_t out_ld, int64_t out_band_stride);
dwt_fuse_status dwt_fuse_check_run_ex(dwt_fuse_wavelet wavelet, int64_t H, int64_t W, int64_t B,
                                      const void *pan, int64_t pan_ld,
                                      const void *ms, int64_t ms_ld, int64_t ms_band_stride,
                                      const float *gain,
                                      const void *out, int64_t out_ld, int64_t out_band_stride,
                                      const dwt_fuse_opts *opts);
dwt_fuse_status dwt_fuse_check_quality(int64_t H, int64_t W, int64_t B,
                                       const float *fused, int64_t fused_ld, int64_t fused_band_stride,
                                       const float *ref, int64_t ref_ld, int64_t ref_band_stride,
                                       const double *out);
dwt_fuse_status dwt_fuse_check_batched(const dwt_fuse_item *items, int64_t n);
dwt_fuse_status dwt_fuse_check_backward_batched(const dwt_fuse_bwd_item *items, int64_t n);
dwt_fuse_status dwt_fuse_check_backward(dwt_fuse_wavelet wavelet, int64_t H, int64_t W, int64_t B,
                                        const float *pan, int64_t pan_ld, const float *gain,
                                        const float *grad_out, int64_t go_ld, int64_t go_band_stride,
                                        const float *grad_pan, const float *grad_ms,
                                        const float *grad_gain);

/* Static description of a status code. */
const char *dwt_fuse_status_str(dwt_fuse_status s);

/* Human-readable detail of the last failure on this context ("" if none). */
const char *dwt_fuse_last_error(const dwt_fuse_ctx *ctx);

/* Tuning.  The launch shape of each call (kernel variant, rows per work
 * unit, waves per workgroup, columns per lane, unit order) comes from a
 * per-context table keyed by wavelet, size class and band count.  With tuning
 * enabled, the first call of each key times the candidate shapes on that
 * call's own buffers (each candidate writes the same output) and keeps the
 * fastest; the first batched call of each batch signature likewise times the
 * kernel variants on the batch.  The table can be saved to / loaded from a
 * small text file (a header line, then one line per key); a file whose
 * header does not match this library build and device, or with a malformed
 * line, is refused as a whole (DWT_FUSE_E_STATE) and the table is unchanged. */
dwt_fuse_status dwt_fuse_set_tuning(dwt_fuse_ctx *ctx, int enable);
dwt_fuse_status dwt_fuse_tune_save(const dwt_fuse_ctx *ctx, const char *path);
dwt_fuse_status dwt_fuse_tune_load(dwt_fuse_ctx *ctx, const char *path);

/* Force a launch shape for all later launches on this context (0 = automatic
 * for that field): coefficient rows per work unit, waves per workgroup,
 * coefficient columns per lane (1 or 2; 4-byte rows always use 1), and the
 * kernel variant (1 = rolling wavefronts that walk seg_rows rows; 2 = one-shot
 * wavefronts of 1 or 2 rows that issue all their loads up front; 3 =
 * LDS-staged workgroups whose wavefronts take seg_rows = 1, 2 or 4 rows each,
 * D4 only, otherwise 2 is used).  Every shape gives bit-identical results.
 * dwt_fuse_run_ex with 8-bit input follows the rows and waves fields (columns
 * 1 / 2 select 4 / 8 per lane), variant 1 (rolling D4) and variant 3
 * (LDS-staged D4, 1 or 2 rows per wavefront); other format combinations use
 * one-shot tiles.  dwt_fuse_backward and dwt_fuse_backward_batched follow the
 * rows, waves and columns fields with the rolling adjoint and variant 2 with
 * one-shot D4 adjoint tiles; variant 3 selects the LDS-staged D4 adjoint
 * (8-byte aligned rows, 1 or 2 rows per wavefront, up to 4 waves; columns 1
 * stages the upstream gradients band after band), which is otherwise the
 * untuned default for D4 on 8-byte aligned rows with 5 or more bands, and
 * in dwt_fuse_backward for scenes too small to fill the GPU with 4-row
 * rolling units.
 * DWT_FUSE_E_SHAPE if a field is out of range. */
dwt_fuse_status dwt_fuse_force_tile(dwt_fuse_ctx *ctx, int seg_rows, int waves_per_block, int cols_per_lane,
                                    int variant);

/* Force LDS-staged D4 launches (dwt_fuse_run, dwt_fuse_run_ex with float
 * formats) to split each tile's bands into work units of bands_per_unit
 * bands (1 .. 8; 0 = automatic: the tuned or default choice, which keeps all
 * bands of a tile in one unit unless tuning found a split faster).  The
 * units of one tile are adjacent, so the PAN rows they share are re-read
 * from L2.  Results are bit-identical for every split.  DWT_FUSE_E_SHAPE if
 * out of range. */
dwt_fuse_status dwt_fuse_force_band_split(dwt_fuse_ctx *ctx, int bands_per_unit);

/* Force the order in which the work units of forward launches (dwt_fuse_run,
 * dwt_fuse_run_ex, the flat dwt_fuse_run_batched form) and of the adjoint
 * are numbered and handed to workgroups: bit 0 set = row bands across the
 * image width (else column strips down the image), bit 1 set = workgroups
 * take units in dispatch order, so the whole GPU advances through them as
 * one front (else each XCD takes a contiguous run); bit 2 set (LDS-staged D4
 * tiles of dwt_fuse_run without a band split; other launches ignore it) =
 * XCD slabs: row bands across the GPU, each of the 8 XCDs taking a
 * contiguous chunk of every band's strips, so neighbouring tiles share an
 * L2; -1 = automatic (the tuned or default order).  Results are
 * bit-identical for every order.  DWT_FUSE_E_SHAPE if out of range
 * (-1 .. 7).  The environment variable DWT_FUSE_FORCE_ORDER sets the same at
 * dwt_fuse_create. */
dwt_fuse_status dwt_fuse_force_order(dwt_fuse_ctx *ctx, int order);

#ifdef __cplusplus
}
#endif
#endif
