// Quality diagnostics of fused bands against reference bands (for example the
// full-resolution truth of a synthetic scene): per band, the sum of squared
// differences and the sum of the reference, accumulated in FP64.
//
// The paper reports no quality metric it defines (section 4 names ERGAS and
// QNR without formulas); these two sums are what RMSE, the relative error and
// an ERGAS-style score need, and a one-wavefront kernel turns them into those
// numbers (in FP64, bands in order).
//
// Every pixel goes to a fixed thread of a fixed block (rows round-robin over
// the blocks of a band, columns strided over the threads, 4 adjacent pixels
// per thread on 16-byte aligned rows), and blocks and bands are combined by
// fixed reduction trees, so the sums are reproducible bit for bit.
// Memory-bound: 8 bytes read per pixel per band.
#include "fuse_internal.h"

namespace dwtf {
namespace {

__device__ __forceinline__ void block_sum2(double &a, double &b, double *sh) {
    const int t = threadIdx.x;
    sh[t] = a;
    sh[256 + t] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) {
            sh[t] += sh[t + s];
            sh[256 + t] += sh[256 + t + s];
        }
        __syncthreads();
    }
    a = sh[0];
    b = sh[256];
}

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void acc1(float fv, float rv, double &sse, double &sr) {
    const double r = (double)rv;
    const double d = (double)fv - r;
    sse = fma(d, d, sse);
    sr += r;
}

// VEC: rows 16-byte aligned with W a multiple of 4 -> 16-byte loads.
template <bool VEC>
__global__ __launch_bounds__(256) void quality_partial_kernel(QualityParams p, double *__restrict__ partial) {
    __shared__ double sh[512];
    const int b = blockIdx.y;
    const float *f = p.fused + (int64_t)b * p.f_bs;
    const float *r = p.ref + (int64_t)b * p.r_bs;
    double sse = 0.0, sr = 0.0;
    for (int y = blockIdx.x; y < p.H; y += gridDim.x) {
        const float *fr = f + (int64_t)y * p.f_ld;
        const float *rr = r + (int64_t)y * p.r_ld;
        if constexpr (VEC) {
            for (int x = 4 * threadIdx.x; x < p.W; x += 1024) {
                const f4 a = *reinterpret_cast<const f4 *>(fr + x);
                const f4 c = *reinterpret_cast<const f4 *>(rr + x);
                acc1(a.x, c.x, sse, sr);
                acc1(a.y, c.y, sse, sr);
                acc1(a.z, c.z, sse, sr);
                acc1(a.w, c.w, sse, sr);
            }
        } else {
            for (int x = threadIdx.x; x < p.W; x += 256) acc1(fr[x], rr[x], sse, sr);
        }
    }
    block_sum2(sse, sr, sh);
    if (threadIdx.x == 0) {
        double *o = partial + 2 * ((int64_t)b * gridDim.x + blockIdx.x);
        o[0] = sse;
        o[1] = sr;
    }
}

__global__ __launch_bounds__(256) void quality_final_kernel(const double *__restrict__ partial, int nblk, int B,
                                                            double *__restrict__ out) {
    __shared__ double sh[512];
    const int b = blockIdx.x;
    double sse = 0.0, sr = 0.0;
    for (int k = threadIdx.x; k < nblk; k += 256) {
        sse += partial[2 * ((int64_t)b * nblk + k)];
        sr += partial[2 * ((int64_t)b * nblk + k) + 1];
    }
    block_sum2(sse, sr, sh);
    if (threadIdx.x == 0) {
        out[b] = sse;
        out[B + b] = sr;
    }
}

// RMSE_b = sqrt(sse_b / n), mean_b = sum_b / n, and the ERGAS-style score
// 100 * (1/2) * sqrt(mean over b of (RMSE_b / mean_b)^2) (1:2 PAN:MS pixel
// size, section 2); a band with mean 0 makes the score +inf.  One thread,
// bands in order: the score is reproducible bit for bit.
__global__ __launch_bounds__(64) void quality_scores_kernel(double *__restrict__ out, int B, double n) {
    if (threadIdx.x != 0) return;
    double acc = 0.0;
    for (int b = 0; b < B; ++b) {
        const double rmse = sqrt(out[b] / n), mean = out[B + b] / n;
        out[2 * B + b] = rmse;
        out[3 * B + b] = mean;
        const double rel = rmse / mean;
        acc += mean != 0.0 ? rel * rel : __builtin_inf();
    }
    out[4 * B] = 100.0 * 0.5 * sqrt(acc / B);
}

}  // namespace

hipError_t launch_quality_scores(const QualityParams &p, double *partial, double *out, hipStream_t s) {
    hipError_t e = launch_quality(p, partial, out, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(quality_scores_kernel, dim3(1), dim3(64), 0, s, out, p.B, (double)p.H * (double)p.W);
    return hipGetLastError();
}

hipError_t launch_quality(const QualityParams &p, double *partial, double *out, hipStream_t s) {
    if (p.B < 1 || p.B > kQualityMaxBands || p.H < 1 || p.W < 1) return hipErrorInvalidValue;
    const auto al16 = [](const float *q, int64_t ld, int64_t bs, int B) {
        return reinterpret_cast<uintptr_t>(q) % 16 == 0 && ld % 4 == 0 && (B == 1 || bs % 4 == 0);
    };
    if (p.W % 4 == 0 && al16(p.fused, p.f_ld, p.f_bs, p.B) && al16(p.ref, p.r_ld, p.r_bs, p.B))
        hipLaunchKernelGGL(quality_partial_kernel<true>, dim3(kQualityBlocks, p.B), dim3(256), 0, s, p, partial);
    else
        hipLaunchKernelGGL(quality_partial_kernel<false>, dim3(kQualityBlocks, p.B), dim3(256), 0, s, p, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(quality_final_kernel, dim3(p.B), dim3(256), 0, s, partial, kQualityBlocks, p.B, out);
    return hipGetLastError();
}

}  // namespace dwtf
