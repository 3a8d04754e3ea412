// The paper's own GPU pipeline (section 3, the per-channel step list), kept
// as an in-repo comparator for the fused kernels: for every MS channel,
//   copy PAN into the working array,
//   1D forward DWT over the rows            (working -> scratch),
//   copy scratch -> working,
//   1D forward DWT over the columns         (working -> scratch),
//   replace the LL quadrant by the MS band  (in scratch),
//   copy scratch -> working,
//   1D inverse DWT over the columns         (working -> scratch),
//   copy scratch -> working,
//   1D inverse DWT over the rows            (working -> output band).
// Every pass reads and writes whole images; one thread per output element,
// as in the paper.  Haar: Eq. 1-2 / 11-12; D4: Eq. 3-6 / 13-16 with the
// periodic wrap, written as the pattern of taps per output element.
#include "fuse_internal.h"

namespace dwtf {
namespace {

// Forward 1D transform of a length-N line: output element i (0 <= i < N) is
// an approximation (i < N/2) or a detail coefficient.
__device__ __forceinline__ float fwd1(const float *s, int64_t stride, int N, int i, int wavelet, const Filters &f) {
    const int half = N >> 1;
    const bool det = i >= half;
    const int j = det ? i - half : i;
    if (wavelet == 0) {  // Eq. 1-2
        const float a = s[(int64_t)(2 * j) * stride], b = s[(int64_t)(2 * j + 1) * stride];
        return det ? (a - b) * 0.5f : (a + b) * 0.5f;
    }
    // Eq. 3-6: taps s_{(2j+k) mod N}; g_k = (-1)^k h_{3-k}
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int n = 2 * j + k;
        n -= (n >= N) ? N : 0;
        n -= (n >= N) ? N : 0;  // N = 2: index up to 2j+3 = 3
        const float c = det ? ((k & 1) ? -f.h[3 - k] : f.h[3 - k]) : f.h[k];
        acc = fmaf(c, s[(int64_t)n * stride], acc);
    }
    return acc;
}

// Inverse 1D transform: sample n from the coefficient line c ([a | d]).
__device__ __forceinline__ float inv1(const float *c, int64_t stride, int N, int n, int wavelet, const Filters &f) {
    const int half = N >> 1;
    if (wavelet == 0) {  // Eq. 11-12
        const int i = n >> 1;
        const float a = c[(int64_t)i * stride], d = c[(int64_t)(half + i) * stride];
        return (n & 1) ? a - d : a + d;
    }
    // Eq. 13-16: sample 2j+p gets a_j h_p + a_{j-1} h_{p+2} + d_j g_p + d_{j-1} g_{p+2} (indices mod N/2)
    const int p = n & 1, j = n >> 1;
    const int jm = (j == 0) ? half - 1 : j - 1;
    const float gp = p ? -f.h[2] : f.h[3];       // g_p     = (-1)^p h_{3-p}
    const float gp2 = p ? -f.h[0] : f.h[1];      // g_{p+2} = (-1)^p h_{1-p}
    float acc = c[(int64_t)j * stride] * f.h[p];
    acc = fmaf(c[(int64_t)jm * stride], f.h[p + 2], acc);
    acc = fmaf(c[(int64_t)(half + j) * stride], gp, acc);
    acc = fmaf(c[(int64_t)(half + jm) * stride], gp2, acc);
    return acc;
}

// dir 0: along rows (each row is a line of length W); dir 1: along columns.
__global__ __launch_bounds__(256) void pass_kernel(const float *__restrict__ in, int64_t in_ld, float *__restrict__ out,
                                                   int64_t out_ld, int H, int W, int dir, int inverse, int wavelet,
                                                   Filters f) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= W || y >= H) return;
    float v;
    if (dir == 0) {
        const float *line = in + (int64_t)y * in_ld;
        v = inverse ? inv1(line, 1, W, x, wavelet, f) : fwd1(line, 1, W, x, wavelet, f);
    } else {
        const float *line = in + x;
        v = inverse ? inv1(line, in_ld, H, y, wavelet, f) : fwd1(line, in_ld, H, y, wavelet, f);
    }
    out[(int64_t)y * out_ld + x] = v;
}

// LL quadrant <- MS band (section 2, step 2).
__global__ __launch_bounds__(256) void replace_kernel(float *__restrict__ X, int64_t ld, const float *__restrict__ ms,
                                                      int64_t ms_ld, int H2, int W2) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= W2 || y >= H2) return;
    X[(int64_t)y * ld + x] = ms[(int64_t)y * ms_ld + x];
}

}  // namespace

hipError_t launch_multipass(int wavelet, int H, int W, int B, const float *pan, int64_t pan_ld, const float *ms,
                            int64_t ms_ld, int64_t ms_bs, float *out, int64_t out_ld, int64_t out_bs, float *work,
                            float *scratch, const Filters &f, hipStream_t s) {
    const dim3 block(256);
    const dim3 grid((W + 255) / 256, H);
    const dim3 grid_ll((W / 2 + 255) / 256, H / 2);
    const size_t row_bytes = sizeof(float) * (size_t)W;
    hipError_t e;
    for (int b = 0; b < B; ++b) {
        // the PAN channel is loaded for every MS channel
        e = hipMemcpy2DAsync(work, row_bytes, pan, sizeof(float) * pan_ld, row_bytes, H, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(pass_kernel, grid, block, 0, s, work, (int64_t)W, scratch, (int64_t)W, H, W, 0, 0, wavelet, f);
        e = hipMemcpyAsync(work, scratch, row_bytes * H, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(pass_kernel, grid, block, 0, s, work, (int64_t)W, scratch, (int64_t)W, H, W, 1, 0, wavelet, f);
        hipLaunchKernelGGL(replace_kernel, grid_ll, block, 0, s, scratch, (int64_t)W, ms + (int64_t)b * ms_bs, ms_ld,
                           H / 2, W / 2);
        e = hipMemcpyAsync(work, scratch, row_bytes * H, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(pass_kernel, grid, block, 0, s, work, (int64_t)W, scratch, (int64_t)W, H, W, 1, 1, wavelet, f);
        e = hipMemcpyAsync(work, scratch, row_bytes * H, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(pass_kernel, grid, block, 0, s, work, (int64_t)W, out + (int64_t)b * out_bs, out_ld, H, W, 0, 1,
                           wavelet, f);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace dwtf
