// Stage 4 of the hot path: tilt displacement (Sec. 2.2 and 3.3).  The first
// two Zernike coefficients shift each pixel after the high-order blur: the
// output pixel (y, x) samples the blurred image at
// (y + s alpha_3(y,x), x + s alpha_2(y,x)), s = 2 q / pi pixels per unit tilt
// coefficient, by bilinear interpolation with the sample position clamped to
// the image.  Bandwidth bound: one thread per pixel, all channels per thread
// so the two tilt planes are read once.  The sample position is formed in
// FP64 so that its rounding does not grow with the pixel index.
#include "internal.hpp"

namespace p2s {
namespace {

// One 64 x 4 pixel block of one frame.
__device__ __forceinline__ void warp_block(const float* __restrict__ in, int C, int H, int W,
                                           const float* __restrict__ tilt, double scale, float* __restrict__ out,
                                           int bx, int by) {
    const int x = bx * 64 + (threadIdx.x & 63);
    const int y = by * 4 + (threadIdx.x >> 6);
    if (x >= W || y >= H) return;
    const size_t HW = (size_t)H * W;
    const size_t i = (size_t)y * W + x;
    // Sample position in FP64: in FP32 the rounding of x + d alone is
    // ulp(x) ~ 1e-5 px on large frames; the interpolation itself stays FP32.
    const double sx = fmin(fmax((double)x + scale * (double)tilt[i], 0.0), (double)(W - 1));
    const double sy = fmin(fmax((double)y + scale * (double)tilt[HW + i], 0.0), (double)(H - 1));
    const double fx0 = floor(sx), fy0 = floor(sy);
    const int xa = (int)fx0, ya = (int)fy0;
    const int xb = min(xa + 1, W - 1), yb = min(ya + 1, H - 1);
    const float fx = (float)(sx - fx0), fy = (float)(sy - fy0);
    for (int c = 0; c < C; ++c) {
        const float* p = in + c * HW;
        const float top = (1.0f - fx) * p[(size_t)ya * W + xa] + fx * p[(size_t)ya * W + xb];
        const float bot = (1.0f - fx) * p[(size_t)yb * W + xa] + fx * p[(size_t)yb * W + xb];
        out[c * HW + i] = (1.0f - fy) * top + fy * bot;
    }
}

__global__ void __launch_bounds__(256) warp_kernel(const float* __restrict__ in, int C, int H, int W,
                                                   const float* __restrict__ tilt, double scale,
                                                   float* __restrict__ out) {
    warp_block(in, C, H, W, tilt, scale, out, blockIdx.x, blockIdx.y);
}

// Batched, persistent form over the (frame, 64 x 4 block) list.
__global__ void __launch_bounds__(256) warp_batch(const FrameDesc* __restrict__ fr, const int* __restrict__ first,
                                                  int n, double scale) {
    const int total = first[n];
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int f = find_frame(first, n, item);
        const FrameDesc& d = fr[f];
        const int l = item - first[f];
        const int by = l / d.warp_tiles_x;
        warp_block(d.blurred, d.C, d.H, d.W, d.fields, scale, d.out, l - by * d.warp_tiles_x, by);
    }
}

}  // namespace

int warp_batch_resident() { return resident_workgroups((const void*)warp_batch, 256, 0); }

hipError_t launch_warp_batch(const BatchLaunch& bl, double scale, hipStream_t s) {
    if (bl.items[ST_WARP] == 0) return hipSuccess;
    hipLaunchKernelGGL(warp_batch, dim3(bl.grid[ST_WARP]), dim3(256), 0, s, bl.frames,
                       bl.first + ST_WARP * (bl.n + 1), bl.n, scale);
    return hipGetLastError();
}

hipError_t launch_warp(const float* in, int C, int H, int W, const float* tilt, double scale, float* out,
                       hipStream_t s) {
    dim3 grid((W + 63) / 64, (H + 3) / 4);
    hipLaunchKernelGGL(warp_kernel, grid, dim3(256), 0, s, in, C, H, W, tilt, scale, out);
    return hipGetLastError();
}

}  // namespace p2s
